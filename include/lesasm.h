/*
 * lesasm — explicit LES momentum-residual assembly on AMD Instinct MI355X.
 *
 * C ABI of the GPU library.  Every call returns an int status (LESASM_OK = 0,
 * negative on error), never throws and never aborts; lesasm_last_error()
 * gives the calling thread's last message.  Device pointers are plain
 * pointers from hipMalloc (or a PyTorch tensor's data_ptr()) on the device
 * that was current when the mesh was created; `stream` is a hipStream_t
 * (NULL = the legacy default stream).  All device work is asynchronous on
 * that stream and no call below synchronises the host unless it says so.
 *
 * What is computed follows Borrell et al., "Heterogeneous CPU/GPU
 * co-execution of CFD simulations on the POWER9 architecture" (FGCS 2020):
 *   - Section 3.2, equation (momentum): the filtered incompressible momentum
 *     equation with rho = 1, kinematic viscosity nu, the EMAC convective form
 *     C(u) = 2 eps(u) u + (div u) u with -|u|^2/2 folded into the modified
 *     pressure p, the viscous term div[2 nu eps(u)] and the subgrid term
 *     div(tau), tau = -2 nu_t eps(u), nu_t from Vreman's model.
 *   - Section 3.2 and Algorithm 1 (step "Element assembly"): Galerkin
 *     finite elements on linear hybrid meshes, assembled element by element.
 *   - Section 3.4.3 (gather, computation, scatter; elements grouped by type
 *     and integration rule into categories).
 * The residual of local node a of element e, component i, is
 *   R_ai = - sum_g w_g detJ_g [ N_a (C_i + dp/dx_i) + dN_a/dx_j 2 (nu + nu_t) eps_ij ]
 * and rhs[node] = sum over the elements touching it, so that M_L du/dt = rhs.
 *
 * Element types, reference nodes (node order of the connectivity) and rules:
 *   LESASM_TET04  (0,0,0) (1,0,0) (0,1,0) (0,0,1); 4-point degree-2 rule.
 *   LESASM_PYR05  (-1,-1,0) (1,-1,0) (1,1,0) (-1,1,0) (0,0,1); rational basis,
 *                 8-point conical product rule (Gauss-Legendre x Gauss-Jacobi).
 *   LESASM_PEN06  (0,0,-1) (1,0,-1) (0,1,-1) (0,0,1) (1,0,1) (0,1,1); 3 x 2 rule.
 *   LESASM_HEX08  (-1,-1,-1) (1,-1,-1) (1,1,-1) (-1,1,-1) then zeta=+1; 2x2x2 Gauss.
 * Filter width Delta_e = (element volume)^(1/3); lumped mass = row sums of
 * the consistent mass matrix (the mass-matrix listing of Section 3.4.3).
 */
#ifndef LESASM_H
#define LESASM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LESASM_VERSION 1

/* ---- status codes ------------------------------------------------------ */
#define LESASM_OK 0
#define LESASM_E_INVALID_ARG -1      /* null/misaligned pointer, bad size, type or index */
#define LESASM_E_INVERTED_ELEMENT -2 /* det J <= 0 at a Gauss point (user element id in message) */
#define LESASM_E_OOM -3              /* device allocation failed */
#define LESASM_E_HIP -4              /* a HIP runtime call failed (text in message) */
#define LESASM_E_STATE -5            /* wrong current device, or object in wrong state */
#define LESASM_E_NONFINITE -6        /* NaN/Inf found by the optional input check */
#define LESASM_E_UNSUPPORTED -7      /* option value not available */

/* ---- element types (value = number of nodes) --------------------------- */
#define LESASM_TET04 4
#define LESASM_PYR05 5
#define LESASM_PEN06 6
#define LESASM_HEX08 8

/* ---- mesh creation flags ----------------------------------------------- */
#define LESASM_MESH_SCATTER_STAGED 0u /* default: elements in chunks (one workgroup each) whose nodes
                                         are staged in LDS; residuals summed in LDS; nodes owned by
                                         the chunk are stored, shared ones written to per-chunk
                                         staging rows that a gather kernel sums (no global atomics) */
#define LESASM_MESH_SCATTER_COLOUR 1u /* greedy element colouring; one launch per colour, plain
                                         read-modify-write scatter, bitwise reproducible */
#define LESASM_MESH_KEEP_ORDER 2u     /* keep the user's element and node order within each type */
#define LESASM_MESH_SCATTER_DIRECT 4u /* one FP64 device atomic per element node and component
                                         (no LDS staging); kept for comparison */
#define LESASM_MESH_SCATTER_CHUNK_ATOMIC 8u /* chunks as in STAGED, shared nodes added with FP64
                                               device atomics instead of staging rows */

typedef struct lesasm_mesh lesasm_mesh;
typedef struct lesasm_mlp lesasm_mlp;

/* Host description of a mesh.  All arrays are host memory, read during
 * lesasm_mesh_create only (the library keeps its own device copies).
 *   n_nodes        geometry nodes; coords[n_nodes][3] (x, y, z).
 *   n_elems        elements; types[n_elems] in {4, 5, 6, 8}.
 *   conn_offsets   [n_elems + 1], conn_offsets[0] = 0, each span = node count.
 *   conn           geometry node ids, 0-based, element node order above.
 *   field_node     [n_nodes] or NULL: unknown (field) node of each geometry
 *                  node, in [0, n_field_nodes).  Periodic copies of a node map
 *                  to the same field node.  NULL means the identity and
 *                  n_field_nodes = n_nodes.
 *   vreman_c       Vreman constant c (nu_t = c sqrt(B_beta / alpha:alpha)).
 *   flags          LESASM_MESH_* bits.                                       */
typedef struct lesasm_mesh_desc {
    int64_t n_nodes;
    const double *coords;
    int64_t n_elems;
    const uint8_t *types;
    const int64_t *conn_offsets;
    const int32_t *conn;
    const int32_t *field_node;
    int64_t n_field_nodes;
    double vreman_c;
    uint32_t flags;
} lesasm_mesh_desc;

typedef struct lesasm_mesh_info {
    int64_t n_nodes;          /* geometry nodes */
    int64_t n_field_nodes;    /* unknowns per component */
    int64_t n_elems;
    int64_t n_per_type[4];    /* TET04, PYR05, PEN06, HEX08 */
    int32_t n_colours[4];     /* per type; 0 unless LESASM_MESH_SCATTER_COLOUR */
    int32_t device;           /* HIP device the mesh lives on */
    uint32_t flags;
    uint64_t device_bytes;    /* device memory owned by the mesh */
} lesasm_mesh_info;

/* Upload and preprocess a mesh on the current HIP device (Section 3.4.3:
 * elements are grouped by type into categories; within a category they are
 * sorted along a Morton curve of their centroids, and nodes are renumbered in
 * first-touch order of that element sequence).  Computes on the GPU, once:
 * det J at every Gauss point (must be > 0), Delta_e and the lumped mass.
 * Synchronises the device before returning.
 * Errors: LESASM_E_INVALID_ARG, LESASM_E_INVERTED_ELEMENT, LESASM_E_OOM,
 * LESASM_E_HIP.  On error *out is NULL and nothing is leaked.               */
int lesasm_mesh_create(const lesasm_mesh_desc *desc, lesasm_mesh **out);

/* Free a mesh and its device memory (synchronises its device).  NULL is a no-op. */
int lesasm_mesh_destroy(lesasm_mesh *mesh);

int lesasm_mesh_get_info(const lesasm_mesh *mesh, lesasm_mesh_info *info);

/* Field arrays passed to the assembly are in the mesh's INTERNAL node order.
 * perm[k] (host, n_field_nodes entries) = user field node of internal node k. */
int lesasm_mesh_node_permutation(const lesasm_mesh *mesh, int32_t *perm);

/* perm[k] (host, n_elems entries) = user element of internal element k. */
int lesasm_mesh_element_permutation(const lesasm_mesh *mesh, int64_t *perm);

/* Reorder a device field of ncomp doubles per node between user and internal
 * order (out-of-place; `in` and `out` must not overlap).
 *   to_internal: out[k][c] = in[perm[k]][c];  to_user: out[perm[k]][c] = in[k][c]. */
int lesasm_fields_to_internal(const lesasm_mesh *mesh, const double *d_user, double *d_internal,
                              int ncomp, void *stream);
int lesasm_fields_to_user(const lesasm_mesh *mesh, const double *d_internal, double *d_user,
                          int ncomp, void *stream);

/* Copy the row-sum lumped mass M_L[n_field_nodes] (internal order) into a
 * caller device buffer. */
int lesasm_mesh_lumped_mass(const lesasm_mesh *mesh, double *d_out, void *stream);

/* Copy Delta_e[n_elems] (internal element order) into a caller device buffer. */
int lesasm_mesh_filter_width(const lesasm_mesh *mesh, double *d_out, void *stream);

/* ---- per-mesh options used by lesasm_assemble_momentum_rhs ------------- */
#define LESASM_OPT_PRECISION 1    /* LESASM_PREC_FP64 (default) or LESASM_PREC_FP32 */
#define LESASM_OPT_RHS_MODE 2     /* LESASM_RHS_RESIDUAL (default) or LESASM_RHS_INCREMENT */
#define LESASM_OPT_CHECK_FINITE 3 /* 1: scan u and p for NaN/Inf first (synchronises) */
#define LESASM_OPT_BLOCK 4        /* threads per block of the assembly kernels: 64, 128 or 256
                                     (default); with 256, FP32 contractions of chunks longer than
                                     512 elements run in blocks of 512 */
#define LESASM_OPT_PROFILE 5      /* 1: record HIP events around every kernel launch */
#define LESASM_OPT_CHUNK 6        /* elements per chunk of the chunked scatters, 32..4096, or 0
                                     (default) for min(512, max(64, 2^floor(log2(n_type/256)))) per
                                     type, 1024 for TET04 and PEN06 when that leaves at least 4096
                                     chunks;
                                     setting it rebuilds the chunks (synchronises) */
#define LESASM_OPT_CONCURRENT 7   /* 1 (default): the element-type kernels of one chunked assembly run
                                     concurrently on forked streams (joined before return); 0: one
                                     after another on the caller's stream (isolated kernel timings) */
#define LESASM_OPT_PERSISTENT 8   /* 0 (default): one workgroup per chunk; 1: the chunk kernels launch
                                     as many workgroups as the GPU holds at once, each looping over
                                     chunks (measured slower: it blocks the concurrent type kernels);
                                     N > 1: at most N workgroups (testing) */

#define LESASM_PREC_FP64 0 /* whole element computation in FP64 */
#define LESASM_PREC_FP32 1 /* element contractions in FP32 on coefficients formed in FP64
                              (modal coefficients, or node-0-shifted values for TET04);
                              gather, nodal accumulation and output stay FP64 */
#define LESASM_RHS_RESIDUAL 0  /* d_rhs = rhs (right-hand side of M_L du/dt = rhs) */
#define LESASM_RHS_INCREMENT 1 /* d_rhs = dt * M_L^{-1} rhs */

int lesasm_mesh_set_option(lesasm_mesh *mesh, int option, int64_t value);
int lesasm_mesh_get_option(const lesasm_mesh *mesh, int option, int64_t *value);

/* One explicit momentum-residual assembly (Algorithm 1, "Element assembly",
 * once per Runge-Kutta stage):
 *   d_u    device [n_field_nodes][3] velocity, internal order, read only.
 *   d_p    device [n_field_nodes] modified pressure, or NULL to drop grad p.
 *   nu     kinematic viscosity.
 *   dt     time step; used only in LESASM_RHS_INCREMENT mode.
 *   d_rhs  device [n_field_nodes][3], overwritten (zero-filled on the stream
 *          first, then scatter-added).  Must not alias d_u or d_p.
 * Pointers must be 8-byte aligned.  Asynchronous on `stream`; a kernel fault
 * shows at the caller's next synchronisation.
 * Streams: calls on one mesh share its staging rows, events and counters.
 * When a call comes on another stream than the mesh's previous call (this
 * entry point, the stepper's, or a batch holding the mesh), the library makes
 * the new stream wait for the previous call's end, so such calls run one
 * after another in the order they were made.  Calls made while the stream is
 * capturing a graph are not ordered this way: replays of a captured call
 * must be ordered against other calls on the same mesh by the caller.
 * Errors: LESASM_E_INVALID_ARG, LESASM_E_STATE (current device differs from
 * the mesh's), LESASM_E_NONFINITE (only with LESASM_OPT_CHECK_FINITE),
 * LESASM_E_HIP (launch failure).                                            */
int lesasm_assemble_momentum_rhs(lesasm_mesh *mesh, const double *d_u, const double *d_p, double nu,
                                 double dt, double *d_rhs, void *stream);

/* Kernel slots reported by lesasm_mesh_kernel_times. */
#define LESASM_KERNEL_FILL 0      /* zero-fill of rhs */
#define LESASM_KERNEL_TET04 1     /* element kernels, one slot per type */
#define LESASM_KERNEL_PYR05 2
#define LESASM_KERNEL_PEN06 3
#define LESASM_KERNEL_HEX08 4
#define LESASM_KERNEL_INCREMENT 5 /* dt M_L^-1 scaling */
#define LESASM_KERNEL_GATHER 6    /* staged scatter: sums of the staging rows of shared nodes */
#define LESASM_NUM_KERNEL_SLOTS 7

/* Per-slot sums of kernel durations (milliseconds, from HIP events recorded on
 * the caller's stream while LESASM_OPT_PROFILE is 1) and launch counts since
 * the last reset.  In colour mode one launch per colour is counted.  Waits for
 * the recorded events (host synchronisation).  ms[] and launches[] are host
 * arrays of LESASM_NUM_KERNEL_SLOTS entries; reset != 0 clears the sums.     */
int lesasm_mesh_kernel_times(lesasm_mesh *mesh, double *ms, int64_t *launches, int reset);

/* ---- fractional-step support (Section 3.2, Algorithm 1) ----------------- */

/* Nodal divergence (D u)_a = int N_a div u dV, d_out[n_field_nodes] overwritten
 * (projection step of the fractional-step scheme).  Asynchronous. */
int lesasm_divergence(lesasm_mesh *mesh, const double *d_u, double *d_out, void *stream);

/* Nodal pressure gradient (G p)_a = int N_a grad p dV, d_out[n_field_nodes][3]
 * overwritten.  Asynchronous. */
int lesasm_gradient(lesasm_mesh *mesh, const double *d_p, double *d_out, void *stream);

typedef struct lesasm_stepper lesasm_stepper;

/* Time stepper of Algorithm 1 on a mesh (which must outlive it): assembles the
 * Laplacian K_ab = int grad N_a . grad N_b dV once (CSR on the device, plus a
 * sliced-ELLPACK copy for the CG's products, see lesasm_stepper_spmv), keeps
 * work vectors, and runs per step three explicit Runge-Kutta stages (Heun's
 * third-order tableau: c = (0, 1/3, 2/3), a21 = 1/3, a32 = 2/3,
 * b = (1/4, 0, 3/4)) and one pressure solve by Jacobi-preconditioned CG to
 * relative residual rtol (at most maxit iterations).  Synchronises. */
int lesasm_stepper_create(lesasm_mesh *mesh, double nu, double dt, double rtol, int maxit, lesasm_stepper **out);
int lesasm_stepper_destroy(lesasm_stepper *stepper);

/* One time step, in place on device arrays in internal order:
 *   u* = u^n + dt (k1/4 + 3 k3/4) with k_s = M_L^-1 rhs(u_s, p^n);
 *   K dp = -(1/dt) D u* (right-hand side projected to zero mean, dp zero mean);
 *   u^n+1 = u* - dt M_L^-1 G dp;  p^n+1 = p^n + dp.
 * The CG convergence test reads the residual on the host every few
 * iterations, so the call synchronises the stream. */
int lesasm_stepper_step(lesasm_stepper *stepper, double *d_u, double *d_p, void *stream);

/* The three explicit stages alone: d_ustar = u* for (d_u, d_p).  Asynchronous. */
int lesasm_stepper_rk3_stages(lesasm_stepper *stepper, const double *d_u, const double *d_p, double *d_ustar,
                              void *stream);

/* Mean-zero solution of K x = b - mean(b) by Jacobi-PCG.  Synchronises. */
int lesasm_pressure_solve(lesasm_stepper *stepper, const double *d_b, double *d_x, void *stream);

/* CG iterations and relative residual of the last pressure solve. */
int lesasm_stepper_stats(const lesasm_stepper *stepper, int *cg_iters, double *cg_rel_residual);

/* ---- step graph: one whole time step as a HIP graph ---------------------- */
/* Algorithm 1's time step (three Runge-Kutta stages with their element
 * assemblies, b = -(1/dt) D u*, the Jacobi-PCG pressure solve, u^n+1 =
 * u* - dt M_L^-1 G dp and p^n+1 = p^n + dp; Section 3.2's fractional step),
 * captured once on `stream` (not the default stream; synchronised first) and
 * replayed with no host synchronisation.  The CG is captured as exactly
 * cg_iters iterations (1..100000); its residual is tested on the device after
 * every iteration and the iterations after the one that met the stepper's
 * rtol return at once (a replay that needs more than cg_iters ends the step
 * with the unconverged solve: lesasm_step_graph_stats tells).  The eager step
 * tests every 16 iterations, so it may run up to 15 more.
 * Bound at creation to d_u [n_field_nodes][3] and d_p [n_field_nodes]
 * (internal order, caller-owned, updated in place by every replay) and to the
 * stepper's work arrays: the stepper and mesh must outlive the graph, and
 * replays must not overlap other calls on the same stepper or mesh.  Errors:
 * LESASM_E_INVALID_ARG (NULL, cg_iters out of range, default stream),
 * LESASM_E_STATE (wrong device, stream already capturing), LESASM_E_OOM,
 * LESASM_E_HIP (capture or instantiation failed). */
typedef struct lesasm_step_graph lesasm_step_graph;
int lesasm_step_graph_create(lesasm_stepper *stepper, double *d_u, double *d_p, int cg_iters,
                             lesasm_step_graph **out, void *stream);

/* Replay on `stream` (asynchronous).  d_u and d_p must be the pointers given
 * at creation, else LESASM_E_STATE. */
int lesasm_step_graph_launch(lesasm_step_graph *graph, double *d_u, double *d_p, void *stream);

/* CG iterations run, relative residual and whether it met rtol, for the last
 * replay (waits for it).  LESASM_E_STATE before the first replay. */
int lesasm_step_graph_stats(lesasm_step_graph *graph, int *cg_iters, double *cg_rel_residual, int *converged);

/* Waits for the last replay, then frees the graph. */
int lesasm_step_graph_destroy(lesasm_step_graph *graph);

/* Copy the assembled Laplacian to host arrays (rowptr[n_field_nodes+1],
 * col[nnz], val[nnz], any of them may be NULL); *nnz receives the count. */
int lesasm_stepper_laplacian(lesasm_stepper *stepper, int32_t *rowptr, int32_t *col, double *val, int64_t *nnz);

/* q = K p with the Laplacian above, by the kernel the pressure CG runs (a
 * sliced-ELLPACK copy of K: slices of 64 consecutive rows, each padded to its
 * longest row and stored column-major; the CSR form if that copy would exceed
 * 2^31 entries).  d_p and d_q are device arrays of n_field_nodes doubles in
 * internal order, must not alias (LESASM_E_INVALID_ARG).  Asynchronous on
 * `stream`; the stepper's reduction buffer is written, so calls must not
 * overlap a pressure solve or step of the same stepper. */
int lesasm_stepper_spmv(lesasm_stepper *stepper, const double *d_p, double *d_q, void *stream);

/* Stored entries of the sliced-ELLPACK copy of K (nonzeros plus padding; 0 if
 * the CSR form serves the CG). */
int lesasm_stepper_sell_entries(const lesasm_stepper *stepper, int64_t *entries);

/* ---- batches of mesh partitions ---------------------------------------- */

typedef struct lesasm_batch lesasm_batch;

#define LESASM_ORDER_MESH 0          /* work queue in mesh, type, chunk order */
#define LESASM_ORDER_LARGEST_FIRST 1 /* chunks by decreasing cost (elements x Gauss points) */
#define LESASM_ORDER_INTERLEAVED 2   /* round-robin over meshes */

/* Group 1..64 non-periodic meshes with the staged scatter (the meshes must
 * outlive the batch and live on the current device).  Work items are
 * (mesh, type, chunk) triples in a device queue; one persistent launch of a
 * grid of grid_per_cu workgroups per compute unit drains it (Section 3.4.3:
 * packs of elements of one category, here pulled from a queue instead of one
 * kernel per pack).  Synchronises. */
int lesasm_batch_create(lesasm_mesh *const *meshes, int n, lesasm_batch **out);
int lesasm_batch_destroy(lesasm_batch *batch);

/* Chunk length (0 = each mesh's default), queue order and workgroups per
 * compute unit; rebuilds chunks and the queue (synchronises). */
int lesasm_batch_configure(lesasm_batch *batch, int chunk, int order, int grid_per_cu);
int lesasm_batch_get_config(const lesasm_batch *batch, int *chunk, int *order, int *grid_per_cu, int *n_items);

/* Kernel layout of the batch: 0 (default) one persistent kernel drains the
 * whole queue, switching on the element type of each item; 1 the queue is
 * ordered type by type (the chosen order kept inside each type) and four
 * persistent kernels, one per element type (each compiled, and resident, for
 * its own type), drain their parts concurrently on forked streams; 2 the same
 * type-ordered queue and four kernels, but one workgroup per item, scheduled
 * by the hardware (no queue counter; grid_per_cu does not apply).  Rebuilds
 * the queue (synchronises).  Errors: LESASM_E_INVALID_ARG, LESASM_E_UNSUPPORTED
 * (a value other than 0, 1 or 2). */
int lesasm_batch_set_per_type(lesasm_batch *batch, int per_type);
int lesasm_batch_get_per_type(const lesasm_batch *batch, int *per_type);

/* Residual assembly of every mesh: host arrays of n device pointers
 * d_u[i] ([n_field_nodes_i][3]), d_p[i] (or d_p == NULL for none), nu[i],
 * d_rhs[i] (overwritten).  Same semantics as lesasm_assemble_momentum_rhs per
 * mesh (residual mode); all meshes use the first mesh's precision option.
 * Asynchronous: one small set-up kernel, the element kernel(s) and the
 * gathers of shared nodes (in the per-type layouts, the nodes of one type
 * only are gathered on that type's stream after its kernel).  A batch shares its members' staging rows: a call on
 * another stream than the previous call on the batch or on any member waits
 * for that call's end (as for lesasm_assemble_momentum_rhs). */
int lesasm_batch_assemble(lesasm_batch *batch, const double *const *d_u, const double *const *d_p,
                          const double *nu, double *const *d_rhs, void *stream);

/* Autotuner: times the batched assembly for chunk lengths {each mesh's own
 * per-type lengths, 128, 256, 512, 1024} x the three queue orders x {2, 4} workgroups per compute unit x the
 * three kernel layouts (the third without a grid size; median of `reps` runs
 * after one warm-up) and keeps the fastest.  With a cache_path, a line "signature chunk order grid per_type
 * ms" is looked up first
 * (signature = compute units and element counts per mesh and type) and
 * appended after tuning.  *best_ms receives the time.  Synchronises. */
int lesasm_batch_tune(lesasm_batch *batch, const double *const *d_u, const double *const *d_p, const double *nu,
                      double *const *d_rhs, const char *cache_path, int reps, double *best_ms);

/* Three explicit Runge-Kutta stages of every mesh, in place on d_u[i] with
 * d_p[i] fixed (Heun's third-order tableau, no pressure projection):
 * k1 = dt M^-1 rhs(u), u2 = u + k1/3, k2 = dt M^-1 rhs(u2), u3 = u + 2 k2/3,
 * k3 = dt M^-1 rhs(u3), u <- u + k1/4 + 3 k3/4.
 *   _graph captures the sequence on `stream` (must not be NULL) into a HIP
 *   graph bound to these pointers (a graph captured before is destroyed
 *   after its last replay has finished); _launch replays it (one host call
 *   per step, ordered against other streams as lesasm_batch_assemble);
 *   _eager runs the same sequence without a graph. */
int lesasm_batch_rk3_graph(lesasm_batch *batch, double *const *d_u, const double *const *d_p, const double *nu,
                           double dt, void *stream);
int lesasm_batch_rk3_launch(lesasm_batch *batch, void *stream);
int lesasm_batch_rk3_eager(lesasm_batch *batch, double *const *d_u, const double *const *d_p, const double *nu,
                           double dt, void *stream);

/* ---- learned subgrid closure -------------------------------------------- */
/* A 10-64-64-6 perceptron replaces Vreman's subgrid stress at the Gauss
 * points (the subgrid term div(tau) of Section 3.2's momentum equation; the
 * paper itself uses Vreman).  Inputs x = [G/|G|_F (9, row-major du_i/dx_j),
 * log(Delta_e/Delta_ref)]; h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2),
 * y = h2 W3 + b3 with components (xx, yy, zz, xy, xz, yz); the stress is
 * tau = Delta_e^2 |G|_F^2 dev(y).  Parameters: 5254 floats in the order
 * W1[10][64], b1[64], W2[64][64], b2[64], W3[64][6], b3[6].               */
#define LESASM_MLP_PARAMS 5254

/* Device copy of the parameters (FP32 master), Adam moments, and the packed
 * BF16 matrix-core operands used by inference.  `params` is host memory. */
int lesasm_mlp_create(const float *params, lesasm_mlp **out);
int lesasm_mlp_destroy(lesasm_mlp *mlp);
int lesasm_mlp_get_params(const lesasm_mlp *mlp, float *params);
/* Replace the parameters (host array), reset Adam, repack (synchronises). */
int lesasm_mlp_set_params(lesasm_mlp *mlp, const float *params);

/* Training, FP32 on the device.  d_x [n][10] inputs, d_t [n][6] targets for
 * dev(y).  Loss L = (1/n) sum w_c (dev(y) - t)_c^2, w = (1,1,1,2,2,2).
 * loss_grad writes dL/dparams to d_grad[5254] (or an internal buffer if NULL)
 * and L to *d_loss (device float, may be NULL); adam applies one step
 * (beta1 0.9, beta2 0.999, eps 1e-8) with the given or internal gradient;
 * train_step = loss_grad + adam.  Asynchronous.  After training, call
 * lesasm_mlp_commit to refresh the BF16 inference copy (synchronises). */
int lesasm_mlp_loss_grad(lesasm_mlp *mlp, const float *d_x, const float *d_t, int n, float *d_grad, float *d_loss,
                         void *stream);
/* lesasm_mlp_loss_grad without any device allocation, for callers that
 * cannot allocate (code under HIP graph capture, serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, kernels and results (bit for bit)
 * as lesasm_mlp_loss_grad, but the work arrays sit in a static device area of
 * 8192 samples (8.6 MB, held by each device the library runs on until the
 * process ends): n > 8192 gives LESASM_E_INVALID_ARG and nothing runs.  The
 * area's address is looked up on the first call on each device.  Every call
 * on one device shares that area: calls that overlap on one device (two
 * streams, or two threads) race and must be ordered by the caller. */
int lesasm_mlp_loss_grad_noalloc(lesasm_mlp *mlp, const float *d_x, const float *d_t, int n, float *d_grad,
                                 float *d_loss, void *stream);
int lesasm_mlp_adam(lesasm_mlp *mlp, const float *d_grad, float lr, void *stream);
int lesasm_mlp_train_step(lesasm_mlp *mlp, const float *d_x, const float *d_t, int n, float lr, float *d_loss,
                          void *stream);
int lesasm_mlp_commit(lesasm_mlp *mlp);

/* Inference of y (before the trace removal) for n samples, d_y [n][6]:
 * _f32 with the FP32 master weights, _bf16 with the matrix-core path the
 * assembly uses (BF16 operands, FP32 sums).  Asynchronous. */
int lesasm_mlp_forward_f32(lesasm_mlp *mlp, const float *d_x, int n, float *d_y, void *stream);
int lesasm_mlp_infer_bf16(lesasm_mlp *mlp, const float *d_x, int n, float *d_y, void *stream);

/* Use the network as the subgrid closure of a mesh (mlp = NULL restores
 * Vreman).  Per element both closures are integrated; the network's residual
 * is kept unless |R_mlp - R_vreman|_2 > fallback_tol |R_vreman|_2 (element
 * vectors), in which case Vreman's is used.  Chunked scatters only; the mlp
 * must outlive its use.  Rebuilds the chunks (synchronises). */
int lesasm_mesh_set_closure(lesasm_mesh *mesh, const lesasm_mlp *mlp, double delta_ref, double fallback_tol);

/* Number of elements that fell back to Vreman since the last call (resets;
 * synchronises). */
int lesasm_mesh_closure_fallbacks(lesasm_mesh *mesh, uint64_t *count);

/* The same per element type: counts[4] in the order TET04, PYR05, PEN06,
 * HEX08 (resets every count; synchronises). */
int lesasm_mesh_closure_fallbacks_by_type(lesasm_mesh *mesh, uint64_t *counts);

/* ---- wall model (boundary assembly) ------------------------------------ */
/* Algorithm 1, "Boundary assembly"; Section 3.2 names a law-of-the-wall
 * model without its formulas.  An equilibrium wall model: for each wall face,
 * the velocity at the vertex average of the face's volume element (the mean
 * of its nodal velocities) and that point's distance y to the face plane give,
 * through Reichardt's law U/u_tau = f(y u_tau/nu) (kappa 0.41, C1 7.8,
 * chi 11), the friction velocity; the traction -u_tau^2 u_t/|u_t| (u_t the
 * tangential part of the velocity) is added to the face nodes, weighted by the
 * face integrals of their shape functions. */
typedef struct lesasm_wall_desc {
    int64_t n_faces;              /* 0 removes the wall */
    const int64_t *face_offsets;  /* host [n_faces+1], face_offsets[0] = 0; 3 or 4 nodes per face */
    const int32_t *face_conn;     /* host, user geometry node ids of each face, as a cycle */
    const int64_t *face_elem;     /* host [n_faces], user id of the volume element the face bounds */
} lesasm_wall_desc;

/* Copies the wall faces (replacing any previous set); host arrays are not
 * retained.  Synchronises.
 * Errors: LESASM_E_INVALID_ARG (NULL, a face of neither 3 nor 4 nodes, node or
 * element out of range), LESASM_E_STATE (wrong device), LESASM_E_OOM,
 * LESASM_E_HIP. */
int lesasm_mesh_set_wall(lesasm_mesh *mesh, const lesasm_wall_desc *desc);

/* d_rhs[n_field][3] += wall-model contributions for velocity d_u[n_field][3]
 * (internal order, device, 8-byte aligned, rhs not aliasing u), kinematic
 * viscosity nu > 0.  Asynchronous on `stream`; a no-op without wall faces.
 * Faces that share a node add with FP64 atomics (summation order varies).
 * Errors: LESASM_E_INVALID_ARG, LESASM_E_STATE, LESASM_E_HIP. */
int lesasm_assemble_wall(lesasm_mesh *mesh, const double *d_u, double nu, double *d_rhs, void *stream);

/* ---- SFC mesh partitioning and load balancing ---------------------------- */
/* Section "Mesh partitioning and load balancing".  The partitioner takes one
 * location per element (the mean of its node coordinates) and optional
 * integer weights (the paper's cost model: one unit per Gauss point), bins the
 * locations on a regular 2^level grid over their bounding box, orders the bins
 * along a Hilbert curve (Skilling's transposed-index construction: bits from
 * the most significant level down, x before y before z) and cuts the weighted
 * curve: bin b, with weight w_b and weight S_b before it on the curve, goes to
 * the part i whose target interval [T_{i-1}, T_i) holds its midpoint
 * S_b + w_b / 2, where T_i = (lambda_1 + ... + lambda_i) W / P (W the total
 * weight, lambda the correction coefficients, all 1 without correction); an
 * element takes the part of its bin.  The bin of a coordinate c on an axis
 * with bounds [lo, hi] is floor((c - lo) / (hi - lo) 2^level), clamped to
 * 2^level - 1 (0 on a flat axis).  Parts are contiguous along the curve; the
 * cumulative weight of parts 0 .. i-1 is within half the largest bin weight
 * of T_i. */

/* d_centroids[n_elems][3] = mean of each element's node coordinates (nodes
 * summed in connectivity order, then divided by their count) and
 * d_weights[n_elems] = its Gauss points (4 nodes: 4, 5: 8, 6: 6, 8: 8).
 * Inputs on the device: d_conn_offsets int64 [n_elems+1] (d_conn_offsets[0]
 * = 0), d_conn int32 [conn_len] node ids, d_coords [n_nodes][3].  d_weights
 * may be NULL.  d_status is a caller-owned device int32 that the call never
 * clears: 1 is OR-ed into it for an element whose node count is not 4, 5, 6
 * or 8 or whose nodes lie outside d_conn, 2 for a node id out of range; such
 * an element's outputs are left unwritten.  Asynchronous on `stream`; read
 * d_status after the stream has finished.
 * Errors: LESASM_E_INVALID_ARG (NULL, negative size), LESASM_E_HIP. */
int lesasm_element_centroids(int64_t n_elems, const int64_t *d_conn_offsets, const int32_t *d_conn, int64_t conn_len,
                             int64_t n_nodes, const double *d_coords, double *d_centroids, int32_t *d_weights,
                             int32_t *d_status, void *stream);

/* Bytes of device workspace lesasm_sfc_partition needs for these sizes
 * (level 1 .. 8, n_parts >= 1).  Errors: LESASM_E_INVALID_ARG. */
int lesasm_sfc_workspace_bytes(int64_t n_elems, int n_parts, int level, size_t *bytes);

/* d_part[n_elems] (int32, device) = part of every element, as described
 * above.  d_centroids [n_elems][3] device, finite; d_weights device int32
 * >= 0 or NULL (weight 1 each); h_lambda host [n_parts] finite, >= 0, or
 * NULL (all 1) -- the sum should be n_parts (the last part takes what the
 * others leave); level 1 .. 8 (8^level bins); d_work a caller-owned device
 * buffer of at least lesasm_sfc_workspace_bytes(), 256-byte aligned.  The
 * total weight must stay below 2^53.  Asynchronous on `stream` (h_lambda is
 * read before the call returns: up to 256 coefficients travel with the
 * launch; with more, the call copies them and waits for the stream); the
 * result is integer arithmetic after the binning, so it does not depend on
 * the launch.  Errors: LESASM_E_INVALID_ARG, LESASM_E_HIP. */
int lesasm_sfc_partition(int64_t n_elems, const double *d_centroids, const int32_t *d_weights, int n_parts,
                         const double *h_lambda, int level, void *d_work, size_t work_bytes, int32_t *d_part,
                         void *stream);

/* Correction coefficients for the next partition from the history of
 * iterations 0 .. n_obs-1 (host arrays, row k = iteration k):
 * h_lambda_hist[n_obs][n_parts] the coefficients used, h_time_hist the
 * measured time of every part.  Per splitting point i = 1 .. n_parts-1 a
 * linear regression of the observations (Lambda_i^k, Upsilon_i^k), with
 * Lambda_i^k = lambda_1^k + ... + lambda_i^k and Upsilon_i^k the time of the
 * first i parts over the mean part time, weighted by growth^k (growth 1: the
 * simple regression; 1.5: the weighted one, each newer observation weighing
 * 50 % more), cut with y = i gives Lambda_i; lambda_out[i] = Lambda_{i+1} -
 * Lambda_i with Lambda_0 = 0, Lambda_P = P.  With a single observation, a
 * spread of Lambda_i below 1e-12 P, or a slope <= 0, the line through the
 * origin and the newest observation is used instead; Lambda is clamped to be
 * non-decreasing within [0, P].  Host only, no device work.
 * Errors: LESASM_E_INVALID_ARG (NULL, n_parts < 1, n_obs < 1, growth <= 0,
 * a coefficient < 0 or not finite, a time < 0 or not finite, or a zero mean
 * time). */
int lesasm_balance_update(int n_parts, int n_obs, const double *h_lambda_hist, const double *h_time_hist,
                          double growth, double *h_lambda_out);

/* Waits for all work queued on `stream` (a hipStream_t; NULL = the null
 * stream) and reports what the asynchronous calls could not: a failed kernel
 * or copy surfaces here as LESASM_E_HIP with the runtime's text.
 * Errors: LESASM_E_HIP. */
int lesasm_check(void *stream);

/* Text of the calling thread's last error ("" if none). */
const char *lesasm_last_error(void);

/* Cap on the device memory this library allocates (meshes, batches,
 * steppers, networks, step graphs; summed over devices), in bytes; 0 removes
 * the cap (the default).  An allocation that would pass it fails with
 * LESASM_E_OOM before any HIP call, and the call that needed it returns that
 * error with nothing created (for tests of the out-of-memory paths and for
 * budgeting).  Caller-supplied buffers are not counted.  Thread-safe. */
int lesasm_set_memory_cap(uint64_t bytes);

/* Device bytes the library holds now (all devices).  Thread-safe. */
int lesasm_memory_in_use(uint64_t *bytes);

int lesasm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LESASM_H */
