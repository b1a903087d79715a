// Momentum-residual assembly: kernels and the lesasm_assemble_momentum_rhs entry.
//
// Algorithm 1, step "Element assembly", run once per Runge-Kutta stage:
// every element gathers its nodes, computes its residual at the Gauss points
// (Section 3.2, equation (momentum), EMAC + viscous + Vreman terms) and
// scatter-adds it into the nodal right-hand side (Section 3.4.3).  One launch
// per element category (type); in colour mode one launch per colour, so no two
// threads of a launch touch the same node and the scatter is a plain
// read-modify-write with a fixed summation order.
#include <algorithm>
#include <cmath>

#include "element.hpp"

namespace lesasm {

template <int T, typename R, bool ATOMIC, bool HAS_P>
__global__ __launch_bounds__(256) void k_assemble(CatView c, const double *__restrict__ xyz,
                                                  const double *__restrict__ u, const double *__restrict__ p,
                                                  double nu, double cv, double *__restrict__ rhs) {
    constexpr int nn = Ref<T>::nn;
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int local = b * blockDim.x + threadIdx.x;
    if (local >= c.n) return;
    const int e = c.off + local;
    ElementData<T, R> d;
    gather<T, R, HAS_P>(d, c, e, xyz, u, p);
    const double dl = c.delta[e];
    R acc[nn][3];
    element_residual<T, R, HAS_P>(d, (R)nu, (R)(cv * dl * dl), acc);
#pragma unroll
    for (int a = 0; a < nn; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double *dst = rhs + 3 * (size_t)d.fid[a] + i;
            if (ATOMIC)
                unsafeAtomicAdd(dst, (double)acc[a][i]);
            else
                *dst += (double)acc[a][i];
        }
}

// Chunked scatters (see chunk_body).  Workgroup w processes chunks w, w + G,
// w + 2G, ... of the G workgroups launched: one chunk each by default
// (G = number of chunks), several with a smaller grid.  The FP32 kernels also
// run in workgroups of 512 threads (see dispatch_chunks).
template <int T, typename R, bool HAS_P, bool PERIODIC, bool STAGED>
__global__ __launch_bounds__(sizeof(R) == 4 ? 512 : 256) void k_assemble_chunk(ChunkView c, int n_chunks, const double *__restrict__ xyz,
                                                        const double *__restrict__ u,
                                                        const double *__restrict__ p, double nu, double cv,
                                                        double *__restrict__ rhs) {
    extern __shared__ __align__(16) double lds[];
    for (int j = xcd_block(blockIdx.x, gridDim.x); j < n_chunks; j += gridDim.x) {
        chunk_body<T, R, HAS_P, PERIODIC, STAGED>(c, j, lds, xyz, u, p, nu, cv, rhs);
        __syncthreads();  // the next chunk's staging overwrites the LDS
    }
}

// The same with the learned closure (network weights after the node data in
// LDS), with a register budget of two wavefronts per SIMD (see mlp_passes).
template <int T, typename R, bool HAS_P, bool PERIODIC, bool STAGED>
__global__ __launch_bounds__(256, 2) void k_assemble_chunk_mlp(ChunkView c, const double *__restrict__ xyz,
                                                            const double *__restrict__ u,
                                                            const double *__restrict__ p, double nu, double cv,
                                                            double *__restrict__ rhs, ClosureView cl,
                                                            int lds_node_doubles) {
    extern __shared__ __align__(16) double lds[];
    chunk_body<T, R, HAS_P, PERIODIC, STAGED, true>(c, xcd_block(blockIdx.x, gridDim.x), lds, xyz, u, p, nu, cv,
                                                    rhs, &cl, lds_node_doubles);
}

// Staged scatter, second phase: every node owned by no chunk sums its staging
// rows (consecutive, in a fixed order: deterministic) and stores the result.
__global__ void k_gather_shared(const int32_t *__restrict__ gnode, const int32_t *__restrict__ goffs,
                                const double *__restrict__ stage, double *__restrict__ rhs, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // A shared node has two rows or more (a node of no element none): the
    // first two are loaded together, before the loop over the rest; the sum
    // still runs in row order.
    const int q0 = goffs[i], q1 = goffs[i + 1];
    const double *r = stage + 3 * (size_t)q0;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, b0 = 0.0, b1 = 0.0, b2 = 0.0;
    if (q1 > q0) a0 = r[0], a1 = r[1], a2 = r[2];
    if (q1 > q0 + 1) b0 = r[3], b1 = r[4], b2 = r[5];
    double s0 = a0 + b0, s1 = a1 + b1, s2 = a2 + b2;
    for (int q = q0 + 2; q < q1; ++q) {
        const double *row = stage + 3 * (size_t)q;
        s0 += row[0];
        s1 += row[1];
        s2 += row[2];
    }
    double *dst = rhs + 3 * (size_t)gnode[i];
    dst[0] = s0;
    dst[1] = s1;
    dst[2] = s2;
}

__global__ void k_fill(double *__restrict__ a, size_t n, double v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        a[i] = v;
}

// rhs <- dt * M_L^-1 rhs
__global__ void k_increment(double *__restrict__ rhs, const double *__restrict__ mass, double dt, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const double s = dt / mass[i];
        rhs[3 * i + 0] *= s;
        rhs[3 * i + 1] *= s;
        rhs[3 * i + 2] *= s;
    }
}

__global__ void k_check_finite(const double *__restrict__ a, size_t n, int *flag) {
    int bad = 0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        bad |= !isfinite(a[i]);
    if (bad) atomicOr(flag, 1);
}

int grid_for(size_t n, int block) {
    size_t g = (n + block - 1) / block;
    return (int)(g < 8192 ? (g ? g : 1) : 8192);
}

template <int T, typename R, bool ATOMIC, bool HAS_P>
static void launch_cat(const CatView &v, int block, hipStream_t s, const double *xyz, const double *u,
                       const double *p, double nu, double cv, double *rhs) {
    const int nb = (v.n + block - 1) / block;
    hipLaunchKernelGGL((k_assemble<T, R, ATOMIC, HAS_P>), dim3(nb), dim3(block), 0, s, v, xyz, u, p, nu, cv, rhs);
}

template <int T, typename R>
static void dispatch_scatter(const CatView &v, bool atomic, bool has_p, int block, hipStream_t s,
                             const double *xyz, const double *u, const double *p, double nu, double cv,
                             double *rhs) {
    if (atomic) {
        if (has_p) launch_cat<T, R, true, true>(v, block, s, xyz, u, p, nu, cv, rhs);
        else launch_cat<T, R, true, false>(v, block, s, xyz, u, p, nu, cv, rhs);
    } else {
        if (has_p) launch_cat<T, R, false, true>(v, block, s, xyz, u, p, nu, cv, rhs);
        else launch_cat<T, R, false, false>(v, block, s, xyz, u, p, nu, cv, rhs);
    }
}

template <int T, typename R, bool STAGED, bool HAS_P, bool PERIODIC>
static void launch_chunk_kernel(const ChunkView &v, int n_chunks, size_t shm, const ClosureView *cl, int block,
                                int persist, hipStream_t s, const double *xyz, const double *u, const double *p,
                                double nu, double cv, double *rhs) {
    const dim3 grid(n_chunks), blk(block);
    if (cl) {
        // network block after the node data, 16-byte aligned (vector reads of the biases)
        const size_t node_doubles = (shm / sizeof(double) + 1) & ~(size_t)1;
        const size_t shm_mlp = node_doubles * sizeof(double) + kMlpLdsBytes + (size_t)(block / 64) * kMlpWaveScratch;
        hipLaunchKernelGGL((k_assemble_chunk_mlp<T, R, HAS_P, PERIODIC, STAGED>), grid, blk, shm_mlp, s, v, xyz, u, p,
                           nu, cv, rhs, *cl, (int)node_doubles);
    } else {
        auto kern = k_assemble_chunk<T, R, HAS_P, PERIODIC, STAGED>;
        int g = n_chunks;
        if (persist > 0) {  // as many workgroups as the GPU holds at once (persist = n_cu), or at most -persist
            int per_cu = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, block, shm) == hipSuccess &&
                per_cu > 0)
                g = std::min(n_chunks, per_cu * persist);
            else
                (void)hipGetLastError();
        } else if (persist < 0) {
            g = std::min(n_chunks, -persist);
        }
        hipLaunchKernelGGL(kern, dim3(g), blk, shm, s, v, n_chunks, xyz, u, p, nu, cv, rhs);
    }
}

template <int T, typename R, bool STAGED>
static void launch_chunks(const ChunkView &v, int n_chunks, size_t shm, const ClosureView *cl, bool has_p,
                          bool periodic, int block, int persist, hipStream_t s, const double *xyz, const double *u,
                          const double *p, double nu, double cv, double *rhs) {
    if (periodic) {
        if (has_p) launch_chunk_kernel<T, R, STAGED, true, true>(v, n_chunks, shm, cl, block, persist, s, xyz, u, p, nu, cv, rhs);
        else launch_chunk_kernel<T, R, STAGED, false, true>(v, n_chunks, shm, cl, block, persist, s, xyz, u, p, nu, cv, rhs);
    } else {
        if (has_p) launch_chunk_kernel<T, R, STAGED, true, false>(v, n_chunks, shm, cl, block, persist, s, xyz, u, p, nu, cv, rhs);
        else launch_chunk_kernel<T, R, STAGED, false, false>(v, n_chunks, shm, cl, block, persist, s, xyz, u, p, nu, cv, rhs);
    }
}

template <typename R, bool STAGED>
static void dispatch_chunks(const Category &c, double *stage, const ClosureView *cl, bool has_p, bool periodic,
                            int block, int persist, hipStream_t s, const double *xyz, const double *u, const double *p, double nu,
                            double cv, double *rhs) {
    ChunkView v{c.d_eoff, c.d_goff, c.d_gnodes, c.d_foff, c.d_fnodes, c.d_fslot, c.d_lg, c.d_lf, c.d_delta, stage,
                (int32_t)c.n};
    const size_t shm = sizeof(double) * (size_t)c.lds_doubles;
    // Chunks longer than 512 elements hold up to 64 KB of node data, so a
    // compute unit keeps two of them: workgroups of 256 threads then cap the
    // FP32 kernels below the wavefronts their registers allow.  Those run in
    // workgroups of 512 threads (20 M hybrid box, FP32: PEN06 373 against 554
    // us, TET04 146 against 164).  Measured and not taken: 384 threads for the
    // FP32 HEX08 kernel (chunks of 512, three wavefronts per SIMD by its
    // registers), 551 against 352 us; 512 threads for the FP64 TET04 kernel,
    // 192 against 184 us.
    if (sizeof(R) == 4 && !cl && block == 256 && c.chunk_elems > 512) block = 512;
    switch (c.type) {
    case LESASM_TET04: launch_chunks<LESASM_TET04, R, STAGED>(v, c.n_chunks, shm, cl, has_p, periodic, block, persist, s, xyz, u, p, nu, cv, rhs); break;
    case LESASM_PYR05: launch_chunks<LESASM_PYR05, R, STAGED>(v, c.n_chunks, shm, cl, has_p, periodic, block, persist, s, xyz, u, p, nu, cv, rhs); break;
    case LESASM_PEN06: launch_chunks<LESASM_PEN06, R, STAGED>(v, c.n_chunks, shm, cl, has_p, periodic, block, persist, s, xyz, u, p, nu, cv, rhs); break;
    case LESASM_HEX08: launch_chunks<LESASM_HEX08, R, STAGED>(v, c.n_chunks, shm, cl, has_p, periodic, block, persist, s, xyz, u, p, nu, cv, rhs); break;
    }
}

ProfileScope::ProfileScope(lesasm_mesh *m_, int slot_, hipStream_t s_) : m(m_), slot(slot_), s(s_) {
    if (!m->profile) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        a = b = nullptr;
        return;
    }
    (void)hipEventRecord(a, s);
}

ProfileScope::~ProfileScope() {
    if (!a) return;
    (void)hipEventRecord(b, s);
    m->pending[slot].push_back({a, b});
}

template <typename R>
static void dispatch_type(int type, const CatView &v, bool atomic, bool has_p, int block, hipStream_t s,
                          const double *xyz, const double *u, const double *p, double nu, double cv, double *rhs) {
    switch (type) {
    case LESASM_TET04: dispatch_scatter<LESASM_TET04, R>(v, atomic, has_p, block, s, xyz, u, p, nu, cv, rhs); break;
    case LESASM_PYR05: dispatch_scatter<LESASM_PYR05, R>(v, atomic, has_p, block, s, xyz, u, p, nu, cv, rhs); break;
    case LESASM_PEN06: dispatch_scatter<LESASM_PEN06, R>(v, atomic, has_p, block, s, xyz, u, p, nu, cv, rhs); break;
    case LESASM_HEX08: dispatch_scatter<LESASM_HEX08, R>(v, atomic, has_p, block, s, xyz, u, p, nu, cv, rhs); break;
    }
}

// Launches every element kernel of one assembly on stream s (rhs already zeroed).
bool mesh_is_chunked(const lesasm_mesh *m) {
    return !(m->flags & (LESASM_MESH_SCATTER_COLOUR | LESASM_MESH_SCATTER_DIRECT));
}

bool mesh_is_staged(const lesasm_mesh *m) {
    return mesh_is_chunked(m) && !(m->flags & LESASM_MESH_SCATTER_CHUNK_ATOMIC);
}

// Shared nodes from which on the gather is split by class: below, one launch
// after the join (the overlap of a few microseconds would not pay for the
// extra launches of a small mesh).
constexpr int kSplitGather = 1 << 18;

// Gather of the staged rows of shared-node classes [c0, c1) (see gather_off) on s.
static void launch_gather(lesasm_mesh *m, int c0, int c1, double *rhs, hipStream_t s) {
    const int a = m->gather_off[c0], n = m->gather_off[c1] - a;
    if (n <= 0) return;
    ProfileScope ps(m, LESASM_KERNEL_GATHER, s);
    hipLaunchKernelGGL(k_gather_shared, dim3((n + 255) / 256), dim3(256), 0, s, m->d_gnode + a, m->d_goffs + a,
                       m->d_stage, rhs, n);
}

// Chunked scatters: the type kernels run concurrently, the first on the
// caller's stream and the others on the device's side streams (fork and join
// through events, so the sequence can be captured in a graph).  Staged, with
// at least kSplitGather shared nodes: the shared nodes whose rows come from one
// type only are gathered on that type's stream right after its kernel (the
// memory-bound gather overlaps the other types' arithmetic), the rest on the
// caller's stream after the join; fewer: all of them after the join.
static int launch_chunked(lesasm_mesh *m, const double *u, const double *p, double nu, double *rhs, hipStream_t s) {
    const bool staged = mesh_is_staged(m);
    ClosureView clv{};
    const ClosureView *cl = nullptr;
    if (m->mlp) {
        clv = ClosureView{mlp_packed(m->mlp), mlp_bias(m->mlp), std::log(m->delta_ref),
                          m->fallback_tol * m->fallback_tol, m->d_fallbacks};
        cl = &clv;
    }
    LESASM_HIP_TRY(hipEventRecord(m->ev_fork, s));
    int used = 0;
    // Launch order of the categories (the first on the caller's stream, the
    // others on the side streams): HEX08, TET04, PYR05, PEN06.  Measured on the
    // hybrid mix, the order sets how the concurrent kernels share the CUs:
    // this one 0.150 ms, TET04-PYR05-PEN06-HEX08 0.157, longest first 0.164.
    static constexpr int kLaunchOrder[kNumCat] = {3, 0, 1, 2};
    for (int kk = 0; kk < kNumCat; ++kk) {
        const int k = kLaunchOrder[kk];
        const Category &c = m->cat[k];
        if (c.n == 0) continue;
        hipStream_t sk = s;
        if (used > 0 && m->concurrent) {
            sk = m->side[(used - 1) % 3];
            if (used <= 3) LESASM_HIP_TRY(hipStreamWaitEvent(sk, m->ev_fork, 0));
        }
        ++used;
        {
            ProfileScope ps(m, LESASM_KERNEL_TET04 + k, sk);
            ClosureView clk{};
            if (cl) {  // fallback counters of this category
                clk = clv;
                clk.fallbacks = m->d_fallbacks + (size_t)k * kFallbackSlots;
                cl = &clk;
            }
            const bool periodic = c.d_lf != c.d_lg;
            const bool f32 = m->precision == LESASM_PREC_FP32;
            if (staged) {
                if (f32) dispatch_chunks<float, true>(c, m->d_stage, cl, p != nullptr, periodic, m->block, m->persist == 1 ? m->n_cu : -m->persist, sk, m->d_xyz, u, p, nu, m->vreman_c, rhs);
                else dispatch_chunks<double, true>(c, m->d_stage, cl, p != nullptr, periodic, m->block, m->persist == 1 ? m->n_cu : -m->persist, sk, m->d_xyz, u, p, nu, m->vreman_c, rhs);
            } else {
                if (f32) dispatch_chunks<float, false>(c, nullptr, cl, p != nullptr, periodic, m->block, m->persist == 1 ? m->n_cu : -m->persist, sk, m->d_xyz, u, p, nu, m->vreman_c, rhs);
                else dispatch_chunks<double, false>(c, nullptr, cl, p != nullptr, periodic, m->block, m->persist == 1 ? m->n_cu : -m->persist, sk, m->d_xyz, u, p, nu, m->vreman_c, rhs);
            }
        }
        if (staged && m->n_gather >= kSplitGather) launch_gather(m, k, k + 1, rhs, sk);
    }
    for (int i = 0; i < (m->concurrent ? std::min(used - 1, 3) : 0); ++i) {
        LESASM_HIP_TRY(hipEventRecord(m->ev_join[i], m->side[i]));
        LESASM_HIP_TRY(hipStreamWaitEvent(s, m->ev_join[i], 0));
    }
    if (staged) launch_gather(m, m->n_gather >= kSplitGather ? kNumCat : 0, kNumCat + 1, rhs, s);
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

int launch_assembly(lesasm_mesh *m, const double *u, const double *p, double nu, double *rhs, hipStream_t s) {
    const bool atomic = !(m->flags & LESASM_MESH_SCATTER_COLOUR);
    if (mesh_is_chunked(m)) return launch_chunked(m, u, p, nu, rhs, s);
    for (int k = 0; k < kNumCat; ++k) {
        const Category &c = m->cat[k];
        if (c.n == 0) continue;
        const size_t nranges = atomic ? 1 : c.colour_off.size() - 1;
        for (size_t r = 0; r < nranges; ++r) {
            CatView v;
            v.cg = c.d_cg;
            v.cf = c.d_cf;
            v.delta = c.d_delta;
            v.ld = (int32_t)c.n;
            v.off = atomic ? 0 : (int32_t)c.colour_off[r];
            v.n = atomic ? (int32_t)c.n : (int32_t)(c.colour_off[r + 1] - c.colour_off[r]);
            if (v.n == 0) continue;
            ProfileScope ps(m, LESASM_KERNEL_TET04 + k, s);
            if (m->precision == LESASM_PREC_FP32)
                dispatch_type<float>(c.type, v, atomic, p != nullptr, m->block, s, m->d_xyz, u, p, nu, m->vreman_c, rhs);
            else
                dispatch_type<double>(c.type, v, atomic, p != nullptr, m->block, s, m->d_xyz, u, p, nu, m->vreman_c, rhs);
        }
    }
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

// One assembly on stream s after argument checks: zero-fill (unless staged),
// element kernels, optional dt M_L^-1 scaling.
int assemble_into(lesasm_mesh *m, const double *u, const double *p, double nu, double dt, double *rhs, hipStream_t s,
                  bool increment) {
    if (m->n_field == 0) return LESASM_OK;
    const size_t n3 = 3 * (size_t)m->n_field;
    bool capturing = false;
    int st = mesh_order_begin(m, s, &capturing);
    if (st) return st;
    if (!mesh_is_staged(m)) {  // the staged scatter writes every node exactly once
        ProfileScope ps(m, LESASM_KERNEL_FILL, s);
        hipLaunchKernelGGL(k_fill, dim3(grid_for(n3, 256)), dim3(256), 0, s, rhs, n3, 0.0);
    }
    st = launch_assembly(m, u, p, nu, rhs, s);
    if (st) return st;
    if (increment) {
        ProfileScope ps(m, LESASM_KERNEL_INCREMENT, s);
        hipLaunchKernelGGL(k_increment, dim3(grid_for(m->n_field, 256)), dim3(256), 0, s, rhs, m->d_mass, dt,
                           (size_t)m->n_field);
    }
    LESASM_HIP_TRY(hipGetLastError());
    return mesh_order_end(m, s, capturing);
}

}  // namespace lesasm

using namespace lesasm;

static bool misaligned(const void *p) { return ((uintptr_t)p & 7u) != 0; }

extern "C" int lesasm_assemble_momentum_rhs(lesasm_mesh *m, const double *d_u, const double *d_p, double nu,
                                            double dt, double *d_rhs, void *stream) {
    if (!m) return fail(LESASM_E_INVALID_ARG, "assemble: mesh is NULL");
    if (m->n_field > 0 && (!d_u || !d_rhs)) return fail(LESASM_E_INVALID_ARG, "assemble: u or rhs is NULL");
    if (misaligned(d_u) || misaligned(d_p) || misaligned(d_rhs))
        return fail(LESASM_E_INVALID_ARG, "assemble: pointers must be 8-byte aligned");
    if (d_rhs && (d_rhs == d_u || (d_p && d_rhs == d_p)))
        return fail(LESASM_E_INVALID_ARG, "assemble: rhs aliases an input");
    int dev = -1;
    LESASM_HIP_TRY(hipGetDevice(&dev));
    if (dev != m->device) return fail(LESASM_E_STATE, "assemble: current device differs from the mesh's device");
    hipStream_t s = (hipStream_t)stream;
    if (m->n_field == 0) return LESASM_OK;
    const size_t n3 = 3 * (size_t)m->n_field;

    if (m->check_finite) {
        int zero = 0, flag = 0;
        LESASM_HIP_TRY(hipMemcpyAsync(m->d_flag, &zero, sizeof(int), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_check_finite, dim3(grid_for(n3, 256)), dim3(256), 0, s, d_u, n3, m->d_flag);
        if (d_p)
            hipLaunchKernelGGL(k_check_finite, dim3(grid_for(m->n_field, 256)), dim3(256), 0, s, d_p,
                               (size_t)m->n_field, m->d_flag);
        LESASM_HIP_TRY(hipMemcpyAsync(&flag, m->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
        LESASM_HIP_TRY(hipStreamSynchronize(s));
        if (flag) return fail(LESASM_E_NONFINITE, "assemble: u or p holds NaN/Inf");
    }

    return assemble_into(m, d_u, d_p, nu, dt, d_rhs, s, m->rhs_mode == LESASM_RHS_INCREMENT);
}

extern "C" int lesasm_mesh_kernel_times(lesasm_mesh *m, double *ms, int64_t *launches, int reset) {
    if (!m || !ms || !launches) return fail(LESASM_E_INVALID_ARG, "kernel_times: NULL argument");
    for (int k = 0; k < LESASM_NUM_KERNEL_SLOTS; ++k) {
        for (auto &ev : m->pending[k]) {
            float t = 0.0f;
            LESASM_HIP_TRY(hipEventSynchronize(ev.second));
            LESASM_HIP_TRY(hipEventElapsedTime(&t, ev.first, ev.second));
            m->prof_ms[k] += t;
            m->prof_n[k] += 1;
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
        m->pending[k].clear();
        ms[k] = m->prof_ms[k];
        launches[k] = m->prof_n[k];
        if (reset) {
            m->prof_ms[k] = 0.0;
            m->prof_n[k] = 0;
        }
    }
    return LESASM_OK;
}
