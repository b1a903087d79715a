// Internal definitions shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "lesasm.h"

struct lesasm_mesh;

namespace lesasm {

// Brackets one kernel launch with HIP events when the mesh profiles.
struct ProfileScope {
    lesasm_mesh *m;
    int slot;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    ProfileScope(lesasm_mesh *m_, int slot_, hipStream_t s_);
    ~ProfileScope();
};

// ---- error model: status code + thread-local message ----------------------
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

#define LESASM_HIP_TRY(expr)                                                                      \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return ::lesasm::fail(e_ == hipErrorOutOfMemory ? LESASM_E_OOM : LESASM_E_HIP,        \
                                  std::string(#expr) + ": " + hipGetErrorString(e_));             \
    } while (0)

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// Remap so that XCD x processes a contiguous run of element blocks, which
// keeps the nodes shared by neighbouring blocks in the same L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    constexpr int X = 8;
    const int q = nb / X, r = nb % X;
    const int x = b % X, slot = b / X;
    return x * q + (x < r ? x : r) + slot;
}

// ---- element categories ----------------------------------------------------
// Category slot k holds type kTypes[k] (the chunked path launches them in its own order).
constexpr int kNumCat = 4;
constexpr int kTypes[kNumCat] = {LESASM_TET04, LESASM_PYR05, LESASM_PEN06, LESASM_HEX08};

inline int cat_of_type(int t) {
    switch (t) {
    case LESASM_TET04: return 0;
    case LESASM_PYR05: return 1;
    case LESASM_PEN06: return 2;
    case LESASM_HEX08: return 3;
    default: return -1;
    }
}

struct Category {
    int type = 0;
    int64_t n = 0;                    // elements of this type
    int64_t first = 0;                // first internal element id of the category
    int32_t *d_cg = nullptr;          // geometry node ids, slot-major [nnode][n]
    int32_t *d_cf = nullptr;          // field node ids, slot-major (aliases d_cg if identical)
    double *d_delta = nullptr;        // filter width per element
    std::vector<int64_t> colour_off;  // colour c = elements [colour_off[c], colour_off[c+1])
    // chunked scatter: consecutive elements grouped so that their nodes fit in LDS
    int32_t n_chunks = 0;
    int32_t *d_eoff = nullptr;     // [n_chunks+1] element offsets within the category
    int32_t *d_goff = nullptr;     // [n_chunks+1] offsets into d_gnodes
    int32_t *d_gnodes = nullptr;   // geometry nodes of each chunk, ascending
    int32_t *d_foff = nullptr;     // [n_chunks+1] offsets into d_fnodes (aliases d_goff without a field map)
    int32_t *d_fnodes = nullptr;   // field nodes of each chunk; bit 31 set if the chunk owns the node
    uint16_t *d_lg = nullptr;      // [nnode][n] chunk-local geometry index of each element slot
    uint16_t *d_lf = nullptr;      // [nnode][n] chunk-local field index (aliases d_lg without a field map)
    int32_t *d_fslot = nullptr;    // per d_fnodes entry: staging slot of a shared node, -1 if owned
    int lds_doubles = 0;           // largest LDS footprint of a chunk, in doubles
    int chunk_elems = 0;           // chunk length used for this category
    std::vector<int32_t> h_cg, h_cf;  // host copies of the internal connectivity (slot-major)
    std::vector<int32_t> h_fnodes;    // host copy of d_fnodes
};

// Arguments of one chunked launch (one workgroup per chunk).
struct ChunkView {
    const int32_t *eoff, *goff, *gnodes, *foff, *fnodes, *fslot;
    const uint16_t *lg, *lf;
    const double *delta;
    double *stage;  // staging rows [slot][3] for shared nodes
    int32_t ld;     // elements in the category
};

constexpr uint32_t kOwnedBit = 0x80000000u;

const short *mlp_packed(const lesasm_mlp *p);
const float *mlp_bias(const lesasm_mlp *p);

// Device memory of the library: every allocation goes through these, which
// count the bytes held and refuse, with LESASM_E_OOM and before any HIP call,
// an allocation that would pass the cap of lesasm_set_memory_cap.
int device_alloc(void **p, size_t bytes, const char *what);
void device_free(void *p);

// Three side streams per device, shared by every mesh and batch on it
// (created on first use, kept until the process ends).
int device_side_streams(int device, hipStream_t out[3]);

// Ordering of calls that share a mesh's mutable state (staging rows, fork and
// join events, fallback counters) across streams: mesh_order_begin makes s
// wait for the previous call's last work when that ran on another stream;
// mesh_order_end records this call's end.  Neither does anything while s is
// capturing a graph (the graph's replays are ordered by their stream).
int mesh_order_begin(lesasm_mesh *m, hipStream_t s, bool *capturing);
int mesh_order_end(lesasm_mesh *m, hipStream_t s, bool capturing);

// Shared between translation units.
int grid_for(size_t n, int block);
int assemble_into(lesasm_mesh *m, const double *u, const double *p, double nu, double dt, double *rhs, hipStream_t s,
                  bool increment);
int launch_wall(lesasm_mesh *m, const double *u, double nu, double *rhs, hipStream_t s);

// Arguments of one assembly launch over a contiguous element range of a category.
struct CatView {
    const int32_t *cg;
    const int32_t *cf;
    const double *delta;
    int32_t ld;   // elements in the category (leading dimension of cg / cf)
    int32_t off;  // first element of the range
    int32_t n;    // elements in the range
};

}  // namespace lesasm

struct lesasm_mesh {
    int device = 0;
    uint32_t flags = 0;
    int64_t n_nodes = 0, n_field = 0, n_elems = 0;
    double vreman_c = 0.1;
    double *d_xyz = nullptr;      // [n_nodes][3], internal geometry order
    double *d_mass = nullptr;     // [n_field], internal field order
    int32_t *d_fperm = nullptr;   // internal -> user field node
    double *d_delta = nullptr;    // [n_elems] filter width, internal element order
    int *d_flag = nullptr;        // small status word for checks
    std::vector<int32_t> h_fperm;
    std::vector<int64_t> h_eperm;
    lesasm::Category cat[lesasm::kNumCat];
    std::vector<void *> allocs;
    uint64_t bytes = 0;
    // options
    int precision = LESASM_PREC_FP64;
    int rhs_mode = LESASM_RHS_RESIDUAL;
    int check_finite = 0;
    int block = 256;
    int profile = 0;
    int concurrent = 1;  // element-type kernels on forked streams
    int persist = 0;     // chunk kernels: 0 one workgroup per chunk, 1 resident workgroups, N > 1 at most N
    int n_cu = 0;        // compute units of the mesh's device
    int chunk_elems = 0;            // elements per chunk of the chunked scatter (0: per-type heuristic)
    std::vector<int32_t> h_finc;    // incidences per internal field node (all types)
    // staged scatter: shared nodes get one staging row per chunk touching them;
    // after the element kernels every non-owned node sums its rows (CSR below)
    double *d_stage = nullptr;      // [n_slots][3]
    int64_t n_slots = 0;
    int32_t n_gather = 0;           // field nodes owned by no chunk
    int32_t *d_gnode = nullptr;     // [n_gather] their ids
    int32_t *d_goffs = nullptr;     // [n_gather+1] first staging row of each shared node (rows consecutive)
    // the shared nodes grouped by the categories whose chunks wrote their rows:
    // class k < kNumCat holds rows of category k only (gathered on that
    // category's stream right after its kernel), class kNumCat the rest
    // (several categories, or no element), gathered after the join;
    // class c is [gather_off[c], gather_off[c+1]) of d_gnode
    int32_t gather_off[lesasm::kNumCat + 2] = {0};
    // side streams and events running the four type kernels concurrently
    hipStream_t side[3] = {nullptr, nullptr, nullptr};
    // learned closure (NULL: Vreman)
    const lesasm_mlp *mlp = nullptr;
    double delta_ref = 1.0, fallback_tol = 0.05;
    int chunk_max_nodes = 800;              // node cap of a chunk (LDS budget)
    unsigned long long *d_fallbacks = nullptr;  // kFallbackSlots counters
    hipEvent_t ev_fork = nullptr, ev_join[3] = {nullptr, nullptr, nullptr};
    // cross-stream ordering: the event marking the end of the last call that
    // used this mesh's state (the mesh's own ev_done, or its batch's), and the
    // stream it was recorded on
    hipEvent_t ev_done = nullptr;
    hipEvent_t order_ev = nullptr;
    hipStream_t order_stream = nullptr;
    // wall model (boundary assembly): per wall face, the nodes of the face and
    // of the volume element it bounds, in internal numbering
    std::vector<int32_t> h_gint, h_fint;  // user geometry node -> internal geometry / field node
    int64_t n_wall = 0;
    int32_t *d_wall_fg = nullptr;  // [n_wall][4] face nodes, geometry ids (-1 pads a triangle)
    int32_t *d_wall_ff = nullptr;  // [n_wall][4] face nodes, field ids
    int32_t *d_wall_eg = nullptr;  // [n_wall][8] element nodes, geometry ids (-1 pads)
    int32_t *d_wall_ef = nullptr;  // [n_wall][8] element nodes, field ids
    // profiling: events pending per kernel slot, accumulated times and counts
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[LESASM_NUM_KERNEL_SLOTS];
    double prof_ms[LESASM_NUM_KERNEL_SLOTS] = {0};
    int64_t prof_n[LESASM_NUM_KERNEL_SLOTS] = {0};
};
