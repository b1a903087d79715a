// Batched assembly of many mesh partitions in one persistent launch.
//
// The paper packs elements of one category into large packs and runs one
// kernel per pack on several streams (Section 3.4.3 and Section 5: pack size,
// threads per block and the number of streams tuned by hand).  Here every
// (mesh, element type, chunk) triple of a batch is one item of a device work
// queue; a grid sized to fill the GPU pulls items with an atomic counter until
// the queue is empty, so uneven partitions need no per-mesh launches.  Chunk
// length and queue order are set by an autotuner.  A three-stage Runge-Kutta
// update of all meshes can be captured into a HIP graph and replayed with one
// host call.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <numeric>
#include <sstream>

#include "element.hpp"

namespace lesasm {

constexpr int kMaxBatch = 64;

// Static description of one (mesh, type) pair.
struct BatchEntry {
    ChunkView v;           // chunk arrays of the type (stage pointer = the mesh's staging rows)
    const double *xyz;
    double cv;             // Vreman constant
    int type;
    int mesh;
};

// Per-call pointers of every mesh (written on the device by k_batch_begin).
struct BatchCall {
    const double *u[kMaxBatch];
    const double *p[kMaxBatch];
    double *rhs[kMaxBatch];
    double nu[kMaxBatch];
};

// Per-mesh arrays for the gather and update kernels.
struct BatchMeshDev {
    const int32_t *gnode, *goffs;
    const double *stage, *mass;
};

constexpr int kHeads = 1 + kNumCat;  // the mixed queue's counter, then one per type

__global__ void k_batch_begin(BatchCall args, BatchCall *dst, int *head) {
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) *dst = args;
        if (threadIdx.x < kHeads) head[threadIdx.x] = 0;
    }
}

template <typename R, bool HAS_P>
__device__ __forceinline__ void batch_item(const BatchEntry &be, const BatchCall *call, int chunk, double *lds) {
    const int mi = be.mesh;
    const double *u = call->u[mi];
    const double *p = HAS_P ? call->p[mi] : nullptr;
    double *rhs = call->rhs[mi];
    const double nu = call->nu[mi];
    switch (be.type) {
    case LESASM_TET04: chunk_body<LESASM_TET04, R, HAS_P, false, true>(be.v, chunk, lds, be.xyz, u, p, nu, be.cv, rhs); break;
    case LESASM_PYR05: chunk_body<LESASM_PYR05, R, HAS_P, false, true>(be.v, chunk, lds, be.xyz, u, p, nu, be.cv, rhs); break;
    case LESASM_PEN06: chunk_body<LESASM_PEN06, R, HAS_P, false, true>(be.v, chunk, lds, be.xyz, u, p, nu, be.cv, rhs); break;
    case LESASM_HEX08: chunk_body<LESASM_HEX08, R, HAS_P, false, true>(be.v, chunk, lds, be.xyz, u, p, nu, be.cv, rhs); break;
    }
}

// Persistent element kernel: each workgroup takes queue items until the
// counter passes the end of the queue (every workgroup reaches that exit).
template <typename R, bool HAS_P>
__global__ __launch_bounds__(256) void k_batch_assemble(const BatchEntry *__restrict__ entries,
                                                        const BatchCall *__restrict__ call,
                                                        const int32_t *__restrict__ wentry,
                                                        const int32_t *__restrict__ wchunk, int nwork, int *head) {
    extern __shared__ __align__(16) double lds[];
    __shared__ int item;
    for (;;) {
        if (threadIdx.x == 0) item = atomicAdd(head, 1);
        __syncthreads();
        const int w = item;
        __syncthreads();
        if (w >= nwork) return;
        batch_item<R, HAS_P>(entries[wentry[w]], call, wchunk[w], lds);
        __syncthreads();
    }
}

// Per-type kernel: the same walk over the items of one element type only, so
// each type is compiled (and occupies registers) on its own and the four run
// concurrently.  PERSISTENT: a grid sized to fill the GPU pulls items from the
// type's counter; otherwise one workgroup per item (item order remapped so
// that each XCD takes a contiguous run), scheduled by the hardware.
template <int T, typename R, bool HAS_P, bool PERSISTENT>
__global__ __launch_bounds__(256) void k_batch_assemble_type(const BatchEntry *__restrict__ entries,
                                                             const BatchCall *__restrict__ call,
                                                             const int32_t *__restrict__ wentry,
                                                             const int32_t *__restrict__ wchunk, int nwork, int *head) {
    extern __shared__ __align__(16) double lds[];
    __shared__ int item;
    for (;;) {
        int w;
        if constexpr (PERSISTENT) {
            if (threadIdx.x == 0) item = atomicAdd(head, 1);
            __syncthreads();
            w = item;
            __syncthreads();
        } else {
            w = xcd_block(blockIdx.x, gridDim.x);
        }
        if (w >= nwork) return;
        const BatchEntry &be = entries[wentry[w]];
        const int mi = be.mesh;
        chunk_body<T, R, HAS_P, false, true>(be.v, wchunk[w], lds, be.xyz, call->u[mi], HAS_P ? call->p[mi] : nullptr,
                                             call->nu[mi], be.cv, call->rhs[mi]);
        if constexpr (!PERSISTENT) return;
        __syncthreads();
    }
}

// A block of at most 256 consecutive nodes of one mesh: the gather and update
// kernels give each workgroup one, so that the mesh index, and every pointer
// read through it, is uniform over the workgroup (scalar loads, no search).
struct BatchBlock {
    int32_t mesh, first, end;  // node range [first, end) of the mesh's list
};
constexpr int kBatchBlock = 256;

// Shared nodes of every mesh: sum of staging rows (fixed order).  One class
// of shared nodes at a time (blocks over the meshes' d_gnode ranges of that
// class), or all of them.
__global__ __launch_bounds__(kBatchBlock) void k_batch_gather(const BatchMeshDev *__restrict__ md,
                                                               const BatchCall *__restrict__ call,
                                                               const BatchBlock *__restrict__ blk) {
    const BatchBlock bk = blk[blockIdx.x];
    const int k = bk.first + (int)threadIdx.x;
    if (k >= bk.end) return;
    const BatchMeshDev d = md[bk.mesh];
    // as k_gather_shared: the first two rows loaded together, summed in row order
    const int q0 = d.goffs[k], q1 = d.goffs[k + 1];
    const double *r = d.stage + 3 * (size_t)q0;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, b0 = 0.0, b1 = 0.0, b2 = 0.0;
    if (q1 > q0) a0 = r[0], a1 = r[1], a2 = r[2];
    if (q1 > q0 + 1) b0 = r[3], b1 = r[4], b2 = r[5];
    double s0 = a0 + b0, s1 = a1 + b1, s2 = a2 + b2;
    for (int q = q0 + 2; q < q1; ++q) {
        const double *row = d.stage + 3 * (size_t)q;
        s0 += row[0];
        s1 += row[1];
        s2 += row[2];
    }
    double *dst = call->rhs[bk.mesh] + 3 * (size_t)d.gnode[k];
    dst[0] = s0;
    dst[1] = s1;
    dst[2] = s2;
}

// Runge-Kutta update over all meshes' nodes (blocks of one mesh each):
//   kout = dt M^-1 rhs (in place in rhs), then y = base + a1 k1 + a2 kout.
struct UpdateArgs {
    const double *base[kMaxBatch];
    double *rhs[kMaxBatch];  // stage residual, scaled in place to dt M^-1 rhs
    const double *k1[kMaxBatch];
    double *y[kMaxBatch];
    double a1, a2, dt;
};

__global__ __launch_bounds__(kBatchBlock) void k_batch_update(UpdateArgs a, const BatchMeshDev *__restrict__ md,
                                                               const BatchBlock *__restrict__ blk) {
    const BatchBlock bk = blk[blockIdx.x];
    const int mi = bk.mesh;
    const size_t k = (size_t)bk.first + threadIdx.x;
    if (k >= (size_t)bk.end) return;
    const double s = a.dt / md[mi].mass[k];
    double *rhs = a.rhs[mi], *y = a.y[mi];
    const double *base = a.base[mi], *k1 = a.k1[mi];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double kv = s * rhs[3 * k + c];
        rhs[3 * k + c] = kv;
        double v = base[3 * k + c] + a.a2 * kv;
        if (k1) v += a.a1 * k1[3 * k + c];
        y[3 * k + c] = v;
    }
}

}  // namespace lesasm

using namespace lesasm;

struct lesasm_batch {
    int device = 0;
    std::vector<lesasm_mesh *> meshes;
    int chunk = 0;   // 0: each mesh's own default
    int order = 0;   // LESASM_ORDER_*
    int grid_per_cu = 2;
    int n_cu = 256;
    // device tables
    BatchEntry *d_entries = nullptr;
    BatchCall *d_call = nullptr;
    BatchMeshDev *d_md = nullptr;
    // node blocks (BatchBlock): row c < kNumCat + 1 the shared-node class c of
    // every mesh (the meshes' gather_off), row kNumCat + 1 every class at once,
    // row kNumCat + 2 every field node (the Runge-Kutta update); row r holds
    // blocks [blk_off[r], blk_off[r + 1]) of d_blk
    BatchBlock *d_blk = nullptr;
    int blk_off[kNumCat + 4] = {0};
    int64_t class_gather[kNumCat + 2] = {0};
    int32_t *d_wentry = nullptr, *d_wchunk = nullptr;
    int *d_head = nullptr;
    int nwork = 0, lds_doubles = 0;
    // per-type mode: the queue is type-major, type category k holds items
    // [type_off[k], type_off[k+1]) and needs type_lds[k] doubles of LDS
    int per_type = 0;
    int type_off[kNumCat + 1] = {0};
    int type_lds[kNumCat] = {0};
    hipStream_t side[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev_fork = nullptr, ev_join[3] = {nullptr, nullptr, nullptr};
    int64_t total_gather = 0, total_nodes = 0;
    std::vector<void *> allocs;
    // Runge-Kutta work arrays (one slab each, per-mesh offsets) and the graph
    double *k1 = nullptr, *k3 = nullptr, *us = nullptr;
    std::vector<int64_t> node_off;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double last_tune_ms = 0.0;
    // end of the last assembly or replay (cross-stream ordering with the
    // member meshes, and the wait before an executable graph is destroyed)
    hipEvent_t ev_done = nullptr;
    bool done_recorded = false;
};

namespace {

template <class T> int balloc(lesasm_batch *b, T **p, size_t n) {
    *p = nullptr;
    if (!n) return LESASM_OK;
    void *q = nullptr;
    int st = device_alloc(&q, n * sizeof(T), "batch");
    if (st) return st;
    b->allocs.push_back(q);
    *p = (T *)q;
    return LESASM_OK;
}

template <class T> void bfree(lesasm_batch *b, T *&p) {
    if (!p) return;
    auto it = std::find(b->allocs.begin(), b->allocs.end(), (void *)p);
    if (it != b->allocs.end()) {
        device_free(p);
        b->allocs.erase(it);
    }
    p = nullptr;
}

void batch_free(lesasm_batch *b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    for (int i = 0; i < 3; ++i)  // (the side streams are the device's)
        if (b->ev_join[i]) (void)hipEventDestroy(b->ev_join[i]);
    if (b->ev_done) {
        for (lesasm_mesh *m : b->meshes)  // the members outlive the batch
            if (m->order_ev == b->ev_done) m->order_ev = nullptr;
        (void)hipEventDestroy(b->ev_done);
    }
    for (void *p : b->allocs) device_free(p);
    delete b;
}

// Cross-stream ordering of a batch call with earlier calls on its member
// meshes (which share their staging rows with the batch) and on the batch
// itself; nothing while s is capturing.
int batch_order_begin(lesasm_batch *b, hipStream_t s, bool *capturing) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    LESASM_HIP_TRY(hipStreamIsCapturing(s, &cs));
    *capturing = cs != hipStreamCaptureStatusNone;
    if (*capturing) return LESASM_OK;
    hipEvent_t last = nullptr;
    for (lesasm_mesh *m : b->meshes)
        if (m->order_ev && m->order_stream != s && m->order_ev != last) {
            LESASM_HIP_TRY(hipStreamWaitEvent(s, m->order_ev, 0));
            last = m->order_ev;
        }
    return LESASM_OK;
}

int batch_order_end(lesasm_batch *b, hipStream_t s, bool capturing) {
    if (capturing) return LESASM_OK;
    LESASM_HIP_TRY(hipEventRecord(b->ev_done, s));
    b->done_recorded = true;
    for (lesasm_mesh *m : b->meshes) {
        m->order_ev = b->ev_done;
        m->order_stream = s;
    }
    return LESASM_OK;
}

// Destroys the captured Runge-Kutta graph after its last replay has finished.
void drop_graph(lesasm_batch *b) {
    if (!b->graph_exec && !b->graph) return;
    if (b->done_recorded) (void)hipEventSynchronize(b->ev_done);
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->graph_exec = nullptr;
    b->graph = nullptr;
}

// Work items ordered by the queue policy.  Cost of a chunk = elements x Gauss
// points of its type (the paper's per-element weight is its number of Gauss
// points).
int build_work(lesasm_batch *b) {
    struct Item {
        int32_t entry, chunk;
        int64_t cost;
        int mesh, cat;
    };
    std::vector<Item> items;
    std::vector<BatchEntry> entries;
    int lds = 0;
    for (int k = 0; k < kNumCat; ++k) b->type_lds[k] = 0;
    for (size_t mi = 0; mi < b->meshes.size(); ++mi) {
        lesasm_mesh *m = b->meshes[mi];
        for (int k = 0; k < kNumCat; ++k) {
            Category &c = m->cat[k];
            if (c.n == 0) continue;
            std::vector<int32_t> eoff(c.n_chunks + 1);
            LESASM_HIP_TRY(hipMemcpy(eoff.data(), c.d_eoff, sizeof(int32_t) * eoff.size(), hipMemcpyDeviceToHost));
            const int ng = c.type == LESASM_TET04 ? 4 : (c.type == LESASM_PEN06 ? 6 : 8);
            const int eid = (int)entries.size();
            BatchEntry be;
            be.v = ChunkView{c.d_eoff, c.d_goff, c.d_gnodes, c.d_foff, c.d_fnodes, c.d_fslot, c.d_lg, c.d_lf,
                             c.d_delta, m->d_stage, (int32_t)c.n};
            be.xyz = m->d_xyz;
            be.cv = m->vreman_c;
            be.type = c.type;
            be.mesh = (int)mi;
            entries.push_back(be);
            lds = std::max(lds, c.lds_doubles);
            b->type_lds[k] = std::max(b->type_lds[k], c.lds_doubles);
            for (int j = 0; j < c.n_chunks; ++j)
                items.push_back({eid, j, (int64_t)(eoff[j + 1] - eoff[j]) * ng, (int)mi, k});
        }
    }
    if (b->order == LESASM_ORDER_LARGEST_FIRST) {
        std::stable_sort(items.begin(), items.end(), [](const Item &x, const Item &y) { return x.cost > y.cost; });
    } else if (b->order == LESASM_ORDER_INTERLEAVED) {
        // round-robin over meshes: the r-th chunk of every mesh, then the (r+1)-th ...
        std::vector<std::vector<Item>> per(b->meshes.size());
        for (const Item &it : items) per[it.mesh].push_back(it);
        items.clear();
        for (size_t r = 0;; ++r) {
            bool any = false;
            for (auto &v : per)
                if (r < v.size()) {
                    items.push_back(v[r]);
                    any = true;
                }
            if (!any) break;
        }
    }
    // per-type mode: the same order inside each type, types one after another
    if (b->per_type)
        std::stable_sort(items.begin(), items.end(), [](const Item &x, const Item &y) { return x.cat < y.cat; });
    for (int k = 0; k <= kNumCat; ++k) b->type_off[k] = 0;
    for (const Item &it : items) b->type_off[it.cat + 1]++;
    for (int k = 0; k < kNumCat; ++k) b->type_off[k + 1] += b->type_off[k];
    std::vector<int32_t> we(items.size()), wc(items.size());
    for (size_t i = 0; i < items.size(); ++i) {
        we[i] = items[i].entry;
        wc[i] = items[i].chunk;
    }
    bfree(b, b->d_entries);
    bfree(b, b->d_wentry);
    bfree(b, b->d_wchunk);
    int st;
    if ((st = balloc(b, &b->d_entries, entries.size())) || (st = balloc(b, &b->d_wentry, we.size())) ||
        (st = balloc(b, &b->d_wchunk, wc.size())))
        return st;
    if (!entries.empty())
        LESASM_HIP_TRY(hipMemcpy(b->d_entries, entries.data(), sizeof(BatchEntry) * entries.size(), hipMemcpyHostToDevice));
    if (!we.empty()) {
        LESASM_HIP_TRY(hipMemcpy(b->d_wentry, we.data(), sizeof(int32_t) * we.size(), hipMemcpyHostToDevice));
        LESASM_HIP_TRY(hipMemcpy(b->d_wchunk, wc.data(), sizeof(int32_t) * wc.size(), hipMemcpyHostToDevice));
    }
    b->nwork = (int)items.size();
    b->lds_doubles = lds;
    return LESASM_OK;
}

int build_tables(lesasm_batch *b) {
    const int n = (int)b->meshes.size();
    constexpr int R = kNumCat + 3;  // rows: the classes, all classes, all field nodes
    std::vector<BatchMeshDev> md(n);
    std::vector<BatchBlock> blk;
    std::vector<int64_t> np(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        lesasm_mesh *m = b->meshes[i];
        md[i] = BatchMeshDev{m->d_gnode, m->d_goffs, m->d_stage, m->d_mass};
        np[i + 1] = np[i] + m->n_field;
    }
    for (int c = 0; c < R; ++c) {
        b->blk_off[c] = (int)blk.size();
        int64_t count = 0;
        for (int i = 0; i < n; ++i) {
            const lesasm_mesh *m = b->meshes[i];
            const int64_t a = c <= kNumCat ? m->gather_off[c] : 0;
            const int64_t e = c <= kNumCat ? m->gather_off[c + 1] : c == kNumCat + 1 ? m->n_gather : m->n_field;
            for (int64_t f = a; f < e; f += kBatchBlock)
                blk.push_back(BatchBlock{i, (int32_t)f, (int32_t)std::min(e, f + kBatchBlock)});
            count += e - a;
        }
        if (c < kNumCat + 2) b->class_gather[c] = count;
        if (blk.size() > (size_t)INT32_MAX) return fail(LESASM_E_UNSUPPORTED, "batch: too many node blocks");
    }
    b->blk_off[R] = (int)blk.size();
    b->total_gather = b->class_gather[kNumCat + 1];
    b->total_nodes = np[n];
    b->node_off = np;
    bfree(b, b->d_md);
    bfree(b, b->d_blk);
    int st;
    if ((st = balloc(b, &b->d_md, (size_t)n)) || (st = balloc(b, &b->d_blk, std::max<size_t>(blk.size(), 1))))
        return st;
    LESASM_HIP_TRY(hipMemcpy(b->d_md, md.data(), sizeof(BatchMeshDev) * n, hipMemcpyHostToDevice));
    if (!blk.empty())
        LESASM_HIP_TRY(hipMemcpy(b->d_blk, blk.data(), sizeof(BatchBlock) * blk.size(), hipMemcpyHostToDevice));
    return LESASM_OK;
}

// Gather of shared-node class c (kNumCat + 1: every class) of every mesh on s.
void launch_batch_gather(lesasm_batch *b, int c, hipStream_t s) {
    const int nb = b->blk_off[c + 1] - b->blk_off[c];
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_batch_gather, dim3((unsigned)nb), dim3(kBatchBlock), 0, s, b->d_md, b->d_call,
                       b->d_blk + b->blk_off[c]);
}

int rebuild(lesasm_batch *b) {
    for (lesasm_mesh *m : b->meshes) {
        if (m->chunk_elems == b->chunk) continue;  // chunks already of this length
        int st = lesasm_mesh_set_option(m, LESASM_OPT_CHUNK, b->chunk);
        if (st) return st;
    }
    int st;
    if ((st = build_tables(b))) return st;
    if ((st = build_work(b))) return st;
    drop_graph(b);  // chunk arrays moved: an instantiated graph is stale
    return LESASM_OK;
}

// Launch of the whole batch assembly (begin, persistent kernel, gather) on s.
template <int T>
void launch_type(lesasm_batch *b, int k, bool has_p, bool fp32, hipStream_t s) {
    const int n = b->type_off[k + 1] - b->type_off[k];
    if (n <= 0) return;
    const bool persistent = b->per_type == 1;
    // persistent: a grid that fills the GPU; else one workgroup per item
    const int grid = persistent ? std::max(1, std::min(n, b->n_cu * b->grid_per_cu)) : n;
    const size_t shm = sizeof(double) * (size_t)b->type_lds[k];
    const int32_t *we = b->d_wentry + b->type_off[k], *wc = b->d_wchunk + b->type_off[k];
    int *head = b->d_head + 1 + k;
#define LESASM_BATCH_TYPE_LAUNCH(RR, HP, PS)                                                                          \
    hipLaunchKernelGGL((k_batch_assemble_type<T, RR, HP, PS>), dim3(grid), dim3(256), shm, s, b->d_entries, b->d_call, \
                       we, wc, n, head)
    if (persistent) {
        if (fp32) {
            if (has_p) LESASM_BATCH_TYPE_LAUNCH(float, true, true);
            else LESASM_BATCH_TYPE_LAUNCH(float, false, true);
        } else {
            if (has_p) LESASM_BATCH_TYPE_LAUNCH(double, true, true);
            else LESASM_BATCH_TYPE_LAUNCH(double, false, true);
        }
    } else {
        if (fp32) {
            if (has_p) LESASM_BATCH_TYPE_LAUNCH(float, true, false);
            else LESASM_BATCH_TYPE_LAUNCH(float, false, false);
        } else {
            if (has_p) LESASM_BATCH_TYPE_LAUNCH(double, true, false);
            else LESASM_BATCH_TYPE_LAUNCH(double, false, false);
        }
    }
#undef LESASM_BATCH_TYPE_LAUNCH
}

int batch_launch(lesasm_batch *b, const BatchCall &call, bool has_p, bool fp32, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_begin, dim3(1), dim3(64), 0, s, call, b->d_call, b->d_head);
    const int grid = std::max(1, std::min(b->nwork, b->n_cu * b->grid_per_cu));
    const size_t shm = sizeof(double) * (size_t)b->lds_doubles;
    if (b->per_type && b->nwork > 0) {
        // the four type kernels on forked streams (order as the single-mesh
        // path: HEX08, TET04, PYR05, PEN06), joined before the gather
        LESASM_HIP_TRY(hipEventRecord(b->ev_fork, s));
        static constexpr int kOrder[kNumCat] = {3, 0, 1, 2};
        int used = 0;
        for (int kk = 0; kk < kNumCat; ++kk) {
            const int k = kOrder[kk];
            if (b->type_off[k + 1] == b->type_off[k]) continue;
            hipStream_t sk = s;
            if (used > 0) {
                sk = b->side[used - 1];
                LESASM_HIP_TRY(hipStreamWaitEvent(sk, b->ev_fork, 0));
            }
            ++used;
            switch (kTypes[k]) {
            case LESASM_TET04: launch_type<LESASM_TET04>(b, k, has_p, fp32, sk); break;
            case LESASM_PYR05: launch_type<LESASM_PYR05>(b, k, has_p, fp32, sk); break;
            case LESASM_PEN06: launch_type<LESASM_PEN06>(b, k, has_p, fp32, sk); break;
            case LESASM_HEX08: launch_type<LESASM_HEX08>(b, k, has_p, fp32, sk); break;
            }
            // the shared nodes of this type only, behind its kernel on its stream
            launch_batch_gather(b, k, sk);
        }
        for (int i = 0; i + 1 < used; ++i) {
            LESASM_HIP_TRY(hipEventRecord(b->ev_join[i], b->side[i]));
            LESASM_HIP_TRY(hipStreamWaitEvent(s, b->ev_join[i], 0));
        }
        launch_batch_gather(b, kNumCat, s);  // nodes of several types, or of none
    } else if (b->nwork > 0) {
        if (fp32) {
            if (has_p) hipLaunchKernelGGL((k_batch_assemble<float, true>), dim3(grid), dim3(256), shm, s, b->d_entries, b->d_call, b->d_wentry, b->d_wchunk, b->nwork, b->d_head);
            else hipLaunchKernelGGL((k_batch_assemble<float, false>), dim3(grid), dim3(256), shm, s, b->d_entries, b->d_call, b->d_wentry, b->d_wchunk, b->nwork, b->d_head);
        } else {
            if (has_p) hipLaunchKernelGGL((k_batch_assemble<double, true>), dim3(grid), dim3(256), shm, s, b->d_entries, b->d_call, b->d_wentry, b->d_wchunk, b->nwork, b->d_head);
            else hipLaunchKernelGGL((k_batch_assemble<double, false>), dim3(grid), dim3(256), shm, s, b->d_entries, b->d_call, b->d_wentry, b->d_wchunk, b->nwork, b->d_head);
        }
    }
    if (!(b->per_type && b->nwork > 0)) launch_batch_gather(b, kNumCat + 1, s);
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

int make_call(lesasm_batch *b, const double *const *u, const double *const *p, const double *nu,
              double *const *rhs, BatchCall &call) {
    std::memset(&call, 0, sizeof(call));
    for (size_t i = 0; i < b->meshes.size(); ++i) {
        if (!u[i] || !rhs[i]) return fail(LESASM_E_INVALID_ARG, "batch: NULL u or rhs pointer");
        call.u[i] = u[i];
        call.p[i] = p ? p[i] : nullptr;
        call.rhs[i] = rhs[i];
        call.nu[i] = nu[i];
        if (p && !p[i]) return fail(LESASM_E_INVALID_ARG, "batch: p must be given for all meshes or none");
    }
    return LESASM_OK;
}

}  // namespace

extern "C" int lesasm_batch_create(lesasm_mesh *const *meshes, int n, lesasm_batch **out) {
    if (!out) return fail(LESASM_E_INVALID_ARG, "batch_create: out is NULL");
    *out = nullptr;
    if (!meshes || n < 1 || n > kMaxBatch)
        return fail(LESASM_E_INVALID_ARG, "batch_create: need 1.." + std::to_string(kMaxBatch) + " meshes");
    int dev = -1;
    LESASM_HIP_TRY(hipGetDevice(&dev));
    for (int i = 0; i < n; ++i) {
        const lesasm_mesh *m = meshes[i];
        if (!m) return fail(LESASM_E_INVALID_ARG, "batch_create: NULL mesh");
        if (m->device != dev) return fail(LESASM_E_STATE, "batch_create: meshes must live on the current device");
        if (m->flags & (LESASM_MESH_SCATTER_COLOUR | LESASM_MESH_SCATTER_DIRECT | LESASM_MESH_SCATTER_CHUNK_ATOMIC))
            return fail(LESASM_E_UNSUPPORTED, "batch_create: meshes must use the staged scatter");
        for (int k = 0; k < kNumCat; ++k)
            if (m->cat[k].d_lf != m->cat[k].d_lg)
                return fail(LESASM_E_UNSUPPORTED, "batch_create: periodic meshes are not batched");
        for (int j = 0; j < i; ++j)
            if (meshes[j] == m) return fail(LESASM_E_INVALID_ARG, "batch_create: a mesh appears twice");
    }
    auto *b = new lesasm_batch();
    struct Guard {
        lesasm_batch *p;
        ~Guard() { batch_free(p); }
    } guard{b};
    b->device = dev;
    b->meshes.assign(meshes, meshes + n);
    hipDeviceProp_t prop;
    LESASM_HIP_TRY(hipGetDeviceProperties(&prop, dev));
    b->n_cu = prop.multiProcessorCount;
    int st;
    if ((st = balloc(b, &b->d_call, 1)) || (st = balloc(b, &b->d_head, kHeads))) return st;
    LESASM_HIP_TRY(hipEventCreate(&b->ev0));
    LESASM_HIP_TRY(hipEventCreate(&b->ev1));
    LESASM_HIP_TRY(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    LESASM_HIP_TRY(hipEventCreateWithFlags(&b->ev_done, hipEventDisableTiming));
    for (int i = 0; i < 3; ++i) LESASM_HIP_TRY(hipEventCreateWithFlags(&b->ev_join[i], hipEventDisableTiming));
    if ((st = device_side_streams(dev, b->side))) return st;
    b->chunk = meshes[0]->chunk_elems;
    if ((st = build_tables(b)) || (st = build_work(b))) return st;
    guard.p = nullptr;
    *out = b;
    return LESASM_OK;
}

extern "C" int lesasm_batch_destroy(lesasm_batch *b) {
    batch_free(b);
    return LESASM_OK;
}

extern "C" int lesasm_batch_configure(lesasm_batch *b, int chunk, int order, int grid_per_cu) {
    if (!b) return fail(LESASM_E_INVALID_ARG, "batch_configure: batch is NULL");
    if (chunk != 0 && (chunk < 32 || chunk > 4096)) return fail(LESASM_E_UNSUPPORTED, "batch_configure: bad chunk");
    if (order < LESASM_ORDER_MESH || order > LESASM_ORDER_INTERLEAVED)
        return fail(LESASM_E_UNSUPPORTED, "batch_configure: bad order");
    if (grid_per_cu < 1 || grid_per_cu > 8) return fail(LESASM_E_UNSUPPORTED, "batch_configure: grid_per_cu in 1..8");
    b->chunk = chunk;
    b->order = order;
    b->grid_per_cu = grid_per_cu;
    return rebuild(b);
}

extern "C" int lesasm_batch_get_config(const lesasm_batch *b, int *chunk, int *order, int *grid_per_cu, int *n_items) {
    if (!b || !chunk || !order || !grid_per_cu || !n_items) return fail(LESASM_E_INVALID_ARG, "batch_get_config: NULL");
    *chunk = b->chunk;
    *order = b->order;
    *grid_per_cu = b->grid_per_cu;
    *n_items = b->nwork;
    return LESASM_OK;
}

extern "C" int lesasm_batch_set_per_type(lesasm_batch *b, int per_type) {
    if (!b) return fail(LESASM_E_INVALID_ARG, "batch_set_per_type: batch is NULL");
    if (per_type < 0 || per_type > 2) return fail(LESASM_E_UNSUPPORTED, "batch_set_per_type: 0, 1 or 2");
    b->per_type = per_type;
    return rebuild(b);
}

extern "C" int lesasm_batch_get_per_type(const lesasm_batch *b, int *per_type) {
    if (!b || !per_type) return fail(LESASM_E_INVALID_ARG, "batch_get_per_type: NULL argument");
    *per_type = b->per_type;
    return LESASM_OK;
}

extern "C" int lesasm_batch_assemble(lesasm_batch *b, const double *const *d_u, const double *const *d_p,
                                     const double *nu, double *const *d_rhs, void *stream) {
    if (!b || !d_u || !nu || !d_rhs) return fail(LESASM_E_INVALID_ARG, "batch_assemble: NULL argument");
    int dev = -1;
    LESASM_HIP_TRY(hipGetDevice(&dev));
    if (dev != b->device) return fail(LESASM_E_STATE, "batch_assemble: wrong current device");
    BatchCall call;
    int st = make_call(b, d_u, d_p, nu, d_rhs, call);
    if (st) return st;
    const bool fp32 = b->meshes[0]->precision == LESASM_PREC_FP32;
    hipStream_t s = (hipStream_t)stream;
    bool capturing = false;
    if ((st = batch_order_begin(b, s, &capturing))) return st;
    if ((st = batch_launch(b, call, d_p != nullptr, fp32, s))) return st;
    return batch_order_end(b, s, capturing);
}

// Autotuner: times the batched assembly for every chunk length in `chunks`
// and every queue order, keeps the fastest.  Results are cached in a text
// file keyed by the batch signature (meshes' element counts per type, CUs).
extern "C" int lesasm_batch_tune(lesasm_batch *b, const double *const *d_u, const double *const *d_p,
                                 const double *nu, double *const *d_rhs, const char *cache_path, int reps,
                                 double *best_ms) {
    if (!b || !d_u || !nu || !d_rhs || reps < 1) return fail(LESASM_E_INVALID_ARG, "batch_tune: bad argument");
    std::ostringstream sig;
    sig << "v3_cu" << b->n_cu;
    for (lesasm_mesh *m : b->meshes)
        for (int k = 0; k < kNumCat; ++k) sig << "_" << m->cat[k].n;
    const std::string key = sig.str();
    LESASM_HIP_TRY(hipDeviceSynchronize());  // earlier calls on any stream end first (the tuner runs on stream 0)
    if (cache_path && *cache_path) {
        std::ifstream in(cache_path);
        std::string k;
        int c, o, g, t;
        double ms;
        while (in >> k >> c >> o >> g >> t >> ms)
            if (k == key) {
                b->chunk = c;
                b->order = o;
                b->grid_per_cu = g;
                b->per_type = t;
                int st = rebuild(b);
                if (st) return st;
                if (best_ms) *best_ms = ms;
                b->last_tune_ms = ms;
                return LESASM_OK;
            }
    }
    BatchCall call;
    int st = make_call(b, d_u, d_p, nu, d_rhs, call);
    if (st) return st;
    const bool fp32 = b->meshes[0]->precision == LESASM_PREC_FP32;
    const int chunks[] = {0, 128, 256, 512, 1024};  // 0: each mesh's own lengths per type
    const int orders[] = {LESASM_ORDER_MESH, LESASM_ORDER_LARGEST_FIRST, LESASM_ORDER_INTERLEAVED};
    const int grids[] = {2, 4};
    double best = 1e30;
    int bc = b->chunk, bo = b->order, bg = b->grid_per_cu, bt = b->per_type;
    for (int c : chunks)
        for (int o : orders)
            for (int g : grids)
                for (int pt = 0; pt < 3; ++pt) {
                    if (pt == 2 && g != grids[0]) continue;  // one workgroup per item: no grid size to choose
                    b->chunk = c;
                    b->order = o;
                    b->grid_per_cu = g;
                    b->per_type = pt;
                    if ((st = rebuild(b))) return st;
                    std::vector<float> t;
                    for (int r = 0; r < reps + 1; ++r) {
                        LESASM_HIP_TRY(hipEventRecord(b->ev0, 0));
                        if ((st = batch_launch(b, call, d_p != nullptr, fp32, 0))) return st;
                        LESASM_HIP_TRY(hipEventRecord(b->ev1, 0));
                        LESASM_HIP_TRY(hipEventSynchronize(b->ev1));
                        float ms = 0;
                        LESASM_HIP_TRY(hipEventElapsedTime(&ms, b->ev0, b->ev1));
                        if (r) t.push_back(ms);  // first run warms up
                    }
                    std::sort(t.begin(), t.end());
                    const double med = t[t.size() / 2];
                    if (med < best) {
                        best = med;
                        bc = c;
                        bo = o;
                        bg = g;
                        bt = pt;
                    }
                }
    b->chunk = bc;
    b->order = bo;
    b->grid_per_cu = bg;
    b->per_type = bt;
    if ((st = rebuild(b))) return st;
    b->last_tune_ms = best;
    if (best_ms) *best_ms = best;
    if (cache_path && *cache_path) {
        std::ofstream outf(cache_path, std::ios::app);
        outf << key << " " << bc << " " << bo << " " << bg << " " << bt << " " << best << "\n";
    }
    return LESASM_OK;
}

// Three-stage Runge-Kutta update of every mesh (Heun's third-order tableau;
// no pressure projection), in place on u, with p fixed:
//   k1 = dt M^-1 rhs(u);  u2 = u + k1/3;  k2 = dt M^-1 rhs(u2);  u3 = u + 2 k2/3;
//   k3 = dt M^-1 rhs(u3); u <- u + k1/4 + 3 k3/4.
static int rk3_record(lesasm_batch *b, double *const *d_u, const double *const *d_p, const double *nu, double dt,
                      hipStream_t s) {
    const int n = (int)b->meshes.size();
    const bool fp32 = b->meshes[0]->precision == LESASM_PREC_FP32;
    const bool has_p = d_p != nullptr;
    std::vector<const double *> u_c(n), us_c(n);
    std::vector<double *> k1(n), k3(n), us(n);
    for (int i = 0; i < n; ++i) {
        k1[i] = b->k1 + 3 * b->node_off[i];
        k3[i] = b->k3 + 3 * b->node_off[i];
        us[i] = b->us + 3 * b->node_off[i];
        u_c[i] = d_u[i];
        us_c[i] = us[i];
    }
    const unsigned gridn = (unsigned)(b->blk_off[kNumCat + 3] - b->blk_off[kNumCat + 2]);
    auto stage = [&](const std::vector<const double *> &uin, const std::vector<double *> &rhs, double a1,
                     const std::vector<double *> *k1v, double a2, std::vector<double *> &y) -> int {
        BatchCall call;
        int st = make_call(b, uin.data(), d_p, nu, rhs.data(), call);
        if (st) return st;
        if ((st = batch_launch(b, call, has_p, fp32, s))) return st;
        UpdateArgs ua;
        std::memset(&ua, 0, sizeof(ua));
        for (int i = 0; i < n; ++i) {
            ua.base[i] = d_u[i];
            ua.rhs[i] = rhs[i];
            ua.k1[i] = k1v ? (*k1v)[i] : nullptr;
            ua.y[i] = y[i];
        }
        ua.a1 = a1;
        ua.a2 = a2;
        ua.dt = dt;
        hipLaunchKernelGGL(k_batch_update, dim3(gridn), dim3(kBatchBlock), 0, s, ua, b->d_md,
                           b->d_blk + b->blk_off[kNumCat + 2]);
        LESASM_HIP_TRY(hipGetLastError());
        return LESASM_OK;
    };
    std::vector<double *> uout(d_u, d_u + n);
    int st;
    if ((st = stage(u_c, k1, 0.0, nullptr, 1.0 / 3.0, us))) return st;   // us = u + k1/3
    if ((st = stage(us_c, k3, 0.0, nullptr, 2.0 / 3.0, us))) return st;  // us = u + 2 k2/3
    return stage(us_c, k3, 0.25, &k1, 0.75, uout);                      // u = u + k1/4 + 3 k3/4
}

extern "C" int lesasm_batch_rk3_graph(lesasm_batch *b, double *const *d_u, const double *const *d_p,
                                      const double *nu, double dt, void *stream) {
    if (!b || !d_u || !nu) return fail(LESASM_E_INVALID_ARG, "batch_rk3_graph: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    if (!s) return fail(LESASM_E_INVALID_ARG, "batch_rk3_graph: capture needs a non-default stream");
    int st;
    if (!b->k1) {
        if ((st = balloc(b, &b->k1, 3 * (size_t)b->total_nodes)) || (st = balloc(b, &b->k3, 3 * (size_t)b->total_nodes)) ||
            (st = balloc(b, &b->us, 3 * (size_t)b->total_nodes)))
            return st;
    }
    drop_graph(b);  // waits for the previous graph's last replay
    LESASM_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    st = rk3_record(b, d_u, d_p, nu, dt, s);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(LESASM_E_HIP, std::string("batch_rk3_graph: capture failed: ") + hipGetErrorString(e));
    b->graph = g;
    LESASM_HIP_TRY(hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0));
    return LESASM_OK;
}

extern "C" int lesasm_batch_rk3_launch(lesasm_batch *b, void *stream) {
    if (!b || !b->graph_exec) return fail(LESASM_E_STATE, "batch_rk3_launch: no captured step");
    hipStream_t s = (hipStream_t)stream;
    bool capturing = false;
    int st = batch_order_begin(b, s, &capturing);
    if (st) return st;
    LESASM_HIP_TRY(hipGraphLaunch(b->graph_exec, s));
    return batch_order_end(b, s, capturing);
}

extern "C" int lesasm_batch_rk3_eager(lesasm_batch *b, double *const *d_u, const double *const *d_p,
                                      const double *nu, double dt, void *stream) {
    if (!b || !d_u || !nu) return fail(LESASM_E_INVALID_ARG, "batch_rk3_eager: NULL argument");
    int st;
    if (!b->k1) {
        if ((st = balloc(b, &b->k1, 3 * (size_t)b->total_nodes)) || (st = balloc(b, &b->k3, 3 * (size_t)b->total_nodes)) ||
            (st = balloc(b, &b->us, 3 * (size_t)b->total_nodes)))
            return st;
    }
    hipStream_t s = (hipStream_t)stream;
    bool capturing = false;
    if ((st = batch_order_begin(b, s, &capturing))) return st;
    if ((st = rk3_record(b, d_u, d_p, nu, dt, s))) return st;
    return batch_order_end(b, s, capturing);
}
