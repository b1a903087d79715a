// Mesh upload and one-time preprocessing (the library's side of Section 3.4.3):
// validation, grouping of elements into categories (one per element type and
// integration rule), Morton ordering of elements inside a category, first-touch
// renumbering of nodes, optional greedy colouring, device upload, and a
// geometry kernel that checks det J > 0 at every Gauss point and computes the
// filter width Delta_e = V_e^(1/3) and the row-sum lumped mass (the
// mass-matrix listing of Section 3.4.3, summed over each row).
#include <algorithm>
#include <mutex>
#include <unordered_map>
#include <climits>
#include <cstring>
#include <memory>
#include <numeric>

#include "element.hpp"

namespace lesasm {

static thread_local std::string g_error;

void set_error(const std::string &msg) { g_error = msg; }

int fail(int code, const std::string &msg) {
    g_error = msg;
    return code;
}

// ---- geometry kernel -------------------------------------------------------
template <int T>
__global__ __launch_bounds__(256) void k_geometry(CatView c, int first, const double *__restrict__ xyz,
                                                  double *__restrict__ mass, double *__restrict__ delta,
                                                  int *__restrict__ bad) {
    using E = Ref<T>;
    constexpr int nn = E::nn;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= c.n) return;
    double x[nn][3];
    int fid[nn];
#pragma unroll
    for (int a = 0; a < nn; ++a) {
        const int g = c.cg[(size_t)a * c.ld + e];
        fid[a] = c.cf[(size_t)a * c.ld + e];
#pragma unroll
        for (int k = 0; k < 3; ++k) x[a][k] = xyz[3 * (size_t)g + k];
    }
#pragma unroll
    for (int a = nn - 1; a >= 0; --a)
#pragma unroll
        for (int k = 0; k < 3; ++k) x[a][k] -= x[0][k];
    double vol = 0.0, m[nn];
#pragma unroll
    for (int a = 0; a < nn; ++a) m[a] = 0.0;
    bool ok = true;
#pragma unroll
    for (int g = 0; g < E::ng; ++g) {
        double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
        for (int a = 1; a < nn; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int k = 0; k < 3; ++k) J[i][k] += x[a][i] * E::tab.dN[g][a][k];
        const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        ok = ok && (det > 0.0);
        const double dv = E::tab.w[g] * det;
        vol += dv;
#pragma unroll
        for (int a = 0; a < nn; ++a) m[a] += dv * E::tab.N[g][a];
    }
    if (!ok) atomicMin(bad, first + e);
    delta[e] = cbrt(vol);
#pragma unroll
    for (int a = 0; a < nn; ++a) unsafeAtomicAdd(mass + fid[a], m[a]);
}

__global__ void k_permute(const double *__restrict__ in, double *__restrict__ out, const int32_t *__restrict__ perm,
                          size_t n, int nc, int to_internal) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n * nc; t += (size_t)gridDim.x * blockDim.x) {
        const size_t k = t / nc;
        const int c = (int)(t - k * nc);
        const size_t uidx = (size_t)perm[k] * nc + c;
        if (to_internal)
            out[t] = in[uidx];
        else
            out[uidx] = in[t];
    }
}

int grid_for(size_t n, int block);

// ---- device memory accounting -------------------------------------------------
namespace {
std::mutex g_mem_mu;
std::unordered_map<void *, size_t> g_mem_sizes;
uint64_t g_mem_in_use = 0, g_mem_cap = 0;  // cap 0: none
std::mutex g_side_mu;
constexpr int kMaxDevices = 64;
hipStream_t g_side[kMaxDevices][3];
}  // namespace

int device_alloc(void **p, size_t bytes, const char *what) {
    *p = nullptr;
    if (bytes == 0) return LESASM_OK;
    {
        std::lock_guard<std::mutex> lk(g_mem_mu);
        if (g_mem_cap && g_mem_in_use + bytes > g_mem_cap)
            return fail(LESASM_E_OOM, std::string(what) + ": allocation of " + std::to_string(bytes) +
                                          " bytes would pass the memory cap (" + std::to_string(g_mem_cap) +
                                          " bytes, " + std::to_string(g_mem_in_use) + " in use)");
        g_mem_in_use += bytes;  // reserved before the allocation
    }
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    std::lock_guard<std::mutex> lk(g_mem_mu);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        g_mem_in_use -= bytes;
        return fail(LESASM_E_OOM, std::string(what) + ": hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                      hipGetErrorString(e));
    }
    g_mem_sizes[q] = bytes;
    *p = q;
    return LESASM_OK;
}

void device_free(void *p) {
    if (!p) return;
    (void)hipFree(p);
    std::lock_guard<std::mutex> lk(g_mem_mu);
    auto it = g_mem_sizes.find(p);
    if (it != g_mem_sizes.end()) {
        g_mem_in_use -= it->second;
        g_mem_sizes.erase(it);
    }
}

int device_side_streams(int device, hipStream_t out[3]) {
    if (device < 0 || device >= kMaxDevices) return fail(LESASM_E_UNSUPPORTED, "side streams: device id too large");
    std::lock_guard<std::mutex> lk(g_side_mu);
    for (int i = 0; i < 3; ++i)
        if (!g_side[device][i]) LESASM_HIP_TRY(hipStreamCreateWithFlags(&g_side[device][i], hipStreamNonBlocking));
    for (int i = 0; i < 3; ++i) out[i] = g_side[device][i];
    return LESASM_OK;
}

int mesh_order_begin(lesasm_mesh *m, hipStream_t s, bool *capturing) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    LESASM_HIP_TRY(hipStreamIsCapturing(s, &cs));
    *capturing = cs != hipStreamCaptureStatusNone;
    if (!*capturing && m->order_ev && m->order_stream != s) LESASM_HIP_TRY(hipStreamWaitEvent(s, m->order_ev, 0));
    return LESASM_OK;
}

int mesh_order_end(lesasm_mesh *m, hipStream_t s, bool capturing) {
    if (capturing) return LESASM_OK;
    LESASM_HIP_TRY(hipEventRecord(m->ev_done, s));
    m->order_ev = m->ev_done;
    m->order_stream = s;
    return LESASM_OK;
}

// ---- host helpers ------------------------------------------------------------
template <class T> static int dalloc(lesasm_mesh *m, T **p, size_t n) {
    *p = nullptr;
    if (n == 0) return LESASM_OK;
    void *q = nullptr;
    int st = device_alloc(&q, n * sizeof(T), "mesh");
    if (st) return st;
    m->allocs.push_back(q);
    m->bytes += n * sizeof(T);
    *p = (T *)q;
    return LESASM_OK;
}

template <class T> static int upload(lesasm_mesh *m, T **p, const std::vector<T> &h) {
    int st = dalloc(m, p, h.size());
    if (st) return st;
    if (!h.empty()) LESASM_HIP_TRY(hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return LESASM_OK;
}

static uint64_t spread3(uint64_t v) {  // 21 bits -> every third bit of 63
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}

static void free_mesh(lesasm_mesh *m) {
    if (!m) return;
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    for (auto &v : m->pending)
        for (auto &ev : v) {
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
    for (int i = 0; i < 3; ++i)  // (the side streams are the device's, not the mesh's)
        if (m->ev_join[i]) (void)hipEventDestroy(m->ev_join[i]);
    if (m->ev_fork) (void)hipEventDestroy(m->ev_fork);
    if (m->ev_done) (void)hipEventDestroy(m->ev_done);
    for (void *p : m->allocs) device_free(p);
    if (have) (void)hipSetDevice(cur);
    delete m;
}

struct MeshGuard {
    lesasm_mesh *m;
    ~MeshGuard() { free_mesh(m); }
};

// Greedy colouring of the elements `order` (user ids) on their field nodes:
// each element takes the lowest colour not used by any element sharing a node.
static std::vector<int> greedy_colour(const std::vector<int64_t> &order, const int64_t *offs, const int32_t *conn,
                                      const int32_t *fmap, int64_t n_field, int &ncol) {
    constexpr int W = 4;  // up to 256 colours
    std::vector<uint64_t> used((size_t)n_field * W, 0);
    std::vector<int> col(order.size());
    ncol = 0;
    for (size_t j = 0; j < order.size(); ++j) {
        const int64_t e = order[j];
        uint64_t forb[W] = {0, 0, 0, 0};
        for (int64_t q = offs[e]; q < offs[e + 1]; ++q) {
            const int64_t f = fmap ? fmap[conn[q]] : conn[q];
            for (int w = 0; w < W; ++w) forb[w] |= used[(size_t)f * W + w];
        }
        int c = -1;
        for (int w = 0; w < W && c < 0; ++w)
            if (~forb[w]) c = 64 * w + __builtin_ctzll(~forb[w]);
        if (c < 0) return {};
        col[j] = c;
        ncol = std::max(ncol, c + 1);
        for (int64_t q = offs[e]; q < offs[e + 1]; ++q) {
            const int64_t f = fmap ? fmap[conn[q]] : conn[q];
            used[(size_t)f * W + c / 64] |= 1ULL << (c % 64);
        }
    }
    return col;
}

template <class T> static void dfree(lesasm_mesh *m, T *&p) {
    if (!p) return;
    auto it = std::find(m->allocs.begin(), m->allocs.end(), (void *)p);
    if (it != m->allocs.end()) {
        device_free(p);
        m->allocs.erase(it);
    }
    p = nullptr;
}

// Chunks for the chunked scatter of category k: runs of consecutive internal
// elements, at most m->chunk_elems long and with at most m->chunk_max_nodes
// distinct geometry and field nodes (800, or 400 when the learned closure
// also needs LDS), so that a chunk's node data fit in LDS.  With the closure,
// PEN06 and HEX08 take 700: their closure kernels hold two workgroups per
// compute unit (registers), so 56 KB of node data beside the 21 KB of weights
// and scratch still fit twice, while the TET04 and PYR05 closure kernels hold
// three (20 M hybrid box: FP32 closure 2.71 against 2.79 ms, FP64 3.92 against
// 4.09 ms).  Node
// lists are sorted ascending (coalesced loads); a field node is owned by a
// chunk when all of its incidences in the mesh lie in that chunk.

static int chunk_length(const lesasm_mesh *m, int type, int64_t n) {
    if (m->chunk_elems) return m->chunk_elems;
    int ce = 64;
    while (ce < 512 && 2 * ce <= n / 256) ce *= 2;
    // TET04 and PEN06 gain from longer chunks (fewer shared nodes per element,
    // so fewer staging rows) once the category still makes at least 4096 of
    // them; HEX08 and PYR05 do not (HEX08 measured slower at 1024)
    if ((type == LESASM_TET04 || type == LESASM_PEN06) && ce == 512 && n / 1024 >= 4096) ce = 1024;
    return ce;
}

static int build_chunks(lesasm_mesh *m, int k) {
    Category &c = m->cat[k];
    dfree(m, c.d_fslot);
    c.h_fnodes.clear();
    dfree(m, c.d_eoff);
    dfree(m, c.d_goff);
    dfree(m, c.d_gnodes);
    if (c.d_foff != c.d_goff) dfree(m, c.d_foff);
    c.d_foff = nullptr;
    dfree(m, c.d_fnodes);
    if (c.d_lf != c.d_lg) dfree(m, c.d_lf);
    c.d_lf = nullptr;
    dfree(m, c.d_lg);
    c.n_chunks = 0;
    c.lds_doubles = 0;
    if (c.n == 0) return LESASM_OK;
    const bool periodic = !c.h_cf.empty();
    const std::vector<int32_t> &cg = c.h_cg, &cf = periodic ? c.h_cf : c.h_cg;
    const int nnode = c.type;
    const int64_t n = c.n;
    const int ce = chunk_length(m, c.type, n);
    const int cap = (m->mlp && (c.type == LESASM_PEN06 || c.type == LESASM_HEX08)) ? 700 : m->chunk_max_nodes;
    c.chunk_elems = ce;
    std::vector<int32_t> eoff{0}, goff{0}, foff{0}, gnodes, fnodes;
    std::vector<uint16_t> lg((size_t)nnode * n), lf(periodic ? (size_t)nnode * n : 0);
    std::vector<int32_t> gslot(m->n_nodes, -1), fslot(m->n_field, -1), fcount(m->n_field, 0);
    std::vector<int32_t> gl, fl;
    int64_t start = 0;
    while (start < n) {
        gl.clear();
        fl.clear();
        int64_t e = start;
        while (e < n && e - start < ce) {
            int newg = 0, newf = 0;
            for (int a = 0; a < nnode; ++a) {
                newg += gslot[cg[(size_t)a * n + e]] < 0;
                newf += fslot[cf[(size_t)a * n + e]] < 0;
            }
            if (e > start && ((int)gl.size() + newg > cap || (int)fl.size() + newf > cap))
                break;
            for (int a = 0; a < nnode; ++a) {
                const int32_t g = cg[(size_t)a * n + e], f = cf[(size_t)a * n + e];
                if (gslot[g] < 0) { gslot[g] = 0; gl.push_back(g); }
                if (fslot[f] < 0) { fslot[f] = 0; fl.push_back(f); }
                fcount[f]++;
            }
            ++e;
        }
        std::sort(gl.begin(), gl.end());
        std::sort(fl.begin(), fl.end());
        for (size_t q = 0; q < gl.size(); ++q) gslot[gl[q]] = (int32_t)q;
        for (size_t q = 0; q < fl.size(); ++q) fslot[fl[q]] = (int32_t)q;
        for (int64_t x = start; x < e; ++x)
            for (int a = 0; a < nnode; ++a) {
                const size_t s = (size_t)a * n + x;
                lg[s] = (uint16_t)gslot[cg[s]];
                if (periodic) lf[s] = (uint16_t)fslot[cf[s]];
            }
        for (int32_t g : gl) {
            gnodes.push_back(g);
            gslot[g] = -1;
        }
        for (int32_t f : fl) {
            fnodes.push_back((int32_t)((uint32_t)f | (fcount[f] == m->h_finc[f] ? kOwnedBit : 0u)));
            fcount[f] = 0;
            fslot[f] = -1;
        }
        c.lds_doubles = std::max(c.lds_doubles, (int)(3 * gl.size() + 7 * fl.size()));
        // chunk node lists are indexed with int32 offsets on the GPU
        if (gnodes.size() >= (size_t)INT32_MAX || fnodes.size() >= (size_t)INT32_MAX)
            return fail(LESASM_E_UNSUPPORTED, "mesh_create: chunk node lists of one element type exceed 2^31 entries");
        eoff.push_back((int32_t)e);
        goff.push_back((int32_t)gnodes.size());
        foff.push_back((int32_t)fnodes.size());
        start = e;
    }
    c.n_chunks = (int32_t)(eoff.size() - 1);
    int st;
    if ((st = upload(m, &c.d_eoff, eoff))) return st;
    if ((st = upload(m, &c.d_goff, goff))) return st;
    if ((st = upload(m, &c.d_gnodes, gnodes))) return st;
    if ((st = upload(m, &c.d_fnodes, fnodes))) return st;
    c.h_fnodes.swap(fnodes);
    if ((st = upload(m, &c.d_lg, lg))) return st;
    if (periodic) {
        if ((st = upload(m, &c.d_foff, foff))) return st;
        if ((st = upload(m, &c.d_lf, lf))) return st;
    } else {
        c.d_foff = c.d_goff;
        c.d_lf = c.d_lg;
    }
    return LESASM_OK;
}

// Staging rows of the staged scatter: one per (chunk, shared node), numbered in
// (type, chunk, node) order, plus the CSR that lets each node owned by no
// chunk sum its rows in that fixed order.
static int build_staging(lesasm_mesh *m) {
    dfree(m, m->d_stage);
    dfree(m, m->d_gnode);
    dfree(m, m->d_goffs);
    m->n_slots = 0;
    m->n_gather = 0;
    for (int g = 0; g < kNumCat + 2; ++g) m->gather_off[g] = 0;
    // Rows of one shared node are consecutive (type and chunk order), so the
    // gather reads them without an index array.  Shared nodes are grouped by
    // the categories that wrote their rows (class k: category k only, class
    // kNumCat: several, or none), node order inside a class.
    std::vector<int32_t> owned(m->n_field, 0), count(m->n_field, 0);
    std::vector<uint8_t> cats(m->n_field, 0);
    int64_t total = 0;
    for (int k = 0; k < kNumCat; ++k) {
        const Category &c = m->cat[k];
        for (size_t q = 0; q < c.h_fnodes.size(); ++q) {
            const uint32_t tag = (uint32_t)c.h_fnodes[q];
            const int32_t f = (int32_t)(tag & ~kOwnedBit);
            if (tag & kOwnedBit) owned[f] = 1;
            else {
                count[f]++;
                total++;
                cats[f] |= (uint8_t)(1u << k);
            }
        }
    }
    if (total >= INT32_MAX) return fail(LESASM_E_UNSUPPORTED, "mesh_create: too many staging rows");
    std::vector<uint8_t> cls(m->n_field, (uint8_t)kNumCat);
    for (int64_t f = 0; f < m->n_field; ++f)
        for (int k = 0; k < kNumCat; ++k)
            if (cats[f] == (1u << k)) cls[f] = (uint8_t)k;
    std::vector<int32_t> gnode, goffs{0};
    std::vector<int32_t> pos(m->n_field, -1);
    m->gather_off[0] = 0;
    for (int g = 0; g <= kNumCat; ++g) {
        for (int64_t f = 0; f < m->n_field; ++f)
            if (!owned[f] && cls[f] == g) {  // includes nodes of no element (count 0): the gather writes their zero
                pos[f] = goffs.back();
                gnode.push_back((int32_t)f);
                goffs.push_back(goffs.back() + count[f]);
            }
        m->gather_off[g + 1] = (int32_t)gnode.size();
    }
    std::vector<std::vector<int32_t>> fslot(kNumCat);
    for (int k = 0; k < kNumCat; ++k) {
        Category &c = m->cat[k];
        dfree(m, c.d_fslot);
        fslot[k].assign(c.h_fnodes.size(), -1);
        for (size_t q = 0; q < c.h_fnodes.size(); ++q) {
            const uint32_t tag = (uint32_t)c.h_fnodes[q];
            if (!(tag & kOwnedBit)) fslot[k][q] = pos[(int32_t)(tag & ~kOwnedBit)]++;
        }
    }
    m->n_slots = total;
    m->n_gather = (int32_t)gnode.size();
    int st;
    if ((st = dalloc(m, &m->d_stage, 3 * (size_t)total))) return st;
    if ((st = upload(m, &m->d_gnode, gnode))) return st;
    if ((st = upload(m, &m->d_goffs, goffs))) return st;
    for (int k = 0; k < kNumCat; ++k)
        if ((st = upload(m, &m->cat[k].d_fslot, fslot[k]))) return st;
    return LESASM_OK;
}

static bool is_chunked(const lesasm_mesh *m) {
    return !(m->flags & (LESASM_MESH_SCATTER_COLOUR | LESASM_MESH_SCATTER_DIRECT));
}

static bool is_staged(const lesasm_mesh *m) { return is_chunked(m) && !(m->flags & LESASM_MESH_SCATTER_CHUNK_ATOMIC); }

static int build_scatter(lesasm_mesh *m) {
    int st;
    for (int k = 0; k < kNumCat; ++k)
        if ((st = build_chunks(m, k))) return st;
    if (is_staged(m) && (st = build_staging(m))) return st;
    if (!m->side[0]) {
        if ((st = device_side_streams(m->device, m->side))) return st;
        for (int i = 0; i < 3; ++i) LESASM_HIP_TRY(hipEventCreateWithFlags(&m->ev_join[i], hipEventDisableTiming));
        LESASM_HIP_TRY(hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming));
    }
    return LESASM_OK;
}

}  // namespace lesasm

using namespace lesasm;

extern "C" const char *lesasm_last_error(void) { return g_error.c_str(); }

extern "C" int lesasm_set_memory_cap(uint64_t bytes) {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    g_mem_cap = bytes;
    return LESASM_OK;
}

extern "C" int lesasm_memory_in_use(uint64_t *bytes) {
    if (!bytes) return fail(LESASM_E_INVALID_ARG, "memory_in_use: NULL argument");
    std::lock_guard<std::mutex> lk(g_mem_mu);
    *bytes = g_mem_in_use;
    return LESASM_OK;
}

extern "C" int lesasm_version(void) { return LESASM_VERSION; }

extern "C" int lesasm_check(void *stream) {
    LESASM_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

extern "C" int lesasm_mesh_create(const lesasm_mesh_desc *d, lesasm_mesh **out) {
    if (!out) return fail(LESASM_E_INVALID_ARG, "mesh_create: out is NULL");
    *out = nullptr;
    if (!d) return fail(LESASM_E_INVALID_ARG, "mesh_create: desc is NULL");
    const int64_t nn = d->n_nodes, ne = d->n_elems;
    if (nn < 0 || ne < 0 || nn >= INT32_MAX || ne >= INT32_MAX)
        return fail(LESASM_E_INVALID_ARG, "mesh_create: node or element count out of range");
    if (ne > 0 && (!d->types || !d->conn_offsets || !d->conn))
        return fail(LESASM_E_INVALID_ARG, "mesh_create: types, conn_offsets or conn is NULL");
    if (nn > 0 && !d->coords) return fail(LESASM_E_INVALID_ARG, "mesh_create: coords is NULL");
    const uint32_t scatter_bits = LESASM_MESH_SCATTER_COLOUR | LESASM_MESH_SCATTER_DIRECT | LESASM_MESH_SCATTER_CHUNK_ATOMIC;
    if (d->flags & ~(scatter_bits | LESASM_MESH_KEEP_ORDER))
        return fail(LESASM_E_INVALID_ARG, "mesh_create: unknown flag bits");
    if (__builtin_popcount(d->flags & scatter_bits) > 1)
        return fail(LESASM_E_INVALID_ARG, "mesh_create: choose one scatter mode");
    if (!(d->vreman_c >= 0.0)) return fail(LESASM_E_INVALID_ARG, "mesh_create: vreman_c must be >= 0");
    const int32_t *fmap = d->field_node;
    const int64_t nf = fmap ? d->n_field_nodes : nn;
    if (fmap) {
        if (nf <= 0 || nf > nn) return fail(LESASM_E_INVALID_ARG, "mesh_create: n_field_nodes out of range");
        for (int64_t g = 0; g < nn; ++g)
            if (fmap[g] < 0 || fmap[g] >= nf)
                return fail(LESASM_E_INVALID_ARG, "mesh_create: field_node[" + std::to_string(g) + "] out of range");
    }
    if (ne > 0 && d->conn_offsets[0] != 0) return fail(LESASM_E_INVALID_ARG, "mesh_create: conn_offsets[0] != 0");
    std::vector<int64_t> order[kNumCat];
    for (int64_t e = 0; e < ne; ++e) {
        const int t = d->types[e];
        const int k = cat_of_type(t);
        if (k < 0)
            return fail(LESASM_E_INVALID_ARG, "mesh_create: element " + std::to_string(e) + " has type " +
                                                  std::to_string(t));
        if (d->conn_offsets[e + 1] - d->conn_offsets[e] != t)
            return fail(LESASM_E_INVALID_ARG, "mesh_create: element " + std::to_string(e) + " has a wrong node count");
        for (int64_t q = d->conn_offsets[e]; q < d->conn_offsets[e + 1]; ++q)
            if (d->conn[q] < 0 || d->conn[q] >= nn)
                return fail(LESASM_E_INVALID_ARG, "mesh_create: element " + std::to_string(e) +
                                                      " references node " + std::to_string(d->conn[q]));
        order[k].push_back(e);
    }

    lesasm_mesh *m = new lesasm_mesh();
    MeshGuard guard{m};
    LESASM_HIP_TRY(hipGetDevice(&m->device));
    LESASM_HIP_TRY(hipDeviceGetAttribute(&m->n_cu, hipDeviceAttributeMultiprocessorCount, m->device));
    m->flags = d->flags;
    m->n_nodes = nn;
    m->n_field = nf;
    m->n_elems = ne;
    m->vreman_c = d->vreman_c;
    const bool keep = d->flags & LESASM_MESH_KEEP_ORDER;
    const bool colour = d->flags & LESASM_MESH_SCATTER_COLOUR;

    // Morton order of element centroids inside each category
    if (!keep && ne > 0) {
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int64_t g = 0; g < nn; ++g)
            for (int k = 0; k < 3; ++k) {
                lo[k] = std::min(lo[k], d->coords[3 * g + k]);
                hi[k] = std::max(hi[k], d->coords[3 * g + k]);
            }
        double scale[3];
        for (int k = 0; k < 3; ++k) scale[k] = hi[k] > lo[k] ? (double)((1 << 21) - 1) / (hi[k] - lo[k]) : 0.0;
        for (int k = 0; k < kNumCat; ++k) {
            std::vector<std::pair<uint64_t, int64_t>> key(order[k].size());
            for (size_t j = 0; j < order[k].size(); ++j) {
                const int64_t e = order[k][j];
                double c[3] = {0, 0, 0};
                const int64_t o = d->conn_offsets[e], n = d->conn_offsets[e + 1] - o;
                for (int64_t a = 0; a < n; ++a)
                    for (int q = 0; q < 3; ++q) c[q] += d->coords[3 * (int64_t)d->conn[o + a] + q];
                uint64_t code = 0;
                for (int q = 0; q < 3; ++q)
                    code |= spread3((uint64_t)((c[q] / n - lo[q]) * scale[q])) << q;
                key[j] = {code, e};
            }
            std::sort(key.begin(), key.end());
            for (size_t j = 0; j < key.size(); ++j) order[k][j] = key[j].second;
        }
    }

    // colour schedule: stable regroup by colour inside each category
    if (colour) {
        for (int k = 0; k < kNumCat; ++k) {
            int ncol = 0;
            std::vector<int> col = greedy_colour(order[k], d->conn_offsets, d->conn, fmap, nf, ncol);
            if (col.empty() && !order[k].empty())
                return fail(LESASM_E_UNSUPPORTED, "mesh_create: more than 256 colours needed");
            std::vector<int64_t> cnt(ncol + 1, 0);
            for (int c : col) cnt[c + 1]++;
            for (int c = 0; c < ncol; ++c) cnt[c + 1] += cnt[c];
            std::vector<int64_t> reordered(order[k].size());
            std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
            for (size_t j = 0; j < col.size(); ++j) reordered[pos[col[j]]++] = order[k][j];
            order[k].swap(reordered);
            m->cat[k].colour_off = cnt;
        }
    }

    // internal element order and first-touch node numbering
    m->h_eperm.reserve(ne);
    int64_t first = 0;
    for (int k = 0; k < kNumCat; ++k) {
        m->cat[k].type = kTypes[k];
        m->cat[k].n = (int64_t)order[k].size();
        m->cat[k].first = first;
        first += m->cat[k].n;
        m->h_eperm.insert(m->h_eperm.end(), order[k].begin(), order[k].end());
    }
    std::vector<int32_t> gnew(nn, -1), fnew(nf, -1);
    if (keep) {
        std::iota(gnew.begin(), gnew.end(), 0);
        std::iota(fnew.begin(), fnew.end(), 0);
    } else {
        int32_t ng = 0, nfc = 0;
        for (int64_t e : m->h_eperm)
            for (int64_t q = d->conn_offsets[e]; q < d->conn_offsets[e + 1]; ++q) {
                const int32_t g = d->conn[q];
                if (gnew[g] < 0) gnew[g] = ng++;
                const int32_t f = fmap ? fmap[g] : g;
                if (fnew[f] < 0) fnew[f] = nfc++;
            }
        for (int64_t g = 0; g < nn; ++g)
            if (gnew[g] < 0) gnew[g] = ng++;
        for (int64_t f = 0; f < nf; ++f)
            if (fnew[f] < 0) fnew[f] = nfc++;
    }
    m->h_fperm.assign(nf, 0);
    for (int64_t f = 0; f < nf; ++f) m->h_fperm[fnew[f]] = (int32_t)f;
    m->h_gint = gnew;
    m->h_fint.assign(nn, 0);
    for (int64_t g = 0; g < nn; ++g) m->h_fint[g] = fnew[fmap ? fmap[g] : g];
    // without a field map the two numberings coincide, so one index array serves both
    const bool alias = (fmap == nullptr);

    int st;
    {
        std::vector<double> xyz((size_t)3 * nn);
        for (int64_t g = 0; g < nn; ++g)
            for (int k = 0; k < 3; ++k) xyz[3 * (size_t)gnew[g] + k] = d->coords[3 * g + k];
        if ((st = upload(m, &m->d_xyz, xyz))) return st;
    }
    if ((st = upload(m, &m->d_fperm, m->h_fperm))) return st;
    if ((st = dalloc(m, &m->d_mass, (size_t)nf))) return st;
    if ((st = dalloc(m, &m->d_flag, 4))) return st;
    if ((st = dalloc(m, &m->d_delta, (size_t)ne))) return st;
    for (int k = 0; k < kNumCat; ++k) {
        Category &c = m->cat[k];
        if (c.n == 0) continue;
        const int nnode = c.type;
        std::vector<int32_t> cg((size_t)nnode * c.n), cf;
        if (!alias) cf.resize(cg.size());
        for (int64_t j = 0; j < c.n; ++j) {
            const int64_t e = order[k][j];
            for (int a = 0; a < nnode; ++a) {
                const int32_t g = d->conn[d->conn_offsets[e] + a];
                cg[(size_t)a * c.n + j] = gnew[g];
                if (!alias) cf[(size_t)a * c.n + j] = fnew[fmap[g]];
            }
        }
        if ((st = upload(m, &c.d_cg, cg))) return st;
        if (alias)
            c.d_cf = c.d_cg;
        else if ((st = upload(m, &c.d_cf, cf)))
            return st;
        c.d_delta = m->d_delta + c.first;
        c.h_cg.swap(cg);
        c.h_cf.swap(cf);
    }
    m->h_finc.assign(nf, 0);
    for (int k = 0; k < kNumCat; ++k) {
        const Category &c = m->cat[k];
        const std::vector<int32_t> &cf = c.h_cf.empty() ? c.h_cg : c.h_cf;
        for (int32_t f : cf) m->h_finc[f]++;
    }
    // every scatter mode orders its calls through this event
    LESASM_HIP_TRY(hipEventCreateWithFlags(&m->ev_done, hipEventDisableTiming));
    if (is_chunked(m) && (st = build_scatter(m))) return st;

    // geometry: det J check, Delta_e, lumped mass
    if (nf > 0) LESASM_HIP_TRY(hipMemset(m->d_mass, 0, sizeof(double) * nf));
    const int big = INT_MAX;
    LESASM_HIP_TRY(hipMemcpy(m->d_flag, &big, sizeof(int), hipMemcpyHostToDevice));
    for (int k = 0; k < kNumCat; ++k) {
        Category &c = m->cat[k];
        if (c.n == 0) continue;
        CatView v{c.d_cg, c.d_cf, c.d_delta, (int32_t)c.n, 0, (int32_t)c.n};
        const dim3 grid((unsigned)((c.n + 255) / 256)), block(256);
        switch (c.type) {
        case LESASM_TET04: hipLaunchKernelGGL(k_geometry<LESASM_TET04>, grid, block, 0, 0, v, (int)c.first, m->d_xyz, m->d_mass, c.d_delta, m->d_flag); break;
        case LESASM_PYR05: hipLaunchKernelGGL(k_geometry<LESASM_PYR05>, grid, block, 0, 0, v, (int)c.first, m->d_xyz, m->d_mass, c.d_delta, m->d_flag); break;
        case LESASM_PEN06: hipLaunchKernelGGL(k_geometry<LESASM_PEN06>, grid, block, 0, 0, v, (int)c.first, m->d_xyz, m->d_mass, c.d_delta, m->d_flag); break;
        case LESASM_HEX08: hipLaunchKernelGGL(k_geometry<LESASM_HEX08>, grid, block, 0, 0, v, (int)c.first, m->d_xyz, m->d_mass, c.d_delta, m->d_flag); break;
        }
        LESASM_HIP_TRY(hipGetLastError());
    }
    LESASM_HIP_TRY(hipDeviceSynchronize());
    int bad = big;
    LESASM_HIP_TRY(hipMemcpy(&bad, m->d_flag, sizeof(int), hipMemcpyDeviceToHost));
    if (bad != big)
        return fail(LESASM_E_INVERTED_ELEMENT, "mesh_create: element " + std::to_string(m->h_eperm[bad]) +
                                                   " has det J <= 0 at a Gauss point");
    guard.m = nullptr;
    *out = m;
    return LESASM_OK;
}

extern "C" int lesasm_mesh_destroy(lesasm_mesh *m) {
    free_mesh(m);
    return LESASM_OK;
}

extern "C" int lesasm_mesh_get_info(const lesasm_mesh *m, lesasm_mesh_info *info) {
    if (!m || !info) return fail(LESASM_E_INVALID_ARG, "get_info: NULL argument");
    std::memset(info, 0, sizeof(*info));
    info->n_nodes = m->n_nodes;
    info->n_field_nodes = m->n_field;
    info->n_elems = m->n_elems;
    for (int k = 0; k < kNumCat; ++k) {
        info->n_per_type[k] = m->cat[k].n;
        info->n_colours[k] = m->cat[k].colour_off.empty() ? 0 : (int32_t)m->cat[k].colour_off.size() - 1;
    }
    info->device = m->device;
    info->flags = m->flags;
    info->device_bytes = m->bytes;
    return LESASM_OK;
}

extern "C" int lesasm_mesh_node_permutation(const lesasm_mesh *m, int32_t *perm) {
    if (!m || (!perm && m->n_field > 0)) return fail(LESASM_E_INVALID_ARG, "node_permutation: NULL argument");
    if (m->n_field) std::memcpy(perm, m->h_fperm.data(), sizeof(int32_t) * m->n_field);
    return LESASM_OK;
}

extern "C" int lesasm_mesh_element_permutation(const lesasm_mesh *m, int64_t *perm) {
    if (!m || (!perm && m->n_elems > 0)) return fail(LESASM_E_INVALID_ARG, "element_permutation: NULL argument");
    if (m->n_elems) std::memcpy(perm, m->h_eperm.data(), sizeof(int64_t) * m->n_elems);
    return LESASM_OK;
}

static int permute(const lesasm_mesh *m, const double *in, double *out, int nc, void *stream, int to_internal) {
    if (!m) return fail(LESASM_E_INVALID_ARG, "permute: mesh is NULL");
    if (nc < 1 || nc > 64) return fail(LESASM_E_INVALID_ARG, "permute: ncomp must be in 1..64");
    if (m->n_field == 0) return LESASM_OK;
    if (!in || !out || in == out) return fail(LESASM_E_INVALID_ARG, "permute: NULL or aliased buffers");
    int dev = -1;
    LESASM_HIP_TRY(hipGetDevice(&dev));
    if (dev != m->device) return fail(LESASM_E_STATE, "permute: current device differs from the mesh's device");
    const size_t n = (size_t)m->n_field;
    hipLaunchKernelGGL(k_permute, dim3(grid_for(n * nc, 256)), dim3(256), 0, (hipStream_t)stream, in, out,
                       m->d_fperm, n, nc, to_internal);
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

extern "C" int lesasm_fields_to_internal(const lesasm_mesh *m, const double *d_user, double *d_internal, int ncomp,
                                         void *stream) {
    return permute(m, d_user, d_internal, ncomp, stream, 1);
}

extern "C" int lesasm_fields_to_user(const lesasm_mesh *m, const double *d_internal, double *d_user, int ncomp,
                                     void *stream) {
    return permute(m, d_internal, d_user, ncomp, stream, 0);
}

extern "C" int lesasm_mesh_lumped_mass(const lesasm_mesh *m, double *d_out, void *stream) {
    if (!m || (!d_out && m->n_field)) return fail(LESASM_E_INVALID_ARG, "lumped_mass: NULL argument");
    if (m->n_field)
        LESASM_HIP_TRY(hipMemcpyAsync(d_out, m->d_mass, sizeof(double) * m->n_field, hipMemcpyDeviceToDevice,
                                      (hipStream_t)stream));
    return LESASM_OK;
}

extern "C" int lesasm_mesh_filter_width(const lesasm_mesh *m, double *d_out, void *stream) {
    if (!m || (!d_out && m->n_elems)) return fail(LESASM_E_INVALID_ARG, "filter_width: NULL argument");
    if (m->n_elems)
        LESASM_HIP_TRY(hipMemcpyAsync(d_out, m->d_delta, sizeof(double) * m->n_elems, hipMemcpyDeviceToDevice,
                                      (hipStream_t)stream));
    return LESASM_OK;
}

extern "C" int lesasm_mesh_set_option(lesasm_mesh *m, int option, int64_t value) {
    if (!m) return fail(LESASM_E_INVALID_ARG, "set_option: mesh is NULL");
    switch (option) {
    case LESASM_OPT_PRECISION:
        if (value != LESASM_PREC_FP64 && value != LESASM_PREC_FP32)
            return fail(LESASM_E_UNSUPPORTED, "set_option: unknown precision");
        m->precision = (int)value;
        return LESASM_OK;
    case LESASM_OPT_RHS_MODE:
        if (value != LESASM_RHS_RESIDUAL && value != LESASM_RHS_INCREMENT)
            return fail(LESASM_E_UNSUPPORTED, "set_option: unknown rhs mode");
        m->rhs_mode = (int)value;
        return LESASM_OK;
    case LESASM_OPT_CHECK_FINITE:
        m->check_finite = value != 0;
        return LESASM_OK;
    case LESASM_OPT_BLOCK:
        if (value != 64 && value != 128 && value != 256)
            return fail(LESASM_E_UNSUPPORTED, "set_option: block must be 64, 128 or 256");
        m->block = (int)value;
        return LESASM_OK;
    case LESASM_OPT_PROFILE:
        m->profile = value != 0;
        return LESASM_OK;
    case LESASM_OPT_CONCURRENT:
        m->concurrent = value != 0;
        return LESASM_OK;
    case LESASM_OPT_PERSISTENT:
        if (value < 0 || value > INT32_MAX) return fail(LESASM_E_UNSUPPORTED, "set_option: persistent must be >= 0");
        m->persist = (int)value;
        return LESASM_OK;
    case LESASM_OPT_CHUNK: {
        if (value != 0 && (value < 32 || value > 4096))
            return fail(LESASM_E_UNSUPPORTED, "set_option: chunk must be 0 or in 32..4096");
        if (!is_chunked(m)) return fail(LESASM_E_STATE, "set_option: chunk size applies to the chunked scatters only");
        int cur = 0;
        LESASM_HIP_TRY(hipGetDevice(&cur));
        if (cur != m->device) return fail(LESASM_E_STATE, "set_option: current device differs from the mesh's device");
        LESASM_HIP_TRY(hipDeviceSynchronize());
        m->chunk_elems = (int)value;
        return build_scatter(m);
    }
    default:
        return fail(LESASM_E_INVALID_ARG, "set_option: unknown option " + std::to_string(option));
    }
}

extern "C" int lesasm_mesh_get_option(const lesasm_mesh *m, int option, int64_t *value) {
    if (!m || !value) return fail(LESASM_E_INVALID_ARG, "get_option: NULL argument");
    switch (option) {
    case LESASM_OPT_PRECISION: *value = m->precision; return LESASM_OK;
    case LESASM_OPT_RHS_MODE: *value = m->rhs_mode; return LESASM_OK;
    case LESASM_OPT_CHECK_FINITE: *value = m->check_finite; return LESASM_OK;
    case LESASM_OPT_BLOCK: *value = m->block; return LESASM_OK;
    case LESASM_OPT_PROFILE: *value = m->profile; return LESASM_OK;
    case LESASM_OPT_CHUNK: *value = m->chunk_elems; return LESASM_OK;
    case LESASM_OPT_CONCURRENT: *value = m->concurrent; return LESASM_OK;
    case LESASM_OPT_PERSISTENT: *value = m->persist; return LESASM_OK;
    default: return fail(LESASM_E_INVALID_ARG, "get_option: unknown option " + std::to_string(option));
    }
}

extern "C" int lesasm_mesh_set_wall(lesasm_mesh *m, const lesasm_wall_desc *d) {
    if (!m || !d) return fail(LESASM_E_INVALID_ARG, "set_wall: NULL argument");
    if (d->n_faces < 0 || (d->n_faces > 0 && (!d->face_offsets || !d->face_conn || !d->face_elem)))
        return fail(LESASM_E_INVALID_ARG, "set_wall: bad face arrays");
    if (d->n_faces > INT32_MAX) return fail(LESASM_E_UNSUPPORTED, "set_wall: too many faces");
    int cur = 0;
    LESASM_HIP_TRY(hipGetDevice(&cur));
    if (cur != m->device) return fail(LESASM_E_STATE, "set_wall: current device differs from the mesh's device");
    const int64_t F = d->n_faces;
    std::vector<int32_t> fg(4 * (size_t)F, -1), ff(4 * (size_t)F, -1), eg(8 * (size_t)F, -1), ef(8 * (size_t)F, -1);
    std::vector<int64_t> einv(m->n_elems, -1);
    for (int64_t i = 0; i < m->n_elems; ++i) einv[m->h_eperm[i]] = i;
    if (d->face_offsets[0] != 0) return fail(LESASM_E_INVALID_ARG, "set_wall: face_offsets[0] must be 0");
    for (int64_t f = 0; f < F; ++f) {
        const int64_t o = d->face_offsets[f], nfn = d->face_offsets[f + 1] - o;
        if (nfn != 3 && nfn != 4)
            return fail(LESASM_E_INVALID_ARG, "set_wall: face " + std::to_string(f) + " has neither 3 nor 4 nodes");
        for (int64_t b = 0; b < nfn; ++b) {
            const int32_t g = d->face_conn[o + b];
            if (g < 0 || g >= m->n_nodes)
                return fail(LESASM_E_INVALID_ARG, "set_wall: face " + std::to_string(f) + " node out of range");
            fg[4 * f + b] = m->h_gint[g];
            ff[4 * f + b] = m->h_fint[g];
        }
        const int64_t e = d->face_elem[f];
        if (e < 0 || e >= m->n_elems)
            return fail(LESASM_E_INVALID_ARG, "set_wall: face " + std::to_string(f) + " element out of range");
        const int64_t i = einv[e];
        int k = 0;
        while (k < kNumCat - 1 && !(i >= m->cat[k].first && i < m->cat[k].first + m->cat[k].n)) ++k;
        const Category &c = m->cat[k];
        const int64_t j = i - c.first;
        const std::vector<int32_t> &cf = c.h_cf.empty() ? c.h_cg : c.h_cf;
        for (int a = 0; a < c.type; ++a) {
            eg[8 * f + a] = c.h_cg[(size_t)a * c.n + j];
            ef[8 * f + a] = cf[(size_t)a * c.n + j];
        }
    }
    LESASM_HIP_TRY(hipDeviceSynchronize());
    dfree(m, m->d_wall_fg);
    dfree(m, m->d_wall_ff);
    dfree(m, m->d_wall_eg);
    dfree(m, m->d_wall_ef);
    m->n_wall = 0;
    int st;
    if (F > 0) {
        if ((st = upload(m, &m->d_wall_fg, fg)) || (st = upload(m, &m->d_wall_ff, ff)) ||
            (st = upload(m, &m->d_wall_eg, eg)) || (st = upload(m, &m->d_wall_ef, ef)))
            return st;
    }
    m->n_wall = F;
    return LESASM_OK;
}

extern "C" int lesasm_assemble_wall(lesasm_mesh *m, const double *d_u, double nu, double *d_rhs, void *stream) {
    if (!m) return fail(LESASM_E_INVALID_ARG, "assemble_wall: mesh is NULL");
    if (m->n_wall == 0) return LESASM_OK;
    if (!d_u || !d_rhs) return fail(LESASM_E_INVALID_ARG, "assemble_wall: u or rhs is NULL");
    if (((uintptr_t)d_u & 7u) || ((uintptr_t)d_rhs & 7u))
        return fail(LESASM_E_INVALID_ARG, "assemble_wall: pointers must be 8-byte aligned");
    if (d_rhs == d_u) return fail(LESASM_E_INVALID_ARG, "assemble_wall: rhs aliases u");
    if (!(nu > 0.0)) return fail(LESASM_E_INVALID_ARG, "assemble_wall: nu must be positive");
    int cur = 0;
    LESASM_HIP_TRY(hipGetDevice(&cur));
    if (cur != m->device) return fail(LESASM_E_STATE, "assemble_wall: current device differs from the mesh's device");
    return launch_wall(m, d_u, nu, d_rhs, (hipStream_t)stream);
}

extern "C" int lesasm_mesh_set_closure(lesasm_mesh *m, const lesasm_mlp *mlp, double delta_ref, double fallback_tol) {
    if (!m) return fail(LESASM_E_INVALID_ARG, "set_closure: mesh is NULL");
    if (mlp && (!(delta_ref > 0.0) || !(fallback_tol >= 0.0)))
        return fail(LESASM_E_INVALID_ARG, "set_closure: need delta_ref > 0 and fallback_tol >= 0");
    if (mlp && !is_chunked(m)) return fail(LESASM_E_UNSUPPORTED, "set_closure: needs a chunked scatter");
    int cur = 0;
    LESASM_HIP_TRY(hipGetDevice(&cur));
    if (cur != m->device) return fail(LESASM_E_STATE, "set_closure: current device differs from the mesh's device");
    LESASM_HIP_TRY(hipDeviceSynchronize());
    if (mlp && !m->d_fallbacks) {  // kFallbackSlots counters per category
        int st = dalloc(m, &m->d_fallbacks, (size_t)kNumCat * kFallbackSlots);
        if (st) return st;
        LESASM_HIP_TRY(hipMemset(m->d_fallbacks, 0, sizeof(unsigned long long) * kNumCat * kFallbackSlots));
    }
    m->mlp = mlp;
    m->delta_ref = mlp ? delta_ref : 1.0;
    m->fallback_tol = mlp ? fallback_tol : 0.05;
    const int cap = mlp ? 400 : 800;
    if (cap != m->chunk_max_nodes) {
        m->chunk_max_nodes = cap;
        return build_scatter(m);
    }
    return LESASM_OK;
}

extern "C" int lesasm_mesh_closure_fallbacks_by_type(lesasm_mesh *m, uint64_t *counts) {
    if (!m || !counts) return fail(LESASM_E_INVALID_ARG, "closure_fallbacks: NULL argument");
    for (int k = 0; k < kNumCat; ++k) counts[k] = 0;
    if (!m->d_fallbacks) return LESASM_OK;
    std::vector<unsigned long long> v((size_t)kNumCat * kFallbackSlots);
    LESASM_HIP_TRY(hipDeviceSynchronize());
    LESASM_HIP_TRY(hipMemcpy(v.data(), m->d_fallbacks, sizeof(unsigned long long) * v.size(), hipMemcpyDeviceToHost));
    LESASM_HIP_TRY(hipMemset(m->d_fallbacks, 0, sizeof(unsigned long long) * v.size()));
    LESASM_HIP_TRY(hipDeviceSynchronize());
    for (int k = 0; k < kNumCat; ++k)
        for (int i = 0; i < kFallbackSlots; ++i) counts[k] += v[(size_t)k * kFallbackSlots + i];
    return LESASM_OK;
}

extern "C" int lesasm_mesh_closure_fallbacks(lesasm_mesh *m, uint64_t *count) {
    if (!count) return fail(LESASM_E_INVALID_ARG, "closure_fallbacks: NULL argument");
    uint64_t c[kNumCat];
    const int st = lesasm_mesh_closure_fallbacks_by_type(m, c);
    if (st) return st;
    *count = c[0] + c[1] + c[2] + c[3];
    return LESASM_OK;
}
