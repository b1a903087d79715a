// Space-filling-curve mesh partitioner and correction-coefficient load
// balancing (Section "Mesh partitioning and load balancing").
//
// Partitioner, on the device, in the paper's five steps:
//   i)   bounding box of the element locations   k_bbox_partial, k_bbox_final
//   ii)  regular 2^L grid in it; iv) Hilbert position of each element's bin;
//   iii) integer bin weights (64-bit atomics)     k_sfc_keys
//   v)   inclusive scan of the bin weights along the curve, targets
//        T_i = Lambda_i W / P, and the midpoint split of every element's bin
//                                                 k_scan_*, k_targets, k_assign
// Everything after the binning is integer arithmetic (weights, prefix sums)
// or the comparison of an exact integer with a target, so the parts do not
// depend on the launch shape or the order of the atomics.
//
// Balancing (host): per splitting point a weighted linear regression of
// (Lambda_i^k, Upsilon_i^k) cut with y = i.
#include <cmath>
#include <vector>

#include "common.hpp"

namespace lesasm {

namespace {

constexpr int kBboxBlocks = 2048;
constexpr int kScanTile = 4096;  // bins per scan block: 1024 threads x 4
constexpr int kMaxLevel = 8;

// Position of bin (x, y, z) on the Hilbert curve of a 2^level grid
// (J. Skilling, "Programming the Hilbert curve", AIP Conf. Proc. 707, 2004):
// the axes are transformed level by level from the top so that each level's
// sub-cube is entered the right way round, Gray-encoded, and the index is read
// from the transposed bits, most significant level first, x before y before z.
__device__ __forceinline__ uint32_t hilbert_position(uint32_t x, uint32_t y, uint32_t z, int level) {
    uint32_t a[3] = {x, y, z};
    for (uint32_t q = 1u << (level - 1); q > 1; q >>= 1) {
        const uint32_t low = q - 1;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (a[i] & q) {
                a[0] ^= low;
            } else {
                const uint32_t t = (a[0] ^ a[i]) & low;
                a[0] ^= t;
                a[i] ^= t;
            }
        }
    }
    a[1] ^= a[0];
    a[2] ^= a[1];
    uint32_t flip = 0;
    for (uint32_t q = 1u << (level - 1); q > 1; q >>= 1)
        if (a[2] & q) flip ^= q - 1;
    uint32_t h = 0;
    for (int b = level - 1; b >= 0; --b)
#pragma unroll
        for (int i = 0; i < 3; ++i) h = (h << 1) | (((a[i] ^ flip) >> b) & 1u);
    return h;
}

// Bin of coordinate c on an axis with bounds lo, hi: floor((c - lo) / (hi -
// lo) * nb), clamped into [0, nb - 1] (0 on a flat axis or for a NaN).
__device__ __forceinline__ uint32_t bin_of(double c, double lo, double hi, int nb) {
    const double ext = hi - lo;
    if (!(ext > 0.0)) return 0;
    const double t = floor((c - lo) / ext * (double)nb);
    if (!(t >= 0.0)) return 0;
    return t >= (double)(nb - 1) ? (uint32_t)(nb - 1) : (uint32_t)t;
}

__global__ __launch_bounds__(256) void k_centroids(int64_t n, const int64_t *__restrict__ off,
                                                   const int32_t *__restrict__ conn, int64_t conn_len, int64_t n_nodes,
                                                   const double *__restrict__ xyz, double *__restrict__ cen,
                                                   int32_t *__restrict__ wts, int32_t *__restrict__ flag) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = off[e], k64 = off[e + 1] - b;
        const int k = (k64 >= 4 && k64 <= 8) ? (int)k64 : 0;
        const int w = k == 4 ? 4 : k == 5 ? 8 : k == 6 ? 6 : k == 8 ? 8 : 0;
        if (!w || b < 0 || b + k > conn_len) {
            atomicOr(flag, 1);
            continue;
        }
        double s[3] = {0.0, 0.0, 0.0};
        bool ok = true;
        for (int a = 0; a < k; ++a) {
            const int32_t g = conn[b + a];
            if (g < 0 || g >= n_nodes) {
                ok = false;
                break;
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) s[d] += xyz[3 * (size_t)g + d];
        }
        if (!ok) {
            atomicOr(flag, 2);
            continue;
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) cen[3 * e + d] = s[d] / (double)k;
        if (wts) wts[e] = w;
    }
}

// Per block: min and max of each coordinate over a grid-stride slice.
__global__ __launch_bounds__(256) void k_bbox_partial(int64_t n, const double *__restrict__ c,
                                                      double *__restrict__ partial) {
    __shared__ double sh[6][256];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double v = c[3 * e + d];
            lo[d] = fmin(lo[d], v);
            hi[d] = fmax(hi[d], v);
        }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        sh[d][threadIdx.x] = lo[d];
        sh[3 + d][threadIdx.x] = hi[d];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                sh[d][threadIdx.x] = fmin(sh[d][threadIdx.x], sh[d][threadIdx.x + w]);
                sh[3 + d][threadIdx.x] = fmax(sh[3 + d][threadIdx.x], sh[3 + d][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) partial[6 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_bbox_final(const double *__restrict__ partial, int nb,
                                                    double *__restrict__ box) {
    __shared__ double sh[6][256];
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nb; b += blockDim.x)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            v[d] = fmin(v[d], partial[6 * b + d]);
            v[3 + d] = fmax(v[3 + d], partial[6 * b + 3 + d]);
        }
#pragma unroll
    for (int d = 0; d < 6; ++d) sh[d][threadIdx.x] = v[d];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                sh[d][threadIdx.x] = fmin(sh[d][threadIdx.x], sh[d][threadIdx.x + w]);
                sh[3 + d][threadIdx.x] = fmax(sh[3 + d][threadIdx.x], sh[3 + d][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) box[threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long *__restrict__ a, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0ull;
}

// Hilbert key of each element's bin; bin weights summed with 64-bit atomics.
// Neighbouring elements mostly share a bin, so each wavefront first merges
// runs of equal keys in lane order (segmented scan over run ids) and only the
// last lane of a run adds the run's weight: integer sums, so the bin weights
// are exact whatever the grouping.
__global__ __launch_bounds__(256) void k_sfc_keys(int64_t n, const double *__restrict__ c,
                                                  const int32_t *__restrict__ wts, const double *__restrict__ box,
                                                  int level, uint32_t *__restrict__ key,
                                                  unsigned long long *__restrict__ binw) {
    const int nb = 1 << level;
    const double lo0 = box[0], lo1 = box[1], lo2 = box[2], hi0 = box[3], hi1 = box[4], hi2 = box[5];
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // the loop runs the same number of times in every lane of a wavefront
    for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
        const int64_t e = base + threadIdx.x;
        const bool valid = e < n;
        uint32_t h = 0xffffffffu;
        unsigned long long v = 0ull;
        if (valid) {
            const uint32_t bx = bin_of(c[3 * e + 0], lo0, hi0, nb);
            const uint32_t by = bin_of(c[3 * e + 1], lo1, hi1, nb);
            const uint32_t bz = bin_of(c[3 * e + 2], lo2, hi2, nb);
            h = hilbert_position(bx, by, bz, level);
            key[e] = h;
            v = (unsigned long long)(long long)(wts ? wts[e] : 1);
        }
        const uint32_t prev = __shfl_up(h, 1);
        const bool head = lane == 0 || prev != h;
        const unsigned long long heads = __ballot(head);
        const int run = __popcll(heads & (~0ull >> (63 - lane)));  // runs started at or before this lane
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned long long up = __shfl_up(v, o);
            const int run_up = __shfl_up(run, o);
            if (lane >= o && run_up == run) v += up;
        }
        const uint32_t next = __shfl_down(h, 1);
        const bool tail = lane == 63 || next != h;
        if (tail && h != 0xffffffffu) atomicAdd(binw + h, v);
    }
}

// Inclusive scan in three passes over tiles of kScanTile bins.
__device__ __forceinline__ unsigned long long block_inclusive_1024(unsigned long long v, unsigned long long *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const unsigned long long add = (int)threadIdx.x >= o ? sh[threadIdx.x - o] : 0ull;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    return sh[threadIdx.x];
}

__global__ __launch_bounds__(1024) void k_scan_tile_sums(const unsigned long long *__restrict__ a, int64_t n,
                                                         unsigned long long *__restrict__ sums) {
    __shared__ unsigned long long sh[1024];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + 4 * threadIdx.x;
    unsigned long long v = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (base + j < n) v += a[base + j];
    v = block_inclusive_1024(v, sh);
    if (threadIdx.x == 1023) sums[blockIdx.x] = v;
}

// Exclusive scan of the tile sums in place (one block, any count).
__global__ __launch_bounds__(1024) void k_scan_tile_offsets(unsigned long long *__restrict__ sums, int nt) {
    __shared__ unsigned long long sh[1024];
    unsigned long long carry = 0;
    for (int b = 0; b < nt; b += 1024) {
        const int i = b + threadIdx.x;
        const unsigned long long v = i < nt ? sums[i] : 0ull;
        const unsigned long long inc = block_inclusive_1024(v, sh);
        if (i < nt) sums[i] = carry + inc - v;
        carry += sh[1023];
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void k_scan_apply(unsigned long long *__restrict__ a, int64_t n,
                                                     const unsigned long long *__restrict__ offs) {
    __shared__ unsigned long long sh[1024];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + 4 * threadIdx.x;
    unsigned long long v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = base + j < n ? a[base + j] : 0ull;
    const unsigned long long own = v[0] + v[1] + v[2] + v[3];
    unsigned long long run = block_inclusive_1024(own, sh) - own + offs[blockIdx.x];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        run += v[j];
        if (base + j < n) a[base + j] = run;
    }
}

// Correction coefficients passed by value (up to kArgLambda parts).
constexpr int kArgLambda = 256;
struct LambdaArg {
    double v[kArgLambda];
};

// t2[i] = 2 T_{i+1} = 2 (Lambda_{i+1} W / P), i < P - 1 (one thread: the
// coefficients are summed in order).  Coefficients from `lam` (device) if set,
// else from `la` if use_arg, else all 1.
__global__ void k_targets(const double *__restrict__ lam, LambdaArg la, int use_arg, int P,
                          const unsigned long long *__restrict__ cum, int64_t nbins, double *__restrict__ t2) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double W = (double)cum[nbins - 1];
    double acc = 0.0;
    for (int i = 0; i + 1 < P; ++i) {
        acc = acc + (lam ? lam[i] : use_arg ? la.v[i] : 1.0);
        t2[i] = 2.0 * (acc * W / (double)P);
    }
}

// part = number of targets at or below the midpoint of the element's bin.
__global__ __launch_bounds__(256) void k_assign(int64_t n, const uint32_t *__restrict__ key,
                                                const unsigned long long *__restrict__ cum,
                                                const double *__restrict__ t2, int P, int32_t *__restrict__ part) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t h = key[e];
        const unsigned long long mid2 = cum[h] + (h ? cum[h - 1] : 0ull);  // 2 S_b + w_b
        const double m = (double)mid2;
        int lo = 0, hi = P - 1;  // first index in [0, P-1) with t2 > m, else P - 1
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (t2[mid] <= m)
                lo = mid + 1;
            else
                hi = mid;
        }
        part[e] = lo;
    }
}

struct Workspace {
    double *partial, *box, *t2, *lam;
    unsigned long long *cum, *tiles;
    uint32_t *key;
    size_t bytes;
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

Workspace layout(void *base, int64_t n, int P, int level) {
    const int64_t nbins = (int64_t)1 << (3 * level);
    const int64_t ntiles = (nbins + kScanTile - 1) / kScanTile;
    char *p = (char *)base;
    size_t o = 0;
    Workspace w{};
    auto take = [&](size_t b) {
        char *q = p ? p + o : nullptr;
        o += align256(b);
        return q;
    };
    w.partial = (double *)take(sizeof(double) * 6 * kBboxBlocks);
    w.box = (double *)take(sizeof(double) * 6);
    w.t2 = (double *)take(sizeof(double) * (size_t)(P > 1 ? P - 1 : 1));
    w.lam = (double *)take(sizeof(double) * (size_t)P);
    w.cum = (unsigned long long *)take(sizeof(unsigned long long) * (size_t)nbins);
    w.tiles = (unsigned long long *)take(sizeof(unsigned long long) * (size_t)ntiles);
    w.key = (uint32_t *)take(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    w.bytes = o;
    return w;
}

}  // namespace

}  // namespace lesasm

using namespace lesasm;

extern "C" int lesasm_element_centroids(int64_t n_elems, const int64_t *d_off, const int32_t *d_conn, int64_t conn_len,
                                        int64_t n_nodes, const double *d_coords, double *d_cen, int32_t *d_wts,
                                        int32_t *d_status, void *stream) {
    if (n_elems < 0 || n_nodes < 0 || conn_len < 0) return fail(LESASM_E_INVALID_ARG, "element_centroids: negative size");
    if (n_elems == 0) return LESASM_OK;
    if (!d_off || !d_conn || !d_coords || !d_cen || !d_status)
        return fail(LESASM_E_INVALID_ARG, "element_centroids: NULL argument");
    hipLaunchKernelGGL(k_centroids, dim3(grid_for((size_t)n_elems, 256)), dim3(256), 0, (hipStream_t)stream, n_elems,
                       d_off, d_conn, conn_len, n_nodes, d_coords, d_cen, d_wts, d_status);
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

extern "C" int lesasm_sfc_workspace_bytes(int64_t n_elems, int n_parts, int level, size_t *bytes) {
    if (!bytes || n_elems < 0 || n_parts < 1 || level < 1 || level > kMaxLevel)
        return fail(LESASM_E_INVALID_ARG, "sfc_workspace_bytes: bad argument");
    *bytes = layout(nullptr, n_elems, n_parts, level).bytes;
    return LESASM_OK;
}

extern "C" int lesasm_sfc_partition(int64_t n, const double *d_cen, const int32_t *d_wts, int P, const double *h_lambda,
                                    int level, void *d_work, size_t work_bytes, int32_t *d_part, void *stream) {
    if (n < 0 || P < 1 || level < 1 || level > kMaxLevel)
        return fail(LESASM_E_INVALID_ARG, "sfc_partition: bad size, part count or level");
    if (n > (int64_t)INT32_MAX) return fail(LESASM_E_INVALID_ARG, "sfc_partition: more than 2^31-1 elements");
    if (n == 0) return LESASM_OK;
    if (!d_cen || !d_part || !d_work) return fail(LESASM_E_INVALID_ARG, "sfc_partition: NULL argument");
    if (((uintptr_t)d_work & 255) != 0) return fail(LESASM_E_INVALID_ARG, "sfc_partition: workspace not 256-byte aligned");
    const Workspace w = layout(d_work, n, P, level);
    if (work_bytes < w.bytes) return fail(LESASM_E_INVALID_ARG, "sfc_partition: workspace too small");
    if (h_lambda)
        for (int i = 0; i < P; ++i)
            if (!std::isfinite(h_lambda[i]) || h_lambda[i] < 0.0)
                return fail(LESASM_E_INVALID_ARG, "sfc_partition: correction coefficient negative or not finite");
    hipStream_t s = (hipStream_t)stream;
    const int64_t nbins = (int64_t)1 << (3 * level);
    const int ntiles = (int)((nbins + kScanTile - 1) / kScanTile);
    // up to kArgLambda coefficients travel in the kernel arguments; more are
    // copied and waited for, so h_lambda is never read after the call returns
    LambdaArg la{};
    const bool by_arg = h_lambda && P <= kArgLambda;
    if (by_arg)
        for (int i = 0; i < P; ++i) la.v[i] = h_lambda[i];
    if (h_lambda && !by_arg) {
        LESASM_HIP_TRY(hipMemcpyAsync(w.lam, h_lambda, sizeof(double) * P, hipMemcpyHostToDevice, s));
        LESASM_HIP_TRY(hipStreamSynchronize(s));
    }
    const int g = grid_for((size_t)n, 256);
    hipLaunchKernelGGL(k_bbox_partial, dim3(kBboxBlocks), dim3(256), 0, s, n, d_cen, w.partial);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(256), 0, s, w.partial, kBboxBlocks, w.box);
    hipLaunchKernelGGL(k_zero_u64, dim3(grid_for((size_t)nbins, 256)), dim3(256), 0, s, w.cum, nbins);
    hipLaunchKernelGGL(k_sfc_keys, dim3(g), dim3(256), 0, s, n, d_cen, d_wts, w.box, level, w.key, w.cum);
    hipLaunchKernelGGL(k_scan_tile_sums, dim3(ntiles), dim3(1024), 0, s, w.cum, nbins, w.tiles);
    hipLaunchKernelGGL(k_scan_tile_offsets, dim3(1), dim3(1024), 0, s, w.tiles, ntiles);
    hipLaunchKernelGGL(k_scan_apply, dim3(ntiles), dim3(1024), 0, s, w.cum, nbins, w.tiles);
    hipLaunchKernelGGL(k_targets, dim3(1), dim3(1), 0, s, (h_lambda && !by_arg) ? w.lam : nullptr, la, by_arg ? 1 : 0,
                       P, w.cum, nbins, w.t2);
    hipLaunchKernelGGL(k_assign, dim3(g), dim3(256), 0, s, n, w.key, w.cum, w.t2, P, d_part);
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

extern "C" int lesasm_balance_update(int P, int K, const double *lam_hist, const double *t_hist, double growth,
                                     double *lam_out) {
    if (!lam_hist || !t_hist || !lam_out || P < 1 || K < 1 || !(growth > 0.0) || !std::isfinite(growth))
        return fail(LESASM_E_INVALID_ARG, "balance_update: bad argument");
    std::vector<double> X((size_t)K * P), Y((size_t)K * P), wk(K);
    for (int k = 0; k < K; ++k) {
        double lam_sum = 0.0, t_sum = 0.0;
        for (int i = 0; i < P; ++i) {
            const double l = lam_hist[(size_t)k * P + i], t = t_hist[(size_t)k * P + i];
            if (!std::isfinite(l) || l < 0.0 || !std::isfinite(t) || t < 0.0)
                return fail(LESASM_E_INVALID_ARG, "balance_update: coefficient or time negative or not finite");
            t_sum += t;
        }
        const double mean = t_sum / P;
        if (!(mean > 0.0)) return fail(LESASM_E_INVALID_ARG, "balance_update: zero mean time");
        double run = 0.0;
        for (int i = 0; i < P; ++i) {
            lam_sum += lam_hist[(size_t)k * P + i];
            run += t_hist[(size_t)k * P + i];
            X[(size_t)k * P + i] = lam_sum;  // Lambda_{i+1}^k
            Y[(size_t)k * P + i] = run / mean;  // Upsilon_{i+1}^k
        }
        wk[k] = std::pow(growth, (double)k);
    }
    std::vector<double> cut(P + 1);
    cut[0] = 0.0;
    cut[P] = (double)P;
    for (int i = 1; i < P; ++i) {
        double next = 0.0;
        bool have = false;
        if (K >= 2) {
            double sw = 0.0, sx = 0.0, sy = 0.0, xmin = INFINITY, xmax = -INFINITY;
            for (int k = 0; k < K; ++k) {
                const double xv = X[(size_t)k * P + i - 1], yv = Y[(size_t)k * P + i - 1];
                sw += wk[k];
                sx += wk[k] * xv;
                sy += wk[k] * yv;
                xmin = std::fmin(xmin, xv);
                xmax = std::fmax(xmax, xv);
            }
            const double mx = sx / sw, my = sy / sw;
            double sxx = 0.0, sxy = 0.0;
            for (int k = 0; k < K; ++k) {
                const double dx = X[(size_t)k * P + i - 1] - mx, dy = Y[(size_t)k * P + i - 1] - my;
                sxx += wk[k] * dx * dx;
                sxy += wk[k] * dx * dy;
            }
            if (xmax - xmin > 1e-12 * P && sxx > 0.0) {
                const double beta = sxy / sxx, alpha = my - beta * mx;
                if (beta > 0.0) {
                    next = ((double)i - alpha) / beta;
                    have = true;
                }
            }
        }
        if (!have) {
            const double xl = X[(size_t)(K - 1) * P + i - 1], yl = Y[(size_t)(K - 1) * P + i - 1];
            next = yl > 0.0 ? (double)i * xl / yl : xl;
        }
        cut[i] = next;
    }
    for (int i = 1; i < P; ++i) cut[i] = std::fmin(std::fmax(cut[i], cut[i - 1]), (double)P);
    for (int i = 0; i < P; ++i) lam_out[i] = cut[i + 1] - cut[i];
    return LESASM_OK;
}
