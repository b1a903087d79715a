// Fractional-step time integration on the GPU (Section 3.2 and Algorithm 1).
//
// Algorithm 1 assembles the Laplacian matrix once before the time loop, then
// per time step runs three Runge-Kutta stages (element assembly, momentum
// update) and one pressure solve by Jacobi-preconditioned conjugate gradients.
// The paper names a third-order Runge-Kutta scheme without its coefficients;
// the tableau here is Heun's third-order method, c = (0, 1/3, 2/3),
// a21 = 1/3, a32 = 2/3, b = (1/4, 0, 3/4).  Projection (incremental):
//   u*     = u^n + dt (k1/4 + 3 k3/4),  k_s = M_L^-1 rhs(u_s, p^n)
//   K dp   = -(1/dt) D u*   (right-hand side projected to zero mean; dp zero mean)
//   u^n+1  = u* - dt M_L^-1 G dp,   p^n+1 = p^n + dp
// with K = int grad N_a . grad N_b, (D u)_a = int N_a div u, (G p)_a = int N_a grad p.
// Everything is FP64.  These are support operations for the assembly; their
// element loops use direct FP64 atomics.
#include <algorithm>
#include <cmath>

#include "element.hpp"

namespace lesasm {

// ---- element operators -----------------------------------------------------

template <int T>
__device__ __forceinline__ void load_geometry(const CatView &c, int e, const double *__restrict__ xyz,
                                              double (&x)[Ref<T>::nn][3], int (&fid)[Ref<T>::nn]) {
    constexpr int nn = Ref<T>::nn;
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
}

// Jacobian at Gauss point g, its inverse (K[k][i] = dxi_k/dx_i) and det.
template <int T>
__device__ __forceinline__ double jac_inverse(const double (&x)[Ref<T>::nn][3], int g, double (&Ki)[3][3]) {
    constexpr int nn = Ref<T>::nn;
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int a = 1; a < nn; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k) J[i][k] += x[a][i] * Ref<T>::tab.dN[g][a][k];
    double adj[3][3];
    adj[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    adj[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    adj[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    adj[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    adj[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    adj[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    adj[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    adj[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    adj[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double det = J[0][0] * adj[0][0] + J[0][1] * adj[1][0] + J[0][2] * adj[2][0];
    const double r = 1.0 / det;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) Ki[i][k] = adj[i][k] * r;
    return det;
}

// (D u)_a += sum_g w det N_a div u
template <int T>
__global__ __launch_bounds__(256) void k_divergence(CatView c, const double *__restrict__ xyz,
                                                    const double *__restrict__ u, double *__restrict__ out) {
    using E = Ref<T>;
    constexpr int nn = E::nn;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= c.n) return;
    double x[nn][3], uu[nn][3], m[nn];
    int fid[nn];
    load_geometry<T>(c, e, xyz, x, fid);
#pragma unroll
    for (int a = 0; a < nn; ++a) {
        m[a] = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) uu[a][k] = u[3 * (size_t)fid[a] + k];
    }
#pragma unroll
    for (int g = 0; g < E::ng; ++g) {
        double Ki[3][3];
        const double det = jac_inverse<T>(x, g, Ki);
        double div = 0.0;
#pragma unroll
        for (int a = 0; a < nn; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double dnx = Ki[0][i] * E::tab.dN[g][a][0] + Ki[1][i] * E::tab.dN[g][a][1] +
                                   Ki[2][i] * E::tab.dN[g][a][2];
                div += uu[a][i] * dnx;
            }
        const double wd = E::tab.w[g] * det * div;
#pragma unroll
        for (int a = 0; a < nn; ++a) m[a] += wd * E::tab.N[g][a];
    }
#pragma unroll
    for (int a = 0; a < nn; ++a) unsafeAtomicAdd(out + fid[a], m[a]);
}

// (G p)_a += sum_g w det N_a grad p
template <int T>
__global__ __launch_bounds__(256) void k_gradient(CatView c, const double *__restrict__ xyz,
                                                  const double *__restrict__ p, double *__restrict__ out) {
    using E = Ref<T>;
    constexpr int nn = E::nn;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= c.n) return;
    double x[nn][3], pp[nn], m[nn][3];
    int fid[nn];
    load_geometry<T>(c, e, xyz, x, fid);
#pragma unroll
    for (int a = 0; a < nn; ++a) {
        pp[a] = p[fid[a]];
        m[a][0] = m[a][1] = m[a][2] = 0.0;
    }
#pragma unroll
    for (int g = 0; g < E::ng; ++g) {
        double Ki[3][3];
        const double det = jac_inverse<T>(x, g, Ki);
        double gp[3] = {0, 0, 0};
#pragma unroll
        for (int a = 0; a < nn; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i)
                gp[i] += pp[a] * (Ki[0][i] * E::tab.dN[g][a][0] + Ki[1][i] * E::tab.dN[g][a][1] +
                                  Ki[2][i] * E::tab.dN[g][a][2]);
        const double wd = E::tab.w[g] * det;
#pragma unroll
        for (int a = 0; a < nn; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) m[a][i] += wd * E::tab.N[g][a] * gp[i];
    }
#pragma unroll
    for (int a = 0; a < nn; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i) unsafeAtomicAdd(out + 3 * (size_t)fid[a] + i, m[a][i]);
}

__device__ __forceinline__ int find_col(const int32_t *__restrict__ col, int lo, int hi, int key) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (col[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// K_ab += sum_g w det grad N_a . grad N_b into the CSR matrix (rows = field nodes)
template <int T>
__global__ __launch_bounds__(256) void k_laplacian(CatView c, const double *__restrict__ xyz,
                                                   const int32_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ col, double *__restrict__ val) {
    using E = Ref<T>;
    constexpr int nn = E::nn;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= c.n) return;
    double x[nn][3], Ke[nn][nn];
    int fid[nn];
    load_geometry<T>(c, e, xyz, x, fid);
#pragma unroll
    for (int a = 0; a < nn; ++a)
#pragma unroll
        for (int b = 0; b < nn; ++b) Ke[a][b] = 0.0;
#pragma unroll
    for (int g = 0; g < E::ng; ++g) {
        double Ki[3][3], dx[nn][3];
        const double det = jac_inverse<T>(x, g, Ki);
#pragma unroll
        for (int a = 0; a < nn; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i)
                dx[a][i] = Ki[0][i] * E::tab.dN[g][a][0] + Ki[1][i] * E::tab.dN[g][a][1] +
                           Ki[2][i] * E::tab.dN[g][a][2];
        const double wd = E::tab.w[g] * det;
#pragma unroll
        for (int a = 0; a < nn; ++a)
#pragma unroll
            for (int b = 0; b < nn; ++b) Ke[a][b] += wd * (dx[a][0] * dx[b][0] + dx[a][1] * dx[b][1] + dx[a][2] * dx[b][2]);
    }
#pragma unroll
    for (int a = 0; a < nn; ++a) {
        const int r0 = rowptr[fid[a]], r1 = rowptr[fid[a] + 1];
#pragma unroll
        for (int b = 0; b < nn; ++b) unsafeAtomicAdd(val + find_col(col, r0, r1, fid[b]), Ke[a][b]);
    }
}

// ---- vector kernels ----------------------------------------------------------

__global__ void k_spmv(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                       const double *__restrict__ val, const double *__restrict__ x, double *__restrict__ y, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int q = rowptr[i]; q < rowptr[i + 1]; ++q) s += val[q] * x[col[q]];
    y[i] = s;
}

constexpr int kRedBlocks = 512;

// Fixed-order two-level reduction: partial[b] = sum over a grid-stride slice.
__global__ void k_dot_partial(const double *__restrict__ a, const double *__restrict__ b, int n,
                              double *__restrict__ partial) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        s += b ? a[i] * b[i] : a[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void k_reduce_final(const double *__restrict__ partial, int nb, double *__restrict__ out) {
    __shared__ double sh[kRedBlocks];
    sh[threadIdx.x] = (int)threadIdx.x < nb ? partial[threadIdx.x] : 0.0;
    __syncthreads();
    for (int w = kRedBlocks / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// Conjugate-gradient kernels.  A fixed grid (kCgBlocks x 256) walks the rows
// in a fixed order, so every reduction is deterministic.  4096 blocks (16 per
// CU) and four row entries in flight per lane keep enough loads outstanding
// to hide the indirect gather's latency (on 1.76 M rows, 38 M nonzeros: 0.168
// ms per iteration against 0.262 with 1024 blocks and one entry per lane).
#ifndef LESASM_CG_BLOCKS
#define LESASM_CG_BLOCKS 4096
#endif
#ifndef LESASM_CG_LANES
#define LESASM_CG_LANES 8
#endif
#ifndef LESASM_CG_UNROLL
#define LESASM_CG_UNROLL 4
#endif
constexpr int kCgBlocks = LESASM_CG_BLOCKS;
constexpr int kMaxCapturedCg = 100000;  // CG iterations a step graph may hold
constexpr int kLanesPerRow = LESASM_CG_LANES;
constexpr int kRowUnroll = LESASM_CG_UNROLL;

// Captured CG iterations (the step graph): iteration `it` runs only while
// it <= *state, where *state is the iteration that met the tolerance
// (INT32_MAX until then).  Eager solves pass state = NULL.
__device__ __forceinline__ bool cg_skip(const int *state, int it) { return state && it > *state; }

// Fixed-order sum of one value per thread of a 256-thread block into out[0].
__device__ __forceinline__ void block_sum_256(double v, double *sh, double *out) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
    __syncthreads();
}

// q = K p with kLanesPerRow lanes per row (coalesced reads of the row's
// entries, kRowUnroll of them in flight per lane, fixed shuffle tree), and
// partial[b] = block sums of p.q.  Each lane adds its entries in row order.
__global__ __launch_bounds__(256) void k_spmv_dot(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                                  const double *__restrict__ val, const double *__restrict__ p,
                                                  double *__restrict__ q, int n, double *__restrict__ partial,
                                                  const int *state = nullptr, int it = 0) {
    if (cg_skip(state, it)) return;
    __shared__ double sh[256];
    const int lane = threadIdx.x % kLanesPerRow;
    const int rows_per_block = 256 / kLanesPerRow;
    double pq = 0.0;
    for (int base = blockIdx.x * rows_per_block; base < n; base += gridDim.x * rows_per_block) {
        const int row = base + (int)threadIdx.x / kLanesPerRow;
        double s = 0.0;
        if (row < n) {
            const int k1 = rowptr[row + 1];
            for (int k = rowptr[row] + lane; k < k1; k += kRowUnroll * kLanesPerRow) {
                int c[kRowUnroll];
                double v[kRowUnroll];
#pragma unroll
                for (int j = 0; j < kRowUnroll; ++j) {
                    const int kk = k + j * kLanesPerRow;
                    c[j] = kk < k1 ? col[kk] : -1;
                    v[j] = kk < k1 ? val[kk] : 0.0;
                }
#pragma unroll
                for (int j = 0; j < kRowUnroll; ++j)
                    if (c[j] >= 0) s += v[j] * p[c[j]];
            }
        }
#pragma unroll
        for (int o = kLanesPerRow / 2; o > 0; o >>= 1) s += __shfl_down(s, o, kLanesPerRow);
        if (lane == 0 && row < n) {
            q[row] = s;
            pq += s * p[row];
        }
    }
    block_sum_256(pq, sh, partial + blockIdx.x);
}

#ifndef LESASM_CG_SELL
#define LESASM_CG_SELL 1
#endif
constexpr int kSlice = 64;  // rows per slice of the sliced-ELLPACK copy (one wavefront)
#ifndef LESASM_SELL_UNROLL
#define LESASM_SELL_UNROLL 4
#endif
#ifndef LESASM_SELL_NT
#define LESASM_SELL_NT 1
#endif
constexpr int kSellUnroll = LESASM_SELL_UNROLL;  // row entries in flight per lane
// the matrix is read once per SpMV: streamed past the caches when LESASM_SELL_NT
template <class T> __device__ __forceinline__ T sell_load(const T *a) {
    if (LESASM_SELL_NT) return __builtin_nontemporal_load(a);
    return *a;
}

// q = K p on the sliced-ELLPACK copy of K: slice s holds rows 64 s .. 64 s +
// 63, padded to its longest row and stored column-major, so entry j of all 64
// rows is one coalesced load; lane l adds row 64 s + l's entries in column
// order (four in flight).  Padding entries hold value 0 and a valid column.
// One wavefront per slice, slices in a fixed grid-stride order; partial[b] =
// block sums of p.q.
__global__ __launch_bounds__(256) void k_spmv_sell_dot(const int32_t *__restrict__ soff,
                                                       const int32_t *__restrict__ scol,
                                                       const double *__restrict__ sval, const double *__restrict__ p,
                                                       double *__restrict__ q, int n, int nslices,
                                                       double *__restrict__ partial, const int *state = nullptr,
                                                       int it = 0) {
    if (cg_skip(state, it)) return;
    __shared__ double sh[256];
    const int lane = threadIdx.x % kSlice, wave = threadIdx.x / kSlice;
    const int waves = 256 / kSlice;
    double pq = 0.0;
    for (int sl = blockIdx.x * waves + wave; sl < nslices; sl += gridDim.x * waves) {
        const int o0 = soff[sl], w = (soff[sl + 1] - o0) / kSlice;
        const int32_t *cc = scol + o0 + lane;
        const double *vv = sval + o0 + lane;
        double s = 0.0;
        int j = 0;
        for (; j + kSellUnroll <= w; j += kSellUnroll) {
            int c[kSellUnroll];
            double v[kSellUnroll];
#pragma unroll
            for (int k = 0; k < kSellUnroll; ++k) {
                c[k] = sell_load(cc + kSlice * (j + k));
                v[k] = sell_load(vv + kSlice * (j + k));
            }
#pragma unroll
            for (int k = 0; k < kSellUnroll; ++k) s += v[k] * p[c[k]];
        }
        for (; j < w; ++j) s += sell_load(vv + kSlice * j) * p[sell_load(cc + kSlice * j)];
        const int row = sl * kSlice + lane;
        if (row < n) {
            q[row] = s;
            pq += s * p[row];
        }
    }
    block_sum_256(pq, sh, partial + blockIdx.x);
}

// sliced-ELLPACK values from the assembled CSR values (src < 0: padding)
__global__ void k_sell_fill(const int32_t *__restrict__ src, const double *__restrict__ val, double *__restrict__ sval,
                            int64_t total) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
        sval[i] = src[i] >= 0 ? val[src[i]] : 0.0;
}

// alpha = rz / pq;  r -= alpha q;  z = r / diag  (x is advanced with the old
// direction by k_cg_direction, which reads p anyway);
// partial[2b] = block sums of r.z, partial[2b+1] = of r.r
__global__ __launch_bounds__(256) void k_cg_update(double *__restrict__ r, double *__restrict__ z,
                                                   const double *__restrict__ q, const double *__restrict__ diag,
                                                   const double *__restrict__ scal, int i_rz, int i_pq, int n,
                                                   double *__restrict__ partial, const int *state = nullptr,
                                                   int it = 0) {
    if (cg_skip(state, it)) return;
    __shared__ double sh[256];
    const double alpha = scal[i_rz] / scal[i_pq];
    double rz = 0.0, rr = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double ri = r[i] - alpha * q[i];
        const double zi = ri / diag[i];
        r[i] = ri;
        z[i] = zi;
        rz += ri * zi;
        rr += ri * ri;
    }
    block_sum_256(rz, sh, partial + 2 * blockIdx.x);
    block_sum_256(rr, sh, partial + 2 * blockIdx.x + 1);
}

// out[j] = fixed-order sum of partial[stride * b + j] over b < nb, for j < m
// (one 1024-thread block).  In a captured CG with conv set, iteration `it`
// that brings out1 (r.r) to at most tol2 * (*bb) records itself in *state.
__global__ __launch_bounds__(1024) void k_reduce_strided(const double *__restrict__ partial, int nb, int stride,
                                                         int m, double *__restrict__ out0, double *__restrict__ out1,
                                                         int *state = nullptr, int it = 0, bool conv = false,
                                                         const double *bb = nullptr, double tol2 = 0.0) {
    if (cg_skip(state, it)) return;
    __shared__ double sh[1024];
    for (int j = 0; j < m; ++j) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nb; b += blockDim.x) v += partial[stride * b + j];
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int w = 512; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) *(j == 0 ? out0 : out1) = sh[0];
        __syncthreads();
    }
    if (conv && threadIdx.x == 0 && *out1 <= tol2 * *bb) *state = it;
}

// x += (rz_old / pq) p;  p = z + (rz_new / rz_old) p
__global__ __launch_bounds__(256) void k_cg_direction(double *__restrict__ x, double *__restrict__ p,
                                                      const double *__restrict__ z, const double *__restrict__ scal,
                                                      int i_new, int i_old, int i_pq, int n,
                                                      const int *state = nullptr, int it = 0) {
    if (cg_skip(state, it)) return;
    const double alpha = scal[i_old] / scal[i_pq];
    const double beta = scal[i_new] / scal[i_old];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double pi = p[i];
        x[i] += alpha * pi;
        p[i] = z[i] + beta * pi;
    }
}

// y = a0 x0 + a1 x1 + a2 x2 (x1, x2 may be NULL)
__global__ void k_lincomb(double *__restrict__ y, double a0, const double *__restrict__ x0, double a1,
                          const double *__restrict__ x1, double a2, const double *__restrict__ x2, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        double v = a0 * x0[i];
        if (x1) v += a1 * x1[i];
        if (x2) v += a2 * x2[i];
        y[i] = v;
    }
}

// y[i] += alpha * x[i] with alpha = scale * (*num) / (*den), read on the device
__global__ void k_axpy_ratio(double *__restrict__ y, const double *__restrict__ x, const double *num,
                             const double *den, double scale, int n) {
    const double alpha = scale * (*num) / (*den);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) y[i] += alpha * x[i];
}

// p = z + (num/den) p
__global__ void k_xpby_ratio(double *__restrict__ p, const double *__restrict__ z, const double *num,
                             const double *den, int n) {
    const double beta = (*num) / (*den);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = z[i] + beta * p[i];
}

// z = x / d (Jacobi)
__global__ void k_jacobi(double *__restrict__ z, const double *__restrict__ x, const double *__restrict__ d, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) z[i] = x[i] / d[i];
}

// x -= (*sum) / n
__global__ void k_sub_mean(double *__restrict__ x, const double *sum, int n) {
    const double m = (*sum) / n;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) x[i] -= m;
}

__global__ void k_diag(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                       const double *__restrict__ val, double *__restrict__ d, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = 0.0;
    for (int q = rowptr[i]; q < rowptr[i + 1]; ++q)
        if (col[q] == i) v = val[q];
    d[i] = v;
}

// u_new = u* - dt M^-1 (G dp)
__global__ void k_correct(double *__restrict__ u, const double *__restrict__ ustar, const double *__restrict__ gdp,
                          const double *__restrict__ mass, double dt, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double s = dt / mass[i];
        u[3 * (size_t)i + 0] = ustar[3 * (size_t)i + 0] - s * gdp[3 * (size_t)i + 0];
        u[3 * (size_t)i + 1] = ustar[3 * (size_t)i + 1] - s * gdp[3 * (size_t)i + 1];
        u[3 * (size_t)i + 2] = ustar[3 * (size_t)i + 2] - s * gdp[3 * (size_t)i + 2];
    }
}

// Start of a captured CG: no iteration yet met the tolerance; with a zero
// right-hand side every iteration is skipped.
__global__ void k_cg_begin(int *state, const double *bb) {
    if (threadIdx.x == 0) state[0] = *bb > 0.0 ? INT32_MAX : 0;
}

// End of a captured CG: rec = {iterations run, relative residual, converged}.
__global__ void k_cg_end(const int *state, const double *scal, int i_rr, int i_bb, int maxit, double *rec) {
    if (threadIdx.x != 0) return;
    const int conv = state[0];
    const double bb = scal[i_bb];
    rec[0] = (double)(conv < maxit ? conv : maxit);
    rec[1] = bb > 0.0 ? sqrt(scal[i_rr] / bb) : 0.0;
    rec[2] = conv <= maxit ? 1.0 : 0.0;
}

__global__ void k_zero(double *__restrict__ a, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        a[i] = 0.0;
}

// Launches KERNEL<type> over every non-empty category of mesh m on stream s.
#define LESASM_PER_CATEGORY(KERNEL, m, s, ...)                                                              \
    for (int k_ = 0; k_ < kNumCat; ++k_) {                                                                 \
        const Category &c_ = (m)->cat[k_];                                                                 \
        if (c_.n == 0) continue;                                                                           \
        CatView v_{c_.d_cg, c_.d_cf, c_.d_delta, (int32_t)c_.n, 0, (int32_t)c_.n};                         \
        const dim3 g_((unsigned)((c_.n + 255) / 256)), b_(256);                                            \
        switch (c_.type) {                                                                                 \
        case LESASM_TET04: hipLaunchKernelGGL(KERNEL<LESASM_TET04>, g_, b_, 0, (s), v_, __VA_ARGS__); break; \
        case LESASM_PYR05: hipLaunchKernelGGL(KERNEL<LESASM_PYR05>, g_, b_, 0, (s), v_, __VA_ARGS__); break; \
        case LESASM_PEN06: hipLaunchKernelGGL(KERNEL<LESASM_PEN06>, g_, b_, 0, (s), v_, __VA_ARGS__); break; \
        case LESASM_HEX08: hipLaunchKernelGGL(KERNEL<LESASM_HEX08>, g_, b_, 0, (s), v_, __VA_ARGS__); break; \
        }                                                                                                  \
    }

}  // namespace lesasm

using namespace lesasm;

struct lesasm_stepper {
    lesasm_mesh *mesh = nullptr;
    double nu = 0.0, dt = 0.0, rtol = 1e-12;
    int maxit = 1000, check_every = 16;
    int n = 0;
    int32_t *rowptr = nullptr, *col = nullptr;
    double *val = nullptr, *diag = nullptr;
    double *k1 = nullptr, *k3 = nullptr, *us = nullptr, *ustar = nullptr, *gdp = nullptr;  // [n][3]
    double *b = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *pv = nullptr, *q = nullptr;  // [n]
    double *partial = nullptr, *scal = nullptr;  // reductions
    std::vector<void *> allocs;
    int last_iters = 0;
    double last_res = 0.0;
    int64_t nnz = 0;
    // sliced-ELLPACK copy of K for the CG's SpMV (empty if not built)
    int32_t *soff = nullptr, *scol = nullptr;
    double *sval = nullptr;
    int nslices = 0;
    int64_t sell_entries = 0;
    int *d_cgstate = nullptr;   // captured CG: iteration that met the tolerance
};

// A whole time step captured in a HIP graph, bound to one (u, p) pair.
struct lesasm_step_graph {
    lesasm_stepper *st = nullptr;
    double *u = nullptr, *p = nullptr;
    int cg_iters = 0;
    double *d_rec = nullptr;        // {iterations, relative residual, converged} of the last replay
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev_last = nullptr;   // recorded after every replay
    bool launched = false;
};

namespace {

template <class T> int salloc(lesasm_stepper *st, T **p, size_t n) {
    *p = nullptr;
    if (!n) return LESASM_OK;
    void *q = nullptr;
    int rc = device_alloc(&q, n * sizeof(T), "stepper");
    if (rc) return rc;
    st->allocs.push_back(q);
    *p = (T *)q;
    return LESASM_OK;
}

void stepper_free(lesasm_stepper *st) {
    if (!st) return;
    (void)hipDeviceSynchronize();
    for (void *p : st->allocs) device_free(p);
    delete st;
}

enum { S_RZ = 0, S_PQ, S_RR, S_RZN, S_BB, S_SUM, S_NUM };

int dot(lesasm_stepper *st, const double *a, const double *b, int which, hipStream_t s) {
    hipLaunchKernelGGL(k_dot_partial, dim3(kRedBlocks), dim3(256), 0, s, a, b, st->n, st->partial);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedBlocks), 0, s, st->partial, kRedBlocks, st->scal + which);
    return LESASM_OK;
}

int pressure_solve(lesasm_stepper *st, const double *b_in, double *x, hipStream_t s) {
    const int n = st->n;
    const int g = grid_for(n, 256);
    // b = b_in - mean(b_in)
    LESASM_HIP_TRY(hipMemcpyAsync(st->b, b_in, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    dot(st, st->b, nullptr, S_SUM, s);
    hipLaunchKernelGGL(k_sub_mean, dim3(g), dim3(256), 0, s, st->b, st->scal + S_SUM, n);
    dot(st, st->b, st->b, S_BB, s);
    hipLaunchKernelGGL(k_zero, dim3(g), dim3(256), 0, s, x, (size_t)n);
    LESASM_HIP_TRY(hipMemcpyAsync(st->r, st->b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_jacobi, dim3(g), dim3(256), 0, s, st->z, st->r, st->diag, n);
    LESASM_HIP_TRY(hipMemcpyAsync(st->pv, st->z, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    dot(st, st->r, st->z, S_RZ, s);
    double host[S_NUM] = {0};
    LESASM_HIP_TRY(hipMemcpyAsync(host, st->scal, sizeof(host), hipMemcpyDeviceToHost, s));
    LESASM_HIP_TRY(hipStreamSynchronize(s));
    const double bnorm = std::sqrt(host[S_BB]);
    int it = 0;
    double res = bnorm;
    if (bnorm > 0.0) {
        // rz lives in two slots used alternately, so no scalar is overwritten
        // while a kernel may still read it.
        int i_rz = S_RZ, i_rzn = S_RZN;
        for (it = 1; it <= st->maxit; ++it) {
            if (st->sval)
                hipLaunchKernelGGL(k_spmv_sell_dot, dim3(kCgBlocks), dim3(256), 0, s, st->soff, st->scol, st->sval,
                                   st->pv, st->q, n, st->nslices, st->partial);
            else
                hipLaunchKernelGGL(k_spmv_dot, dim3(kCgBlocks), dim3(256), 0, s, st->rowptr, st->col, st->val, st->pv,
                                   st->q, n, st->partial);
            hipLaunchKernelGGL(k_reduce_strided, dim3(1), dim3(1024), 0, s, st->partial, kCgBlocks, 1, 1,
                               st->scal + S_PQ, st->scal + S_PQ);
            hipLaunchKernelGGL(k_cg_update, dim3(kCgBlocks), dim3(256), 0, s, st->r, st->z, st->q, st->diag,
                               st->scal, i_rz, S_PQ, n, st->partial);
            hipLaunchKernelGGL(k_reduce_strided, dim3(1), dim3(1024), 0, s, st->partial, kCgBlocks, 2, 2,
                               st->scal + i_rzn, st->scal + S_RR);
            hipLaunchKernelGGL(k_cg_direction, dim3(kCgBlocks), dim3(256), 0, s, x, st->pv, st->z, st->scal, i_rzn,
                               i_rz, S_PQ, n);
            std::swap(i_rz, i_rzn);
            if (it % st->check_every == 0 || it == st->maxit) {
                LESASM_HIP_TRY(hipMemcpyAsync(host, st->scal, sizeof(host), hipMemcpyDeviceToHost, s));
                LESASM_HIP_TRY(hipStreamSynchronize(s));
                res = std::sqrt(host[S_RR]);
                if (res <= st->rtol * bnorm) break;
            }
        }
    }
    st->last_iters = std::min(it, st->maxit);
    st->last_res = bnorm > 0.0 ? res / bnorm : 0.0;
    dot(st, x, nullptr, S_SUM, s);
    hipLaunchKernelGGL(k_sub_mean, dim3(g), dim3(256), 0, s, x, st->scal + S_SUM, n);
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

// The same solve for graph capture: no host reads and no copies through the
// copy engine.  Exactly cg_iters iterations are captured; once the residual
// meets the tolerance (tested after every iteration, on the device) the
// remaining iterations return at once.  rec receives the iteration count,
// relative residual and convergence flag.
int pressure_solve_captured(lesasm_stepper *st, const double *b_in, double *x, hipStream_t s, int cg_iters,
                            double *rec) {
    const int n = st->n;
    const int g = grid_for(n, 256);
    hipLaunchKernelGGL(k_lincomb, dim3(g), dim3(256), 0, s, st->b, 1.0, b_in, 0.0, nullptr, 0.0, nullptr, (size_t)n);
    dot(st, st->b, nullptr, S_SUM, s);
    hipLaunchKernelGGL(k_sub_mean, dim3(g), dim3(256), 0, s, st->b, st->scal + S_SUM, n);
    dot(st, st->b, st->b, S_BB, s);
    hipLaunchKernelGGL(k_zero, dim3(g), dim3(256), 0, s, x, (size_t)n);
    hipLaunchKernelGGL(k_lincomb, dim3(g), dim3(256), 0, s, st->r, 1.0, st->b, 0.0, nullptr, 0.0, nullptr, (size_t)n);
    hipLaunchKernelGGL(k_jacobi, dim3(g), dim3(256), 0, s, st->z, st->r, st->diag, n);
    hipLaunchKernelGGL(k_lincomb, dim3(g), dim3(256), 0, s, st->pv, 1.0, st->z, 0.0, nullptr, 0.0, nullptr, (size_t)n);
    dot(st, st->r, st->z, S_RZ, s);
    hipLaunchKernelGGL(k_cg_begin, dim3(1), dim3(64), 0, s, st->d_cgstate, st->scal + S_BB);
    const double tol2 = st->rtol * st->rtol;
    int i_rz = S_RZ, i_rzn = S_RZN;
    int *state = st->d_cgstate;
    for (int it = 1; it <= cg_iters; ++it) {
        if (st->sval)
            hipLaunchKernelGGL(k_spmv_sell_dot, dim3(kCgBlocks), dim3(256), 0, s, st->soff, st->scol, st->sval, st->pv,
                               st->q, n, st->nslices, st->partial, (const int *)state, it);
        else
            hipLaunchKernelGGL(k_spmv_dot, dim3(kCgBlocks), dim3(256), 0, s, st->rowptr, st->col, st->val, st->pv,
                               st->q, n, st->partial, (const int *)state, it);
        hipLaunchKernelGGL(k_reduce_strided, dim3(1), dim3(1024), 0, s, st->partial, kCgBlocks, 1, 1,
                           st->scal + S_PQ, st->scal + S_PQ, state, it, false, (const double *)nullptr, 0.0);
        hipLaunchKernelGGL(k_cg_update, dim3(kCgBlocks), dim3(256), 0, s, st->r, st->z, st->q, st->diag, st->scal,
                           i_rz, S_PQ, n, st->partial, (const int *)state, it);
        hipLaunchKernelGGL(k_reduce_strided, dim3(1), dim3(1024), 0, s, st->partial, kCgBlocks, 2, 2,
                           st->scal + i_rzn, st->scal + S_RR, state, it, true, (const double *)(st->scal + S_BB),
                           tol2);
        hipLaunchKernelGGL(k_cg_direction, dim3(kCgBlocks), dim3(256), 0, s, x, st->pv, st->z, st->scal, i_rzn, i_rz,
                           S_PQ, n, (const int *)state, it);
        std::swap(i_rz, i_rzn);
    }
    hipLaunchKernelGGL(k_cg_end, dim3(1), dim3(64), 0, s, (const int *)state, (const double *)st->scal, (int)S_RR,
                       (int)S_BB, cg_iters, rec);
    dot(st, x, nullptr, S_SUM, s);
    hipLaunchKernelGGL(k_sub_mean, dim3(g), dim3(256), 0, s, x, st->scal + S_SUM, n);
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

}  // namespace

extern "C" int lesasm_divergence(lesasm_mesh *m, const double *d_u, double *d_out, void *stream) {
    if (!m || (m->n_field && (!d_u || !d_out))) return fail(LESASM_E_INVALID_ARG, "divergence: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    if (!m->n_field) return LESASM_OK;
    hipLaunchKernelGGL(k_zero, dim3(grid_for(m->n_field, 256)), dim3(256), 0, s, d_out, (size_t)m->n_field);
    LESASM_PER_CATEGORY(k_divergence, m, s, (const double *)m->d_xyz, d_u, d_out);
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

extern "C" int lesasm_gradient(lesasm_mesh *m, const double *d_p, double *d_out, void *stream) {
    if (!m || (m->n_field && (!d_p || !d_out))) return fail(LESASM_E_INVALID_ARG, "gradient: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    if (!m->n_field) return LESASM_OK;
    hipLaunchKernelGGL(k_zero, dim3(grid_for(3 * (size_t)m->n_field, 256)), dim3(256), 0, s, d_out,
                       3 * (size_t)m->n_field);
    LESASM_PER_CATEGORY(k_gradient, m, s, (const double *)m->d_xyz, d_p, d_out);
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

extern "C" int lesasm_stepper_create(lesasm_mesh *m, double nu, double dt, double rtol, int maxit,
                                     lesasm_stepper **out) {
    if (!out) return fail(LESASM_E_INVALID_ARG, "stepper_create: out is NULL");
    *out = nullptr;
    if (!m || !(dt > 0.0) || !(rtol > 0.0) || maxit < 1)
        return fail(LESASM_E_INVALID_ARG, "stepper_create: need a mesh, dt > 0, rtol > 0, maxit >= 1");
    int dev = -1;
    LESASM_HIP_TRY(hipGetDevice(&dev));
    if (dev != m->device) return fail(LESASM_E_STATE, "stepper_create: current device differs from the mesh's");
    auto *st = new lesasm_stepper();
    struct Guard {
        lesasm_stepper *p;
        ~Guard() { stepper_free(p); }
    } guard{st};
    st->mesh = m;
    st->nu = nu;
    st->dt = dt;
    st->rtol = rtol;
    st->maxit = maxit;
    st->n = (int)m->n_field;
    const int n = st->n;

    // CSR pattern of K: for each field node, the field nodes of its elements
    std::vector<int32_t> ninc(n + 1, 0);
    for (int k = 0; k < kNumCat; ++k) {
        const Category &c = m->cat[k];
        const std::vector<int32_t> &cf = c.h_cf.empty() ? c.h_cg : c.h_cf;
        for (int32_t f : cf) ninc[f + 1]++;
    }
    for (int i = 0; i < n; ++i) ninc[i + 1] += ninc[i];
    std::vector<int64_t> elem_of(ninc[n]);
    std::vector<int32_t> fill(ninc.begin(), ninc.end() - 1);
    int64_t gbase = 0;
    for (int k = 0; k < kNumCat; ++k) {
        const Category &c = m->cat[k];
        const std::vector<int32_t> &cf = c.h_cf.empty() ? c.h_cg : c.h_cf;
        for (int a = 0; a < c.type; ++a)
            for (int64_t e = 0; e < c.n; ++e) elem_of[fill[cf[(size_t)a * c.n + e]]++] = gbase + e;
        gbase += c.n;
    }
    auto elem_nodes = [&](int64_t ge, std::vector<int32_t> &outv) {
        for (int k = 0; k < kNumCat; ++k) {
            const Category &c = m->cat[k];
            if (ge < c.first || ge >= c.first + c.n) continue;
            const std::vector<int32_t> &cf = c.h_cf.empty() ? c.h_cg : c.h_cf;
            for (int a = 0; a < c.type; ++a) outv.push_back(cf[(size_t)a * c.n + (ge - c.first)]);
            return;
        }
    };
    std::vector<int32_t> rowptr(n + 1, 0), col, tmp;
    for (int i = 0; i < n; ++i) {
        tmp.clear();
        tmp.push_back(i);
        for (int32_t q = ninc[i]; q < ninc[i + 1]; ++q) elem_nodes(elem_of[q], tmp);
        std::sort(tmp.begin(), tmp.end());
        tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
        col.insert(col.end(), tmp.begin(), tmp.end());
        rowptr[i + 1] = (int32_t)col.size();
    }
    st->nnz = (int64_t)col.size();
    int rc;
    if ((rc = salloc(st, &st->rowptr, rowptr.size())) || (rc = salloc(st, &st->col, col.size())) ||
        (rc = salloc(st, &st->val, col.size())) || (rc = salloc(st, &st->diag, (size_t)n)) ||
        (rc = salloc(st, &st->k1, 3 * (size_t)n)) || (rc = salloc(st, &st->k3, 3 * (size_t)n)) ||
        (rc = salloc(st, &st->us, 3 * (size_t)n)) || (rc = salloc(st, &st->ustar, 3 * (size_t)n)) ||
        (rc = salloc(st, &st->gdp, 3 * (size_t)n)) || (rc = salloc(st, &st->b, (size_t)n)) ||
        (rc = salloc(st, &st->x, (size_t)n)) || (rc = salloc(st, &st->r, (size_t)n)) ||
        (rc = salloc(st, &st->z, (size_t)n)) || (rc = salloc(st, &st->pv, (size_t)n)) ||
        (rc = salloc(st, &st->q, (size_t)n)) || (rc = salloc(st, &st->partial, 2 * kCgBlocks)) ||
        (rc = salloc(st, &st->scal, S_NUM)) || (rc = salloc(st, &st->d_cgstate, 4)))
        return rc;
    if (n) {
        LESASM_HIP_TRY(hipMemcpy(st->rowptr, rowptr.data(), sizeof(int32_t) * rowptr.size(), hipMemcpyHostToDevice));
        LESASM_HIP_TRY(hipMemcpy(st->col, col.data(), sizeof(int32_t) * col.size(), hipMemcpyHostToDevice));
        LESASM_HIP_TRY(hipMemset(st->val, 0, sizeof(double) * col.size()));
        hipStream_t s0 = 0;
        LESASM_PER_CATEGORY(k_laplacian, m, s0, (const double *)m->d_xyz, (const int32_t *)st->rowptr,
                            (const int32_t *)st->col, st->val);
        hipLaunchKernelGGL(k_diag, dim3((n + 255) / 256), dim3(256), 0, 0, st->rowptr, st->col, st->val, st->diag, n);
        LESASM_HIP_TRY(hipGetLastError());
        if (LESASM_CG_SELL) {
            // slices of kSlice rows, each padded to its longest row, column-major
            const int ns = (n + kSlice - 1) / kSlice;
            std::vector<int32_t> soff(ns + 1, 0);
            int64_t total = 0;
            for (int sl = 0; sl < ns; ++sl) {
                int w = 0;
                for (int r = sl * kSlice; r < std::min(n, (sl + 1) * kSlice); ++r) w = std::max(w, rowptr[r + 1] - rowptr[r]);
                total += (int64_t)w * kSlice;
                soff[sl + 1] = (int32_t)std::min<int64_t>(total, INT32_MAX);
            }
            if (total < INT32_MAX) {  // otherwise the CSR kernel serves the CG
                std::vector<int32_t> scol((size_t)total), src((size_t)total);
                for (int sl = 0; sl < ns; ++sl) {
                    const int w = (soff[sl + 1] - soff[sl]) / kSlice;
                    for (int l = 0; l < kSlice; ++l) {
                        const int r = sl * kSlice + l;
                        const int len = r < n ? rowptr[r + 1] - rowptr[r] : 0;
                        for (int j = 0; j < w; ++j) {
                            const size_t at = (size_t)soff[sl] + (size_t)j * kSlice + l;
                            if (j < len) {
                                scol[at] = col[(size_t)rowptr[r] + j];
                                src[at] = rowptr[r] + j;
                            } else {
                                scol[at] = r < n ? r : 0;
                                src[at] = -1;
                            }
                        }
                    }
                }
                int32_t *d_src = nullptr;
                if ((rc = salloc(st, &st->soff, soff.size())) || (rc = salloc(st, &st->scol, scol.size())) ||
                    (rc = salloc(st, &st->sval, scol.size())) || (rc = salloc(st, &d_src, src.size())))
                    return rc;
                LESASM_HIP_TRY(hipMemcpy(st->soff, soff.data(), sizeof(int32_t) * soff.size(), hipMemcpyHostToDevice));
                LESASM_HIP_TRY(hipMemcpy(st->scol, scol.data(), sizeof(int32_t) * scol.size(), hipMemcpyHostToDevice));
                LESASM_HIP_TRY(hipMemcpy(d_src, src.data(), sizeof(int32_t) * src.size(), hipMemcpyHostToDevice));
                hipLaunchKernelGGL(k_sell_fill, dim3(grid_for((size_t)total, 256)), dim3(256), 0, 0, d_src, st->val,
                                   st->sval, total);
                LESASM_HIP_TRY(hipGetLastError());
                LESASM_HIP_TRY(hipDeviceSynchronize());
                st->allocs.erase(std::find(st->allocs.begin(), st->allocs.end(), (void *)d_src));
                device_free(d_src);
                st->nslices = ns;
                st->sell_entries = total;
            }
        }
        LESASM_HIP_TRY(hipDeviceSynchronize());
    }
    guard.p = nullptr;
    *out = st;
    return LESASM_OK;
}

extern "C" int lesasm_stepper_destroy(lesasm_stepper *st) {
    stepper_free(st);
    return LESASM_OK;
}

extern "C" int lesasm_stepper_laplacian(lesasm_stepper *st, int32_t *rowptr, int32_t *col, double *val, int64_t *nnz) {
    if (!st || !nnz) return fail(LESASM_E_INVALID_ARG, "stepper_laplacian: NULL argument");
    *nnz = st->nnz;
    if (rowptr) LESASM_HIP_TRY(hipMemcpy(rowptr, st->rowptr, sizeof(int32_t) * (st->n + 1), hipMemcpyDeviceToHost));
    if (col) LESASM_HIP_TRY(hipMemcpy(col, st->col, sizeof(int32_t) * st->nnz, hipMemcpyDeviceToHost));
    if (val) LESASM_HIP_TRY(hipMemcpy(val, st->val, sizeof(double) * st->nnz, hipMemcpyDeviceToHost));
    return LESASM_OK;
}

extern "C" int lesasm_stepper_spmv(lesasm_stepper *st, const double *d_p, double *d_q, void *stream) {
    if (!st || (st->n && (!d_p || !d_q))) return fail(LESASM_E_INVALID_ARG, "stepper_spmv: NULL argument");
    if (d_p == d_q) return fail(LESASM_E_INVALID_ARG, "stepper_spmv: p and q must not alias");
    if (!st->n) return LESASM_OK;
    hipStream_t s = (hipStream_t)stream;
    if (st->sval)
        hipLaunchKernelGGL(k_spmv_sell_dot, dim3(kCgBlocks), dim3(256), 0, s, st->soff, st->scol, st->sval, d_p, d_q,
                           st->n, st->nslices, st->partial);
    else
        hipLaunchKernelGGL(k_spmv_dot, dim3(kCgBlocks), dim3(256), 0, s, st->rowptr, st->col, st->val, d_p, d_q,
                           st->n, st->partial);
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

extern "C" int lesasm_stepper_sell_entries(const lesasm_stepper *st, int64_t *entries) {
    if (!st || !entries) return fail(LESASM_E_INVALID_ARG, "stepper_sell_entries: NULL argument");
    *entries = st->sell_entries;
    return LESASM_OK;
}

extern "C" int lesasm_pressure_solve(lesasm_stepper *st, const double *d_b, double *d_x, void *stream) {
    if (!st || (st->n && (!d_b || !d_x))) return fail(LESASM_E_INVALID_ARG, "pressure_solve: NULL argument");
    if (!st->n) return LESASM_OK;
    return pressure_solve(st, d_b, d_x, (hipStream_t)stream);
}

// Three explicit stages only: d_ustar = u^n + dt (k1/4 + 3 k3/4).
static int rk3_stages(lesasm_stepper *st, const double *u, const double *p, double *ustar, hipStream_t s) {
    lesasm_mesh *m = st->mesh;
    const size_t n3 = 3 * (size_t)st->n;
    const int g = grid_for(n3, 256);
    int rc;
    // stage 1: k1 = dt M^-1 rhs(u^n); u2 = u^n + k1/3
    if ((rc = assemble_into(m, u, p, st->nu, st->dt, st->k1, s, true))) return rc;
    hipLaunchKernelGGL(k_lincomb, dim3(g), dim3(256), 0, s, st->us, 1.0, u, 1.0 / 3.0, st->k1, 0.0, nullptr, n3);
    // stage 2: k2 = dt M^-1 rhs(u2); u3 = u^n + 2 k2/3   (k2 held in k3)
    if ((rc = assemble_into(m, st->us, p, st->nu, st->dt, st->k3, s, true))) return rc;
    hipLaunchKernelGGL(k_lincomb, dim3(g), dim3(256), 0, s, st->us, 1.0, u, 2.0 / 3.0, st->k3, 0.0, nullptr, n3);
    // stage 3: k3 = dt M^-1 rhs(u3); u* = u^n + k1/4 + 3 k3/4
    if ((rc = assemble_into(m, st->us, p, st->nu, st->dt, st->k3, s, true))) return rc;
    hipLaunchKernelGGL(k_lincomb, dim3(g), dim3(256), 0, s, ustar, 1.0, u, 0.25, st->k1, 0.75, st->k3, n3);
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

extern "C" int lesasm_stepper_rk3_stages(lesasm_stepper *st, const double *d_u, const double *d_p, double *d_ustar,
                                         void *stream) {
    if (!st || (st->n && (!d_u || !d_ustar))) return fail(LESASM_E_INVALID_ARG, "rk3_stages: NULL argument");
    if (!st->n) return LESASM_OK;
    return rk3_stages(st, d_u, d_p, d_ustar, (hipStream_t)stream);
}

// One time step on s: the stages, b = -(1/dt) D u*, the pressure solve (eager
// with host convergence checks, or captured with cg_iters device-terminated
// iterations when rec is given), the correction and the pressure update.
static int step_body(lesasm_stepper *st, double *d_u, double *d_p, hipStream_t s, int cg_iters, double *rec) {
    lesasm_mesh *m = st->mesh;
    const int n = st->n;
    int rc;
    if ((rc = rk3_stages(st, d_u, d_p, st->ustar, s))) return rc;
    // b = -(1/dt) D u*
    if ((rc = lesasm_divergence(m, st->ustar, st->q, s))) return rc;
    hipLaunchKernelGGL(k_lincomb, dim3(grid_for(n, 256)), dim3(256), 0, s, st->q, -1.0 / st->dt, st->q, 0.0, nullptr,
                       0.0, nullptr, (size_t)n);
    if (rec) rc = pressure_solve_captured(st, st->q, st->x, s, cg_iters, rec);
    else rc = pressure_solve(st, st->q, st->x, s);
    if (rc) return rc;
    if ((rc = lesasm_gradient(m, st->x, st->gdp, s))) return rc;
    hipLaunchKernelGGL(k_correct, dim3(grid_for(n, 256)), dim3(256), 0, s, d_u, st->ustar, st->gdp, m->d_mass,
                       st->dt, n);
    hipLaunchKernelGGL(k_lincomb, dim3(grid_for(n, 256)), dim3(256), 0, s, d_p, 1.0, d_p, 1.0, st->x, 0.0, nullptr,
                       (size_t)n);
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

extern "C" int lesasm_stepper_step(lesasm_stepper *st, double *d_u, double *d_p, void *stream) {
    if (!st || (st->n && (!d_u || !d_p))) return fail(LESASM_E_INVALID_ARG, "stepper_step: NULL argument");
    int dev = -1;
    LESASM_HIP_TRY(hipGetDevice(&dev));
    if (dev != st->mesh->device) return fail(LESASM_E_STATE, "stepper_step: wrong current device");
    if (!st->n) return LESASM_OK;
    return step_body(st, d_u, d_p, (hipStream_t)stream, 0, nullptr);
}

// ---- step graph ----------------------------------------------------------------

static void step_graph_free(lesasm_step_graph *g) {
    if (!g) return;
    // a replay may still be queued: wait for the last one before the
    // executable graph goes away
    if (g->launched && g->ev_last) (void)hipEventSynchronize(g->ev_last);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->ev_last) (void)hipEventDestroy(g->ev_last);
    device_free(g->d_rec);
    delete g;
}

extern "C" int lesasm_step_graph_create(lesasm_stepper *st, double *d_u, double *d_p, int cg_iters,
                                        lesasm_step_graph **out, void *stream) {
    if (!out) return fail(LESASM_E_INVALID_ARG, "step_graph_create: out is NULL");
    *out = nullptr;
    if (!st || !d_u || !d_p) return fail(LESASM_E_INVALID_ARG, "step_graph_create: NULL argument");
    if (cg_iters < 1 || cg_iters > kMaxCapturedCg)
        return fail(LESASM_E_INVALID_ARG, "step_graph_create: cg_iters must be in 1.." + std::to_string(kMaxCapturedCg));
    if (!st->n) return fail(LESASM_E_INVALID_ARG, "step_graph_create: the mesh has no field nodes");
    hipStream_t s = (hipStream_t)stream;
    if (!s) return fail(LESASM_E_INVALID_ARG, "step_graph_create: capture needs a non-default stream");
    int dev = -1;
    LESASM_HIP_TRY(hipGetDevice(&dev));
    if (dev != st->mesh->device) return fail(LESASM_E_STATE, "step_graph_create: wrong current device");
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    LESASM_HIP_TRY(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone) return fail(LESASM_E_STATE, "step_graph_create: stream is already capturing");
    auto *g = new lesasm_step_graph();
    struct Guard {
        lesasm_step_graph *p;
        ~Guard() { step_graph_free(p); }
    } guard{g};
    g->st = st;
    g->u = d_u;
    g->p = d_p;
    g->cg_iters = cg_iters;
    {
        void *q = nullptr;
        const int rc = device_alloc(&q, 4 * sizeof(double), "step graph");
        if (rc) return rc;
        g->d_rec = (double *)q;
    }
    LESASM_HIP_TRY(hipEventCreateWithFlags(&g->ev_last, hipEventDisableTiming));
    // the mesh's previous work must not overlap the capture's first launches
    LESASM_HIP_TRY(hipStreamSynchronize(s));
    LESASM_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = step_body(st, d_u, d_p, s, cg_iters, g->d_rec);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(LESASM_E_HIP, std::string("step_graph_create: capture failed: ") + hipGetErrorString(e));
    g->graph = graph;
    LESASM_HIP_TRY(hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0));
    guard.p = nullptr;
    *out = g;
    return LESASM_OK;
}

extern "C" int lesasm_step_graph_launch(lesasm_step_graph *g, double *d_u, double *d_p, void *stream) {
    if (!g) return fail(LESASM_E_INVALID_ARG, "step_graph_launch: graph is NULL");
    if (d_u != g->u || d_p != g->p)
        return fail(LESASM_E_STATE, "step_graph_launch: u and p must be the buffers the graph was captured with");
    int dev = -1;
    LESASM_HIP_TRY(hipGetDevice(&dev));
    if (dev != g->st->mesh->device) return fail(LESASM_E_STATE, "step_graph_launch: wrong current device");
    hipStream_t s = (hipStream_t)stream;
    LESASM_HIP_TRY(hipGraphLaunch(g->exec, s));
    LESASM_HIP_TRY(hipEventRecord(g->ev_last, s));
    g->launched = true;
    return LESASM_OK;
}

extern "C" int lesasm_step_graph_stats(lesasm_step_graph *g, int *cg_iters, double *cg_rel_residual, int *converged) {
    if (!g || !cg_iters || !cg_rel_residual || !converged)
        return fail(LESASM_E_INVALID_ARG, "step_graph_stats: NULL argument");
    if (!g->launched) return fail(LESASM_E_STATE, "step_graph_stats: the graph has not been launched");
    LESASM_HIP_TRY(hipEventSynchronize(g->ev_last));
    double rec[3] = {0.0, 0.0, 0.0};
    LESASM_HIP_TRY(hipMemcpy(rec, g->d_rec, sizeof(rec), hipMemcpyDeviceToHost));
    *cg_iters = (int)rec[0];
    *cg_rel_residual = rec[1];
    *converged = rec[2] != 0.0;
    return LESASM_OK;
}

extern "C" int lesasm_step_graph_destroy(lesasm_step_graph *g) {
    step_graph_free(g);
    return LESASM_OK;
}

extern "C" int lesasm_stepper_stats(const lesasm_stepper *st, int *cg_iters, double *cg_rel_residual) {
    if (!st || !cg_iters || !cg_rel_residual) return fail(LESASM_E_INVALID_ARG, "stepper_stats: NULL argument");
    *cg_iters = st->last_iters;
    *cg_rel_residual = st->last_res;
    return LESASM_OK;
}
