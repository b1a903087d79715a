// Learned subgrid closure: parameters, GPU training kernels (FP32 master
// weights, forward, backward, Adam) and BF16 matrix-core inference.
//
// Parameter order (float32, 5254 values): W1[10][64], b1[64], W2[64][64],
// b2[64], W3[64][6], b3[6]; a layer computes h_out = h_in W + b.  Loss:
// L = (1/N) sum_n sum_c w_c (z_nc - t_nc)^2 with z = y minus the trace of its
// (xx, yy, zz) part and w = (1, 1, 1, 2, 2, 2) (Frobenius norm of the
// symmetric tensor).  Adam: bias-corrected moments, beta1 0.9, beta2 0.999,
// eps 1e-8.  Every reduction over samples runs in a fixed order.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "mlp.hpp"

namespace lesasm {

constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + kMlpIn * kMlpH, OFF_W2 = OFF_B1 + kMlpH, OFF_B2 = OFF_W2 + kMlpH * kMlpH,
              OFF_W3 = OFF_B2 + kMlpH, OFF_B3 = OFF_W3 + kMlpH * kMlpOut;

__device__ __forceinline__ void deviatoric6(float (&y)[kMlpOut]) {
    const float tr = (y[0] + y[1] + y[2]) * (1.0f / 3.0f);
    y[0] -= tr;
    y[1] -= tr;
    y[2] -= tr;
}

// FP32 forward of one sample with parameters P (global or LDS); keeps h1, h2.
__device__ __forceinline__ void fwd_f32(const float *P, const float *x, float *h1, float *h2, float (&y)[kMlpOut]) {
    for (int j = 0; j < kMlpH; ++j) {
        float s = P[OFF_B1 + j];
        for (int k = 0; k < kMlpIn; ++k) s += x[k] * P[OFF_W1 + k * kMlpH + j];
        h1[j] = s > 0.f ? s : 0.f;
    }
    for (int j = 0; j < kMlpH; ++j) {
        float s = P[OFF_B2 + j];
        for (int k = 0; k < kMlpH; ++k) s += h1[k] * P[OFF_W2 + k * kMlpH + j];
        h2[j] = s > 0.f ? s : 0.f;
    }
    for (int o = 0; o < kMlpOut; ++o) {
        float s = P[OFF_B3 + o];
        for (int k = 0; k < kMlpH; ++k) s += h2[k] * P[OFF_W3 + k * kMlpOut + o];
        y[o] = s;
    }
}

// Per sample: activations, loss term and dL/dy (through the trace projection).
__global__ __launch_bounds__(128) void k_mlp_fwd_train(const float *__restrict__ P, const float *__restrict__ X,
                                                       const float *__restrict__ Tg, int n, float *__restrict__ H1,
                                                       float *__restrict__ H2, float *__restrict__ DY,
                                                       float *__restrict__ loss) {
    __shared__ float sP[kMlpParams];
    for (int k = threadIdx.x; k < kMlpParams; k += blockDim.x) sP[k] = P[k];
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[kMlpIn], y[kMlpOut];
    for (int k = 0; k < kMlpIn; ++k) x[k] = X[(size_t)i * kMlpIn + k];
    float *h1 = H1 + (size_t)i * kMlpH, *h2 = H2 + (size_t)i * kMlpH;
    fwd_f32(sP, x, h1, h2, y);
    deviatoric6(y);
    const float w[kMlpOut] = {1.f, 1.f, 1.f, 2.f, 2.f, 2.f};
    float l = 0.f, dz[kMlpOut];
    for (int o = 0; o < kMlpOut; ++o) {
        const float r = y[o] - Tg[(size_t)i * kMlpOut + o];
        l += w[o] * r * r;
        dz[o] = 2.f * w[o] * r / (float)n;
    }
    const float m = (dz[0] + dz[1] + dz[2]) * (1.0f / 3.0f);
    for (int o = 0; o < kMlpOut; ++o) DY[(size_t)i * kMlpOut + o] = o < 3 ? dz[o] - m : dz[o];
    loss[i] = l / (float)n;
}

// Per sample: back-propagated pre-activation gradients of both hidden layers.
__global__ __launch_bounds__(128) void k_mlp_bwd_act(const float *__restrict__ P, const float *__restrict__ H1,
                                                     const float *__restrict__ H2, const float *__restrict__ DY,
                                                     int n, float *__restrict__ DA1, float *__restrict__ DA2) {
    __shared__ float sP[kMlpParams];
    for (int k = threadIdx.x; k < kMlpParams; k += blockDim.x) sP[k] = P[k];
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float dy[kMlpOut], da2[kMlpH];
    for (int o = 0; o < kMlpOut; ++o) dy[o] = DY[(size_t)i * kMlpOut + o];
    for (int j = 0; j < kMlpH; ++j) {
        float s = 0.f;
        for (int o = 0; o < kMlpOut; ++o) s += dy[o] * sP[OFF_W3 + j * kMlpOut + o];
        da2[j] = H2[(size_t)i * kMlpH + j] > 0.f ? s : 0.f;
        DA2[(size_t)i * kMlpH + j] = da2[j];
    }
    for (int j = 0; j < kMlpH; ++j) {
        float s = 0.f;
        for (int k = 0; k < kMlpH; ++k) s += da2[k] * sP[OFF_W2 + j * kMlpH + k];
        DA1[(size_t)i * kMlpH + j] = H1[(size_t)i * kMlpH + j] > 0.f ? s : 0.f;
    }
}

// Weight gradients: one block per weight row (or bias vector), threads over
// columns, samples summed in order.  Row r < 10: W1 (inputs X, grads DA1);
// r < 74: W2 (H1, DA2); r < 138: W3 (H2, DY); r = 138, 139, 140: b1, b2, b3.
__global__ void k_mlp_wgrad(const float *__restrict__ X, const float *__restrict__ H1, const float *__restrict__ H2,
                            const float *__restrict__ DA1, const float *__restrict__ DA2,
                            const float *__restrict__ DY, int n, float *__restrict__ grad) {
    const int r = blockIdx.x, j = threadIdx.x;
    const float *in = nullptr, *d = nullptr;
    int ldin = 0, ldd = 0, cols = 0, row = 0, off = 0;
    if (r < 10) { in = X; ldin = kMlpIn; d = DA1; ldd = kMlpH; cols = kMlpH; row = r; off = OFF_W1 + r * kMlpH; }
    else if (r < 74) { in = H1; ldin = kMlpH; d = DA2; ldd = kMlpH; cols = kMlpH; row = r - 10; off = OFF_W2 + row * kMlpH; }
    else if (r < 138) { in = H2; ldin = kMlpH; d = DY; ldd = kMlpOut; cols = kMlpOut; row = r - 74; off = OFF_W3 + row * kMlpOut; }
    else if (r == 138) { d = DA1; ldd = kMlpH; cols = kMlpH; off = OFF_B1; }
    else if (r == 139) { d = DA2; ldd = kMlpH; cols = kMlpH; off = OFF_B2; }
    else { d = DY; ldd = kMlpOut; cols = kMlpOut; off = OFF_B3; }
    if (j >= cols) return;
    float s = 0.f;
    if (in)
        for (int i = 0; i < n; ++i) s += in[(size_t)i * ldin + row] * d[(size_t)i * ldd + j];
    else
        for (int i = 0; i < n; ++i) s += d[(size_t)i * ldd + j];
    grad[off + j] = s;
}

__global__ void k_sum_f32(const float *__restrict__ a, int n, float *__restrict__ out) {
    __shared__ float sh[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) s += a[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

__global__ void k_adam(float *__restrict__ P, float *__restrict__ M, float *__restrict__ V,
                       const float *__restrict__ g, int n, float lr, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float m = 0.9f * M[i] + 0.1f * gi;
    const float v = 0.999f * V[i] + 0.001f * gi * gi;
    M[i] = m;
    V[i] = v;
    P[i] -= lr * (m / c1) / (sqrtf(v / c2) + 1e-8f);
}

__global__ __launch_bounds__(128) void k_mlp_forward_f32(const float *__restrict__ P, const float *__restrict__ X,
                                                         int n, float *__restrict__ Y) {
    __shared__ float sP[kMlpParams];
    for (int k = threadIdx.x; k < kMlpParams; k += blockDim.x) sP[k] = P[k];
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[kMlpIn], h1[kMlpH], h2[kMlpH], y[kMlpOut];
    for (int k = 0; k < kMlpIn; ++k) x[k] = X[(size_t)i * kMlpIn + k];
    fwd_f32(sP, x, h1, h2, y);
    for (int o = 0; o < kMlpOut; ++o) Y[(size_t)i * kMlpOut + o] = y[o];
}

// Matrix-core inference of N samples: each wavefront takes 64 samples at a
// time (the last group padded by repeating the final sample).
__global__ __launch_bounds__(256) void k_mlp_infer_bf16(const short *__restrict__ packed,
                                                        const float *__restrict__ bias, const float *__restrict__ X,
                                                        int n, float *__restrict__ Y) {
    extern __shared__ __align__(16) unsigned char smem[];
    const MlpLds w = mlp_stage(packed, bias, smem);
    __syncthreads();
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    unsigned char *scratch = smem + kMlpLdsBytes + wave * kMlpWaveScratch;
    const int waves = gridDim.x * (blockDim.x / 64);
    for (int base = (blockIdx.x * (blockDim.x / 64) + wave) * 64; base < n; base += waves * 64) {
        const int i = min(base + lane, n - 1);
        float x[kMlpIn], y[kMlpOut];
        for (int k = 0; k < kMlpIn; ++k) x[k] = X[(size_t)i * kMlpIn + k];
        mlp_wave(w, x, y, scratch);
        if (base + lane < n)
            for (int o = 0; o < kMlpOut; ++o) Y[(size_t)i * kMlpOut + o] = y[o];
    }
}

// Packs float parameters into the A tiles of mlp_wave (bf16) and the bias block.
static void pack_weights(const float *P, std::vector<short> &tiles, std::vector<float> &bias) {
    auto bf = [](float f) -> short {
        uint32_t u;
        std::memcpy(&u, &f, 4);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return (short)(u >> 16);
    };
    tiles.assign(kMlpPackedShorts, 0);
    auto put = [&](int tile, int i, int k, float v) {  // A[i][k] of a 16x16 tile
        const int lane = i + 16 * (k / 4);
        tiles[((size_t)tile * 64 + lane) * 4 + (k % 4)] = bf(v);
    };
    for (int mt = 0; mt < 4; ++mt)  // W1^T: rows = hidden, k = input
        for (int i = 0; i < 16; ++i)
            for (int k = 0; k < 16; ++k) put(mt, i, k, k < kMlpIn ? P[OFF_W1 + k * kMlpH + 16 * mt + i] : 0.f);
    // W2^T tiles (mt, kb) of K = 32: A[i][k] in lane i + 16 (k/8), slot k%8;
    // K index k of block kb is hidden unit 16 (2 kb + s/4) + 4 (k/8) + s%4, s = k%8
    for (int mt = 0; mt < 4; ++mt)
        for (int kb = 0; kb < 2; ++kb)
            for (int i = 0; i < 16; ++i)
                for (int k = 0; k < 32; ++k) {
                    const int q = k / 8, s = k % 8;
                    const int unit = 16 * (2 * kb + s / 4) + 4 * q + s % 4;
                    const int lane = i + 16 * q;
                    tiles[kMlpW2Shorts + ((size_t)(2 * mt + kb) * 64 + lane) * 8 + s] =
                        bf(P[OFF_W2 + unit * kMlpH + 16 * mt + i]);
                }
    for (int ks = 0; ks < 4; ++ks)  // W3^T: rows = outputs (6 used)
        for (int i = 0; i < 16; ++i)
            for (int k = 0; k < 16; ++k)
                put(kMlpW3Tile + ks, i, k, i < kMlpOut ? P[OFF_W3 + (16 * ks + k) * kMlpOut + i] : 0.f);
    bias.assign(kMlpH + kMlpH + 8, 0.f);
    for (int j = 0; j < kMlpH; ++j) {
        bias[j] = P[OFF_B1 + j];
        bias[kMlpH + j] = P[OFF_B2 + j];
    }
    for (int o = 0; o < kMlpOut; ++o) bias[2 * kMlpH + o] = P[OFF_B3 + o];
}

}  // namespace lesasm

using namespace lesasm;

struct lesasm_mlp {
    int device = 0;
    float *params = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    short *packed = nullptr;
    float *bias = nullptr;
    int step = 0;
    // training work arrays, grown on demand
    int cap = 0;
    float *H1 = nullptr, *H2 = nullptr, *DY = nullptr, *DA1 = nullptr, *DA2 = nullptr, *loss = nullptr;
};

static void mlp_free_work(lesasm_mlp *p) {
    for (float *q : {p->H1, p->H2, p->DY, p->DA1, p->DA2, p->loss}) device_free(q);
    p->H1 = p->H2 = p->DY = p->DA1 = p->DA2 = p->loss = nullptr;
    p->cap = 0;
}

static void mlp_free(lesasm_mlp *p) {
    if (!p) return;
    (void)hipDeviceSynchronize();
    mlp_free_work(p);
    for (void *q : {(void *)p->params, (void *)p->m, (void *)p->v, (void *)p->grad, (void *)p->packed, (void *)p->bias})
        device_free(q);
    delete p;
}

static int mlp_repack(lesasm_mlp *p) {
    std::vector<float> host(kMlpParams);
    LESASM_HIP_TRY(hipMemcpy(host.data(), p->params, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
    std::vector<short> tiles;
    std::vector<float> bias;
    pack_weights(host.data(), tiles, bias);
    LESASM_HIP_TRY(hipMemcpy(p->packed, tiles.data(), sizeof(short) * tiles.size(), hipMemcpyHostToDevice));
    LESASM_HIP_TRY(hipMemcpy(p->bias, bias.data(), sizeof(float) * bias.size(), hipMemcpyHostToDevice));
    return LESASM_OK;
}

static int mlp_work(lesasm_mlp *p, int n) {
    if (n <= p->cap) return LESASM_OK;
    mlp_free_work(p);
    const size_t N = (size_t)n;
    for (auto pr : {std::make_pair(&p->H1, N * kMlpH), std::make_pair(&p->H2, N * kMlpH),
                    std::make_pair(&p->DY, N * kMlpOut), std::make_pair(&p->DA1, N * kMlpH),
                    std::make_pair(&p->DA2, N * kMlpH), std::make_pair(&p->loss, N)}) {
        const int st = device_alloc((void **)pr.first, pr.second * sizeof(float), "mlp work arrays");
        if (st) {
            mlp_free_work(p);
            return st;
        }
    }
    p->cap = n;
    return LESASM_OK;
}

extern "C" int lesasm_mlp_create(const float *params, lesasm_mlp **out) {
    if (!out || !params) return fail(LESASM_E_INVALID_ARG, "mlp_create: NULL argument");
    *out = nullptr;
    auto *p = new lesasm_mlp();
    struct Guard {
        lesasm_mlp *q;
        ~Guard() { mlp_free(q); }
    } guard{p};
    LESASM_HIP_TRY(hipGetDevice(&p->device));
    for (auto pr : {std::make_pair((void **)&p->params, sizeof(float) * kMlpParams),
                    std::make_pair((void **)&p->m, sizeof(float) * kMlpParams),
                    std::make_pair((void **)&p->v, sizeof(float) * kMlpParams),
                    std::make_pair((void **)&p->grad, sizeof(float) * kMlpParams),
                    std::make_pair((void **)&p->packed, sizeof(short) * kMlpPackedShorts),
                    std::make_pair((void **)&p->bias, sizeof(float) * (2 * kMlpH + 8))}) {
        const int st = device_alloc(pr.first, pr.second, "mlp_create");
        if (st) return st;
    }
    LESASM_HIP_TRY(hipMemcpy(p->params, params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    LESASM_HIP_TRY(hipMemset(p->m, 0, sizeof(float) * kMlpParams));
    LESASM_HIP_TRY(hipMemset(p->v, 0, sizeof(float) * kMlpParams));
    int st = mlp_repack(p);
    if (st) return st;
    guard.q = nullptr;
    *out = p;
    return LESASM_OK;
}

extern "C" int lesasm_mlp_destroy(lesasm_mlp *p) {
    mlp_free(p);
    return LESASM_OK;
}

extern "C" int lesasm_mlp_get_params(const lesasm_mlp *p, float *params) {
    if (!p || !params) return fail(LESASM_E_INVALID_ARG, "mlp_get_params: NULL argument");
    LESASM_HIP_TRY(hipMemcpy(params, p->params, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
    return LESASM_OK;
}

extern "C" int lesasm_mlp_set_params(lesasm_mlp *p, const float *params) {
    if (!p || !params) return fail(LESASM_E_INVALID_ARG, "mlp_set_params: NULL argument");
    LESASM_HIP_TRY(hipMemcpy(p->params, params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    LESASM_HIP_TRY(hipMemset(p->m, 0, sizeof(float) * kMlpParams));
    LESASM_HIP_TRY(hipMemset(p->v, 0, sizeof(float) * kMlpParams));
    p->step = 0;
    return mlp_repack(p);
}

extern "C" int lesasm_mlp_loss_grad(lesasm_mlp *p, const float *d_x, const float *d_t, int n, float *d_grad,
                                    float *d_loss, void *stream) {
    if (!p || !d_x || !d_t || n < 1) return fail(LESASM_E_INVALID_ARG, "mlp_loss_grad: bad argument");
    int st = mlp_work(p, n);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    const dim3 g((n + 127) / 128), b(128);
    hipLaunchKernelGGL(k_mlp_fwd_train, g, b, 0, s, p->params, d_x, d_t, n, p->H1, p->H2, p->DY, p->loss);
    hipLaunchKernelGGL(k_mlp_bwd_act, g, b, 0, s, p->params, p->H1, p->H2, p->DY, n, p->DA1, p->DA2);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(141), dim3(64), 0, s, d_x, p->H1, p->H2, p->DA1, p->DA2, p->DY, n,
                       d_grad ? d_grad : p->grad);
    if (d_loss) hipLaunchKernelGGL(k_sum_f32, dim3(1), dim3(256), 0, s, p->loss, n, d_loss);
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

// ---- loss gradient without allocation -------------------------------------------
// The training work arrays of lesasm_mlp_loss_grad_noalloc live in one
// file-scope device array, H1, H2, DA1, DA2 [n][64], DY [n][6], loss [n] for
// n up to kNoAllocMaxSamples (8.6 MB; each device holds its own copy until the
// process ends).  Host code never passes the array's name to a kernel: its
// device address is taken once per device with hipGetSymbolAddress and kept
// in g_scratch.  Every kernel writes each work entry of samples < n before
// any kernel reads it, so nothing is cleared between calls.
namespace {
constexpr int kNoAllocMaxSamples = 8192;
constexpr size_t kScratchPerSample = 4 * kMlpH + kMlpOut + 1;
constexpr int kScratchDevices = 64;
}  // namespace

static __device__ __align__(256) float scratch[(size_t)kNoAllocMaxSamples * kScratchPerSample];

static std::mutex g_scratch_mu;
static float *g_scratch[kScratchDevices];

static int scratch_address(int device, float **out) {
    if (device < 0 || device >= kScratchDevices)
        return fail(LESASM_E_UNSUPPORTED, "mlp_loss_grad_noalloc: device id too large");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(LESASM_E_HIP, std::string("mlp_loss_grad_noalloc: hipGetSymbolAddress failed: ") +
                                          hipGetErrorString(e));
        g_scratch[device] = (float *)ptr;
    }
    *out = g_scratch[device];
    return LESASM_OK;
}

extern "C" int lesasm_mlp_loss_grad_noalloc(lesasm_mlp *p, const float *d_x, const float *d_t, int n,
                                            float *d_grad, float *d_loss, void *stream) {
    if (!p || !d_x || !d_t || n < 1) return fail(LESASM_E_INVALID_ARG, "mlp_loss_grad_noalloc: bad argument");
    if (n > kNoAllocMaxSamples)
        return fail(LESASM_E_INVALID_ARG, "mlp_loss_grad_noalloc: n = " + std::to_string(n) + " exceeds the " +
                                              std::to_string(kNoAllocMaxSamples) + " samples of the static work area");
    int dev = -1;
    LESASM_HIP_TRY(hipGetDevice(&dev));
    if (dev != p->device) return fail(LESASM_E_STATE, "mlp_loss_grad_noalloc: current device differs from the mlp's");
    float *w = nullptr;
    int st = scratch_address(dev, &w);
    if (st) return st;
    const size_t N = (size_t)n;
    float *H1 = w, *H2 = H1 + N * kMlpH, *DA1 = H2 + N * kMlpH, *DA2 = DA1 + N * kMlpH, *DY = DA2 + N * kMlpH,
          *loss = DY + N * kMlpOut;
    hipStream_t s = (hipStream_t)stream;
    const dim3 g((n + 127) / 128), b(128);
    hipLaunchKernelGGL(k_mlp_fwd_train, g, b, 0, s, p->params, d_x, d_t, n, H1, H2, DY, loss);
    hipLaunchKernelGGL(k_mlp_bwd_act, g, b, 0, s, p->params, H1, H2, DY, n, DA1, DA2);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(141), dim3(64), 0, s, d_x, H1, H2, DA1, DA2, DY, n, d_grad ? d_grad : p->grad);
    if (d_loss) hipLaunchKernelGGL(k_sum_f32, dim3(1), dim3(256), 0, s, loss, n, d_loss);
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

extern "C" int lesasm_mlp_adam(lesasm_mlp *p, const float *d_grad, float lr, void *stream) {
    if (!p) return fail(LESASM_E_INVALID_ARG, "mlp_adam: NULL argument");
    p->step += 1;
    const float c1 = 1.f - std::pow(0.9f, (float)p->step), c2 = 1.f - std::pow(0.999f, (float)p->step);
    hipLaunchKernelGGL(k_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, (hipStream_t)stream, p->params, p->m,
                       p->v, d_grad ? d_grad : p->grad, kMlpParams, lr, c1, c2);
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

extern "C" int lesasm_mlp_train_step(lesasm_mlp *p, const float *d_x, const float *d_t, int n, float lr,
                                     float *d_loss, void *stream) {
    int st = lesasm_mlp_loss_grad(p, d_x, d_t, n, nullptr, d_loss, stream);
    if (st) return st;
    return lesasm_mlp_adam(p, nullptr, lr, stream);
}

extern "C" int lesasm_mlp_commit(lesasm_mlp *p) {
    if (!p) return fail(LESASM_E_INVALID_ARG, "mlp_commit: NULL argument");
    LESASM_HIP_TRY(hipDeviceSynchronize());
    return mlp_repack(p);
}

extern "C" int lesasm_mlp_forward_f32(lesasm_mlp *p, const float *d_x, int n, float *d_y, void *stream) {
    if (!p || !d_x || !d_y || n < 0) return fail(LESASM_E_INVALID_ARG, "mlp_forward_f32: bad argument");
    if (!n) return LESASM_OK;
    hipLaunchKernelGGL(k_mlp_forward_f32, dim3((n + 127) / 128), dim3(128), 0, (hipStream_t)stream, p->params, d_x, n, d_y);
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

extern "C" int lesasm_mlp_infer_bf16(lesasm_mlp *p, const float *d_x, int n, float *d_y, void *stream) {
    if (!p || !d_x || !d_y || n < 0) return fail(LESASM_E_INVALID_ARG, "mlp_infer_bf16: bad argument");
    if (!n) return LESASM_OK;
    const int groups = (n + 63) / 64;
    const int blocks = std::min((groups + 3) / 4, 1024);
    const size_t shm = kMlpLdsBytes + 4 * kMlpWaveScratch;
    hipLaunchKernelGGL(k_mlp_infer_bf16, dim3(blocks), dim3(256), shm, (hipStream_t)stream, p->packed, p->bias, d_x,
                       n, d_y);
    LESASM_HIP_TRY(hipGetLastError());
    return LESASM_OK;
}

// Internal accessors for the fused closure.
namespace lesasm {
const short *mlp_packed(const lesasm_mlp *p) { return p->packed; }
const float *mlp_bias(const lesasm_mlp *p) { return p->bias; }
}  // namespace lesasm
