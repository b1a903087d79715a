// Learned subgrid closure: a 10-64-64-6 perceptron evaluated by one wavefront
// for 64 samples at once with BF16 matrix-core instructions (FP32 sums).
//
// The chain is computed transposed, H^T = W^T X^T, so that a layer's 16x16
// accumulator tiles are, element for element, the B operand of the next
// layer (rows = hidden units = the K index, columns = samples):
//   v_mfma_f32_16x16x16_bf16:  A[i][k] in lane i + 16 (k/4), slot k%4
//                              B[k][j] in lane j + 16 (k/4), slot k%4
//                              D[i][j] in lane j + 16 (i/4), slot i%4
// Layer 2 uses gfx950's v_mfma_f32_16x16x32_bf16 (K = 32 per instruction:
// A[i][k] in lane i + 16 (k/8), slot k%8, B likewise), with its 32 K values
// taken from two row tiles t0, t1 of H1: slot s of lane j + 16 q holds hidden
// unit 16 t0 + 4 q + s (s < 4) or 16 t1 + 4 q + s - 4, which is exactly what
// that lane holds of the two tiles, so H1 needs no movement between lanes; the
// W2 tiles are packed with the same numbering of the hidden units.
// Weights are packed once into those A tiles (W1^T: 4 row tiles, K padded
// from 10 to 16; W2^T: 4 x 2 tiles of K = 32; W3^T: 1 row tile, 6 of 16 rows
// used, 4 K tiles).
// Inputs:  x = [G / |G|_F (9), log(Delta / Delta_ref)], outputs 6 symmetric
// components (xx, yy, zz, xy, xz, yz) before the trace removal.
#pragma once

#include "common.hpp"

namespace lesasm {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kMlpIn = 10, kMlpH = 64, kMlpOut = 6;
constexpr int kMlpParams = kMlpIn * kMlpH + kMlpH + kMlpH * kMlpH + kMlpH + kMlpH * kMlpOut + kMlpOut;  // 5254
// packed A tiles: 4 (W1, 64 lanes x 4 bf16), 8 (W2, 64 lanes x 8 bf16), 4 (W3,
// 64 lanes x 4 bf16); in units of 64 lanes x 4 bf16: 4 + 16 + 4
constexpr int kMlpTiles = 4 + 16 + 4;
constexpr int kMlpPackedShorts = kMlpTiles * 64 * 4;
constexpr int kMlpW2Shorts = 4 * 64 * 4;   // offset of the W2 tiles
constexpr int kMlpW3Tile = 20;              // first W3 tile, in 64 x 4 units
// LDS bytes of the packed weights and biases (b1, b2, b3 padded to 8)
constexpr int kMlpLdsBytes = kMlpPackedShorts * 2 + (kMlpH + kMlpH + 8) * 4;
// per-wavefront LDS scratch: 64 samples x 16 bf16 inputs (32 bytes per sample),
// over which the 64 x 8 float outputs (32 bytes per sample) are written once
// the sample's inputs have been read
constexpr int kMlpWaveScratch = 64 * 16 * 2;

// Round-to-nearest-even float -> bf16 bits (finite inputs).
__device__ __forceinline__ short f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

struct MlpLds {
    const bf16x4_t *tiles;  // W1 and W3 tiles, [tile][64] in 64 x 4 units
    const bf16x8_t *w2;     // W2 tiles, [2 mt + kb][64]
    const float *b1, *b2, *b3;
};

// View of packed weights already staged in LDS at `lds`.
__device__ __forceinline__ MlpLds mlp_lds_view(const unsigned char *lds) {
    const short *t = (const short *)lds;
    const float *b = (const float *)(lds + kMlpPackedShorts * 2);
    return MlpLds{(const bf16x4_t *)t, (const bf16x8_t *)(t + kMlpW2Shorts), b, b + kMlpH, b + 2 * kMlpH};
}

// Copy packed weights (global, bf16 tiles + f32 biases) into LDS; call with the
// whole workgroup, followed by a barrier.
__device__ __forceinline__ MlpLds mlp_stage(const short *__restrict__ packed, const float *__restrict__ bias,
                                            unsigned char *lds) {
    short *t = (short *)lds;
    for (int k = threadIdx.x; k < kMlpPackedShorts / 4; k += blockDim.x)
        ((bf16x4_t *)t)[k] = ((const bf16x4_t *)packed)[k];
    float *b = (float *)(lds + kMlpPackedShorts * 2);
    for (int k = threadIdx.x; k < kMlpH + kMlpH + 8; k += blockDim.x) b[k] = bias[k];
    return mlp_lds_view(lds);
}

// Two floats to two bf16 (round to nearest even, the hardware conversion),
// packed low-first into 32 bits.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
    const f32x2_t v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}
__device__ __forceinline__ bf16x4_t pack_bf16x4(float a, float b, float c, float d) {
    const uint32_t lo = pack_bf16(a, b), hi = pack_bf16(c, d);
    typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
    const u32x2_t v = {lo, hi};
    return __builtin_bit_cast(bf16x4_t, v);
}
// max(v, 0) on four bf16 values: a negative bf16 is a negative 16-bit
// integer, so two packed integer maxima clear the negative values; rounding
// then rectifying equals rectifying then rounding.
__device__ __forceinline__ bf16x4_t relu_bf16x4(bf16x4_t v) {
    return __builtin_elementwise_max(v, bf16x4_t{0, 0, 0, 0});
}
// Two bf16x4 register quads as one bf16x8 operand (slots 0-3, then 4-7).
__device__ __forceinline__ bf16x8_t cat_bf16x8(bf16x4_t lo, bf16x4_t hi) {
    typedef short s16x8_t __attribute__((ext_vector_type(8)));
    const s16x8_t v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    return __builtin_bit_cast(bf16x8_t, v);
}

// Whole-wavefront evaluation: every lane supplies the 10 inputs of its own
// sample and receives its 6 outputs.  All 64 lanes must call it together
// (matrix instructions ignore the execution mask).  scratch: kMlpWaveScratch
// bytes of LDS private to this wavefront.  Biases enter as the accumulator
// input of the first matrix instruction of each tile; layer 2 and layer 3 run
// row tile by row tile, so only one row tile of H2 is ever held.  PASSES = 2
// or 4 runs the chain on 32 or 16 samples at a time (a half or a quarter of
// the live activations, the weight tiles read as many times), for kernels
// whose occupancy that raises.
template <int PASSES = 1>
__device__ __forceinline__ void mlp_wave(const MlpLds &w, const float (&x)[kMlpIn], float (&y)[kMlpOut],
                                         unsigned char *scratch) {
    static_assert(PASSES == 1 || PASSES == 2 || PASSES == 4, "one, two or four passes");
    constexpr int NT = 4 / PASSES;  // sample tiles of 16 per pass
    const int lane = __lane_id();
    const int lq = lane >> 4, lr = lane & 15;
    short *xs = (short *)scratch;  // [64][16] inputs
    float *ys = (float *)scratch;  // [64][8] outputs, sample j over input row j
    {
        const bf16x4_t v0 = pack_bf16x4(x[0], x[1], x[2], x[3]);
        const bf16x4_t v1 = pack_bf16x4(x[4], x[5], x[6], x[7]);
        const bf16x4_t v2 = pack_bf16x4(x[8], x[9], 0.f, 0.f);
        const bf16x4_t v3 = {0, 0, 0, 0};
        bf16x4_t *dst = (bf16x4_t *)(xs + 16 * lane);
        dst[0] = v0;
        dst[1] = v1;
        dst[2] = v2;
        dst[3] = v3;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll 1
    for (int pass = 0; pass < PASSES; ++pass) {  // not unrolled: the passes reuse the same registers
        // B operands of layer 1: X^T[k][sample], sample = 16 nt + lr, k = 4 lq + t
        bf16x4_t bx[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) bx[t] = ((const bf16x4_t *)(xs + 16 * (16 * (NT * pass + t) + lr)))[lq];

        // layer 1: H1^T = relu(W1^T X^T + b1), 4 row tiles x NT sample tiles
        bf16x4_t h1[4][NT];  // [k-step = row tile][sample tile]
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bf16x4_t a = w.tiles[mt * 64 + lane];
            const f32x4_t b = *(const f32x4_t *)(w.b1 + 16 * mt + 4 * lq);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const f32x4_t acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bx[t], b, 0, 0, 0);
                h1[mt][t] = relu_bf16x4(pack_bf16x4(acc[0], acc[1], acc[2], acc[3]));
            }
        }
        // layers 2 and 3 by row tile of H2: H2^T = relu(W2^T H1^T + b2), Y^T += W3^T H2^T
        f32x4_t acc3[NT];
        {
            const f32x4_t b3 = lq < 2 ? *(const f32x4_t *)(w.b3 + 4 * lq) : f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int t = 0; t < NT; ++t) acc3[t] = b3;
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const f32x4_t b = *(const f32x4_t *)(w.b2 + 16 * mt + 4 * lq);
            f32x4_t acc[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = b;
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                const bf16x8_t a = w.w2[(2 * mt + kb) * 64 + lane];
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, cat_bf16x8(h1[2 * kb][t], h1[2 * kb + 1][t]),
                                                                     acc[t], 0, 0, 0);
            }
            const bf16x4_t a3 = w.tiles[(kMlpW3Tile + mt) * 64 + lane];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const bf16x4_t h2 = relu_bf16x4(pack_bf16x4(acc[t][0], acc[t][1], acc[t][2], acc[t][3]));
                acc3[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a3, h2, acc3[t], 0, 0, 0);
            }
        }
        // Y^T rows 0..5 (lanes with lq < 2 hold rows 0..7), over the input rows
        // of this pass's samples, which no later pass reads
        if (lq < 2)
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) ys[8 * (16 * (NT * pass + t) + lr) + 4 * lq + q] = acc3[t][q];
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o) y[o] = ys[8 * lane + o];
    __builtin_amdgcn_wave_barrier();
}

// Inputs of one Gauss point: G (row-major du_i/dx_j) and log(Delta/Delta_ref).
template <typename R>
__device__ __forceinline__ void mlp_features(const R (&G)[3][3], float logd, float (&x)[kMlpIn], R &gnorm2) {
    gnorm2 = (R)0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) gnorm2 += G[i][j] * G[i][j];
    const float inv = gnorm2 > (R)0 ? __builtin_amdgcn_rsqf((float)gnorm2) : 0.f;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) x[3 * i + j] = (float)G[i][j] * inv;
    x[9] = logd;
}

}  // namespace lesasm
