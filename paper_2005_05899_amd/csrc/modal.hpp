// Modal (monomial) form of the linear pyramid, prism and hexahedron.
//
// Each of these elements spans a small space of functions of the reference
// coordinates, so a nodal field v_a is rewritten once per element as
// coefficients c_m of fixed monomials phi_m:  v(xi) = sum_m c_m phi_m(xi),
// with N_a = sum_m B[a][m] phi_m.  At a Gauss point the value and the three
// reference derivatives then cost a few multiply-adds with point scalars
// instead of one multiply-add per node and direction; the test side is the
// transpose: F_m = sum_g (phi_m f_g + grad phi_m . T_g), R_a = sum_m B[a][m] F_m.
// The algebra is exact: the same residual, with fewer operations.
//
//  HEX08  phi = {1, x, y, z, xy, xz, yz, xyz} on [-1,1]^3;
//         N_a = (1+sx x)(1+sy y)(1+sz z)/8, so B[a][m] = s^m_a / 8
//         (s^m_a the product of the node's signs over the monomial's variables).
//  PEN06  phi = {1, r, s, z, rz, sz};  N_(i,l) = L_i (1 + sigma_l z)/2,
//         L = (1-r-s, r, s), sigma = (-1, +1) for the bottom / top triangle.
//  PYR05  phi = {1, xi, eta, zeta, q} with q = xi eta / (1 - zeta);
//         N_a = (1 - zeta + sx xi + sy eta + sx sy q)/4 (base), N_4 = zeta.
//         At a point of the collapsed rule (A, B, c): xi = A(1-c), eta = B(1-c),
//         zeta = c, q = AB(1-c) and grad q = (B, A, AB).
//
// Trial coefficients are formed in FP64 from the FP64 nodal values; the
// coordinate field keeps only its non-constant coefficients (all differences
// of node values), so converting them to FP32 loses nothing to cancellation.
// Per-point scalars live in constant memory (uniform, scalar loads).
#pragma once

#include "refelem.hpp"

namespace lesasm {

template <int NQ, int NG> struct ModalPts {
    double w[NG];      // Gauss weight times the sign and scale folded from B
    double q[NG][NQ];  // point scalars (see each type)
};

// HEX08: q = {x, y, z, xy, xz, yz, xyz}; w = -1/8 (B = s/8 and R = -F folded).
__host__ __device__ constexpr ModalPts<7, 8> make_modal_hex08() {
    ModalPts<7, 8> t{};
    for (int g = 0; g < 8; ++g) {
        const double X = (g & 1 ? 1 : -1) * kInvSqrt3;
        const double Y = (g & 2 ? 1 : -1) * kInvSqrt3;
        const double Z = (g & 4 ? 1 : -1) * kInvSqrt3;
        t.w[g] = -0.125;
        t.q[g][0] = X;
        t.q[g][1] = Y;
        t.q[g][2] = Z;
        t.q[g][3] = X * Y;
        t.q[g][4] = X * Z;
        t.q[g][5] = Y * Z;
        t.q[g][6] = X * Y * Z;
    }
    return t;
}

// PEN06: q = {r, s, z, rz, sz}; w = -(1/6)(1/2).
__host__ __device__ constexpr ModalPts<5, 6> make_modal_pen06() {
    ModalPts<5, 6> t{};
    const double tr[3][2] = {{1.0 / 6.0, 1.0 / 6.0}, {2.0 / 3.0, 1.0 / 6.0}, {1.0 / 6.0, 2.0 / 3.0}};
    for (int g = 0; g < 6; ++g) {
        const double r = tr[g % 3][0], s = tr[g % 3][1];
        const double z = (g < 3 ? -1 : 1) * kInvSqrt3;
        t.w[g] = -1.0 / 12.0;
        t.q[g][0] = r;
        t.q[g][1] = s;
        t.q[g][2] = z;
        t.q[g][3] = r * z;
        t.q[g][4] = s * z;
    }
    return t;
}

// PYR05: q = {xi, eta, zeta, q, A, B, AB}; w = -W (the sign of R = -F folded;
// the base nodes' 1/4 is applied when the modal residual is distributed).
__host__ __device__ constexpr ModalPts<7, 8> make_modal_pyr05() {
    ModalPts<7, 8> t{};
    for (int g = 0; g < 8; ++g) {
        const double A = (g & 1 ? 1 : -1) * kInvSqrt3;
        const double B = (g & 2 ? 1 : -1) * kInvSqrt3;
        const double c = kPyrC[g >> 2];
        t.w[g] = -kPyrW[g >> 2];
        t.q[g][0] = A * (1.0 - c);
        t.q[g][1] = B * (1.0 - c);
        t.q[g][2] = c;
        t.q[g][3] = A * B * (1.0 - c);
        t.q[g][4] = A;
        t.q[g][5] = B;
        t.q[g][6] = A * B;
    }
    return t;
}

static __constant__ ModalPts<7, 8> c_modal_hex08 = make_modal_hex08();
static __constant__ ModalPts<5, 6> c_modal_pen06 = make_modal_pen06();
static __constant__ ModalPts<7, 8> c_modal_pyr05 = make_modal_pyr05();

template <int T> struct Modal;

// ---------------------------------------------------------------- HEX08
template <> struct Modal<LESASM_HEX08> {
    static constexpr int nn = 8, nm = 8, nq = 7, ng = 8;
    __device__ static const ModalPts<7, 8> &pts() { return c_modal_hex08; }
    // c[m] = sum_a s^m_a v_a / 8, m = {1, x, y, z, xy, xz, yz, xyz}; node
    // order: (x, y) = (-,-), (+,-), (+,+), (-,+) on z = -1, then on z = +1.
    __host__ __device__ static void to_modal(const double (&v)[8], double (&c)[8]) {
        // tensor index t = ix + 2 iy + 4 iz of node a
        const double h[8] = {v[0], v[1], v[3], v[2], v[4], v[5], v[7], v[6]};
        double a1[8], a2[8];
#pragma unroll
        for (int k = 0; k < 4; ++k) {  // x stage: pairs t, t+1
            a1[2 * k] = h[2 * k] + h[2 * k + 1];
            a1[2 * k + 1] = h[2 * k + 1] - h[2 * k];
        }
#pragma unroll
        for (int k = 0; k < 2; ++k)  // y stage: pairs t, t+2
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                a2[4 * k + j] = a1[4 * k + j] + a1[4 * k + j + 2];
                a2[4 * k + j + 2] = a1[4 * k + j + 2] - a1[4 * k + j];
            }
        double a3[8];
#pragma unroll
        for (int j = 0; j < 4; ++j) {  // z stage: pairs t, t+4
            a3[j] = a2[j] + a2[j + 4];
            a3[j + 4] = a2[j + 4] - a2[j];
        }
        // a3[t]: t bit0 = x, bit1 = y, bit2 = z factor present
        c[0] = 0.125 * a3[0];
        c[1] = 0.125 * a3[1];
        c[2] = 0.125 * a3[2];
        c[3] = 0.125 * a3[4];
        c[4] = 0.125 * a3[3];
        c[5] = 0.125 * a3[5];
        c[6] = 0.125 * a3[6];
        c[7] = 0.125 * a3[7];
    }
    // value (with c[0]) and reference gradient at point scalars q
    template <typename R> __host__ __device__ static void grad(const R *c, const double *q, R (&d)[3]) {
        // c indexed {1, x, y, z, xy, xz, yz, xyz}
        d[0] = c[1] + (R)q[1] * c[4] + (R)q[2] * c[5] + (R)q[5] * c[7];
        d[1] = c[2] + (R)q[0] * c[4] + (R)q[2] * c[6] + (R)q[4] * c[7];
        d[2] = c[3] + (R)q[0] * c[5] + (R)q[1] * c[6] + (R)q[3] * c[7];
    }
    template <typename R> __host__ __device__ static R value(const R *c, const double *q, const R (&)[3]) {
        return c[0] + (R)q[0] * c[1] + (R)q[1] * c[2] + (R)q[2] * c[3] + (R)q[3] * c[4] + (R)q[4] * c[5] +
               (R)q[5] * c[6] + (R)q[6] * c[7];
    }
    // F_m += phi_m f + grad phi_m . t  (WF false: the gradient part only)
    template <bool WF, typename R> __host__ __device__ static void test(R *F, const double *q, R f, const R (&t)[3]) {
        const R x = (R)q[0], y = (R)q[1], z = (R)q[2], xy = (R)q[3], xz = (R)q[4], yz = (R)q[5], xyz = (R)q[6];
        if (WF) {
            F[0] += f;
            F[1] += x * f;
            F[2] += y * f;
            F[3] += z * f;
            F[4] += xy * f;
            F[5] += xz * f;
            F[6] += yz * f;
            F[7] += xyz * f;
        }
        F[1] += t[0];
        F[2] += t[1];
        F[3] += t[2];
        F[4] += y * t[0] + x * t[1];
        F[5] += z * t[0] + x * t[2];
        F[6] += z * t[1] + y * t[2];
        F[7] += yz * t[0] + xz * t[1] + xy * t[2];
    }
    // R_a = sum_m s^m_a F_m (scale and sign are in the weights)
    template <typename R> __host__ __device__ static void to_nodal(const R (&F)[8], R (&r)[8]) {
        // inverse tensor transform: r[t] = sum over monomials of signs
        const R a3[8] = {F[0], F[1], F[2], F[4], F[3], F[5], F[6], F[7]};  // index by bit mask
        R a2[8], a1[8], h[8];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a2[j] = a3[j] - a3[j + 4];
            a2[j + 4] = a3[j] + a3[j + 4];
        }
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                a1[4 * k + j] = a2[4 * k + j] - a2[4 * k + j + 2];
                a1[4 * k + j + 2] = a2[4 * k + j] + a2[4 * k + j + 2];
            }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            h[2 * k] = a1[2 * k] - a1[2 * k + 1];
            h[2 * k + 1] = a1[2 * k] + a1[2 * k + 1];
        }
        r[0] = h[0];
        r[1] = h[1];
        r[2] = h[3];
        r[3] = h[2];
        r[4] = h[4];
        r[5] = h[5];
        r[6] = h[7];
        r[7] = h[6];
    }
};

// ---------------------------------------------------------------- PEN06
template <> struct Modal<LESASM_PEN06> {
    static constexpr int nn = 6, nm = 6, nq = 5, ng = 6;
    __device__ static const ModalPts<5, 6> &pts() { return c_modal_pen06; }
    // nodes 0..2 bottom triangle (z = -1), 3..5 top; c = {1, r, s, z, rz, sz}
    __host__ __device__ static void to_modal(const double (&v)[6], double (&c)[6]) {
        const double m0 = 0.5 * (v[0] + v[3]), m1 = 0.5 * (v[1] + v[4]), m2 = 0.5 * (v[2] + v[5]);
        const double d0 = 0.5 * (v[3] - v[0]), d1 = 0.5 * (v[4] - v[1]), d2 = 0.5 * (v[5] - v[2]);
        c[0] = m0;
        c[1] = m1 - m0;
        c[2] = m2 - m0;
        c[3] = d0;
        c[4] = d1 - d0;
        c[5] = d2 - d0;
    }
    template <typename R> __host__ __device__ static void grad(const R *c, const double *q, R (&d)[3]) {
        d[0] = c[1] + (R)q[2] * c[4];
        d[1] = c[2] + (R)q[2] * c[5];
        d[2] = c[3] + (R)q[0] * c[4] + (R)q[1] * c[5];
    }
    // value from the z-derivative d[2] of grad(): c0 + r c_r + s c_s + z d_z
    template <typename R> __host__ __device__ static R value(const R *c, const double *q, const R (&d)[3]) {
        return c[0] + (R)q[0] * c[1] + (R)q[1] * c[2] + (R)q[2] * d[2];
    }
    template <bool WF, typename R> __host__ __device__ static void test(R *F, const double *q, R f, const R (&t)[3]) {
        const R r = (R)q[0], s = (R)q[1], z = (R)q[2], rz = (R)q[3], sz = (R)q[4];
        if (WF) {
            F[0] += f;
            F[1] += r * f;
            F[2] += s * f;
            F[3] += z * f;
            F[4] += rz * f;
            F[5] += sz * f;
        }
        F[1] += t[0];
        F[2] += t[1];
        F[3] += t[2];
        F[4] += z * t[0] + r * t[2];
        F[5] += z * t[1] + s * t[2];
    }
    // R_(i,l) = sum_m 2 B[(i,l)][m] F_m (the 1/2 and the sign are in the weights)
    template <typename R> __host__ __device__ static void to_nodal(const R (&F)[6], R (&r)[6]) {
        const R a = F[0] - F[1] - F[2], b = F[3] - F[4] - F[5];
        r[0] = a - b;
        r[3] = a + b;
        r[1] = F[1] - F[4];
        r[4] = F[1] + F[4];
        r[2] = F[2] - F[5];
        r[5] = F[2] + F[5];
    }
};

// ---------------------------------------------------------------- PYR05
template <> struct Modal<LESASM_PYR05> {
    static constexpr int nn = 5, nm = 5, nq = 7, ng = 8;
    __device__ static const ModalPts<7, 8> &pts() { return c_modal_pyr05; }
    // base nodes (sx, sy) = (-,-), (+,-), (+,+), (-,+), apex 4; c = {1, xi, eta, zeta, q}
    __host__ __device__ static void to_modal(const double (&v)[5], double (&c)[5]) {
        const double p = v[0] + v[1], m = v[1] - v[0], P = v[2] + v[3], M = v[2] - v[3];
        c[0] = 0.25 * (p + P);
        c[1] = 0.25 * (m + M);
        c[2] = 0.25 * (P - p);
        c[3] = v[4] - c[0];
        c[4] = 0.25 * (M - m);
    }
    template <typename R> __host__ __device__ static void grad(const R *c, const double *q, R (&d)[3]) {
        d[0] = c[1] + (R)q[5] * c[4];
        d[1] = c[2] + (R)q[4] * c[4];
        d[2] = c[3] + (R)q[6] * c[4];
    }
    template <typename R> __host__ __device__ static R value(const R *c, const double *q, const R (&)[3]) {
        return c[0] + (R)q[0] * c[1] + (R)q[1] * c[2] + (R)q[2] * c[3] + (R)q[3] * c[4];
    }
    template <bool WF, typename R> __host__ __device__ static void test(R *F, const double *q, R f, const R (&t)[3]) {
        if (WF) {
            F[0] += f;
            F[1] += (R)q[0] * f;
            F[2] += (R)q[1] * f;
            F[3] += (R)q[2] * f;
            F[4] += (R)q[3] * f;
        }
        F[1] += t[0];
        F[2] += t[1];
        F[3] += t[2];
        F[4] += (R)q[5] * t[0] + (R)q[4] * t[1] + (R)q[6] * t[2];
    }
    template <typename R> __host__ __device__ static void to_nodal(const R (&F)[5], R (&r)[5]) {
        const R b = F[0] - F[3];
        r[0] = (R)0.25 * (b - F[1] - F[2] + F[4]);
        r[1] = (R)0.25 * (b + F[1] - F[2] - F[4]);
        r[2] = (R)0.25 * (b + F[1] + F[2] + F[4]);
        r[3] = (R)0.25 * (b - F[1] + F[2] - F[4]);
        r[4] = F[3];
    }
};

}  // namespace lesasm
