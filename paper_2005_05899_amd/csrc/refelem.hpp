// Reference elements of the GPU path, built at compile time.
//
// For each linear element type: Gauss points, weights, shape-function values
// N[g][a] and reference derivatives dN[g][a][k] at those points.  Written for
// the device kernels in tensor / collapsed form; the kernels only ever see
// compile-time constants, which the compiler folds into the instruction
// stream after full unrolling (zeros and ones disappear).
//
//  TET04  unit simplex, N = (1-r-s-t, r, s, t); 4-point rule exact to degree 2
//         (barycentric (a,b,b,b), a = (5+3 sqrt5)/20, b = (5-sqrt5)/20, w = 1/24).
//  PYR05  base [-1,1]^2 at zeta=0, apex (0,0,1).  Evaluated in collapsed
//         coordinates xi = A(1-c), eta = B(1-c), zeta = c, where the rational
//         basis becomes polynomial: N_base = (1-c)(1+sx A)(1+sy B)/4 with
//         dN/dxi = sx(1+sy B)/4, dN/deta = sy(1+sx A)/4,
//         dN/dzeta = (sx sy A B - 1)/4; apex N = c, gradient (0,0,1).
//         Rule: A, B = +-1/sqrt3 times the 2-point Gauss-Jacobi rule of weight
//         (1-c)^2 on [0,1]: c = 1/3 -+ sqrt10/15, W = 1/6 +- sqrt10/48.
//  PEN06  triangle (1-r-s, r, s) x line ((1-z)/2, (1+z)/2); 3 x 2 points, w = 1/6.
//  HEX08  trilinear on [-1,1]^3, 2 x 2 x 2 Gauss-Legendre, w = 1.
#pragma once

#include "lesasm.h"

namespace lesasm {

// decimal expansions, correctly rounded by the compiler
constexpr double kInvSqrt3 = 0.577350269189625764509148780502;
constexpr double kTetA = 0.585410196624968454461376050310;
constexpr double kTetB = 0.138196601125010515179541316563;
constexpr double kPyrC[2] = {0.122514822655441377866740430371, 0.544151844011225288799926236296};
constexpr double kPyrW[2] = {0.232547451253507902749976948842, 0.100785882079825430583356384491};

template <int T> struct Ref;

template <int NN, int NG> struct RefTable {
    double w[NG];
    double N[NG][NN];
    double dN[NG][NN][3];
};

__host__ __device__ constexpr RefTable<8, 8> make_hex08() {
    RefTable<8, 8> t{};
    const int sx[8] = {-1, 1, 1, -1, -1, 1, 1, -1};
    const int sy[8] = {-1, -1, 1, 1, -1, -1, 1, 1};
    const int sz[8] = {-1, -1, -1, -1, 1, 1, 1, 1};
    for (int g = 0; g < 8; ++g) {
        const double X = (g & 1 ? 1 : -1) * kInvSqrt3;
        const double Y = (g & 2 ? 1 : -1) * kInvSqrt3;
        const double Z = (g & 4 ? 1 : -1) * kInvSqrt3;
        t.w[g] = 1.0;
        for (int a = 0; a < 8; ++a) {
            const double fx = 1.0 + sx[a] * X, fy = 1.0 + sy[a] * Y, fz = 1.0 + sz[a] * Z;
            t.N[g][a] = 0.125 * fx * fy * fz;
            t.dN[g][a][0] = 0.125 * sx[a] * fy * fz;
            t.dN[g][a][1] = 0.125 * sy[a] * fx * fz;
            t.dN[g][a][2] = 0.125 * sz[a] * fx * fy;
        }
    }
    return t;
}

template <> struct Ref<LESASM_HEX08> {
    static constexpr int nn = 8, ng = 8;
    static constexpr RefTable<8, 8> tab = make_hex08();
};

__host__ __device__ constexpr RefTable<4, 4> make_tet04() {
    RefTable<4, 4> t{};
    for (int g = 0; g < 4; ++g) {
        // point g has barycentric coordinate a on vertex g, b elsewhere
        double L[4] = {kTetB, kTetB, kTetB, kTetB};
        L[g] = kTetA;
        t.w[g] = 1.0 / 24.0;
        for (int a = 0; a < 4; ++a) {
            t.N[g][a] = L[a];
            for (int k = 0; k < 3; ++k) t.dN[g][a][k] = (a == 0) ? -1.0 : (a == k + 1 ? 1.0 : 0.0);
        }
    }
    return t;
}

template <> struct Ref<LESASM_TET04> {
    static constexpr int nn = 4, ng = 4;
    static constexpr RefTable<4, 4> tab = make_tet04();
};

__host__ __device__ constexpr RefTable<6, 6> make_pen06() {
    RefTable<6, 6> t{};
    const double tr[3][2] = {{1.0 / 6.0, 1.0 / 6.0}, {2.0 / 3.0, 1.0 / 6.0}, {1.0 / 6.0, 2.0 / 3.0}};
    for (int g = 0; g < 6; ++g) {
        const double r = tr[g % 3][0], s = tr[g % 3][1];
        const double z = (g < 3 ? -1 : 1) * kInvSqrt3;
        const double L[3] = {1.0 - r - s, r, s};
        const double Lr[3] = {-1.0, 1.0, 0.0}, Ls[3] = {-1.0, 0.0, 1.0};
        const double Zf[2] = {0.5 * (1.0 - z), 0.5 * (1.0 + z)};
        const double Zd[2] = {-0.5, 0.5};
        t.w[g] = 1.0 / 6.0;
        for (int lvl = 0; lvl < 2; ++lvl)
            for (int i = 0; i < 3; ++i) {
                const int a = 3 * lvl + i;
                t.N[g][a] = L[i] * Zf[lvl];
                t.dN[g][a][0] = Lr[i] * Zf[lvl];
                t.dN[g][a][1] = Ls[i] * Zf[lvl];
                t.dN[g][a][2] = L[i] * Zd[lvl];
            }
    }
    return t;
}

template <> struct Ref<LESASM_PEN06> {
    static constexpr int nn = 6, ng = 6;
    static constexpr RefTable<6, 6> tab = make_pen06();
};

__host__ __device__ constexpr RefTable<5, 8> make_pyr05() {
    RefTable<5, 8> t{};
    const int sx[4] = {-1, 1, 1, -1};
    const int sy[4] = {-1, -1, 1, 1};
    for (int g = 0; g < 8; ++g) {
        const double A = (g & 1 ? 1 : -1) * kInvSqrt3;
        const double B = (g & 2 ? 1 : -1) * kInvSqrt3;
        const double c = kPyrC[g >> 2];
        t.w[g] = kPyrW[g >> 2];
        for (int a = 0; a < 4; ++a) {
            t.N[g][a] = 0.25 * (1.0 - c) * (1.0 + sx[a] * A) * (1.0 + sy[a] * B);
            t.dN[g][a][0] = 0.25 * sx[a] * (1.0 + sy[a] * B);
            t.dN[g][a][1] = 0.25 * sy[a] * (1.0 + sx[a] * A);
            t.dN[g][a][2] = 0.25 * (sx[a] * sy[a] * A * B - 1.0);
        }
        t.N[g][4] = c;
        t.dN[g][4][0] = 0.0;
        t.dN[g][4][1] = 0.0;
        t.dN[g][4][2] = 1.0;
    }
    return t;
}

template <> struct Ref<LESASM_PYR05> {
    static constexpr int nn = 5, ng = 8;
    static constexpr RefTable<5, 8> tab = make_pyr05();
};

// The same tables in constant memory, for kernels that loop over Gauss points
// instead of unrolling them (indexing with a uniform loop counter becomes
// scalar loads, keeping register pressure to one Gauss point at a time).
static __constant__ RefTable<8, 8> c_hex08 = make_hex08();
static __constant__ RefTable<4, 4> c_tet04 = make_tet04();
static __constant__ RefTable<6, 6> c_pen06 = make_pen06();
static __constant__ RefTable<5, 8> c_pyr05 = make_pyr05();

template <int T> struct RefConst;
template <> struct RefConst<LESASM_HEX08> { __device__ static const RefTable<8, 8> &tab() { return c_hex08; } };
template <> struct RefConst<LESASM_TET04> { __device__ static const RefTable<4, 4> &tab() { return c_tet04; } };
template <> struct RefConst<LESASM_PEN06> { __device__ static const RefTable<6, 6> &tab() { return c_pen06; } };
template <> struct RefConst<LESASM_PYR05> { __device__ static const RefTable<5, 8> &tab() { return c_pyr05; } };

}  // namespace lesasm
