// Device-side element computation: gather, geometry, interpolation, Vreman,
// residual contraction (Algorithm 1 "Element assembly"; Section 3.4.3
// gather / computation / scatter).
//
// One thread owns one element; its node data and residual live in registers.
// Loops over nodes are unrolled; the Gauss-point loop is not (tables come from
// constant memory through scalar loads), so only one point's temporaries are
// live at a time.  Node data enter as FP64 and are turned into modal
// coefficients (PYR05, PEN06, HEX08) or node-0-shifted values (TET04) before
// the contraction precision R is applied, so that in FP32 no absolute
// coordinate is ever subtracted.
#pragma once

#include "common.hpp"
#include "refelem.hpp"
#include "mlp.hpp"
#include "modal.hpp"

#ifndef LESASM_SPREAD_WAVES
#define LESASM_SPREAD_WAVES 1
#endif

namespace lesasm {

// Element data in registers.  PYR05, PEN06 and HEX08 hold the modal
// coefficients of coordinates, velocity and pressure (modal.hpp); the affine
// TET04 holds node values shifted by local node 0 (in FP64, before the
// contraction precision R is applied), since its closed form works on nodes.
template <int T, typename R> struct ElementData {
    static constexpr int nn = Ref<T>::nn, nm = Modal<T>::nm;
    int fid[nn];    // field node ids (scatter targets)
    R X[3][nm];     // coordinate coefficients (X[i][0], the mean, is unused)
    R U[3][nm];     // velocity coefficients
    R P[nm];        // pressure coefficients (P[0] unused)
};

template <typename R> struct ElementData<LESASM_TET04, R> {
    static constexpr int nn = 4;
    int fid[nn];
    R x[nn][3];     // coordinates relative to node 0
    R du[nn][3];    // velocity relative to node 0
    R dp[nn];       // pressure relative to node 0
    double u0[3];   // velocity at node 0
};

// Fill d from FP64 node values given by accessors xa(a, k), ua(a, k), pa(a).
template <int T, typename R, bool HAS_P, class XA, class UA, class PA>
__device__ __forceinline__ void load_element(ElementData<T, R> &d, XA xa, UA ua, PA pa) {
    constexpr int nn = Ref<T>::nn;
    if constexpr (T == LESASM_TET04) {
        double x0[3], p0 = HAS_P ? pa(0) : 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            x0[k] = xa(0, k);
            d.u0[k] = ua(0, k);
        }
#pragma unroll
        for (int a = 0; a < nn; ++a) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                d.x[a][k] = a ? (R)(xa(a, k) - x0[k]) : (R)0;
                d.du[a][k] = a ? (R)(ua(a, k) - d.u0[k]) : (R)0;
            }
            d.dp[a] = (HAS_P && a) ? (R)(pa(a) - p0) : (R)0;
        }
    } else {
        using M = Modal<T>;
        double v[nn], c[nn];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
#pragma unroll
            for (int a = 0; a < nn; ++a) v[a] = xa(a, k);
            M::to_modal(v, c);
#pragma unroll
            for (int m = 0; m < nn; ++m) d.X[k][m] = (R)c[m];
#pragma unroll
            for (int a = 0; a < nn; ++a) v[a] = ua(a, k);
            M::to_modal(v, c);
#pragma unroll
            for (int m = 0; m < nn; ++m) d.U[k][m] = (R)c[m];
        }
        if constexpr (HAS_P) {
#pragma unroll
            for (int a = 0; a < nn; ++a) v[a] = pa(a);
            M::to_modal(v, c);
#pragma unroll
            for (int m = 0; m < nn; ++m) d.P[m] = (R)c[m];
        } else {
#pragma unroll
            for (int m = 0; m < nn; ++m) d.P[m] = (R)0;
        }
    }
}

template <int T, typename R, bool HAS_P>
__device__ __forceinline__ void gather(ElementData<T, R> &d, const CatView &c, int e,
                                       const double *__restrict__ xyz, const double *__restrict__ u,
                                       const double *__restrict__ p) {
    constexpr int nn = Ref<T>::nn;
    int gid[nn];
#pragma unroll
    for (int a = 0; a < nn; ++a) {
        gid[a] = c.cg[(size_t)a * c.ld + e];
        d.fid[a] = (c.cf == c.cg) ? gid[a] : c.cf[(size_t)a * c.ld + e];
    }
    load_element<T, R, HAS_P>(
        d, [&](int a, int k) { return xyz[3 * (size_t)gid[a] + k]; },
        [&](int a, int k) { return u[3 * (size_t)d.fid[a] + k]; }, [&](int a) { return p[d.fid[a]]; });
}

// Element data from chunk-staged LDS arrays: node coordinates sx[k][3] by
// local geometry slot, velocity su[k][3] and pressure sp[k] by local field slot.
template <int T, typename R, bool HAS_P>
__device__ __forceinline__ void gather_lds(ElementData<T, R> &d, const int (&lg)[Ref<T>::nn],
                                           const int (&lf)[Ref<T>::nn], const double *sx, const double *su,
                                           const double *sp) {
    constexpr int nn = Ref<T>::nn;
#pragma unroll
    for (int a = 0; a < nn; ++a) d.fid[a] = lf[a];
    load_element<T, R, HAS_P>(
        d, [&](int a, int k) { return sx[3 * lg[a] + k]; }, [&](int a, int k) { return su[3 * lf[a] + k]; },
        [&](int a) { return sp[lf[a]]; });
}

// Reciprocal and reciprocal square root from the hardware estimates refined
// by two Newton steps (quadratic convergence: ~2^-26 -> ~2^-52 -> below FP64
// rounding), cheaper than the IEEE division and square-root sequences.
__device__ __forceinline__ double fast_rcp(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float fast_rcp(float d) { return __builtin_amdgcn_rcpf(d); }

__device__ __forceinline__ double fast_rsqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x, y * y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-x, y * y, 1.0);
    return fma(0.5 * y, e, y);
}
__device__ __forceinline__ float fast_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }

// Vreman: with alpha = G^T, beta = Delta^2 G G^T and alpha:alpha = tr(G G^T).
// nu_t = c Delta^2 sqrt(B'/A) with B' the sum of the principal 2x2 minors of
// G G^T (B_beta = Delta^4 B') and A its trace; 0 when A = 0; B' clamped at 0.
template <typename R>
__device__ __forceinline__ R vreman_nut(const R G[3][3], R cd2) {
    const R m00 = G[0][0] * G[0][0] + G[0][1] * G[0][1] + G[0][2] * G[0][2];
    const R m11 = G[1][0] * G[1][0] + G[1][1] * G[1][1] + G[1][2] * G[1][2];
    const R m22 = G[2][0] * G[2][0] + G[2][1] * G[2][1] + G[2][2] * G[2][2];
    const R m01 = G[0][0] * G[1][0] + G[0][1] * G[1][1] + G[0][2] * G[1][2];
    const R m02 = G[0][0] * G[2][0] + G[0][1] * G[2][1] + G[0][2] * G[2][2];
    const R m12 = G[1][0] * G[2][0] + G[1][1] * G[2][1] + G[1][2] * G[2][2];
    const R A = m00 + m11 + m22;
    const R B = m00 * m11 - m01 * m01 + m00 * m22 - m02 * m02 + m11 * m22 - m12 * m12;
    // zero when B <= 0 (clamp) or A = 0.  FP64: sqrt(B/A) = B / sqrt(A B) (no
    // overflow risk for |G|^6 in FP64); FP32: sqrt(B * (1/A)) keeps the range.
    if (!(A > (R)0 && B > (R)0)) return (R)0;
    if constexpr (sizeof(R) == 8)
        return cd2 * B * fast_rsqrt(A * B);
    else
        return cd2 * __builtin_amdgcn_sqrtf(B * fast_rcp(A));
}

// Learned-closure context of one wavefront (weights in LDS, private scratch).
struct MlpCtx {
    MlpLds w;
    unsigned char *scratch;
    float logd;  // log(Delta_e / Delta_ref)
};

// Passes of the network per round of 64 Gauss points (mlp_wave), chosen per
// kernel by measurement on the 20 M hybrid box.  FP32: two for TET04 and PYR05
// (162 -> 130 and 200 -> 166 registers, three wavefronts per SIMD), one for
// PEN06 and HEX08 (which stay at two wavefronts either way; one pass reads the
// weight tiles once).  FP64: together with a two-wavefront register budget on
// the kernel (which spills 68 bytes per lane for PEN06 and 260 for HEX08),
// two for TET04 and PEN06, four for PYR05 and HEX08: the FP64 closure assembly
// 4.08 against 4.63 ms with one pass (PEN06 and HEX08 then at one wavefront).
template <int T, typename R>
constexpr int mlp_passes() {
    if constexpr (sizeof(R) == 4) return (T == LESASM_TET04 || T == LESASM_PYR05) ? 2 : 1;
    else return (T == LESASM_TET04 || T == LESASM_PEN06) ? 2 : 4;
}

// Subgrid stress of the network minus Vreman's (-nu_t S, S = G + G^T), as the
// stress-flux tile T'_ik = w sum_j dtau_ij adj_kj of one Gauss point.
template <typename R, int PASSES>
__device__ __forceinline__ void mlp_stress_flux(const MlpCtx &mc, const R (&G)[3][3], const R (&S)[3][3], R nut,
                                                R d2, R adj[3][3], R w, R (&Tp)[3][3]) {
    float x[kMlpIn], y[kMlpOut];
    R gn2;
    mlp_features<R>(G, mc.logd, x, gn2);
    mlp_wave<PASSES>(mc.w, x, y, mc.scratch);
    const float tr = (y[0] + y[1] + y[2]) * (1.0f / 3.0f);
    const R sc = d2 * gn2;
    R dt[3][3];
    dt[0][0] = sc * (R)(y[0] - tr) + nut * S[0][0];
    dt[1][1] = sc * (R)(y[1] - tr) + nut * S[1][1];
    dt[2][2] = sc * (R)(y[2] - tr) + nut * S[2][2];
    dt[0][1] = dt[1][0] = sc * (R)y[3] + nut * S[0][1];
    dt[0][2] = dt[2][0] = sc * (R)y[4] + nut * S[0][2];
    dt[1][2] = dt[2][1] = sc * (R)y[5] + nut * S[1][2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) Tp[i][k] = w * (dt[i][0] * adj[k][0] + dt[i][1] * adj[k][1] + dt[i][2] * adj[k][2]);
}

// TET04 is affine: J, G, grad p and nu_t are constant over the element, and
// the 4-point rule integrates N_a N_b exactly (degree 2), so its quadrature
// sums collapse to closed forms of the same value:
//   sum_g w_g N_a(g) = 1/24,   sum_g w_g N_a(g) N_b(g) = (1 + delta_ab) / 120.
// With M = S + tr(G) I the EMAC term is C(u) = M u (linear in u), hence
//   R_a = -det [ M (u_a + sum_b u_b) / 120 + grad p / 24 ] - T dN_a,
//   T = (1/6) (nu + nu_t) S adj^T,  dN_0 = (-1,-1,-1), dN_a = e_(a-1).
template <typename R, bool HAS_P, bool MLP>
__device__ __forceinline__ void tet_residual(const ElementData<LESASM_TET04, R> &d, R nu, R cd2, R d2, R acc[4][3],
                                             R dacc[4][3], const MlpCtx *mc) {
    R J[3][3], Gx[3][3], px[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            J[i][k] = d.x[k + 1][i];
            Gx[i][k] = d.du[k + 1][i];
        }
#pragma unroll
    for (int k = 0; k < 3; ++k) px[k] = HAS_P ? d.dp[k + 1] : (R)0;
    R adj[3][3];
    adj[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    adj[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    adj[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    adj[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    adj[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    adj[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    adj[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    adj[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    adj[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const R det = J[0][0] * adj[0][0] + J[0][1] * adj[1][0] + J[0][2] * adj[2][0];
    const R rdet = fast_rcp(det);
    R G[3][3], q[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
            G[i][j] = (Gx[i][0] * adj[0][j] + Gx[i][1] * adj[1][j] + Gx[i][2] * adj[2][j]) * rdet;
        q[i] = HAS_P ? (px[0] * adj[0][i] + px[1] * adj[1][i] + px[2] * adj[2][i]) * rdet : (R)0;
    }
    const R nut = vreman_nut<R>(G, cd2);
    R S[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) S[i][j] = G[i][j] + G[j][i];
    const R divu = G[0][0] + G[1][1] + G[2][2];
    const R wvis = (R)(1.0 / 6.0) * (nu + nut);
    R Tm[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            Tm[i][k] = wvis * (S[i][0] * adj[k][0] + S[i][1] * adj[k][1] + S[i][2] * adj[k][2]);
    // sum_b u_b = 4 u0 + sum_b du_b
    R su[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) su[i] = (R)4 * (R)d.u0[i] + d.du[1][i] + d.du[2][i] + d.du[3][i];
    const R c120 = det * (R)(1.0 / 120.0), c24 = det * (R)(1.0 / 24.0);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        R v[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) v[i] = (R)d.u0[i] + d.du[a][i] + su[i];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const R Cm = S[i][0] * v[0] + S[i][1] * v[1] + S[i][2] * v[2] + divu * v[i];
            const R visc = a ? Tm[i][a - 1] : -(Tm[i][0] + Tm[i][1] + Tm[i][2]);
            acc[a][i] = -(c120 * Cm + c24 * q[i] + visc);
        }
    }
    if constexpr (MLP) {  // constant gradient: one network evaluation per element
        R Tp[3][3];
        mlp_stress_flux<R, mlp_passes<LESASM_TET04, R>()>(*mc, G, S, nut, d2, adj, (R)(1.0 / 6.0), Tp);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            dacc[0][i] = -(Tp[i][0] + Tp[i][1] + Tp[i][2]);
#pragma unroll
            for (int a = 1; a < 4; ++a) dacc[a][i] = Tp[i][a - 1];
        }
    }
}

// Per Gauss point, from J = dx/dxi, Gx = du/dxi, px = dp/dxi and u_g:
// adj = det J^-1, G = Gx adj / det, grad p likewise, nu_t, S = G + G^T,
// C = S u_g + tr(G) u_g, f = w det (C + grad p), T = w (nu + nu_t) S adj^T
// (= dV sigma J^-T, the flux paired with the reference gradients).
// UNSCALED (FP64 without the learned closure): G, S and grad p are kept
// multiplied by det, which cancels from f, and 1/det is applied once to
// nu_t (homogeneous of degree 1 in G) and to the viscous weight.  FP32 keeps
// the scaled form, whose magnitudes stay in range for any element size.
template <typename R, bool HAS_P> struct PointFlux {
    R f[3], T[3][3];
    R G[3][3], S[3][3], adj[3][3], nut;
};

template <typename R, bool HAS_P, bool UNSCALED>
__device__ __forceinline__ void point_flux(const R (&J)[3][3], const R (&Gx)[3][3], const R (&px)[3],
                                           const R (&ug)[3], R w, R nu, R cd2, PointFlux<R, HAS_P> &o) {
    R(&adj)[3][3] = o.adj;
    adj[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    adj[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    adj[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    adj[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    adj[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    adj[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    adj[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    adj[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    adj[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const R det = J[0][0] * adj[0][0] + J[0][1] * adj[1][0] + J[0][2] * adj[2][0];
    const R rdet = fast_rcp(det);
    const R sc = UNSCALED ? (R)1 : rdet;
    R q[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const R g = Gx[i][0] * adj[0][j] + Gx[i][1] * adj[1][j] + Gx[i][2] * adj[2][j];
            o.G[i][j] = UNSCALED ? g : g * sc;
        }
        const R qi = HAS_P ? px[0] * adj[0][i] + px[1] * adj[1][i] + px[2] * adj[2][i] : (R)0;
        q[i] = UNSCALED ? qi : qi * sc;
    }
    o.nut = UNSCALED ? vreman_nut<R>(o.G, cd2) * rdet : vreman_nut<R>(o.G, cd2);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) o.S[i][j] = o.G[i][j] + o.G[j][i];
    const R divu = o.G[0][0] + o.G[1][1] + o.G[2][2];
    const R wdet = UNSCALED ? w : w * det;
    const R wvis = UNSCALED ? w * (nu + o.nut) * rdet : w * (nu + o.nut);
    // viscous stress times the weight, symmetric: 6 products
    const R s00 = wvis * o.S[0][0], s11 = wvis * o.S[1][1], s22 = wvis * o.S[2][2];
    const R s01 = wvis * o.S[0][1], s02 = wvis * o.S[0][2], s12 = wvis * o.S[1][2];
    const R sw[3][3] = {{s00, s01, s02}, {s01, s11, s12}, {s02, s12, s22}};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const R C = o.S[i][0] * ug[0] + o.S[i][1] * ug[1] + o.S[i][2] * ug[2] + divu * ug[i];
        o.f[i] = wdet * (C + q[i]);
#pragma unroll
        for (int k = 0; k < 3; ++k) o.T[i][k] = sw[i][0] * adj[k][0] + sw[i][1] * adj[k][1] + sw[i][2] * adj[k][2];
    }
}

// Residual of one element into acc[a][i] (overwritten).  PYR05, PEN06 and
// HEX08 evaluate trial values and reference gradients from the modal
// coefficients and accumulate the test side as modal sums F[i][m], mapped
// to the nodes once per element (the weights carry the sign of the residual
// and the scale of the nodal map).
// With MLP, dacc receives the residual change from replacing Vreman's stress
// by the network's: dacc_a = int dN_a/dx_j (tau_mlp - tau_vreman)_ij dV.
template <int T, typename R, bool HAS_P, bool MLP = false>
__device__ __forceinline__ void element_residual(const ElementData<T, R> &d, R nu, R cd2,
                                                 R acc[Ref<T>::nn][3], R d2 = (R)0,
                                                 R (*dacc)[3] = nullptr, const MlpCtx *mc = nullptr) {
    if constexpr (T == LESASM_TET04) {
        tet_residual<R, HAS_P, MLP>(d, nu, cd2, d2, acc, dacc, mc);
        return;
    } else {
        using M = Modal<T>;
        constexpr int nn = Ref<T>::nn, nm = M::nm;
        const auto &pt = M::pts();
        R F[3][nm], dF[3][MLP ? nm : 1];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
#pragma unroll
            for (int m = 0; m < nm; ++m) F[i][m] = (R)0;
            if constexpr (MLP)
#pragma unroll
                for (int m = 0; m < nm; ++m) dF[i][m] = (R)0;
        }
        // point scalars loaded one point ahead, so that their scalar-cache
        // latency overlaps the previous point's arithmetic
        double qn[M::nq], wn = pt.w[0];
#pragma unroll
        for (int k = 0; k < M::nq; ++k) qn[k] = pt.q[0][k];
#pragma unroll 1
        for (int g = 0; g < M::ng; ++g) {
            double qc[M::nq];
#pragma unroll
            for (int k = 0; k < M::nq; ++k) qc[k] = qn[k];
            const double wc = wn;
            if (g + 1 < M::ng) {
#pragma unroll
                for (int k = 0; k < M::nq; ++k) qn[k] = pt.q[g + 1][k];
                wn = pt.w[g + 1];
            }
            const double *q = qc;
            R J[3][3], Gx[3][3], px[3] = {(R)0, (R)0, (R)0}, ug[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                M::grad(d.X[i], q, J[i]);
                M::grad(d.U[i], q, Gx[i]);
                ug[i] = M::value(d.U[i], q, Gx[i]);
            }
            if constexpr (HAS_P) M::grad(d.P, q, px);
            const R w = (R)wc;
            PointFlux<R, HAS_P> o;
            point_flux<R, HAS_P, sizeof(R) == 8 && !MLP>(J, Gx, px, ug, w, nu, cd2, o);
#pragma unroll
            for (int i = 0; i < 3; ++i) M::template test<true>(F[i], q, o.f[i], o.T[i]);
            if constexpr (MLP) {
                R Tp[3][3];
                mlp_stress_flux<R, mlp_passes<T, R>()>(*mc, o.G, o.S, o.nut, d2, o.adj, -w, Tp);
#pragma unroll
                for (int i = 0; i < 3; ++i) M::template test<false>(dF[i], q, (R)0, Tp[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            R r[nn];
            M::to_nodal(F[i], r);
#pragma unroll
            for (int a = 0; a < nn; ++a) acc[a][i] = r[a];
            if constexpr (MLP) {
                M::to_nodal(dF[i], r);
#pragma unroll
                for (int a = 0; a < nn; ++a) dacc[a][i] = r[a];
            }
        }
    }
}

// One chunk of consecutive elements, processed by one workgroup.  The
// chunk's distinct nodes are loaded once into LDS (coordinates, velocity,
// pressure), every element reads them from there, and element residuals are
// summed into per-node LDS accumulators.  Afterwards each node is written once:
// a plain store when every element touching it lies in this chunk (owned), an
// staged row (STAGED) or FP64 device atomic otherwise.  LDS layout (doubles):
//   x[ng][3] | u[nf][3] | p[nf] | acc[nf][3].
// Learned closure of a launch: packed weights, filter-width reference and
// the fallback threshold (squared), plus the counters of Vreman fallbacks.
// Vreman-fallback counts: workgroup b adds to counter b % kFallbackSlots
// (spread over many addresses: one shared counter made every chunk's closing
// atomic wait on the others)
constexpr int kFallbackSlots = 4096;
struct ClosureView {
    const short *packed;
    const float *bias;
    double log_delta_ref;
    double tol2;
    unsigned long long *fallbacks;
};

template <int T, typename R, bool HAS_P, bool PERIODIC, bool STAGED, bool MLP = false>
__device__ __forceinline__ void chunk_body(const ChunkView &c, int j, double *lds, const double *__restrict__ xyz,
                                           const double *__restrict__ u, const double *__restrict__ p, double nu,
                                           double cv, double *__restrict__ rhs, const ClosureView *cl = nullptr,
                                           int lds_node_doubles = 0) {
    constexpr int nn = Ref<T>::nn;
    const int e0 = c.eoff[j], e1 = c.eoff[j + 1];
    const int g0 = c.goff[j], ng = c.goff[j + 1] - g0;
    const int f0 = PERIODIC ? c.foff[j] : g0;
    const int nf = PERIODIC ? c.foff[j + 1] - f0 : ng;
    double *sx = lds, *su = sx + 3 * ng, *sp = su + 3 * nf, *sacc = sp + nf;

    for (int k = threadIdx.x; k < ng; k += blockDim.x) {
        const size_t g = (size_t)c.gnodes[g0 + k];
        sx[3 * k + 0] = xyz[3 * g + 0];
        sx[3 * k + 1] = xyz[3 * g + 1];
        sx[3 * k + 2] = xyz[3 * g + 2];
    }
    for (int k = threadIdx.x; k < nf; k += blockDim.x) {
        const size_t f = (size_t)((uint32_t)c.fnodes[f0 + k] & ~kOwnedBit);
        su[3 * k + 0] = u[3 * f + 0];
        su[3 * k + 1] = u[3 * f + 1];
        su[3 * k + 2] = u[3 * f + 2];
        sp[k] = HAS_P ? p[f] : 0.0;
        sacc[3 * k + 0] = sacc[3 * k + 1] = sacc[3 * k + 2] = 0.0;
    }
    if constexpr (MLP) mlp_stage(cl->packed, cl->bias, (unsigned char *)(lds + lds_node_doubles));
    __syncthreads();

    if constexpr (!MLP) {
        for (int base = e0; base < e1; base += blockDim.x) {
#if LESASM_SPREAD_WAVES
            // In a full block, wavefront w takes every (blockDim/64)-th element
            // starting at w: neighbouring elements (which share nodes) go to
            // different wavefronts, so fewer lanes of one LDS atomic hit the
            // same node.
            const int e = base + (int)blockDim.x <= e1
                              ? base + (int)(threadIdx.x & 63) * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6)
                              : base + (int)threadIdx.x;
#else
            const int e = base + (int)threadIdx.x;
#endif
            if (e >= e1) break;
            int lg[nn], lf[nn];
#pragma unroll
            for (int a = 0; a < nn; ++a) {
                lg[a] = c.lg[(size_t)a * c.ld + e];
                lf[a] = PERIODIC ? (int)c.lf[(size_t)a * c.ld + e] : lg[a];
            }
            ElementData<T, R> d;
            gather_lds<T, R, HAS_P>(d, lg, lf, sx, su, sp);
            const double dl = c.delta[e];
            R acc[nn][3];
            element_residual<T, R, HAS_P>(d, (R)nu, (R)(cv * dl * dl), acc);
#pragma unroll
            for (int a = 0; a < nn; ++a)
#pragma unroll
                for (int i = 0; i < 3; ++i) unsafeAtomicAdd(sacc + 3 * lf[a] + i, (double)acc[a][i]);
        }
    } else {
        // Learned closure: whole wavefronts step through the elements together
        // (the network runs on matrix instructions across all 64 lanes); lanes
        // past the end repeat the last element and discard it.
        unsigned char *mlds = (unsigned char *)(lds + lds_node_doubles);
        MlpCtx mc;
        mc.w = mlp_lds_view(mlds);
        mc.scratch = mlds + kMlpLdsBytes + (threadIdx.x / 64) * kMlpWaveScratch;
        unsigned fallbacks = 0;
        const int wave0 = (threadIdx.x / 64) * 64;
        for (int base = e0; base < e1; base += blockDim.x) {
            if (base + wave0 >= e1) break;  // whole wavefront past the end (uniform)
            const bool active = base + (int)threadIdx.x < e1;
            const int e = active ? base + (int)threadIdx.x : e1 - 1;
            int lg[nn], lf[nn];
#pragma unroll
            for (int a = 0; a < nn; ++a) {
                lg[a] = c.lg[(size_t)a * c.ld + e];
                lf[a] = PERIODIC ? (int)c.lf[(size_t)a * c.ld + e] : lg[a];
            }
            ElementData<T, R> d;
            gather_lds<T, R, HAS_P>(d, lg, lf, sx, su, sp);
            const double dl = c.delta[e];
            mc.logd = (float)(log(dl) - cl->log_delta_ref);
            R acc[nn][3], dacc[nn][3];
            element_residual<T, R, HAS_P, true>(d, (R)nu, (R)(cv * dl * dl), acc, (R)(dl * dl), dacc, &mc);
            // fallback test: |R_mlp - R_vreman| <= tol |R_vreman| (element 2-norms)
            R nd = (R)0, na = (R)0;
#pragma unroll
            for (int a = 0; a < nn; ++a)
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    nd += dacc[a][i] * dacc[a][i];
                    na += acc[a][i] * acc[a][i];
                }
            const bool use_mlp = (double)nd <= cl->tol2 * (double)na;
            if (active) {
                fallbacks += !use_mlp;
#pragma unroll
                for (int a = 0; a < nn; ++a)
#pragma unroll
                    for (int i = 0; i < 3; ++i)
                        unsafeAtomicAdd(sacc + 3 * lf[a] + i, (double)(use_mlp ? acc[a][i] + dacc[a][i] : acc[a][i]));
            }
        }
        if (fallbacks) atomicAdd(cl->fallbacks + (blockIdx.x & (kFallbackSlots - 1)), (unsigned long long)fallbacks);
    }
    __syncthreads();

    for (int k = threadIdx.x; k < nf; k += blockDim.x) {
        const uint32_t tag = (uint32_t)c.fnodes[f0 + k];
        double *dst = rhs + 3 * (size_t)(tag & ~kOwnedBit);
        if (tag & kOwnedBit) {
            dst[0] = sacc[3 * k + 0];
            dst[1] = sacc[3 * k + 1];
            dst[2] = sacc[3 * k + 2];
        } else if (STAGED) {
            double *row = c.stage + 3 * (size_t)c.fslot[f0 + k];
            row[0] = sacc[3 * k + 0];
            row[1] = sacc[3 * k + 1];
            row[2] = sacc[3 * k + 2];
        } else {
            unsafeAtomicAdd(dst + 0, sacc[3 * k + 0]);
            unsafeAtomicAdd(dst + 1, sacc[3 * k + 1]);
            unsafeAtomicAdd(dst + 2, sacc[3 * k + 2]);
        }
    }
}

}  // namespace lesasm
