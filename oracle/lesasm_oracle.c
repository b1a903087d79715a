/*
 * Plain FP64 CPU oracle for the explicit LES momentum-residual assembly.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library; it is the definition of what
 * the GPU path must compute, written out as plainly as possible:
 * straightforward loops over elements, Gauss points and nodes in that order,
 * no blocking, fusion or reordering.
 *
 * What is computed (Borrell et al., FGCS 2020):
 *   * Section 3.2, equation (momentum): filtered incompressible Navier-Stokes
 *     with rho = 1 and kinematic viscosity nu.  The convective bracket is used
 *     in its EMAC form, C(u) = 2 eps(u) u + (div u) u, with the -|u|^2/2
 *     gradient absorbed into the modified pressure p; the viscous term
 *     div[2 nu eps(u)] and the subgrid term div(tau), tau = -2 nu_t eps(u),
 *     are integrated by parts with the natural boundary terms dropped.
 *   * Section 3.2: Vreman's eddy viscosity for nu_t (model only cited by the
 *     paper; the published formula is written out in oracle_vreman below).
 *   * Section 3.2: Galerkin finite elements on linear hybrid meshes
 *     (Section 3.3: tetrahedra, prisms, pyramids; hexahedra as well).
 *   * Section 3.4.3 (element assembly: gather, compute, scatter) and the
 *     mass-matrix listing there, whose row sums give the lumped mass.
 *
 * Residual of local node a, component i, of element e (sum over j):
 *   R_ai = - sum_g dV_g [ N_a (C_i + dp/dx_i) + dN_a/dx_j * 2 (nu + nu_t) eps_ij ]
 * scattered as rhs[field(a)] += R_a, so that M_L du/dt = rhs.
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   quadrature per type (TET 4-pt degree 2, PEN 3x2, PYR 8-pt collapsed
 *   conical product, HEX 2x2x2 Gauss), rational pyramid basis, filter width
 *   Delta_e = (element volume)^(1/3), nu_t = 0 where alpha:alpha = 0 and
 *   B_beta clamped at 0.
 *
 * Pins: every function here is checked by tests against closed forms,
 * invariants, exact rational integration or brute force (see tests/).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_NODE 8
#define ORACLE_MAX_GAUSS 8

/* term selection for oracle_assemble / oracle_element_residual */
#define TERM_CONV 1      /* EMAC convection                              */
#define TERM_PRES 2      /* pressure gradient                            */
#define TERM_VISC 4      /* molecular viscosity, 2 nu eps(u)             */
#define TERM_SGS 8       /* Vreman eddy viscosity, 2 nu_t eps(u)         */
#define TERM_LITERAL 16  /* convective form read literally (subtract grad |u|^2/2) */
#define TERM_ALL (TERM_CONV | TERM_PRES | TERM_VISC | TERM_SGS)

static long long g_bad_element = -1;

long long oracle_bad_element(void) { return g_bad_element; }

/* ------------------------------------------------------------------------ */
/* Reference elements                                                       */
/* ------------------------------------------------------------------------ */

int oracle_nnode(int type)
{
    switch (type) {
    case 4: return 4;
    case 5: return 5;
    case 6: return 6;
    case 8: return 8;
    default: return -1;
    }
}

int oracle_ngauss(int type)
{
    switch (type) {
    case 4: return 4;
    case 5: return 8;
    case 6: return 6;
    case 8: return 8;
    default: return -1;
    }
}

/* Shape functions N[a] and reference derivatives dN[a*3 + k] = dN_a/dxi_k at
 * xi = (xi, eta, zeta).  Standard linear isoparametric bases:
 *   TET04: N = (1-r-s-t, r, s, t) on the unit simplex.
 *   PYR05: base (-1,-1),(1,-1),(1,1),(-1,1) at zeta = 0, apex (0,0,1);
 *          N_a = (1-zeta+xi_a xi)(1-zeta+eta_a eta) / (4 (1-zeta)), N_5 = zeta
 *          (rational basis; at the apex itself the base functions are 0 and
 *          the derivatives are left as 0).
 *   PEN06: triangle (1-r-s, r, s) times line ((1-zeta)/2, (1+zeta)/2).
 *   HEX08: N_a = (1 + xi_a xi)(1 + eta_a eta)(1 + zeta_a zeta) / 8.        */
int oracle_shape(int type, const double *xi, double *N, double *dN)
{
    const double r = xi[0], s = xi[1], t = xi[2];
    if (type == 4) {
        N[0] = 1.0 - r - s - t; N[1] = r; N[2] = s; N[3] = t;
        const double d[12] = {-1, -1, -1, 1, 0, 0, 0, 1, 0, 0, 0, 1};
        memcpy(dN, d, sizeof d);
        return 0;
    }
    if (type == 5) {
        static const double sa[4] = {-1, 1, 1, -1};
        static const double ta[4] = {-1, -1, 1, 1};
        const double q = 1.0 - t;
        if (q <= 0.0) {
            for (int a = 0; a < 4; ++a) { N[a] = 0.0; dN[3 * a] = dN[3 * a + 1] = dN[3 * a + 2] = 0.0; }
        } else {
            for (int a = 0; a < 4; ++a) {
                const double A = q + sa[a] * r, B = q + ta[a] * s;
                N[a] = A * B / (4.0 * q);
                dN[3 * a + 0] = sa[a] * B / (4.0 * q);
                dN[3 * a + 1] = ta[a] * A / (4.0 * q);
                /* d/dzeta of A B / (4 q) with dq/dzeta = -1 */
                dN[3 * a + 2] = (-(A + B) * q + A * B) / (4.0 * q * q);
            }
        }
        N[4] = t;
        dN[12] = 0.0; dN[13] = 0.0; dN[14] = 1.0;
        return 0;
    }
    if (type == 6) {
        const double L[3] = {1.0 - r - s, r, s};
        const double dLr[3] = {-1, 1, 0}, dLs[3] = {-1, 0, 1};
        const double Z[2] = {0.5 * (1.0 - t), 0.5 * (1.0 + t)};
        const double dZ[2] = {-0.5, 0.5};
        for (int j = 0; j < 2; ++j)
            for (int i = 0; i < 3; ++i) {
                const int a = i + 3 * j;
                N[a] = L[i] * Z[j];
                dN[3 * a + 0] = dLr[i] * Z[j];
                dN[3 * a + 1] = dLs[i] * Z[j];
                dN[3 * a + 2] = L[i] * dZ[j];
            }
        return 0;
    }
    if (type == 8) {
        static const double xa[8] = {-1, 1, 1, -1, -1, 1, 1, -1};
        static const double ya[8] = {-1, -1, 1, 1, -1, -1, 1, 1};
        static const double za[8] = {-1, -1, -1, -1, 1, 1, 1, 1};
        for (int a = 0; a < 8; ++a) {
            const double fx = 1.0 + xa[a] * r, fy = 1.0 + ya[a] * s, fz = 1.0 + za[a] * t;
            N[a] = 0.125 * fx * fy * fz;
            dN[3 * a + 0] = 0.125 * xa[a] * fy * fz;
            dN[3 * a + 1] = 0.125 * ya[a] * fx * fz;
            dN[3 * a + 2] = 0.125 * za[a] * fx * fy;
        }
        return 0;
    }
    return -1;
}

/* Gauss rules: points pts[g*3 + k] and weights w[g].
 *   TET04: 4 points, barycentric permutations of (a, b, b, b),
 *          a = (5 + 3 sqrt5)/20, b = (5 - sqrt5)/20, w = 1/24 (degree 2).
 *   PYR05: conical product: xi = A (1-c), eta = B (1-c), zeta = c with
 *          A, B in +-1/sqrt3 (Gauss-Legendre) and c the 2-point Gauss-Jacobi
 *          rule for the weight (1-c)^2 on [0, 1]:
 *          c = 1/3 -+ sqrt10/15, W = 1/6 +- sqrt10/48.
 *   PEN06: triangle points (1/6,1/6), (2/3,1/6), (1/6,2/3) (weight 1/6 each)
 *          times zeta = -+1/sqrt3 (weight 1).
 *   HEX08: 2x2x2 Gauss-Legendre, +-1/sqrt3, weight 1.                       */
int oracle_gauss(int type, double *pts, double *w)
{
    const double g = 1.0 / sqrt(3.0);
    if (type == 4) {
        const double a = (5.0 + 3.0 * sqrt(5.0)) / 20.0, b = (5.0 - sqrt(5.0)) / 20.0;
        const double p[12] = {b, b, b, a, b, b, b, a, b, b, b, a};
        memcpy(pts, p, sizeof p);
        for (int q = 0; q < 4; ++q) w[q] = 1.0 / 24.0;
        return 4;
    }
    if (type == 5) {
        const double c[2] = {1.0 / 3.0 - sqrt(10.0) / 15.0, 1.0 / 3.0 + sqrt(10.0) / 15.0};
        const double W[2] = {1.0 / 6.0 + sqrt(10.0) / 48.0, 1.0 / 6.0 - sqrt(10.0) / 48.0};
        const double ab[2] = {-g, g};
        int q = 0;
        for (int k = 0; k < 2; ++k)
            for (int j = 0; j < 2; ++j)
                for (int i = 0; i < 2; ++i, ++q) {
                    pts[3 * q + 0] = ab[i] * (1.0 - c[k]);
                    pts[3 * q + 1] = ab[j] * (1.0 - c[k]);
                    pts[3 * q + 2] = c[k];
                    w[q] = W[k];
                }
        return 8;
    }
    if (type == 6) {
        const double tr[3][2] = {{1.0 / 6.0, 1.0 / 6.0}, {2.0 / 3.0, 1.0 / 6.0}, {1.0 / 6.0, 2.0 / 3.0}};
        const double zl[2] = {-g, g};
        int q = 0;
        for (int k = 0; k < 2; ++k)
            for (int i = 0; i < 3; ++i, ++q) {
                pts[3 * q + 0] = tr[i][0];
                pts[3 * q + 1] = tr[i][1];
                pts[3 * q + 2] = zl[k];
                w[q] = 1.0 / 6.0;
            }
        return 6;
    }
    if (type == 8) {
        const double l[2] = {-g, g};
        int q = 0;
        for (int k = 0; k < 2; ++k)
            for (int j = 0; j < 2; ++j)
                for (int i = 0; i < 2; ++i, ++q) {
                    pts[3 * q + 0] = l[i];
                    pts[3 * q + 1] = l[j];
                    pts[3 * q + 2] = l[k];
                    w[q] = 1.0;
                }
        return 8;
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Vreman eddy viscosity                                                    */
/* ------------------------------------------------------------------------ */

/* G[i*3 + j] = du_i/dx_j.  Vreman (2004): alpha_ij = du_j/dx_i,
 * beta_ij = Delta^2 alpha_mi alpha_mj,
 * B = b11 b22 - b12^2 + b11 b33 - b13^2 + b22 b33 - b23^2,
 * nu_t = c sqrt(B / (alpha_ij alpha_ij)), and 0 when alpha_ij alpha_ij = 0.
 * Rounding can push B slightly below 0, so it is clamped at 0.               */
double oracle_vreman(const double *G, double delta, double c)
{
    double alpha[3][3], beta[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            alpha[i][j] = G[j * 3 + i];
    double aa = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            aa += alpha[i][j] * alpha[i][j];
    if (aa == 0.0) return 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int m = 0; m < 3; ++m) s += alpha[m][i] * alpha[m][j];
            beta[i][j] = delta * delta * s;
        }
    double B = beta[0][0] * beta[1][1] - beta[0][1] * beta[0][1]
             + beta[0][0] * beta[2][2] - beta[0][2] * beta[0][2]
             + beta[1][1] * beta[2][2] - beta[1][2] * beta[1][2];
    if (B < 0.0) B = 0.0;
    return c * sqrt(B / aa);
}

/* ------------------------------------------------------------------------ */
/* One element                                                              */
/* ------------------------------------------------------------------------ */

static double det3(const double J[3][3])
{
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
         - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
         + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

static void inv3(const double J[3][3], double det, double K[3][3])
{
    K[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    K[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    K[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    K[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    K[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    K[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    K[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    K[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    K[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
}

/* Jacobian J_ij = sum_a x_ai dN_a/dxi_j at one point. */
static void jacobian(int n, const double *x, const double *dN, double J[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int a = 0; a < n; ++a) s += x[3 * a + i] * dN[3 * a + j];
            J[i][j] = s;
        }
}

/* Element volume sum_g w_g det J_g; returns -1 on a bad type and -2 when
 * det J <= 0 at some Gauss point. */
int oracle_element_volume(int type, const double *x, double *vol)
{
    double pts[3 * ORACLE_MAX_GAUSS], w[ORACLE_MAX_GAUSS], N[ORACLE_MAX_NODE], dN[3 * ORACLE_MAX_NODE];
    const int n = oracle_nnode(type);
    const int ng = oracle_gauss(type, pts, w);
    if (n < 0 || ng < 0) return -1;
    double v = 0.0;
    for (int q = 0; q < ng; ++q) {
        double J[3][3];
        oracle_shape(type, pts + 3 * q, N, dN);
        jacobian(n, x, dN, J);
        const double d = det3(J);
        if (!(d > 0.0)) return -2;
        v += w[q] * d;
    }
    *vol = v;
    return 0;
}

/* Residual R[a*3 + i] of one element from its node coordinates x[a*3+k],
 * velocities u[a*3+i] and pressures p[a] (p may be NULL).  If gp is not
 * NULL it receives, per Gauss point, 18 doubles:
 *   detJ, w, u_0..2, G_00..G_22 (row-major, G_ij = du_i/dx_j), dp/dx_0..2, nu_t.
 * delta_out (may be NULL) receives Delta_e.                                 */
int oracle_element_residual(int type, const double *x, const double *u, const double *p,
                            double nu, double c, int terms, double *R, double *gp, double *delta_out)
{
    double pts[3 * ORACLE_MAX_GAUSS], w[ORACLE_MAX_GAUSS];
    double N[ORACLE_MAX_NODE], dN[3 * ORACLE_MAX_NODE], dNdx[3 * ORACLE_MAX_NODE];
    const int n = oracle_nnode(type);
    const int ng = oracle_gauss(type, pts, w);
    if (n < 0 || ng < 0) return -1;

    double vol;
    const int st = oracle_element_volume(type, x, &vol);
    if (st) return st;
    const double delta = cbrt(vol);
    if (delta_out) *delta_out = delta;

    for (int k = 0; k < 3 * n; ++k) R[k] = 0.0;

    for (int q = 0; q < ng; ++q) {
        double J[3][3], K[3][3];
        oracle_shape(type, pts + 3 * q, N, dN);
        jacobian(n, x, dN, J);
        const double det = det3(J);
        inv3(J, det, K);
        const double dV = w[q] * det;

        /* dN_a/dx_i = sum_j (J^-1)_ji dN_a/dxi_j */
        for (int a = 0; a < n; ++a)
            for (int i = 0; i < 3; ++i) {
                double s = 0.0;
                for (int j = 0; j < 3; ++j) s += K[j][i] * dN[3 * a + j];
                dNdx[3 * a + i] = s;
            }

        double ug[3] = {0, 0, 0}, G[3][3] = {{0}}, dp[3] = {0, 0, 0};
        for (int a = 0; a < n; ++a)
            for (int i = 0; i < 3; ++i) {
                ug[i] += N[a] * u[3 * a + i];
                for (int j = 0; j < 3; ++j) G[i][j] += u[3 * a + i] * dNdx[3 * a + j];
                if (p) dp[i] += p[a] * dNdx[3 * a + i];
            }

        const double nut = oracle_vreman(&G[0][0], delta, c);

        /* EMAC convection C_i = (G_ij + G_ji) u_j + G_jj u_i */
        double C[3], S[3][3];
        const double divu = G[0][0] + G[1][1] + G[2][2];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) S[i][j] = G[i][j] + G[j][i];
        for (int i = 0; i < 3; ++i) {
            double s = 0.0;
            for (int j = 0; j < 3; ++j) s += S[i][j] * ug[j];
            C[i] = s + divu * ug[i];
            if (terms & TERM_LITERAL) {
                /* minus grad(|u|^2/2): (grad |u|^2/2)_i = sum_j u_j G_ji */
                double gk = 0.0;
                for (int j = 0; j < 3; ++j) gk += ug[j] * G[j][i];
                C[i] -= gk;
            }
        }

        double visc = 0.0;
        if (terms & TERM_VISC) visc += nu;
        if (terms & TERM_SGS) visc += nut;

        for (int a = 0; a < n; ++a)
            for (int i = 0; i < 3; ++i) {
                double f = 0.0;
                if (terms & TERM_CONV) f += C[i];
                if (terms & TERM_PRES) f += dp[i];
                double s = 0.0;
                for (int j = 0; j < 3; ++j) s += dNdx[3 * a + j] * visc * S[i][j];
                R[3 * a + i] -= dV * (N[a] * f + s);
            }

        if (gp) {
            double *o = gp + 18 * q;
            o[0] = det; o[1] = w[q];
            for (int i = 0; i < 3; ++i) o[2 + i] = ug[i];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) o[5 + 3 * i + j] = G[i][j];
            for (int i = 0; i < 3; ++i) o[14 + i] = dp[i];
            o[17] = nut;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Whole mesh                                                               */
/* ------------------------------------------------------------------------ */

/* Gathers element e; returns the number of nodes or a negative error. */
static int gather(long long e, int64_t n_nodes, const double *coords, const uint8_t *types,
                  const int64_t *offs, const int32_t *conn, const int32_t *field_node, int64_t n_field,
                  const double *u, const double *p, double *x, double *ue, double *pe, int64_t *fid)
{
    const int type = types[e];
    const int n = oracle_nnode(type);
    if (n < 0 || offs[e + 1] - offs[e] != n) return -1;
    for (int a = 0; a < n; ++a) {
        const int64_t g = conn[offs[e] + a];
        if (g < 0 || g >= n_nodes) return -1;
        const int64_t f = field_node ? (int64_t)field_node[g] : g;
        if (f < 0 || f >= n_field) return -1;
        fid[a] = f;
        for (int k = 0; k < 3; ++k) x[3 * a + k] = coords[3 * g + k];
        if (u)
            for (int k = 0; k < 3; ++k) ue[3 * a + k] = u[3 * f + k];
        if (pe) pe[a] = p ? p[f] : 0.0;
    }
    return n;
}

/* rhs[n_field][3] is overwritten.  u[n_field][3]; p[n_field] or NULL.       */
int oracle_assemble(int64_t n_nodes, const double *coords, int64_t n_elems, const uint8_t *types,
                    const int64_t *offs, const int32_t *conn, const int32_t *field_node, int64_t n_field,
                    const double *u, const double *p, double nu, double c, int terms, double *rhs)
{
    double x[3 * ORACLE_MAX_NODE], ue[3 * ORACLE_MAX_NODE], pe[ORACLE_MAX_NODE], R[3 * ORACLE_MAX_NODE];
    int64_t fid[ORACLE_MAX_NODE];
    g_bad_element = -1;
    for (int64_t k = 0; k < 3 * n_field; ++k) rhs[k] = 0.0;
    for (int64_t e = 0; e < n_elems; ++e) {
        const int n = gather(e, n_nodes, coords, types, offs, conn, field_node, n_field, u, p, x, ue, pe, fid);
        if (n < 0) { g_bad_element = e; return -1; }
        const int st = oracle_element_residual(types[e], x, ue, p ? pe : NULL, nu, c, terms, R, NULL, NULL);
        if (st) { g_bad_element = e; return st; }
        for (int a = 0; a < n; ++a)
            for (int i = 0; i < 3; ++i) rhs[3 * fid[a] + i] += R[3 * a + i];
    }
    return 0;
}

/* Timing leg of the benchmark's CPU baseline: the same element loop as
 * oracle_assemble, the elements split into nthreads contiguous ranges run by
 * OpenMP threads, each thread summing into a private right-hand side; the
 * private arrays are then added node by node in thread order (deterministic).
 * The result equals oracle_assemble's up to the order of the nodal sums.
 * Needs 3 * n_field * nthreads doubles of host memory; returns -3 if they
 * cannot be allocated. */
int oracle_assemble_threads(int64_t n_nodes, const double *coords, int64_t n_elems, const uint8_t *types,
                            const int64_t *offs, const int32_t *conn, const int32_t *field_node, int64_t n_field,
                            const double *u, const double *p, double nu, double c, int terms, int nthreads,
                            double *rhs)
{
    if (nthreads < 1) nthreads = 1;
    const int64_t len = 3 * n_field;
    double *priv = (double *)calloc((size_t)nthreads * (size_t)(len > 0 ? len : 1), sizeof(double));
    if (!priv) return -3;
    int status = 0;
    long long bad = -1;
    g_bad_element = -1;
#pragma omp parallel num_threads(nthreads)
    {
        const int t = omp_get_thread_num(), nt = omp_get_num_threads();
        const int64_t e0 = n_elems * t / nt, e1 = n_elems * (t + 1) / nt;
        double *mine = priv + (size_t)t * (size_t)len;
        double x[3 * ORACLE_MAX_NODE], ue[3 * ORACLE_MAX_NODE], pe[ORACLE_MAX_NODE], R[3 * ORACLE_MAX_NODE];
        int64_t fid[ORACLE_MAX_NODE];
        for (int64_t e = e0; e < e1; ++e) {
            const int n = gather(e, n_nodes, coords, types, offs, conn, field_node, n_field, u, p, x, ue, pe, fid);
            const int st = n < 0 ? -1 : oracle_element_residual(types[e], x, ue, p ? pe : NULL, nu, c, terms, R,
                                                                 NULL, NULL);
            if (st) {
#pragma omp critical
                if (bad < 0 || e < bad) { bad = e; status = st; }
                break;
            }
            for (int a = 0; a < n; ++a)
                for (int i = 0; i < 3; ++i) mine[3 * fid[a] + i] += R[3 * a + i];
        }
#pragma omp barrier
#pragma omp for schedule(static)
        for (int64_t k = 0; k < len; ++k) {
            double s = 0.0;
            for (int q = 0; q < nt; ++q) s += priv[(size_t)q * (size_t)len + k];
            rhs[k] = s;
        }
    }
    free(priv);
    if (status) { g_bad_element = bad; return status; }
    return 0;
}

/* Threads oracle_assemble_threads would use with nthreads = 0 (the OpenMP default). */
int oracle_max_threads(void) { return omp_get_max_threads(); }

/* Row-sum lumped mass M[f] = sum_e sum_g w_g det J_g N_a(xi_g), M[n_field]. */
int oracle_lumped_mass(int64_t n_nodes, const double *coords, int64_t n_elems, const uint8_t *types,
                       const int64_t *offs, const int32_t *conn, const int32_t *field_node, int64_t n_field,
                       double *M)
{
    double x[3 * ORACLE_MAX_NODE], pts[3 * ORACLE_MAX_GAUSS], w[ORACLE_MAX_GAUSS];
    double N[ORACLE_MAX_NODE], dN[3 * ORACLE_MAX_NODE];
    int64_t fid[ORACLE_MAX_NODE];
    g_bad_element = -1;
    for (int64_t k = 0; k < n_field; ++k) M[k] = 0.0;
    for (int64_t e = 0; e < n_elems; ++e) {
        const int n = gather(e, n_nodes, coords, types, offs, conn, field_node, n_field, NULL, NULL, x, NULL, NULL, fid);
        if (n < 0) { g_bad_element = e; return -1; }
        const int ng = oracle_gauss(types[e], pts, w);
        for (int q = 0; q < ng; ++q) {
            double J[3][3];
            oracle_shape(types[e], pts + 3 * q, N, dN);
            jacobian(n, x, dN, J);
            const double d = det3(J);
            if (!(d > 0.0)) { g_bad_element = e; return -2; }
            for (int a = 0; a < n; ++a) M[fid[a]] += w[q] * d * N[a];
        }
    }
    return 0;
}

/* Filter width Delta_e = (sum_g w_g det J_g)^(1/3) per element. */
int oracle_filter_width(int64_t n_nodes, const double *coords, int64_t n_elems, const uint8_t *types,
                        const int64_t *offs, const int32_t *conn, double *delta)
{
    double x[3 * ORACLE_MAX_NODE];
    int64_t fid[ORACLE_MAX_NODE];
    g_bad_element = -1;
    for (int64_t e = 0; e < n_elems; ++e) {
        const int n = gather(e, n_nodes, coords, types, offs, conn, NULL, n_nodes, NULL, NULL, x, NULL, NULL, fid);
        if (n < 0) { g_bad_element = e; return -1; }
        double v;
        const int st = oracle_element_volume(types[e], x, &v);
        if (st) { g_bad_element = e; return st; }
        delta[e] = cbrt(v);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Pressure step operators (Algorithm 1: Laplacian assembled once before the */
/* time loop; projection step of the fractional-step scheme, Section 3.2)   */
/* ------------------------------------------------------------------------ */

/* Element Laplacian K[a*n + b] = sum_g w_g det J_g dN_a/dx . dN_b/dx. */
int oracle_element_laplacian(int type, const double *x, double *K)
{
    double pts[3 * ORACLE_MAX_GAUSS], w[ORACLE_MAX_GAUSS];
    double N[ORACLE_MAX_NODE], dN[3 * ORACLE_MAX_NODE], dNdx[3 * ORACLE_MAX_NODE];
    const int n = oracle_nnode(type);
    const int ng = oracle_gauss(type, pts, w);
    if (n < 0 || ng < 0) return -1;
    for (int k = 0; k < n * n; ++k) K[k] = 0.0;
    for (int q = 0; q < ng; ++q) {
        double J[3][3], Ki[3][3];
        oracle_shape(type, pts + 3 * q, N, dN);
        jacobian(n, x, dN, J);
        const double det = det3(J);
        if (!(det > 0.0)) return -2;
        inv3(J, det, Ki);
        for (int a = 0; a < n; ++a)
            for (int i = 0; i < 3; ++i) {
                double s = 0.0;
                for (int j = 0; j < 3; ++j) s += Ki[j][i] * dN[3 * a + j];
                dNdx[3 * a + i] = s;
            }
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
                double s = 0.0;
                for (int i = 0; i < 3; ++i) s += dNdx[3 * a + i] * dNdx[3 * b + i];
                K[a * n + b] += w[q] * det * s;
            }
    }
    return 0;
}

/* Nodal divergence (D u)[f] = sum_e sum_g dV N_a div u, out[n_field]. */
int oracle_divergence(int64_t n_nodes, const double *coords, int64_t n_elems, const uint8_t *types,
                      const int64_t *offs, const int32_t *conn, const int32_t *field_node, int64_t n_field,
                      const double *u, double *out)
{
    double x[3 * ORACLE_MAX_NODE], ue[3 * ORACLE_MAX_NODE], pts[3 * ORACLE_MAX_GAUSS], w[ORACLE_MAX_GAUSS];
    double N[ORACLE_MAX_NODE], dN[3 * ORACLE_MAX_NODE];
    int64_t fid[ORACLE_MAX_NODE];
    g_bad_element = -1;
    for (int64_t k = 0; k < n_field; ++k) out[k] = 0.0;
    for (int64_t e = 0; e < n_elems; ++e) {
        const int n = gather(e, n_nodes, coords, types, offs, conn, field_node, n_field, u, NULL, x, ue, NULL, fid);
        if (n < 0) { g_bad_element = e; return -1; }
        const int ng = oracle_gauss(types[e], pts, w);
        for (int q = 0; q < ng; ++q) {
            double J[3][3], Ki[3][3];
            oracle_shape(types[e], pts + 3 * q, N, dN);
            jacobian(n, x, dN, J);
            const double det = det3(J);
            if (!(det > 0.0)) { g_bad_element = e; return -2; }
            inv3(J, det, Ki);
            double div = 0.0;
            for (int a = 0; a < n; ++a)
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) div += ue[3 * a + i] * Ki[j][i] * dN[3 * a + j];
            for (int a = 0; a < n; ++a) out[fid[a]] += w[q] * det * N[a] * div;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Residual of a given subgrid stress                                       */
/* ------------------------------------------------------------------------ */

/* R[a*3 + i] = sum_g w_g det J_g dN_a/dx_j tau_g,ij for a symmetric stress
 * given per Gauss point as tau[g*6 + c], c = (xx, yy, zz, xy, xz, yz).  This
 * is the weak form of -div(tau) moved to the right-hand side (the natural
 * boundary term dropped), i.e. the subgrid part of the residual for a closure
 * that supplies tau directly (with Vreman, tau = -2 nu_t eps(u)).           */
int oracle_element_stress_residual(int type, const double *x, const double *tau, double *R)
{
    double pts[3 * ORACLE_MAX_GAUSS], w[ORACLE_MAX_GAUSS];
    double N[ORACLE_MAX_NODE], dN[3 * ORACLE_MAX_NODE], dNdx[3 * ORACLE_MAX_NODE];
    const int n = oracle_nnode(type);
    const int ng = oracle_gauss(type, pts, w);
    if (n < 0 || ng < 0) return -1;
    for (int k = 0; k < 3 * n; ++k) R[k] = 0.0;
    for (int q = 0; q < ng; ++q) {
        double J[3][3], K[3][3];
        oracle_shape(type, pts + 3 * q, N, dN);
        jacobian(n, x, dN, J);
        const double det = det3(J);
        if (!(det > 0.0)) return -2;
        inv3(J, det, K);
        for (int a = 0; a < n; ++a)
            for (int i = 0; i < 3; ++i) {
                double s = 0.0;
                for (int j = 0; j < 3; ++j) s += K[j][i] * dN[3 * a + j];
                dNdx[3 * a + i] = s;
            }
        const double *t = tau + 6 * q;
        const double T[3][3] = {{t[0], t[3], t[4]}, {t[3], t[1], t[5]}, {t[4], t[5], t[2]}};
        for (int a = 0; a < n; ++a)
            for (int i = 0; i < 3; ++i) {
                double s = 0.0;
                for (int j = 0; j < 3; ++j) s += dNdx[3 * a + j] * T[i][j];
                R[3 * a + i] += w[q] * det * s;
            }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Boundary assembly: equilibrium wall model (Algorithm 1, "Boundary        */
/* assembly"; Section 3.2 names a law-of-the-wall model without formulas)   */
/* ------------------------------------------------------------------------ */
/*
 * Reading (listed in the design notes):
 *   exchange point  x_e = vertex average of the wall face's volume element,
 *                   u_e = mean of its nodal velocities (the finite-element
 *                   interpolant at x_e for every linear type);
 *   wall distance   y = |n . (x_e - x_f)|, x_f the face's vertex average and
 *                   n its unit normal (triangle: (x1-x0) x (x2-x0); quad:
 *                   (x2-x0) x (x3-x1));
 *   tangential velocity u_t = u_e - (u_e . n) n, U = |u_t|;
 *   law of the wall (Reichardt): U / u_tau = f(y u_tau / nu),
 *     f(y+) = ln(1 + kappa y+)/kappa + C1 (1 - exp(-y+/chi) - (y+/chi) exp(-y+/3)),
 *     kappa = 0.41, C1 = 7.8, chi = 11, solved for u_tau by Newton's method;
 *   wall shear stress tau_w = u_tau^2 (rho = 1) against the flow:
 *     t = -tau_w u_t / U (t = 0 when U = 0);
 *   nodal contribution rhs[a] += t * int_face N_a dA (linear triangle, or
 *     bilinear quadrilateral with the 2 x 2 Gauss rule).
 */
#define WALL_KAPPA 0.41
#define WALL_C1 7.8
#define WALL_CHI 11.0

double oracle_wall_law(double yp)
{
    return log(1.0 + WALL_KAPPA * yp) / WALL_KAPPA +
           WALL_C1 * (1.0 - exp(-yp / WALL_CHI) - (yp / WALL_CHI) * exp(-yp / 3.0));
}

static double wall_law_slope(double yp)
{
    return 1.0 / (1.0 + WALL_KAPPA * yp) +
           WALL_C1 * (exp(-yp / WALL_CHI) / WALL_CHI - exp(-yp / 3.0) / WALL_CHI + (yp / WALL_CHI) * exp(-yp / 3.0) / 3.0);
}

/* u_tau with U = u_tau f(y u_tau / nu); 0 when U = 0.  Newton's method on
 * g(u) = u f(y u / nu) - U from the viscous-sublayer value sqrt(nu U / y). */
double oracle_friction_velocity(double U, double y, double nu)
{
    if (!(U > 0.0)) return 0.0;
    double ut = sqrt(nu * U / y);
    for (int it = 0; it < 100; ++it) {
        const double yp = y * ut / nu;
        const double g = ut * oracle_wall_law(yp) - U;
        const double dg = oracle_wall_law(yp) + yp * wall_law_slope(yp);
        const double step = g / dg;
        ut -= step;
        if (fabs(step) <= 1e-15 * ut) break;
    }
    return ut;
}

/* Face integrals of the face's own shape functions, int N_a dA, for a
 * triangle (n = 3) or a bilinear quadrilateral (n = 4), and the unit normal. */
static int face_geometry(int n, const double *xf, double *wa, double *nrm)
{
    double c[3];
    if (n == 3) {
        double d1[3], d2[3];
        for (int k = 0; k < 3; ++k) {
            d1[k] = xf[3 + k] - xf[k];
            d2[k] = xf[6 + k] - xf[k];
        }
        c[0] = d1[1] * d2[2] - d1[2] * d2[1];
        c[1] = d1[2] * d2[0] - d1[0] * d2[2];
        c[2] = d1[0] * d2[1] - d1[1] * d2[0];
        const double area = 0.5 * sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        for (int a = 0; a < 3; ++a) wa[a] = area / 3.0;
    } else if (n == 4) {
        double d1[3], d2[3];
        for (int k = 0; k < 3; ++k) {
            d1[k] = xf[6 + k] - xf[k];
            d2[k] = xf[9 + k] - xf[3 + k];
        }
        c[0] = d1[1] * d2[2] - d1[2] * d2[1];
        c[1] = d1[2] * d2[0] - d1[0] * d2[2];
        c[2] = d1[0] * d2[1] - d1[1] * d2[0];
        /* nodes counter-clockwise: (-1,-1), (1,-1), (1,1), (-1,1) */
        const double s[4] = {-1, 1, 1, -1}, t[4] = {-1, -1, 1, 1};
        const double gq = 1.0 / sqrt(3.0);
        for (int a = 0; a < 4; ++a) wa[a] = 0.0;
        for (int gi = 0; gi < 2; ++gi)
            for (int gj = 0; gj < 2; ++gj) {
                const double xi = gi ? gq : -gq, eta = gj ? gq : -gq;
                double dx[3] = {0, 0, 0}, dy[3] = {0, 0, 0};
                for (int a = 0; a < 4; ++a)
                    for (int k = 0; k < 3; ++k) {
                        dx[k] += 0.25 * s[a] * (1.0 + t[a] * eta) * xf[3 * a + k];
                        dy[k] += 0.25 * t[a] * (1.0 + s[a] * xi) * xf[3 * a + k];
                    }
                const double cx = dx[1] * dy[2] - dx[2] * dy[1];
                const double cy = dx[2] * dy[0] - dx[0] * dy[2];
                const double cz = dx[0] * dy[1] - dx[1] * dy[0];
                const double jac = sqrt(cx * cx + cy * cy + cz * cz);
                for (int a = 0; a < 4; ++a) wa[a] += 0.25 * (1.0 + s[a] * xi) * (1.0 + t[a] * eta) * jac;
            }
    } else {
        return -1;
    }
    const double len = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    if (!(len > 0.0)) return -2;
    for (int k = 0; k < 3; ++k) nrm[k] = c[k] / len;
    return 0;
}

/* Wall-model contribution of every wall face into out[n_field][3]
 * (overwritten).  Face f has the user nodes face_conn[face_offs[f] ..
 * face_offs[f+1]) (3 or 4) and lies on volume element face_elem[f].  Optional
 * per-face diagnostics: y, U, u_tau (each [n_faces], may be NULL). */
int oracle_wall_assemble(int64_t n_nodes, const double *coords, int64_t n_elems, const uint8_t *types,
                         const int64_t *offs, const int32_t *conn, const int32_t *field_node, int64_t n_field,
                         const double *u, double nu, int64_t n_faces, const int64_t *face_offs,
                         const int32_t *face_conn, const int64_t *face_elem, double *out, double *diag_y,
                         double *diag_U, double *diag_ut)
{
    double x[3 * ORACLE_MAX_NODE], ue[3 * ORACLE_MAX_NODE];
    int64_t fid[ORACLE_MAX_NODE];
    g_bad_element = -1;
    for (int64_t k = 0; k < 3 * n_field; ++k) out[k] = 0.0;
    for (int64_t f = 0; f < n_faces; ++f) {
        const int64_t e = face_elem[f];
        const int nf = (int)(face_offs[f + 1] - face_offs[f]);
        if (e < 0 || e >= n_elems || (nf != 3 && nf != 4)) { g_bad_element = f; return -1; }
        const int n = gather(e, n_nodes, coords, types, offs, conn, field_node, n_field, u, NULL, x, ue, NULL, fid);
        if (n < 0) { g_bad_element = f; return -1; }
        double xe[3] = {0, 0, 0}, uel[3] = {0, 0, 0};
        for (int a = 0; a < n; ++a)
            for (int k = 0; k < 3; ++k) {
                xe[k] += x[3 * a + k] / n;
                uel[k] += ue[3 * a + k] / n;
            }
        double xf[12], xc[3] = {0, 0, 0};
        int64_t ff[4];
        for (int b = 0; b < nf; ++b) {
            const int64_t g = face_conn[face_offs[f] + b];
            if (g < 0 || g >= n_nodes) { g_bad_element = f; return -1; }
            ff[b] = field_node ? (int64_t)field_node[g] : g;
            for (int k = 0; k < 3; ++k) {
                xf[3 * b + k] = coords[3 * g + k];
                xc[k] += coords[3 * g + k] / nf;
            }
        }
        double wa[4], nrm[3];
        const int st = face_geometry(nf, xf, wa, nrm);
        if (st) { g_bad_element = f; return st; }
        double y = 0.0, un = 0.0;
        for (int k = 0; k < 3; ++k) {
            y += nrm[k] * (xe[k] - xc[k]);
            un += nrm[k] * uel[k];
        }
        y = fabs(y);
        if (!(y > 0.0)) { g_bad_element = f; return -2; }
        double ut[3], U = 0.0;
        for (int k = 0; k < 3; ++k) {
            ut[k] = uel[k] - un * nrm[k];
            U += ut[k] * ut[k];
        }
        U = sqrt(U);
        const double utau = oracle_friction_velocity(U, y, nu);
        double t[3] = {0, 0, 0};
        if (U > 0.0)
            for (int k = 0; k < 3; ++k) t[k] = -utau * utau * ut[k] / U;
        for (int b = 0; b < nf; ++b)
            for (int k = 0; k < 3; ++k) out[3 * ff[b] + k] += t[k] * wa[b];
        if (diag_y) diag_y[f] = y;
        if (diag_U) diag_U[f] = U;
        if (diag_ut) diag_ut[f] = utau;
    }
    return 0;
}
