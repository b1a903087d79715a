"""Single-element pins by exact rational integration.

The residual of one affine element is built here from scratch with exact
polynomial arithmetic (tests/polyexact.py): basis functions as polynomials,
physical gradients through the inverse of the affine map, and closed-form
monomial integrals over the reference domain -- no quadrature, no floating
point.  Wherever the oracle's Gauss rule is exact for the integrand (argued per
case below), the two must agree to rounding.  Textbook values (tetrahedron
mass matrix, unit-cube gradient integrals, nodal volumes) are checked too.
"""
from fractions import Fraction

import numpy as np
import pytest

from tests.polyexact import Poly, collapsed_pyramid_mono, cube_mono, det3, inv3, prism_mono, simplex_mono

F = Fraction


def ref_basis(t):
    """(N_a, dN_a/dxi_k, monomial integral) in the integration variables of type t."""
    v0, v1, v2 = Poly.var(0), Poly.var(1), Poly.var(2)
    one = Poly.const(1)
    if t == 8:
        signs = [(-1, -1, -1), (1, -1, -1), (1, 1, -1), (-1, 1, -1), (-1, -1, 1), (1, -1, 1), (1, 1, 1), (-1, 1, 1)]
        N = [F(1, 8) * (one + sx * v0) * (one + sy * v1) * (one + sz * v2) for sx, sy, sz in signs]
        dN = [[n.diff(k) for k in range(3)] for n in N]
        return N, dN, cube_mono(-1, 1)
    if t == 4:
        N = [one - v0 - v1 - v2, v0, v1, v2]
        dN = [[n.diff(k) for k in range(3)] for n in N]
        return N, dN, simplex_mono
    if t == 6:
        L = [one - v0 - v1, v0, v1]
        Z = [F(1, 2) * (one - v2), F(1, 2) * (one + v2)]
        N = [L[i] * Z[j] for j in range(2) for i in range(3)]
        dN = [[n.diff(k) for k in range(3)] for n in N]
        return N, dN, prism_mono
    if t == 5:
        # collapsed coordinates a, b, c: xi = a (1-c), eta = b (1-c), zeta = c.
        # Base: N = (1-c)(1 + xa a)(1 + ya b)/4, with reference derivatives
        # dN/dxi = xa (1 + ya b)/4, dN/deta = ya (1 + xa a)/4,
        # dN/dzeta = -1/4 + xa ya a b / 4.  Apex: N = c, gradient (0, 0, 1).
        a, b, c = v0, v1, v2
        N, dN = [], []
        for xa, ya in [(-1, -1), (1, -1), (1, 1), (-1, 1)]:
            N.append(F(1, 4) * (one - c) * (one + xa * a) * (one + ya * b))
            dN.append([F(xa, 4) * (one + ya * b), F(ya, 4) * (one + xa * a),
                       F(-1, 4) * one + F(xa * ya, 4) * a * b])
        N.append(c)
        dN.append([Poly(), Poly(), one])
        return N, dN, collapsed_pyramid_mono
    raise ValueError(t)


REF_NODES = {
    4: [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)],
    5: [(-1, -1, 0), (1, -1, 0), (1, 1, 0), (-1, 1, 0), (0, 0, 1)],
    6: [(0, 0, -1), (1, 0, -1), (0, 1, -1), (0, 0, 1), (1, 0, 1), (0, 1, 1)],
    8: [(-1, -1, -1), (1, -1, -1), (1, 1, -1), (-1, 1, -1), (-1, -1, 1), (1, -1, 1), (1, 1, 1), (-1, 1, 1)],
}

# A non-symmetric affine map with dyadic entries (exact in binary floating point)
B_MAP = [[F(3, 4), F(1, 8), F(-1, 4)], [F(-1, 8), F(5, 8), F(1, 16)], [F(1, 16), F(-3, 16), F(7, 8)]]
X0 = [F(1, 2), F(-3, 4), F(5, 4)]


def physical_nodes(t, B=B_MAP, x0=X0):
    return [[sum(B[i][k] * F(xi[k]) for k in range(3)) + x0[i] for i in range(3)] for xi in REF_NODES[t]]


def exact_residual(t, u_nodes, p_nodes, nu, B=B_MAP, terms=("conv", "pres", "visc")):
    """-det(B) * int_ref [N_a (C_i + dp/dx_i) + dN_a/dx_j nu (G_ij + G_ji)]."""
    N, dNref, mono = ref_basis(t)
    n = len(N)
    K = inv3(B)
    detB = det3(B)
    dNdx = [[sum((dNref[a][k] * K[k][i] for k in range(3)), Poly()) for i in range(3)] for a in range(n)]
    u = [sum((N[a] * u_nodes[a][i] for a in range(n)), Poly()) for i in range(3)]
    G = [[sum((dNdx[a][j] * u_nodes[a][i] for a in range(n)), Poly()) for j in range(3)] for i in range(3)]
    q = [sum((dNdx[a][i] * p_nodes[a] for a in range(n)), Poly()) for i in range(3)]
    divu = G[0][0] + G[1][1] + G[2][2]
    C = [sum(((G[i][j] + G[j][i]) * u[j] for j in range(3)), Poly()) + divu * u[i] for i in range(3)]
    R = np.zeros((n, 3))
    for a in range(n):
        for i in range(3):
            f = Poly()
            if "conv" in terms:
                f = f + C[i]
            if "pres" in terms:
                f = f + q[i]
            integrand = N[a] * f
            if "visc" in terms:
                integrand = integrand + sum((dNdx[a][j] * (G[i][j] + G[j][i]) * nu for j in range(3)), Poly())
            R[a, i] = float(-detB * integrand.integrate(mono))
    return R


def dyadic_values(rng, shape, den=16):
    return [[F(int(v), den) for v in row] for row in rng.integers(-2 * den, 2 * den, size=shape)]


# Gauss rule exact for arbitrary nodal data: HEX (degree <= 3 per variable on an
# affine hexahedron), TET (degree 2), PYR (in collapsed coordinates a, b <= 3,
# c <= 2 against the (1-c)^2 weight).  PEN: only for linear fields, because
# N_a u G reaches degree 3 on the triangle where the 3-point rule stops at 2.
@pytest.mark.parametrize("t", [4, 5, 8])
def test_single_element_residual_arbitrary_fields(orc, t):
    rng = np.random.default_rng(10 + t)
    n = len(REF_NODES[t])
    u = dyadic_values(rng, (n, 3))
    p = [row[0] for row in dyadic_values(rng, (n, 1))]
    nu = F(3, 8)
    exact = exact_residual(t, u, p, nu)
    x = np.array([[float(v) for v in row] for row in physical_nodes(t)])
    R, _, _ = orc.element_residual(t, x, np.array(u, float), np.array(p, float), float(nu), 0.0)
    scale = np.abs(exact).max()
    assert scale > 0.1
    assert np.abs(R - exact).max() < 1e-14 * scale * 10, np.abs(R - exact).max()


@pytest.mark.parametrize("t", [4, 5, 6, 8])
def test_single_element_residual_linear_fields(orc, t):
    rng = np.random.default_rng(20 + t)
    A = dyadic_values(rng, (3, 3), den=8)
    b = [F(1, 4), F(-1, 2), F(3, 8)]
    g = [F(1, 2), F(-1, 8), F(1, 4)]
    X = physical_nodes(t)
    u = [[sum(A[i][k] * X[a][k] for k in range(3)) + b[i] for i in range(3)] for a in range(len(X))]
    p = [sum(g[k] * X[a][k] for k in range(3)) + F(1, 2) for a in range(len(X))]
    nu = F(5, 16)
    exact = exact_residual(t, u, p, nu)
    x = np.array([[float(v) for v in row] for row in X])
    R, gp, _ = orc.element_residual(t, x, np.array(u, float), np.array(p, float), float(nu), 0.0)
    assert np.abs(R - exact).max() < 1e-13 * np.abs(exact).max()
    # isoparametric reproduction: G = A and grad p = g at every Gauss point
    An = np.array(A, float)
    for rec in gp:
        assert np.abs(rec[5:14].reshape(3, 3) - An).max() < 1e-13
        assert np.abs(rec[14:17] - np.array(g, float)).max() < 1e-13


@pytest.mark.parametrize("t", [4, 5, 6, 8])
def test_single_element_vreman_term_linear_fields(orc, t):
    """With G = A constant, nu_t is constant on the element, so the subgrid part
    of the residual is -nu_t int dN_a/dx_j (A + A^T)_ij dV."""
    rng = np.random.default_rng(30 + t)
    A = dyadic_values(rng, (3, 3), den=8)
    X = physical_nodes(t)
    u = [[sum(A[i][k] * X[a][k] for k in range(3)) for i in range(3)] for a in range(len(X))]
    x = np.array([[float(v) for v in row] for row in X])
    c = 0.1
    vol = float(det3(B_MAP)) * {4: 1 / 6, 5: 4 / 3, 6: 1.0, 8: 8.0}[t]
    nut = orc.vreman(np.array(A, float), vol ** (1 / 3), c)
    assert nut > 0
    R, gp, delta = orc.element_residual(t, x, np.array(u, float), None, 0.0, c, terms=orc.TERM_SGS)
    assert delta == pytest.approx(vol ** (1 / 3), rel=1e-14)
    unit = exact_residual(t, u, [F(0)] * len(X), F(1), terms=("visc",))
    assert np.abs(R - nut * unit).max() < 1e-13 * np.abs(nut * unit).max()
    assert np.abs(gp[:, 17] - nut).max() < 1e-14 * nut


def test_tet_consistent_mass_closed_form(orc):
    """int N_a N_b = V (1 + delta_ab) / 20, so for u = A x + b the convective
    residual is -M (V/20)(u_a + sum_b u_b) with M = A + A^T + tr(A) I."""
    rng = np.random.default_rng(40)
    x = np.array([[0.1, 0.2, 0.0], [1.3, 0.1, 0.2], [0.2, 0.9, -0.1], [0.3, 0.4, 1.1]])
    A = rng.standard_normal((3, 3))
    b = rng.standard_normal(3)
    u = x @ A.T + b
    V = np.dot(x[1] - x[0], np.cross(x[2] - x[0], x[3] - x[0])) / 6
    M = A + A.T + np.trace(A) * np.eye(3)
    expect = -np.array([M @ ((V / 20) * (u[a] + u.sum(axis=0))) for a in range(4)])
    R, _, _ = orc.element_residual(4, x, u, None, 0.0, 0.0, terms=orc.TERM_CONV)
    assert np.abs(R - expect).max() < 1e-14 * np.abs(expect).max() * 10


def test_unit_cube_gradient_integrals(orc):
    """On the unit cube, int dN_b/dx_j = +-1/4 (sign of node b's offset along j)."""
    x = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], float)
    u = np.zeros((8, 3))
    for b in range(8):
        p = np.zeros(8)
        p[b] = 1.0
        R, _, _ = orc.element_residual(8, x, u, p, 0.0, 0.0, terms=orc.TERM_PRES)
        expect = np.where(x[b] > 0.5, 0.25, -0.25)
        assert np.abs(-R.sum(axis=0) - expect).max() < 1e-15


@pytest.mark.parametrize("t,shares", [(4, [1 / 4] * 4), (6, [1 / 6] * 6), (8, [1 / 8] * 8),
                                      (5, [3 / 16] * 4 + [1 / 4])])
def test_single_element_lumped_mass(orc, t, shares):
    """Nodal volume shares of affine elements: tet V/4, prism V/6, hex V/8,
    pyramid 3V/16 per base node and V/4 at the apex."""
    class M:
        pass
    X = np.array([[float(v) for v in row] for row in physical_nodes(t)])
    m = M()
    m.coords, m.types = X, np.array([t], np.uint8)
    m.conn_offsets = np.array([0, len(X)], np.int64)
    m.conn = np.arange(len(X), dtype=np.int32)
    m.field_node, m.n_field_nodes = None, len(X)
    V = float(det3(B_MAP)) * {4: 1 / 6, 5: 4 / 3, 6: 1.0, 8: 8.0}[t]
    assert np.abs(orc.lumped_mass(m) - V * np.array(shares)).max() < 1e-15 * 10
