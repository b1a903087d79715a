"""Pins of the oracle's pressure-step operators and RK3 stages.

Element Laplacians against exact rational integration; divergence of linear
fields against the lumped mass; divergence/gradient duality on the periodic
cube; the mean-zero pressure solve; third-order accuracy of the RK3 stages.
"""
from fractions import Fraction

import numpy as np
import pytest

from paper_2005_05899_amd import meshgen as mg
from tests.polyexact import Poly, det3, inv3
from tests.test_oracle_exact import B_MAP, physical_nodes, ref_basis


def exact_element_laplacian(t, B=B_MAP):
    N, dNref, mono = ref_basis(t)
    K = inv3(B)
    detB = det3(B)
    n = len(N)
    dNdx = [[sum((dNref[a][k] * K[k][i] for k in range(3)), Poly()) for i in range(3)] for a in range(n)]
    out = np.zeros((n, n))
    for a in range(n):
        for b in range(n):
            integrand = sum((dNdx[a][i] * dNdx[b][i] for i in range(3)), Poly())
            out[a, b] = float(detB * integrand.integrate(mono))
    return out


@pytest.mark.parametrize("t", [4, 5, 6, 8])
def test_element_laplacian_exact(orc, t):
    """grad N . grad N is integrated exactly on affine elements of every type."""
    x = np.array([[float(v) for v in row] for row in physical_nodes(t)])
    K = orc.element_laplacian(t, x)
    ex = exact_element_laplacian(t)
    assert np.abs(K - ex).max() < 1e-14 * np.abs(ex).max() * 10
    assert np.abs(K - K.T).max() == 0.0 or np.abs(K - K.T).max() < 1e-15
    assert np.abs(K.sum(axis=1)).max() < 1e-14


def test_unit_cube_and_reference_tet_stiffness(orc):
    """Textbook values: unit-cube trilinear stiffness has 1/3 on the diagonal,
    0 along edges, -1/12 across face and body diagonals; the reference tet has
    K = V grad N_a . grad N_b with V = 1/6."""
    x = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], float)
    K = orc.element_laplacian(8, x)
    for a in range(8):
        for b in range(8):
            d = int(np.abs(x[a] - x[b]).sum())
            expect = {0: 1 / 3, 1: 0.0, 2: -1 / 12, 3: -1 / 12}[d]
            assert abs(K[a, b] - expect) < 1e-15
    xt = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    g = np.array([[-1, -1, -1], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    assert np.abs(orc.element_laplacian(4, xt) - (g @ g.T) / 6).max() < 1e-16


def test_divergence_of_linear_field_is_trace_times_mass(orc):
    c = mg.small_hybrid_case(nx=4, ny=3, seed=5)
    rng = np.random.default_rng(3)
    A, b = rng.standard_normal((3, 3)), rng.standard_normal(3)
    u = c.mesh.coords @ A.T + b
    D = orc.divergence(c.mesh, u)
    M = orc.lumped_mass(c.mesh)
    assert np.abs(D - np.trace(A) * M).max() < 1e-13 * np.abs(np.trace(A) * M).max()


def test_divergence_gradient_duality_on_periodic_cube(orc):
    """sum_a p_a (D u)_a + sum_a u_a . (G p)_a = int div(p u) = 0 (periodic,
    exactly integrated on the uniform cube)."""
    from oracle import step
    c = mg.periodic_tg_case(6)
    rng = np.random.default_rng(4)
    u = rng.standard_normal((c.mesh.n_field_nodes, 3))
    p = rng.standard_normal(c.mesh.n_field_nodes)
    D = orc.divergence(c.mesh, u)
    G = step.gradient(c.mesh, p)
    lhs = (p * D).sum() + (u * G).sum()
    assert abs(lhs) < 1e-13 * (np.abs(p * D).sum() + np.abs(u * G).sum())


def test_pressure_solve_mean_zero(orc):
    from oracle import step
    c = mg.periodic_tg_case(6)
    K = step.laplacian(c.mesh)
    rng = np.random.default_rng(5)
    b = rng.standard_normal(c.mesh.n_field_nodes)
    x = step.pressure_solve(K, b)
    assert abs(x.mean()) < 1e-14
    assert np.abs(K @ x - (b - b.mean())).max() < 1e-10 * np.abs(b).max()


def test_rk3_stages_are_third_order(orc):
    """One RK3 step of the semi-discrete momentum system u' = M^-1 rhs(u) has a
    local error O(dt^4): halving dt divides it by about 16."""
    from oracle import step
    c = mg.periodic_tg_case(4, noise=0.05)
    M = orc.lumped_mass(c.mesh)

    def reference(dt, sub=64):
        u = c.u
        for _ in range(sub):
            u = step.rk3_momentum(c.mesh, u, c.p, 0.05, 0.1, dt / sub, M)
        return u

    errs = []
    for dt in (0.2, 0.1):
        errs.append(np.abs(step.rk3_momentum(c.mesh, c.u, c.p, 0.05, 0.1, dt, M) - reference(dt)).max())
    ratio = errs[0] / errs[1]
    assert 12 < ratio < 20, (errs, ratio)
