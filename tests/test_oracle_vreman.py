"""Pins of the oracle's Vreman eddy viscosity (closed forms and invariants)."""
import math

import numpy as np
import pytest


def test_zero_gradient_gives_exact_zero(orc):
    assert orc.vreman(np.zeros((3, 3)), 0.7, 0.1) == 0.0


def test_pure_shear_gives_zero(orc):
    # u = (gamma y, 0, 0): alpha has rank one, so B_beta = 0
    G = np.zeros((3, 3))
    G[0, 1] = 3.7
    assert orc.vreman(G, 0.5, 0.1) == 0.0


@pytest.mark.parametrize("omega", [0.3, -2.0, 11.0])
def test_solid_rotation(orc, omega):
    # u = (-omega y, omega x, 0): nu_t = c Delta^2 |omega| / sqrt(2)
    G = np.array([[0, -omega, 0], [omega, 0, 0], [0, 0, 0]], float)
    d, c = 0.3, 0.1
    assert orc.vreman(G, d, c) == pytest.approx(c * d * d * abs(omega) / math.sqrt(2), rel=1e-14)


def test_plane_strain(orc):
    G = np.diag([1.0, -1.0, 0.0])
    d, c = 0.25, 0.07
    assert orc.vreman(G, d, c) == pytest.approx(c * d * d / math.sqrt(2), rel=1e-14)


def test_axisymmetric_strain(orc):
    # G = diag(a, a, -2a): alpha^T alpha = a^2 diag(1,1,4); B = D^4 a^4 (1 + 4 + 4),
    # alpha:alpha = 6 a^2 -> nu_t = c D^2 |a| sqrt(9/6)
    a, d, c = 1.7, 0.2, 0.1
    G = np.diag([a, a, -2 * a])
    assert orc.vreman(G, d, c) == pytest.approx(c * d * d * abs(a) * math.sqrt(1.5), rel=1e-14)


def test_matches_invariant_form(orc):
    """B_beta is Delta^4 times the second invariant of M = G G^T (sum of the
    principal 2x2 minors), so nu_t = c D^2 sqrt(((tr M)^2 - tr M^2) / (2 tr M))."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        G = rng.standard_normal((3, 3)) * rng.uniform(0.01, 100)
        d, c = rng.uniform(0.01, 2), rng.uniform(0.01, 0.3)
        M = G @ G.T
        tr = np.trace(M)
        inv2 = 0.5 * (tr * tr - np.trace(M @ M))
        expect = c * d * d * math.sqrt(max(inv2, 0) / tr)
        assert orc.vreman(G, d, c) == pytest.approx(expect, rel=1e-11)


def test_rotation_invariance_and_scaling(orc):
    rng = np.random.default_rng(6)
    for _ in range(50):
        G = rng.standard_normal((3, 3))
        Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        v = orc.vreman(G, 0.4, 0.1)
        assert orc.vreman(Q @ G @ Q.T, 0.4, 0.1) == pytest.approx(v, rel=1e-12)
        # homogeneous of degree 1 in G and 2 in Delta, linear in c
        assert orc.vreman(3.0 * G, 0.4, 0.1) == pytest.approx(3.0 * v, rel=1e-13)
        assert orc.vreman(G, 0.8, 0.1) == pytest.approx(4.0 * v, rel=1e-13)
        assert orc.vreman(G, 0.4, 0.2) == pytest.approx(2.0 * v, rel=1e-14)
