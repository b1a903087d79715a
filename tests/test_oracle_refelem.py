"""Pins of the oracle's reference elements: shape functions and quadrature.

Checked against closed forms only (partition of unity, Kronecker property,
linear completeness, finite differences of N, exact monomial integrals).
"""
from fractions import Fraction
from math import factorial

import numpy as np
import pytest

from tests.polyexact import collapsed_pyramid_mono, cube_mono, prism_mono, simplex_mono

NODES = {
    4: [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)],
    5: [(-1, -1, 0), (1, -1, 0), (1, 1, 0), (-1, 1, 0), (0, 0, 1)],
    6: [(0, 0, -1), (1, 0, -1), (0, 1, -1), (0, 0, 1), (1, 0, 1), (0, 1, 1)],
    8: [(-1, -1, -1), (1, -1, -1), (1, 1, -1), (-1, 1, -1), (-1, -1, 1), (1, -1, 1), (1, 1, 1), (-1, 1, 1)],
}
VOLUME = {4: 1.0 / 6.0, 5: 4.0 / 3.0, 6: 1.0, 8: 8.0}
TYPES = (4, 5, 6, 8)


def interior_points(t, n=20, seed=0):
    """Random points strictly inside the reference element of type t."""
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        if t == 8:
            pts.append(rng.uniform(-0.95, 0.95, 3))
        elif t == 4:
            p = rng.uniform(0.02, 0.9, 3)
            if p.sum() < 0.95:
                pts.append(p)
        elif t == 6:
            r, s = rng.uniform(0.02, 0.9, 2)
            if r + s < 0.95:
                pts.append(np.array([r, s, rng.uniform(-0.95, 0.95)]))
        else:
            z = rng.uniform(0.02, 0.9)
            q = 1 - z
            pts.append(np.array([rng.uniform(-0.95, 0.95) * q, rng.uniform(-0.95, 0.95) * q, z]))
    return pts


@pytest.mark.parametrize("t", TYPES)
def test_partition_of_unity_and_derivative_sum(orc, t):
    pts = list(orc.gauss(t)[0]) + interior_points(t)
    for xi in pts:
        N, dN = orc.shape(t, xi)
        assert abs(N.sum() - 1.0) < 1e-14
        assert np.abs(dN.sum(axis=0)).max() < 1e-14


@pytest.mark.parametrize("t", TYPES)
def test_kronecker_property(orc, t):
    for b, xb in enumerate(NODES[t]):
        N, _ = orc.shape(t, np.array(xb, float))
        expect = np.zeros(len(N))
        expect[b] = 1.0
        assert np.abs(N - expect).max() < 1e-15, (t, b, N)


@pytest.mark.parametrize("t", TYPES)
def test_linear_completeness(orc, t):
    """sum_a N_a xi_a = xi and sum_a xi_a (x) dN_a = I at any interior point."""
    X = np.array(NODES[t], float)
    for xi in list(orc.gauss(t)[0]) + interior_points(t, seed=1):
        N, dN = orc.shape(t, xi)
        assert np.abs(N @ X - xi).max() < 1e-14
        assert np.abs(X.T @ dN - np.eye(3)).max() < 1e-14


@pytest.mark.parametrize("t", TYPES)
def test_derivatives_match_finite_differences(orc, t):
    h = 1e-6
    for xi in interior_points(t, n=10, seed=2):
        _, dN = orc.shape(t, xi)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            fd = (orc.shape(t, xi + e)[0] - orc.shape(t, xi - e)[0]) / (2 * h)
            assert np.abs(fd - dN[:, k]).max() < 1e-8


def test_pyramid_basis_vanishes_on_opposite_faces(orc):
    """Base function a vanishes on the two triangular faces not containing node a."""
    rng = np.random.default_rng(3)
    # face x = 1 - z (nodes 1, 2, apex): N_0 and N_3 vanish there
    for _ in range(10):
        z = rng.uniform(0.05, 0.9)
        y = rng.uniform(-1, 1) * (1 - z)
        N, _ = orc.shape(5, np.array([1 - z, y, z]))
        assert abs(N[0]) < 1e-15 and abs(N[3]) < 1e-15


@pytest.mark.parametrize("t", TYPES)
def test_weights_sum_to_reference_volume(orc, t):
    _, w = orc.gauss(t)
    assert abs(w.sum() - VOLUME[t]) < 1e-15
    assert (w > 0).all()


def _quad(orc, t, f):
    pts, w = orc.gauss(t)
    return sum(wq * f(*p) for p, wq in zip(pts, w))


def test_hex_rule_exact_to_degree_3_per_variable(orc):
    mono = cube_mono(-1, 1)
    for i in range(4):
        for j in range(4):
            for k in range(4):
                q = _quad(orc, 8, lambda x, y, z: x ** i * y ** j * z ** k)
                assert abs(q - float(mono(i, j, k))) < 1e-14
    # degree 4 in one variable is not integrated exactly by 2 points
    assert abs(_quad(orc, 8, lambda x, y, z: x ** 4) - float(mono(4, 0, 0))) > 1e-3


def test_tet_rule_exact_to_total_degree_2(orc):
    for i in range(3):
        for j in range(3 - i):
            for k in range(3 - i - j):
                q = _quad(orc, 4, lambda r, s, t: r ** i * s ** j * t ** k)
                assert abs(q - float(simplex_mono(i, j, k))) < 1e-15
    assert abs(_quad(orc, 4, lambda r, s, t: r ** 3) - float(simplex_mono(3, 0, 0))) > 1e-5


def test_prism_rule_exact_tri_degree_2_line_degree_3(orc):
    for i in range(3):
        for j in range(3 - i):
            for k in range(4):
                q = _quad(orc, 6, lambda r, s, z: r ** i * s ** j * z ** k)
                assert abs(q - float(prism_mono(i, j, k))) < 1e-15


def pyramid_mono(i, j, k):
    """Integral of xi^i eta^j zeta^k over the reference pyramid (closed form):
    int_0^1 zeta^k [int_{-q}^{q} xi^i][int_{-q}^{q} eta^j] dzeta, q = 1 - zeta."""
    if i % 2 or j % 2:
        return Fraction(0)
    # (2 q^{i+1}/(i+1)) (2 q^{j+1}/(j+1)) -> 4/((i+1)(j+1)) * B(k+1, i+j+3)
    beta = Fraction(factorial(k) * factorial(i + j + 2), factorial(k + i + j + 3))
    return Fraction(4, (i + 1) * (j + 1)) * beta


def test_pyramid_rule_exact_on_monomials(orc):
    """In collapsed coordinates xi^i eta^j zeta^k = a^i b^j (1-c)^(i+j) c^k, so
    the conical 2x2x2 rule is exact for i+j+k <= 3."""
    for i in range(4):
        for j in range(4):
            for k in range(4):
                if i + j + k > 3:
                    continue
                q = _quad(orc, 5, lambda x, y, z: x ** i * y ** j * z ** k)
                assert abs(q - float(pyramid_mono(i, j, k))) < 1e-15, (i, j, k)


def test_pyramid_basis_integrals(orc):
    """int N_base = 1/4 and int N_apex = 1/3 over the reference pyramid
    (collapsed form N_base = (1-c)(1 +- a)(1 +- b)/4, N_apex = c)."""
    pts, w = orc.gauss(5)
    tot = np.zeros(5)
    for p, wq in zip(pts, w):
        tot += wq * orc.shape(5, p)[0]
    assert np.abs(tot[:4] - 0.25).max() < 1e-15
    assert abs(tot[4] - 1.0 / 3.0) < 1e-15
    # same numbers from the collapsed-coordinate closed forms
    base =(collapsed_pyramid_mono(0, 0, 0) - collapsed_pyramid_mono(0, 0, 1)) / 4
    assert base == Fraction(1, 4)
    assert collapsed_pyramid_mono(0, 0, 1) == Fraction(1, 3)
