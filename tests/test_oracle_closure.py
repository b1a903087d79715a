"""Pins of the oracle's stress-residual helper used by the learned closure:
with tau = -2 nu_t eps(u) it must reproduce the Vreman part of the residual,
and a constant stress gives the closed-form face integrals."""
import numpy as np
import pytest

from paper_2005_05899_amd import meshgen as mg


def test_stress_residual_reproduces_vreman_term(orc):
    c = mg.small_hybrid_case(nx=3, ny=3, seed=9)
    m = c.mesh
    for e in range(0, m.n_elems, 7):
        nodes = m.element_nodes(e)
        t = int(m.types[e])
        R, gp, _ = orc.element_residual(t, m.coords[nodes], c.u[nodes], None, 0.0, 0.1, terms=orc.TERM_SGS)
        G = gp[:, 5:14].reshape(-1, 3, 3)
        eps = 0.5 * (G + G.transpose(0, 2, 1))
        tau = -2.0 * gp[:, 17][:, None, None] * eps
        t6 = np.stack([tau[:, 0, 0], tau[:, 1, 1], tau[:, 2, 2], tau[:, 0, 1], tau[:, 0, 2], tau[:, 1, 2]], axis=1)
        Rs = orc.element_stress_residual(t, m.coords[nodes], t6)
        assert np.abs(Rs - R).max() <= 1e-13 * max(np.abs(R).max(), 1e-300)


def test_constant_stress_on_unit_cube(orc):
    """A constant tau_xy on the unit cube: R_a = int dN_a/dx_j tau_ij, i.e.
    +-1/4 tau_xy in x from the y-derivative and in y from the x-derivative."""
    x = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], float)
    R = orc.element_stress_residual(8, x, [[0, 0, 0, 2.0, 0, 0]] * 8)
    sx = np.where(x[:, 0] > 0.5, 0.25, -0.25)
    sy = np.where(x[:, 1] > 0.5, 0.25, -0.25)
    assert np.abs(R[:, 0] - 2.0 * sy).max() < 1e-15
    assert np.abs(R[:, 1] - 2.0 * sx).max() < 1e-15
    assert np.abs(R[:, 2]).max() < 1e-15
