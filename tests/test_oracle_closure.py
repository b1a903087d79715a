"""Pins of the learned-closure oracle (`oracle/closure.py`), the checker of the
GPU's fused closure.  The closure replaces Vreman's stress tau_v = -nu_t (G +
G^T) in the subgrid term div(tau) of the momentum equation (Section 3.2) by
the network's tau_m = Delta^2 |G|_F^2 dev(y) and falls back to Vreman per
element where |R_mlp - R_vreman| > tol |R_vreman| (element 2-norms).  What
pins it, none of it re-typing the oracle:

* tol = 0 keeps Vreman everywhere: bit for bit the plain assembly;
* a network whose output is zero turns the subgrid term off, so with every
  element kept the result is the plain assembly of the other three terms;
* a "perfect Vreman network" (its output written from Vreman's invariant
  form, B = (tr^2 M - tr M^2) / 2 with M = G G^T) gives tau_m = dev(tau_v):
  for a trace-free linear field the stresses agree and every element keeps
  the network with a zero difference; for any field the difference is the
  trace term (2/3) nu_t (div u) I, integrated against grad N;
* the stress difference conserves momentum element by element;
* the fallback decision flips at the stated threshold, on the element norm.

The module under test may be swapped for a planted-mistake copy through
LESASM_CLOSURE_ORACLE (used by the mutation tests).  Also pinned here: the
stress-residual helper the closure uses."""
import importlib.util
import math
import os

import numpy as np
import pytest

from oracle import mlp as omlp
from paper_2005_05899_amd import meshgen as mg


def _load():
    path = os.environ.get("LESASM_CLOSURE_ORACLE")
    if not path:
        from oracle import closure
        return closure
    # a copy in another directory, loaded as a module of the oracle package so
    # that its relative imports resolve
    spec = importlib.util.spec_from_file_location("oracle.closure_variant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


CL = _load()


@pytest.fixture(scope="module")
def case():
    return mg.small_hybrid_case(nx=3, ny=3, layers=[(mg.PEN06, 1), (mg.TET04, 1), (mg.PYR05, 1), (mg.HEX08, 1)],
                                seed=21)


def _params(seed, scale=1.0):
    p = omlp.init_params(seed)
    rng = np.random.default_rng(seed + 1)
    for k in p:  # nonzero biases
        if k[0] == "b":
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    p["W3"] *= scale
    p["b3"] *= scale
    return p


def _width_ref(mesh):
    from oracle import filter_width
    return float(np.median(filter_width(mesh)))


def _vreman_network(c):
    """Network stand-in whose output, from x[:, :9] = G/|G|_F alone, is
    y = -c sqrt(B(Gh)) (Gh + Gh^T) with B from the invariant form of Vreman's
    B_beta at unit width: B = (tr^2 M - tr M^2)/2, M = Gh Gh^T.  Then
    Delta^2 |G|^2 y = -nu_t (G + G^T) = tau_v (nu_t = c Delta^2 sqrt(B(G)/|G|^2),
    B homogeneous of degree 4, so sqrt(B(G)/|G|^2) = |G| sqrt(B(Gh)))."""
    def forward(params, x):
        Gh = np.asarray(x, np.float64)[:, :9].reshape(-1, 3, 3)
        M = Gh @ Gh.transpose(0, 2, 1)
        tr = np.trace(M, axis1=1, axis2=2)
        tr2 = np.einsum("nij,nji->n", M, M)
        B = np.maximum(0.5 * (tr * tr - tr2), 0.0)
        S = Gh + Gh.transpose(0, 2, 1)
        s6 = np.stack([S[:, 0, 0], S[:, 1, 1], S[:, 2, 2], S[:, 0, 1], S[:, 0, 2], S[:, 1, 2]], axis=1)
        return -c * np.sqrt(B)[:, None] * s6
    return forward


def test_zero_tolerance_is_the_plain_assembly(orc, case):
    m = case.mesh
    rhs, use, eps = CL.assemble(m, case.u, case.p, case.nu, case.vreman_c, _params(3), _width_ref(m), tol=0.0)
    assert not use.any() and (eps > 0).all()
    assert np.array_equal(rhs, orc.assemble(m, case.u, case.p, case.nu, case.vreman_c))


@pytest.mark.parametrize("bf16", [True, False])
def test_zero_network_turns_the_subgrid_term_off(orc, case, bf16):
    m = case.mesh
    p = _params(5)
    p["W3"][:] = 0.0
    p["b3"][:] = 0.0
    rhs, use, _ = CL.assemble(m, case.u, case.p, case.nu, case.vreman_c, p, _width_ref(m), tol=math.inf, bf16=bf16)
    assert use.all()
    want = orc.assemble(m, case.u, case.p, case.nu, case.vreman_c, terms=orc.TERM_CONV | orc.TERM_PRES | orc.TERM_VISC)
    full = orc.assemble(m, case.u, case.p, case.nu, case.vreman_c)
    assert np.abs(full - want).max() > 1e-3 * np.abs(want).max()  # the subgrid term is not negligible here
    assert np.abs(rhs - want).max() <= 1e-13 * np.abs(want).max()


def test_vreman_network_on_a_trace_free_linear_field_keeps_every_element(orc, case, monkeypatch):
    m = case.mesh
    rng = np.random.default_rng(31)
    A = rng.standard_normal((3, 3))
    A -= np.trace(A) / 3.0 * np.eye(3)  # div u = 0
    xf = m.field_coords()
    u = xf @ A.T + rng.standard_normal(3)
    c = 0.17
    monkeypatch.setattr(CL._mlp, "forward_bf16", _vreman_network(c))
    # widths far from Delta_ref: the scaling by Delta^2 must use each element's own width
    rhs, use, eps = CL.assemble(m, u, case.p, case.nu, c, _params(7), 3.0 * _width_ref(m), tol=1e-9)
    assert use.all(), eps.max()
    assert eps.max() < 1e-12
    want = orc.assemble(m, u, case.p, case.nu, c)
    assert np.abs(rhs - want).max() <= 1e-12 * np.abs(want).max()


def test_parts_hold_the_network_stress_term_and_the_differences(orc, case, monkeypatch):
    # diagnostics of the closure oracle (the tolerance of the GPU closure tests
    # is built from them): with the Vreman stand-in on a trace-free linear
    # field every element is kept and the network's stress term is Vreman's,
    # i.e. the subgrid term of the plain assembly; the per-element differences
    # assemble to the closure residual minus the plain one
    m = case.mesh
    rng = np.random.default_rng(33)
    A = rng.standard_normal((3, 3))
    A -= np.trace(A) / 3.0 * np.eye(3)
    u = m.field_coords() @ A.T + rng.standard_normal(3)
    c = 0.13
    monkeypatch.setattr(CL._mlp, "forward_bf16", _vreman_network(c))
    rhs, use, eps, parts = CL.assemble(m, u, case.p, case.nu, c, _params(9), _width_ref(m), tol=math.inf,
                                       parts=True)
    assert use.all()
    sgs = orc.assemble(m, u, case.p, case.nu, c, terms=orc.TERM_SGS)
    assert np.abs(sgs).max() > 0
    assert np.abs(parts["share"] - sgs).max() <= 1e-12 * np.abs(sgs).max()
    monkeypatch.undo()
    rhs, use, eps, parts = CL.assemble(m, case.u, case.p, case.nu, case.vreman_c, _params(5, 0.05), _width_ref(m),
                                       tol=math.inf, parts=True)
    assert use.all() and len(parts["D"]) == m.n_elems
    dsum = np.zeros_like(rhs)
    fn = m.field_node
    for e in range(m.n_elems):
        nodes = m.conn[m.conn_offsets[e]:m.conn_offsets[e + 1]]
        np.add.at(dsum, nodes if fn is None else fn[nodes], parts["D"][e])
    plain = orc.assemble(m, case.u, case.p, case.nu, case.vreman_c)
    assert np.abs(dsum).max() > 1e-6 * np.abs(plain).max()
    assert np.abs(plain + dsum - rhs).max() <= 1e-12 * np.abs(rhs).max()


def test_vreman_network_leaves_the_trace_term(orc, case, monkeypatch):
    # tau_m - tau_v = dev(tau_v) - tau_v = -(tr tau_v / 3) I = (2/3) nu_t div(u) I
    m = case.mesh
    c = case.vreman_c
    monkeypatch.setattr(CL._mlp, "forward_bf16", _vreman_network(c))
    rhs, use, _ = CL.assemble(m, case.u, case.p, case.nu, c, _params(7), _width_ref(m), tol=math.inf)
    assert use.all()
    want = orc.assemble(m, case.u, case.p, case.nu, c)
    for e in range(m.n_elems):
        nodes = m.element_nodes(e)
        f = nodes if m.field_node is None else m.field_node[nodes]
        t = int(m.types[e])
        _, gp, _ = orc.element_residual(t, m.coords[nodes], case.u[f], case.p[f], case.nu, c)
        divu = gp[:, 5] + gp[:, 9] + gp[:, 13]
        k = (2.0 / 3.0) * gp[:, 17] * divu
        tau = np.stack([k, k, k, 0 * k, 0 * k, 0 * k], axis=1)
        np.add.at(want, f, orc.element_stress_residual(t, m.coords[nodes], tau))
    assert np.abs(rhs - want).max() <= 1e-12 * np.abs(want).max()
    assert np.abs(rhs - orc.assemble(m, case.u, case.p, case.nu, c)).max() > 1e-6 * np.abs(want).max()


def test_network_input_orientation_and_width(orc, case, monkeypatch):
    # a stand-in whose output copies entries of x = [G/|G|, log(Delta/Delta_ref)]:
    # y = (1 + x_9) (Gh_00, Gh_11, Gh_22, Gh_01, Gh_02, Gh_12) (not symmetric in
    # G, so a transposed input changes it); the expected substitution is built
    # from the oracle's Gauss-point gradients and widths
    m = case.mesh
    c = case.vreman_c
    dref = 0.7 * _width_ref(m)

    def forward(params, x):
        x = np.asarray(x, np.float64)
        return (1.0 + x[:, 9:10]) * x[:, [0, 4, 8, 1, 2, 5]]
    monkeypatch.setattr(CL._mlp, "forward_bf16", forward)
    rhs, use, _ = CL.assemble(m, case.u, case.p, case.nu, c, _params(13), dref, tol=math.inf)
    assert use.all()
    want = orc.assemble(m, case.u, case.p, case.nu, c)
    for e in range(m.n_elems):
        nodes = m.element_nodes(e)
        f = nodes if m.field_node is None else m.field_node[nodes]
        t = int(m.types[e])
        _, gp, delta = orc.element_residual(t, m.coords[nodes], case.u[f], case.p[f], case.nu, c)
        G = gp[:, 5:14].reshape(-1, 3, 3)
        gn = np.sqrt((G * G).sum(axis=(1, 2)))
        y = (1.0 + math.log(delta / dref)) * np.stack([G[:, 0, 0], G[:, 1, 1], G[:, 2, 2], G[:, 0, 1], G[:, 0, 2],
                                                        G[:, 1, 2]], axis=1) / gn[:, None]
        y[:, :3] -= y[:, :3].mean(axis=1, keepdims=True)
        tau_m = (delta ** 2 * gn ** 2)[:, None] * y
        S = G + G.transpose(0, 2, 1)
        tau_v = -gp[:, 17][:, None] * np.stack([S[:, 0, 0], S[:, 1, 1], S[:, 2, 2], S[:, 0, 1], S[:, 0, 2],
                                                S[:, 1, 2]], axis=1)
        np.add.at(want, f, orc.element_stress_residual(t, m.coords[nodes], tau_m - tau_v))
    assert np.abs(rhs - want).max() <= 1e-12 * np.abs(want).max()


def test_stress_difference_conserves_momentum(orc, case):
    # per element sum_a grad N_a = 0, so the substituted stress adds nothing
    # to the total momentum: every kept element's difference sums to zero
    m = case.mesh
    p = _params(9, scale=0.02)
    r_inf, use, _ = CL.assemble(m, case.u, case.p, case.nu, case.vreman_c, p, _width_ref(m), tol=math.inf)
    r_0, _, _ = CL.assemble(m, case.u, case.p, case.nu, case.vreman_c, p, _width_ref(m), tol=0.0)
    d = r_inf - r_0
    assert use.all() and np.abs(d).max() > 0
    assert np.abs(d.sum(axis=0)).max() <= 1e-13 * np.abs(d).sum(axis=0).max()


def test_fallback_decision_flips_at_the_threshold(orc, case):
    # single-element meshes: the result is R_v + D when kept and R_v when not;
    # the choice flips between tol just above and just below |D| / |R_v|
    m = case.mesh
    p = _params(11, scale=0.02)
    dref = _width_ref(m)
    for t in (mg.TET04, mg.PYR05, mg.PEN06, mg.HEX08):
        e = int(np.where(m.types == t)[0][1])
        sub, fids = mg.submesh(m, [e])
        args = (sub, case.u[fids], case.p[fids], case.nu, case.vreman_c, p, dref)
        r_inf, _, eps = CL.assemble(*args, tol=math.inf)
        r_0, _, _ = CL.assemble(*args, tol=0.0)
        rv = orc.assemble(sub, case.u[fids], case.p[fids], case.nu, case.vreman_c)
        D = r_inf - rv
        e0 = float(eps[0])
        assert 0 < e0 < math.inf
        assert abs(np.linalg.norm(D) / np.linalg.norm(rv) - e0) <= 1e-12 * e0
        above, use_a, _ = CL.assemble(*args, tol=e0 * (1 + 1e-9))
        below, use_b, _ = CL.assemble(*args, tol=e0 * (1 - 1e-9))
        assert use_a[0] and not use_b[0]
        assert np.array_equal(above, r_inf) and np.array_equal(below, r_0)
        assert np.array_equal(r_0, rv)


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


def test_features_depend_on_the_direction_of_G_and_the_width_ratio():
    rng = np.random.default_rng(12)
    G = rng.standard_normal((20, 3, 3))
    d = rng.uniform(0.5, 2.0, 20)
    x1, g1 = omlp.features(G, d, 1.0)
    x2, g2 = omlp.features(2.5 * G, d, 1.0)
    assert np.allclose(x1, x2, rtol=0, atol=1e-15) and np.allclose(g2, 6.25 * g1, rtol=1e-14)
    assert np.allclose(np.linalg.norm(x1[:, :9], axis=1), 1.0, rtol=0, atol=1e-15)
    assert np.allclose(x1[:, :9].reshape(-1, 3, 3), G / np.sqrt(g1)[:, None, None], rtol=0, atol=1e-15)
    assert np.allclose(x1[:, 9], np.log(d), rtol=0, atol=1e-15)
    x3, _ = omlp.features(G, 2.0 * d, 2.0)
    assert np.allclose(x3[:, 9], x1[:, 9], rtol=0, atol=1e-15)
