"""Mesh-level pins of the oracle: invariants, special cases, consistency.

* constant fields give a zero residual; nu_t is exactly 0 where G = 0
* linear fields are reproduced exactly on distorted hybrid elements
* periodic cube: EMAC conserves discrete kinetic energy and every term
  conserves momentum (the literal convective form does not conserve energy)
* per element the viscous and subgrid residuals sum to zero and dissipate
* Taylor-Green: rhs / M_L converges to the continuous operator at O(h^2)
* patch test on a uniform hex grid; rotation equivariance; scatter bookkeeping
"""
import math

import numpy as np
import pytest

from paper_2005_05899_amd import meshgen as mg


@pytest.fixture(scope="module")
def hyb():
    return mg.small_hybrid_case(nx=4, ny=3, layers=[(mg.PEN06, 2), (mg.TET04, 2), (mg.PYR05, 1), (mg.HEX08, 2)], seed=3)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_constant_fields_give_zero_residual(orc, hyb):
    m = hyb.mesh
    u = np.tile([0.3, -1.2, 2.0], (m.n_field_nodes, 1))
    p = np.full(m.n_field_nodes, 4.5)
    rhs = orc.assemble(m, u, p, nu=0.1, c=0.1)
    assert np.abs(rhs).max() < 1e-14 * 2.0
    # nu_t is rounding-small for constant u and exactly zero where G = 0 exactly
    zero = np.zeros_like(u)
    for e in range(m.n_elems):
        nodes = m.element_nodes(e)
        _, gp, _ = orc.element_residual(int(m.types[e]), m.coords[nodes], u[nodes], p[nodes], 0.1, 0.1)
        assert np.abs(gp[:, 17]).max() < 1e-15
        _, gp0, _ = orc.element_residual(int(m.types[e]), m.coords[nodes], zero[nodes], p[nodes], 0.1, 0.1)
        assert (gp0[:, 17] == 0.0).all() and (gp0[:, 5:14] == 0.0).all()


def test_linear_fields_reproduced_on_distorted_elements(orc, hyb):
    m = hyb.mesh
    rng = np.random.default_rng(1)
    A, b, g = rng.standard_normal((3, 3)), rng.standard_normal(3), rng.standard_normal(3)
    u = m.coords @ A.T + b
    p = m.coords @ g + 0.3
    for e in range(m.n_elems):
        nodes = m.element_nodes(e)
        _, gp, _ = orc.element_residual(int(m.types[e]), m.coords[nodes], u[nodes], p[nodes], 0.1, 0.1)
        assert np.abs(gp[:, 5:14] - A.reshape(1, 9)).max() < 1e-12, e
        assert np.abs(gp[:, 14:17] - g).max() < 1e-12, e


def test_lumped_mass_and_filter_width(orc, hyb):
    m = hyb.mesh
    M = orc.lumped_mass(m)
    assert (M > 0).all()
    # the only geometric gap is the non-conforming tet/pyramid plane
    assert abs(M.sum() - (2 * math.pi) ** 3) < 1e-3 * (2 * math.pi) ** 3
    d = orc.filter_width(m)
    vols = np.array([orc.element_volume(int(m.types[e]), m.coords[m.element_nodes(e)]) for e in range(m.n_elems)])
    assert np.abs(d ** 3 - vols).max() < 1e-13 * vols.max()
    cube = mg.periodic_hex_cube(8)
    Mc = orc.lumped_mass(cube)
    assert np.abs(Mc - (2 * math.pi / 8) ** 3).max() < 1e-13


@pytest.fixture(scope="module")
def tg16():
    return mg.periodic_tg_case(16)


def test_periodic_momentum_conservation(orc, tg16):
    c = tg16
    rhs = orc.assemble(c.mesh, c.u, c.p, c.nu, c.vreman_c)
    scale = np.abs(rhs).sum(axis=0)
    assert (np.abs(rhs.sum(axis=0)) < 1e-13 * scale).all()
    for term in (orc.TERM_CONV, orc.TERM_PRES, orc.TERM_VISC, orc.TERM_SGS):
        r = orc.assemble(c.mesh, c.u, c.p, 0.3, 0.1, terms=term)
        assert (np.abs(r.sum(axis=0)) < 1e-13 * np.abs(r).sum(axis=0) + 1e-300).all(), term


def test_periodic_emac_energy_conservation(orc, tg16):
    """sum_a u_a . R_a^conv = -int div(u |u|^2) = 0, integrated exactly by the
    2x2x2 rule on the uniform cube; the noisy field is not solenoidal, so the
    literal form (grad |u|^2/2 subtracted) leaves -1/2 int (div u)|u|^2."""
    c = tg16
    noisy = c.u + mg.uniform_noise(c.u.shape, 0.2, 9)
    r = orc.assemble(c.mesh, noisy, None, 0.0, 0.0, terms=orc.TERM_CONV)
    e = (noisy * r).sum()
    scale = np.abs(noisy * r).sum()
    assert abs(e) < 1e-14 * scale
    r_lit = orc.assemble(c.mesh, noisy, None, 0.0, 0.0, terms=orc.TERM_CONV | orc.TERM_LITERAL)
    assert abs((noisy * r_lit).sum()) > 1e-6 * scale


def test_per_element_viscous_sums_and_dissipation(orc, hyb):
    m = hyb.mesh
    rng = np.random.default_rng(2)
    u = rng.standard_normal((m.n_field_nodes, 3))
    for e in range(m.n_elems):
        nodes = m.element_nodes(e)
        t = int(m.types[e])
        Rv, _, _ = orc.element_residual(t, m.coords[nodes], u[nodes], None, 0.7, 0.1, terms=orc.TERM_VISC)
        Rs, _, _ = orc.element_residual(t, m.coords[nodes], u[nodes], None, 0.7, 0.1, terms=orc.TERM_SGS)
        sc = np.abs(Rv).max()
        assert np.abs(Rv.sum(axis=0)).max() < 1e-13 * sc
        assert np.abs(Rs.sum(axis=0)).max() < 1e-13 * max(np.abs(Rs).max(), 1e-300)
        assert (u[nodes] * (Rv + Rs)).sum() <= 1e-14 * sc


def test_distorted_periodic_hex_momentum_balance(orc):
    """Sum over nodes of every term vanishes on a perturbed periodic hex mesh
    (Piola identity: the divergence-form integrands are exact per element)."""
    cube = mg.periodic_hex_cube(6)
    rng = np.random.default_rng(4)
    h = 2 * math.pi / 6
    # perturb field nodes consistently so periodic copies move together
    shift = rng.uniform(-0.15, 0.15, (cube.n_field_nodes, 3)) * h
    cube.coords = cube.coords + shift[cube.field_node]
    u = rng.standard_normal((cube.n_field_nodes, 3))
    p = rng.standard_normal(cube.n_field_nodes)
    for term in (orc.TERM_VISC, orc.TERM_SGS, orc.TERM_PRES):
        r = orc.assemble(cube, u, p, 0.2, 0.1, terms=term)
        assert np.abs(r.sum(axis=0)).max() < 1e-12 * np.abs(r).sum(axis=0).max(), term


def tg_operator(x, nu):
    """Continuous -(C + grad p) + nu lap u for Taylor-Green with p = p_TG - |u|^2/2."""
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    return np.stack([
        -np.sin(2 * X) * np.cos(2 * Z) / 8 - 3 * nu * np.sin(X) * np.cos(Y) * np.cos(Z),
        -np.sin(2 * Y) * np.cos(2 * Z) / 8 + 3 * nu * np.cos(X) * np.sin(Y) * np.cos(Z),
        (np.cos(2 * X) + np.cos(2 * Y)) * np.sin(2 * Z) / 8,
    ], axis=1)


@pytest.mark.parametrize("nu", [0.0, 1.0])
def test_taylor_green_second_order_consistency(orc, nu):
    errs = []
    for n in (16, 32, 64):
        c = mg.periodic_tg_case(n, noise=0.0)
        rhs = orc.assemble(c.mesh, c.u, c.p, nu, 0.0)
        M = orc.lumped_mass(c.mesh)
        f = tg_operator(c.mesh.field_coords(), nu)
        errs.append(np.abs(rhs / M[:, None] - f).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 0.006 * (1 + 3 * nu)
    assert rates[0] > 1.8 and rates[1] > 1.93, (errs, rates)


def test_patch_test_uniform_hex(orc):
    """Linear u on a uniform grid: interior viscous residual is 0 and the
    convective one is -h^3 C(x_a) with C = (A + A^T + tr A I) u(x_a)."""
    n, L = 5, 1.0
    m = mg.uniform_hex_box((n, n, n), (L, L, L))
    h = L / n
    rng = np.random.default_rng(5)
    A, b = rng.standard_normal((3, 3)), rng.standard_normal(3)
    u = m.coords @ A.T + b
    interior = np.all((m.coords > 0.5 * h) & (m.coords < L - 0.5 * h), axis=1)
    rv = orc.assemble(m, u, None, 1.0, 0.0, terms=orc.TERM_VISC)
    assert np.abs(rv[interior]).max() < 1e-14 * np.abs(rv).max()
    rc = orc.assemble(m, u, None, 0.0, 0.0, terms=orc.TERM_CONV)
    Mm = A + A.T + np.trace(A) * np.eye(3)
    expect = -(h ** 3) * (u[interior] @ Mm.T)
    assert rel(rc[interior], expect) < 1e-13


def test_rotation_equivariance(orc, hyb):
    """Rotating mesh and fields rotates the residual: R(Qx, Qu) = Q R(x, u)."""
    m = hyb.mesh
    rng = np.random.default_rng(6)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    u = hyb.u
    r0 = orc.assemble(m, u, hyb.p, hyb.nu, 0.1)

    class Rot:
        pass
    mr = Rot()
    mr.coords = m.coords @ Q.T + np.array([1.0, -2.0, 0.5])
    mr.types, mr.conn_offsets, mr.conn = m.types, m.conn_offsets, m.conn
    mr.field_node, mr.n_field_nodes = m.field_node, m.n_field_nodes
    r1 = orc.assemble(mr, u @ Q.T, hyb.p, hyb.nu, 0.1)
    assert rel(r1, r0 @ Q.T) < 1e-12


def test_scatter_matches_per_element_sum(orc, hyb):
    """The assembled rhs equals a plain Python scatter of per-element residuals."""
    m = hyb.mesh
    rhs = orc.assemble(m, hyb.u, hyb.p, hyb.nu, 0.1)
    acc = np.zeros_like(rhs)
    for e in range(m.n_elems):
        nodes = m.element_nodes(e)
        R, _, _ = orc.element_residual(int(m.types[e]), m.coords[nodes], hyb.u[nodes], hyb.p[nodes], hyb.nu, 0.1)
        np.add.at(acc, nodes, R)
    assert rel(rhs, acc) < 1e-14


def test_periodic_map_equals_folded_assembly(orc):
    """Assembling on the periodic cube equals assembling on the unfolded
    (n+1)^3 grid with copied fields and summing periodic images."""
    c = mg.periodic_tg_case(4)
    m = c.mesh
    r_per = orc.assemble(m, c.u, c.p, 0.3, 0.1)

    class Open:
        pass
    o = Open()
    o.coords, o.types, o.conn_offsets, o.conn = m.coords, m.types, m.conn_offsets, m.conn
    o.field_node, o.n_field_nodes = None, m.n_nodes
    r_open = orc.assemble(o, c.u[m.field_node], c.p[m.field_node], 0.3, 0.1)
    folded = np.zeros_like(r_per)
    np.add.at(folded, m.field_node, r_open)
    assert rel(r_per, folded) < 1e-14


def test_error_paths(orc):
    from oracle.oracle import OracleError
    m = mg.uniform_hex_box((2, 1, 1))
    u = np.zeros((m.n_nodes, 3))
    bad = mg.Mesh(m.coords, m.types, m.conn_offsets, m.conn.copy())
    # invert element 1 by swapping bottom and top faces
    o = bad.conn_offsets[1]
    bad.conn[o:o + 8] = np.concatenate([bad.conn[o + 4:o + 8], bad.conn[o:o + 4]])
    with pytest.raises(OracleError) as ei:
        orc.assemble(bad, u)
    assert ei.value.code == -2 and ei.value.element == 1
    oob = mg.Mesh(m.coords, m.types, m.conn_offsets, m.conn.copy())
    oob.conn[3] = m.n_nodes
    with pytest.raises(OracleError) as ei:
        orc.assemble(oob, u)
    assert ei.value.code == -1 and ei.value.element == 0
    bt = mg.Mesh(m.coords, np.array([8, 7], np.uint8), m.conn_offsets, m.conn)
    with pytest.raises(OracleError):
        orc.assemble(bt, u)
