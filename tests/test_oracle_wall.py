"""Pins of the oracle's wall model (boundary assembly, Algorithm 1): limits of
the law of the wall, the inverse for the friction velocity, closed-form wall
forces on flat walls, and invariances.  None of them re-types the law."""
import math

import numpy as np
import pytest

import oracle
from paper_2005_05899_amd import meshgen as mg

KAPPA = 0.41


def test_law_viscous_sublayer_limit():
    # u+ = y+ to first order at the wall
    for yp in (1e-8, 1e-6, 1e-4):
        assert abs(oracle.wall_law(yp) / yp - 1.0) < 2e-3 * max(yp * 1e3, 1e-3)
    assert oracle.wall_law(0.0) == 0.0


def test_law_logarithmic_slope():
    # far from the wall the law is logarithmic with slope 1/kappa
    for a, b in ((1e5, 1e6), (1e6, 1e7)):
        slope = (oracle.wall_law(b) - oracle.wall_law(a)) / math.log(b / a)
        assert abs(slope - 1.0 / KAPPA) < 1e-4


def test_law_increasing():
    yp = np.logspace(-3, 6, 400)
    f = np.array([oracle.wall_law(v) for v in yp])
    assert (np.diff(f) > 0).all()


@pytest.mark.parametrize("y,nu", [(1e-3, 1e-5), (0.05, 1.5e-5), (0.3, 1e-3), (1e-4, 1e-2)])
def test_friction_velocity_inverts_the_law(y, nu):
    for ut in (1e-4, 1e-2, 0.05, 1.0, 3.0):
        U = ut * oracle.wall_law(y * ut / nu)
        got = oracle.friction_velocity(U, y, nu)
        assert abs(got - ut) <= 1e-12 * ut


def test_friction_velocity_zero_and_sublayer():
    assert oracle.friction_velocity(0.0, 0.1, 1e-5) == 0.0
    # deep in the sublayer the law is linear: u_tau = sqrt(nu U / y)
    U, y, nu = 1e-6, 1e-3, 1e-2
    assert abs(oracle.friction_velocity(U, y, nu) / math.sqrt(nu * U / y) - 1.0) < 1e-4


def _box(nx, ny, nz, lx=2.0, ly=1.5, lz=1.0):
    m = mg.uniform_hex_box((nx, ny, nz), (lx, ly, lz))
    return m


def test_uniform_flow_over_flat_hex_wall_closed_form():
    nx, ny, nz, lx, ly, lz = 4, 3, 2, 2.0, 1.5, 1.0
    m = _box(nx, ny, nz, lx, ly, lz)
    fo, fc, fe = mg.wall_faces(m)
    assert len(fe) == nx * ny and (np.diff(fo) == 4).all()
    U0, nu = 0.8, 1e-3
    u = np.tile([U0, 0.0, 0.0], (m.n_nodes, 1))
    out, y, U, ut = oracle.wall_assemble(m, u, nu, fo, fc, fe)
    h = lz / nz
    assert np.allclose(y, h / 2, rtol=0, atol=1e-15) and np.allclose(U, U0, rtol=1e-15)
    tau = ut[0] ** 2
    # total force on the wall: -tau * area along the flow
    F = out.sum(axis=0)
    assert abs(F[0] + tau * lx * ly) < 1e-13 and abs(F[1]) < 1e-15 and abs(F[2]) < 1e-15
    # nodal shares: a quarter of each touching face
    A = (lx / nx) * (ly / ny)
    z0 = np.where(m.coords[:, 2] == 0.0)[0]
    ix = np.round(m.coords[z0, 0] / (lx / nx)).astype(int)
    iy = np.round(m.coords[z0, 1] / (ly / ny)).astype(int)
    nfaces = (1 + ((ix > 0) & (ix < nx))) * (1 + ((iy > 0) & (iy < ny)))
    assert np.allclose(out[z0, 0], -tau * A * nfaces / 4, rtol=1e-13, atol=0)
    off = np.setdiff1d(np.arange(m.n_nodes), z0)
    assert (out[off] == 0).all()


def test_wall_normal_velocity_and_constant_shift_do_not_matter():
    m = _box(3, 3, 2)
    fo, fc, fe = mg.wall_faces(m)
    rng = np.random.default_rng(5)
    u = rng.uniform(-1, 1, (m.n_nodes, 3))
    base, *_ = oracle.wall_assemble(m, u, 1e-3, fo, fc, fe)
    u2 = u.copy()
    u2[:, 2] += 0.7  # normal to the wall z = 0
    moved, *_ = oracle.wall_assemble(m, u2, 1e-3, fo, fc, fe)
    assert np.allclose(moved, base, rtol=1e-13, atol=1e-16)


def test_force_opposes_tangential_flow():
    c = mg.small_hybrid_case(nx=4, ny=3, seed=7)
    fo, fc, fe = mg.wall_faces(c.mesh)
    out, y, U, ut = oracle.wall_assemble(c.mesh, c.u, c.nu, fo, fc, fe)
    assert (y > 0).all() and (ut > 0).all()
    # every face pushes against its own tangential velocity: rebuild per face
    tot = 0.0
    for f in range(len(fe)):
        one, *_ = oracle.wall_assemble(c.mesh, c.u, c.nu, fo[f:f + 2] - fo[f], fc[fo[f]:fo[f + 1]], fe[f:f + 1])
        e = fe[f]
        en = c.mesh.conn[c.mesh.conn_offsets[e]:c.mesh.conn_offsets[e + 1]]
        ue = c.u[en].mean(axis=0)
        ue[2] = 0.0  # wall z = 0: tangential part
        F = one.sum(axis=0)
        assert F @ ue < 0
        assert abs(np.linalg.norm(F) - ut[f] ** 2 * _face_area(c.mesh.coords[fc[fo[f]:fo[f + 1]]])) < 1e-12
        tot += F
    assert np.allclose(tot, out.sum(axis=0), rtol=1e-12, atol=1e-15)


def _face_area(x):
    # planar polygon area by the shoelace rule in the wall plane z = 0
    xs, ys = x[:, 0], x[:, 1]
    return 0.5 * abs(np.dot(xs, np.roll(ys, -1)) - np.dot(ys, np.roll(xs, -1)))


def test_rotation_equivariance():
    c = mg.small_hybrid_case(nx=3, ny=3, seed=3)
    fo, fc, fe = mg.wall_faces(c.mesh)
    out, *_ = oracle.wall_assemble(c.mesh, c.u, c.nu, fo, fc, fe)
    th = 0.7
    Q = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]]) @ \
        np.array([[1, 0, 0], [0, math.cos(0.3), -math.sin(0.3)], [0, math.sin(0.3), math.cos(0.3)]])
    m2 = mg.Mesh(c.mesh.coords @ Q.T, c.mesh.types, c.mesh.conn_offsets, c.mesh.conn, c.mesh.field_node,
                 c.mesh.n_field_nodes if c.mesh.field_node is not None else 0)
    out2, *_ = oracle.wall_assemble(m2, c.u @ Q.T, c.nu, fo, fc, fe)
    assert np.allclose(out2, out @ Q.T, rtol=0, atol=1e-13 * np.abs(out).max())


def test_nonplanar_quad_area_by_subdivision():
    # one hex whose bottom face is a twisted (non-planar) quad: the face weights
    # sum to the bilinear surface area, computed by fine triangulation
    x = np.array([[0, 0, 0], [1, 0, 0.0], [1, 1, 0.0], [0, 1, 0.0], [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], float)
    x[2, 2] = 0.2  # lift one corner of the bottom face
    m = mg.Mesh(x, np.array([mg.HEX08], np.uint8), np.array([0, 8], np.int64), np.arange(8, dtype=np.int32), None, 0)
    u = np.tile([1.0, 0.0, 0.0], (8, 1))
    fo, fc, fe = np.array([0, 4]), np.array([0, 1, 2, 3], np.int32), np.array([0])
    out, y, U, ut = oracle.wall_assemble(m, u, 1e-3, fo, fc, fe)
    n = 400
    s = np.linspace(-1, 1, n + 1)

    def P(a, b):
        w = np.array([(1 - a) * (1 - b), (1 + a) * (1 - b), (1 + a) * (1 + b), (1 - a) * (1 + b)]) / 4
        return w.T @ x[:4]
    area = 0.0
    for i in range(n):
        A = P(s[i], s[:-1]); B = P(s[i + 1], s[:-1]); C = P(s[i + 1], s[1:]); D = P(s[i], s[1:])
        area += 0.5 * np.linalg.norm(np.cross(B - A, C - A), axis=1).sum()
        area += 0.5 * np.linalg.norm(np.cross(C - A, D - A), axis=1).sum()
    # |F| = tau * sum of weights (t is constant on the face)
    assert abs(np.linalg.norm(out.sum(axis=0)) / ut[0] ** 2 - area) < 1e-5


def test_translation_invariance():
    c = mg.small_hybrid_case(nx=3, ny=2, seed=4)
    fo, fc, fe = mg.wall_faces(c.mesh)
    out, *_ = oracle.wall_assemble(c.mesh, c.u, c.nu, fo, fc, fe)
    m2 = mg.Mesh(c.mesh.coords + np.array([0.3, -1.1, 2.5]), c.mesh.types, c.mesh.conn_offsets, c.mesh.conn,
                 c.mesh.field_node, c.mesh.n_field_nodes if c.mesh.field_node is not None else 0)
    out2, *_ = oracle.wall_assemble(m2, c.u, c.nu, fo, fc, fe)
    assert np.allclose(out2, out, rtol=0, atol=1e-12 * np.abs(out).max())
