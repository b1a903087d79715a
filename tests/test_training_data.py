"""Pins of the learned closure's training data (`training.py`), on the CPU:
the box filter, the subgrid stress of the filtered field, the Gauss-point
gradients of the coarse finite-element field and the normalised samples.

* the (1/4, 1/2, 1/4) filter multiplies a periodic Fourier mode by
  cos^2(k h / 2) per direction, and keeps the periodic mean;
* a constant field has a zero subgrid stress (exactly for dyadic values);
* tau = filter(u u^T) - filter(u) filter(u)^T is a covariance under a positive
  kernel of unit sum, so it is positive semi-definite at every node;
* for u = (sin k y, 0, 0) tau_xx has a closed form at both filter levels and
  every other component vanishes;
* the Gauss-point values and gradients of a field linear in the grid indices
  are exact on cells away from the periodic seam;
* samples carry unit-norm gradient directions, the log width ratio of their
  level, and deviatoric targets scaled by Delta^2 |G|^2.

The module under test may be swapped for a planted-mistake copy through
LESASM_TRAINING_MODULE (used by the mutation tests)."""
import importlib.util
import math
import os

import numpy as np

from paper_2005_05899_amd import meshgen as mg  # noqa: F401  (the package, for the variant's relative imports)


def _load():
    path = os.environ.get("LESASM_TRAINING_MODULE")
    if not path:
        from paper_2005_05899_amd import training
        return training
    spec = importlib.util.spec_from_file_location("paper_2005_05899_amd.training_variant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


TR = _load()


def _grid(n):
    return np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")  # k (z), j (y), i (x)


def test_box_filter_on_a_fourier_mode():
    n = 16
    k, j, i = _grid(n)
    kx, ky, kz = 1, 3, 5
    th = 2 * math.pi / n
    f = np.cos(kx * th * i + 0.3) * np.sin(ky * th * j - 0.2) * np.cos(kz * th * k + 1.1)
    g = TR.box_filter(f[..., None])[..., 0]
    factor = (math.cos(kx * th / 2) * math.cos(ky * th / 2) * math.cos(kz * th / 2)) ** 2
    assert np.abs(g - factor * f).max() <= 1e-14


def test_box_filter_keeps_the_periodic_mean():
    f = np.random.default_rng(1).standard_normal((12, 12, 12, 3))
    g = TR.box_filter(f)
    assert np.abs(g.mean(axis=(0, 1, 2)) - f.mean(axis=(0, 1, 2))).max() <= 1e-15


def test_constant_field_has_no_subgrid_stress():
    u = np.broadcast_to(np.array([1.5, -0.75, 2.0]), (16, 16, 16, 3)).copy()
    for lev in (1, 2):
        ub, tau = TR.filter_level(u, lev)
        assert ub.shape == (16 >> lev,) * 3 + (3,)
        assert (tau == 0.0).all() and (ub == u[0, 0, 0]).all()
    u = np.broadcast_to(np.random.default_rng(2).standard_normal(3), (8, 8, 8, 3)).copy()
    _, tau = TR.filter_level(u, 1)
    assert np.abs(tau).max() <= 1e-15


def test_subgrid_stress_is_positive_semidefinite():
    u = np.random.default_rng(3).standard_normal((16, 16, 16, 3))
    for lev in (1, 2):
        _, t = TR.filter_level(u, lev)
        T = np.stack([np.stack([t[..., 0], t[..., 3], t[..., 4]], -1),
                      np.stack([t[..., 3], t[..., 1], t[..., 5]], -1),
                      np.stack([t[..., 4], t[..., 5], t[..., 2]], -1)], -2)
        ev = np.linalg.eigvalsh(T.reshape(-1, 3, 3))
        assert ev.min() >= -1e-14 * ev.max()
        assert ev.max() > 0


def test_shear_mode_stress_closed_form():
    # u = (sin k y, 0, 0): filtering along y multiplies sin by c1 = cos^2(k h/2)
    # and cos 2ky by c2 = cos^2(k h); at level 2 the second pass has width 4h
    n, kk = 32, 3
    h = 2 * math.pi / n
    _, j, _ = _grid(n)
    y = j * h
    u = np.zeros((n, n, n, 3))
    u[..., 0] = np.sin(kk * y)
    for lev in (1, 2):
        ub, tau = TR.filter_level(u, lev)
        a = b = 1.0
        for L in range(lev):
            hl = h * 2 ** L
            a *= math.cos(kk * hl / 2) ** 2
            b *= math.cos(kk * hl) ** 2
        yc = y[:: 1 << lev, :: 1 << lev, :: 1 << lev]
        want = 0.5 - 0.5 * b * np.cos(2 * kk * yc) - a * a * np.sin(kk * yc) ** 2
        assert np.abs(tau[..., 0] - want).max() <= 1e-14
        assert np.abs(tau[..., 1:]).max() <= 1e-15
        assert np.abs(ub[..., 0] - a * np.sin(kk * yc)).max() <= 1e-14


def test_gauss_point_values_and_gradients_of_a_linear_field():
    m, h = 6, 0.25
    k, j, i = _grid(m)
    a, b, c, d = 0.7, -1.3, 2.1, 0.4
    f = (a * i + b * j + c * k + d)[..., None]
    vals, grads = TR.gauss_point_fields(f, h)
    g1 = TR.GAUSS_1D
    pts = [(gz, gy, gx) for gz in g1 for gy in g1 for gx in g1]
    # cells whose 8 corners avoid the periodic seam: index < m - 1 in every axis
    inner = ((k < m - 1) & (j < m - 1) & (i < m - 1)).reshape(-1)
    for q, (gz, gy, gx) in enumerate(pts):
        v = vals[q * m ** 3:(q + 1) * m ** 3, 0]
        want = a * (i + gx) + b * (j + gy) + c * (k + gz) + d
        assert np.abs(v[inner] - want.reshape(-1)[inner]).max() <= 1e-13
        gq = grads[q * m ** 3:(q + 1) * m ** 3, 0]
        assert np.abs(gq[inner] - np.array([a, b, c]) / h).max() <= 1e-13
    assert abs(g1[0] + g1[1] - 1.0) < 1e-15 and abs((g1[1] - g1[0]) - 1 / math.sqrt(3.0)) < 1e-15


def test_samples_are_normalised_and_deviatoric():
    n = 16
    rng = np.random.default_rng(4)
    k, j, i = _grid(n)
    th = 2 * math.pi / n
    u = np.stack([np.sin(th * j + 0.1) + 0.3 * np.cos(2 * th * k), np.cos(th * k) * np.sin(th * i),
                  np.sin(3 * th * i - 0.5)], -1) + 0.05 * rng.standard_normal((n, n, n, 3))
    data, dref = TR.samples_from_snapshot(u, levels=(1, 2), length=2 * math.pi)
    assert abs(dref - 2 * math.pi / (n // 2)) < 1e-15
    x, t, G, tau, delta = (data[q] for q in ("x", "t", "G", "tau", "delta"))
    g2 = (G.reshape(-1, 9) ** 2).sum(axis=1)
    assert np.allclose(x[:, :9], (G.reshape(-1, 9) / np.sqrt(g2)[:, None]).astype(np.float32), rtol=0, atol=1e-7)
    assert set(np.round(np.unique(delta), 12)) == {round(2 * math.pi / 8, 12), round(2 * math.pi / 4, 12)}
    assert np.allclose(x[:, 9], np.log(delta / dref), rtol=0, atol=1e-7)
    assert np.abs(tau[:, :3].sum(axis=1)).max() <= 1e-14 * np.abs(tau).max()
    assert np.allclose(t, tau / (delta ** 2 * g2)[:, None], rtol=1e-6, atol=1e-7 * np.abs(t).max())


# ---- samples on hybrid elements -----------------------------------------------------

def test_gauss_jacobi_rule_is_exact_to_degree_three():
    c, w = TR._gauss_jacobi2()
    for k in range(4):
        exact = 2.0 / ((k + 1) * (k + 2) * (k + 3))  # int_0^1 c^k (1 - c)^2 dc
        assert abs((w * c ** k).sum() - exact) <= 1e-15, k
    assert ((c > 0) & (c < 1)).all() and (w > 0).all()


def test_reference_elements_reproduce_linear_fields():
    # partition of unity, rule weights summing to the reference volume, and
    # linear completeness: sum_a N_a xi_a = xi and sum_a xi_a (x) dN_a = I at
    # every Gauss point (node coordinates written out per type)
    nodes = {
        mg.TET04: [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]],
        mg.PYR05: [[-1, -1, 0], [1, -1, 0], [1, 1, 0], [-1, 1, 0], [0, 0, 1]],
        mg.PEN06: [[0, 0, -1], [1, 0, -1], [0, 1, -1], [0, 0, 1], [1, 0, 1], [0, 1, 1]],
        mg.HEX08: [[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1], [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]],
    }
    vol = {mg.TET04: 1 / 6, mg.PYR05: 4 / 3, mg.PEN06: 1.0, mg.HEX08: 8.0}
    for t, xn in nodes.items():
        xn = np.array(xn, float)
        xi, w = TR.reference_rule(t)
        N, dN = TR.reference_shape(t, xi)
        assert abs(w.sum() - vol[t]) <= 1e-15, t
        assert np.abs(N.sum(axis=1) - 1).max() <= 1e-15, t
        assert np.abs(N @ xn - xi).max() <= 1e-15, t
        assert np.abs(np.einsum("ak,gaj->gkj", xn, dN) - np.eye(3)).max() <= 1e-14, t
        # each node's function is 1 there and 0 at the other nodes (at the nodes,
        # the pyramid apex excepted: its base functions are singular there)
        pts = xn if t != mg.PYR05 else xn[:4]
        Nn, _ = TR.reference_shape(t, pts)
        assert np.abs(Nn - np.eye(len(xn))[:len(pts)]).max() <= 1e-15, t


def test_hybrid_samples_of_a_linear_field():
    # a velocity linear in x on the grid: every Gauss point of every element
    # away from the periodic seam sees G = A (isoparametric completeness on the
    # perturbed, graded elements); the widths' cubes add up to the box volume;
    # a constant stress field gives its deviatoric part everywhere
    m, L = 12, 2 * math.pi
    h = L / m
    rng = np.random.default_rng(3)
    A = rng.standard_normal((3, 3))
    k, j, i = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    x = np.stack([i * h, j * h, k * h], axis=-1)
    ub = x @ A.T + rng.standard_normal(3)
    t6 = rng.standard_normal(6)
    tau = np.broadcast_to(t6, (m, m, m, 6)).copy()
    raw = TR.hybrid_element_samples(ub, tau, L, seed=5)
    n = len(raw["delta"])
    assert raw["G"].shape == (n, 3, 3) and raw["tau"].shape == (n, 6) and raw["etype"].shape == (n,)
    assert set(np.unique(raw["etype"])) == {mg.TET04, mg.PYR05, mg.PEN06, mg.HEX08}
    dev = t6.copy()
    dev[:3] -= t6[:3].mean()
    assert np.abs(raw["tau"] - dev).max() <= 1e-14
    # elements away from the seam: rebuild the same box and take the elements
    # whose nodes all lie below L - h in x, y and z (their Gauss points follow
    # the per-type order of the sampler)
    mesh = mg.hybrid_box(m, m, mg.hybrid_layers(m * m, int(m ** 3 / (0.4 / 6 + 0.4 / 2 + 0.05 / 6 + 0.15))),
                         length=(L,) * 3, seed=5)
    o, checked, vol = 0, 0, 0.0
    for t in (mg.TET04, mg.PYR05, mg.PEN06, mg.HEX08):
        idx = np.flatnonzero(mesh.types == t)
        ng = len(TR.reference_rule(t)[1])
        conn = mesh.conn[mesh.conn_offsets[idx][:, None] + np.arange(mg.NNODE[t])[None, :]]
        inner = (mesh.coords[conn] < L - h - 1e-9).all(axis=(1, 2))
        G = raw["G"][o:o + ng * len(idx)].reshape(len(idx), ng, 3, 3)
        d = raw["delta"][o:o + ng * len(idx)].reshape(len(idx), ng)
        assert np.abs(G[inner] - A).max() <= 1e-11 * np.abs(A).max(), t
        vol += (d[:, 0] ** 3).sum()
        checked += int(inner.sum())
        o += ng * len(idx)
    assert o == n and checked > 0.3 * mesh.n_elems
    # the generator's one non-conforming interface plane (bilinear quad faces
    # against pairs of triangles, perturbed) leaves slivers: 1e-5 of the volume
    assert abs(vol - L ** 3) <= 1e-4 * L ** 3


def test_hybrid_network_samples_are_normalised():
    m, L = 8, 2 * math.pi
    rng = np.random.default_rng(4)
    ub = rng.standard_normal((m, m, m, 3))
    tau = rng.standard_normal((m, m, m, 6))
    raw = TR.hybrid_element_samples(ub, tau, L, seed=6)
    dref = 0.7 * L / m
    s = TR.network_samples(raw, dref)
    g2 = (s["G"].reshape(-1, 9) ** 2).sum(axis=1)
    assert np.abs(np.linalg.norm(s["x"][:, :9], axis=1) - 1).max() <= 1e-6
    assert np.allclose(s["x"][:, 9], np.log(s["delta"] / dref), atol=1e-6)
    assert np.allclose(s["t"], s["tau"] / (s["delta"] ** 2 * g2)[:, None], rtol=1e-6)
    assert np.abs(s["t"][:, :3].sum(axis=1)).max() <= 1e-5 * np.abs(s["t"]).max()
    # tetrahedra of a cube cell are narrower than the hexahedra: widths ~0.55 h against ~h
    w_tet = np.median(s["delta"][s["etype"] == mg.TET04])
    w_hex = np.median(s["delta"][s["etype"] == mg.HEX08])
    assert 0.45 < w_tet / (L / m) < 0.65 and 0.85 < w_hex / (L / m) < 1.15


def test_gathered_samples_weights_and_levels():
    # both sample kinds and both filter levels are present; the drawing weight
    # is (Delta / level width)^4 with the level width the geometric mean of
    # that level's hybrid-element widths, and the width input is relative to
    # the level-1 width
    rng = np.random.default_rng(8)
    u = rng.standard_normal((16, 16, 16, 3))
    d, dref = TR.gathered_samples([u], seed0=3)
    n = len(d["x"])
    assert all(len(d[k]) == n for k in ("t", "G", "tau", "delta", "etype", "level", "hybrid", "w"))
    assert d["hybrid"].any() and (~d["hybrid"]).any()
    assert set(np.unique(d["level"])) == {1, 2}
    for lev in (1, 2):
        hy = d["hybrid"] & (d["level"] == lev)
        assert abs(np.log(d["w"][hy]).mean() / 4) <= 1e-12, lev
    h1 = 2 * math.pi / 8
    assert np.allclose(d["delta"][~d["hybrid"] & (d["level"] == 1)], h1)
    assert np.allclose(d["delta"][~d["hybrid"] & (d["level"] == 2)], 2 * h1)
    assert abs(np.log(d["delta"][d["hybrid"] & (d["level"] == 1)] / dref).mean()) <= 1e-12
    assert np.allclose(d["x"][:, 9], np.log(d["delta"] / dref), atol=1e-6)
