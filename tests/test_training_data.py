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
