"""Pins of the oracle's SFC partitioner and correction-coefficient balancing
(Section "Mesh partitioning and load balancing"): properties that any Hilbert
curve has, closed-form partitions of uniform grids, the weight bound of the
one-dimensional split, and the regression's exactness on affine data and its
agreement with numpy's least-squares fit.  None of them re-types the oracle.

The module under test may be swapped for a planted-mistake copy through
LESASM_PARTITION_ORACLE (used by the mutation tests)."""
import importlib.util
import itertools
import os

import numpy as np
import pytest

from paper_2005_05899_amd import meshgen as mg


def _load():
    path = os.environ.get("LESASM_PARTITION_ORACLE")
    if not path:
        from oracle import partition
        return partition
    spec = importlib.util.spec_from_file_location("partition_variant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


P = _load()


def _cells(level):
    n = 1 << level
    c = np.array(list(itertools.product(range(n), repeat=3)), np.int64)
    return c, P.hilbert_index(c[:, 0], c[:, 1], c[:, 2], level)


@pytest.mark.parametrize("level", [1, 2, 3, 4])
def test_hilbert_is_a_bijection(level):
    _, h = _cells(level)
    assert np.array_equal(np.sort(h), np.arange(8 ** level))


@pytest.mark.parametrize("level", [1, 2, 3, 4])
def test_hilbert_steps_to_a_face_neighbour(level):
    c, h = _cells(level)
    path = c[np.argsort(h)]
    step = np.abs(np.diff(path, axis=0)).sum(axis=1)
    assert (step == 1).all()


@pytest.mark.parametrize("level", [2, 3, 4])
def test_hilbert_blocks_fill_aligned_cubes(level):
    c, h = _cells(level)
    path = c[np.argsort(h)]
    for m in range(1, level):
        side = 1 << m
        for blk in path.reshape(-1, side ** 3, 3):
            lo, hi = blk.min(axis=0), blk.max(axis=0)
            assert (hi - lo == side - 1).all() and (lo % side == 0).all()


def test_hilbert_starts_at_the_origin():
    for level in (1, 3, 5):
        assert int(P.hilbert_index(0, 0, 0, level)) == 0


def test_bins_of_box_corners_and_flat_axes():
    c = np.array([[0.0, 1.0, 5.0], [1.0, 1.0, 5.0], [0.5, 1.0, 5.0], [0.999999, 1.0, 5.0]])
    b = P.bins(c, 3)
    assert b[:, 0].tolist() == [0, 7, 4, 7] and (b[:, 1:] == 0).all()


def test_bins_scale_and_translation_invariant():
    rng = np.random.default_rng(3)
    c = rng.uniform(-1, 1, (500, 3))
    assert np.array_equal(P.bins(c, 5), P.bins(2.0 * c + 8.0, 5))


def _uniform(level):
    n = 1 << level
    m = mg.uniform_hex_box((n, n, n), (1.0, 1.0, 1.0))
    return m, n


@pytest.mark.parametrize("parts", [8, 64])
def test_uniform_grid_splits_into_aligned_sub_cubes(parts):
    level = 3
    m, n = _uniform(level)
    cen, w = P.element_centroids(m.coords, m.conn_offsets, m.conn)
    part, key, _ = P.sfc_partition(cen, w, parts, level=level)
    cell = np.floor(cen * n).astype(int)
    side = round(n / round(parts ** (1 / 3)))
    for i in range(parts):
        sel = cell[part == i]
        assert len(sel) == n ** 3 // parts
        lo, hi = sel.min(axis=0), sel.max(axis=0)
        assert (hi - lo == side - 1).all() and (lo % side == 0).all()


def test_centroids_and_gauss_point_weights():
    import oracle
    c = mg.small_hybrid_case(nx=3, ny=3, seed=2)
    m = c.mesh
    cen, w = P.element_centroids(m.coords, m.conn_offsets, m.conn)
    for e in range(m.n_elems):
        nodes = m.conn[m.conn_offsets[e]:m.conn_offsets[e + 1]]
        # the mean is the point that makes the node offsets sum to zero
        assert np.abs((m.coords[nodes] - cen[e]).sum(axis=0)).max() < 1e-13
        assert w[e] == oracle.ngauss(int(m.types[e]))
    assert set(np.unique(m.types)) == {mg.TET04, mg.PYR05, mg.PEN06, mg.HEX08}


def _random_case(n=3000, seed=1):
    rng = np.random.default_rng(seed)
    cen = rng.normal(size=(n, 3)) * [1.0, 2.0, 0.5]
    w = rng.integers(1, 9, n)
    return cen, w


@pytest.mark.parametrize("parts,level", [(5, 3), (7, 4), (16, 2), (3, 5)])
def test_split_points_within_half_a_bin_of_the_targets(parts, level):
    cen, w = _random_case()
    lam = np.random.default_rng(parts).uniform(0.5, 1.5, parts)
    lam *= parts / lam.sum()
    part, key, binw = P.sfc_partition(cen, w, parts, lam=lam, level=level)
    W = int(w.sum())
    assert binw.sum() == W
    cum = np.cumsum([w[part == i].sum() for i in range(parts)])
    goal = np.cumsum(lam) * W / parts
    assert np.all(np.abs(cum[:-1] - goal[:-1]) <= binw.max() / 2 + 1e-9)
    assert cum[-1] == W


def test_parts_are_contiguous_along_the_curve():
    cen, w = _random_case(seed=4)
    part, key, _ = P.sfc_partition(cen, w, 9, level=4)
    order = np.argsort(key, kind="stable")
    assert (np.diff(part[order]) >= 0).all()
    # elements of one bin share a part
    for k in np.unique(key)[:200]:
        assert len(np.unique(part[key == k])) == 1


def test_zero_coefficient_gives_an_empty_part_and_doubled_neighbour():
    cen, w = _random_case(n=20000, seed=5)
    part, _, binw = P.sfc_partition(cen, w, 4, lam=[2.0, 0.0, 1.0, 1.0], level=5)
    W = w.sum()
    assert (part == 1).sum() == 0
    assert abs(w[part == 0].sum() - W / 2) <= binw.max()


def test_permutation_invariance_and_trivial_cases():
    cen, w = _random_case(seed=6)
    part, _, _ = P.sfc_partition(cen, w, 6, level=4)
    perm = np.random.default_rng(0).permutation(len(w))
    part2, _, _ = P.sfc_partition(cen[perm], w[perm], 6, level=4)
    assert np.array_equal(part2, part[perm])
    one, _, _ = P.sfc_partition(cen, w, 1, level=4)
    assert (one == 0).all()
    empty, _, _ = P.sfc_partition(np.zeros((0, 3)), None, 4, level=3)
    assert len(empty) == 0


# ---- balancing ---------------------------------------------------------------

def _times(lam, density):
    """Times of parts laid on a work continuum [0, P] with the given
    cumulative work function R: part i covers [Lambda_{i-1}, Lambda_i]."""
    edges = np.concatenate([[0.0], np.cumsum(lam)])
    return np.diff(density(edges))


def test_equal_times_leave_the_coefficients_unchanged():
    lam = np.array([0.7, 1.3, 1.1, 0.9])
    new = P.balance_update([lam], [[2.0, 2.0, 2.0, 2.0]])
    assert np.allclose(new, lam, rtol=0, atol=1e-14)


def test_affine_response_is_balanced_after_two_observations():
    Pn = 6
    R = lambda s: np.where(s < 1.0, 2.0 * s, s + 1.0)  # noqa: E731  work density 2 then 1
    lam0 = np.ones(Pn)
    lam1 = np.array([1.2, 0.9, 1.0, 1.1, 0.7, 1.1])  # every split moves
    t0, t1 = _times(lam0, R), _times(lam1, R)
    for growth in (1.0, 1.5):
        new = P.balance_update([lam0, lam1], [t0, t1], growth=growth)
        assert abs(new.sum() - Pn) < 1e-13 and (new >= 0).all()
        t = _times(new, R)
        ups = np.cumsum(t) / t.mean()
        # splitting points 2 .. P-1 lie on the affine branch: exactly balanced
        assert np.allclose(ups[1:-1], np.arange(2, Pn), rtol=0, atol=1e-12)


def test_regression_matches_numpy_least_squares():
    rng = np.random.default_rng(8)
    Pn, K = 5, 4
    R = lambda s: s + 0.2 * s ** 2  # noqa: E731
    lams = rng.uniform(0.6, 1.4, (K, Pn))
    lams *= Pn / lams.sum(axis=1, keepdims=True)
    ts = np.array([_times(lam, R) for lam in lams]) * rng.uniform(0.97, 1.03, (K, Pn))
    Lam = np.cumsum(lams, axis=1)
    Ups = np.cumsum(ts, axis=1) / ts.mean(axis=1, keepdims=True)
    for growth in (1.0, 1.5):
        new = P.balance_update(lams, ts, growth=growth)
        want = [0.0]
        for i in range(1, Pn):
            beta, alpha = np.polyfit(Lam[:, i - 1], Ups[:, i - 1], 1, w=np.sqrt(growth ** np.arange(K)))
            assert beta > 0
            want.append((i - alpha) / beta)
        want.append(Pn)
        assert (np.diff(want) > 0).all()  # no clamping on this data
        got = np.concatenate([[0.0], np.cumsum(new)])
        assert np.allclose(got, want, rtol=1e-12, atol=1e-12)


def _origin_line(lam, t):
    """Splitting points of the fallback: each on the line through the origin
    and its newest observation, Lambda_i = i Lambda_i^K / Upsilon_i^K (then
    clamped non-decreasing into [0, P])."""
    Pn = len(lam)
    Lam, Ups = np.cumsum(lam), np.cumsum(t) / np.mean(t)
    pts = [0.0] + [i * Lam[i - 1] / Ups[i - 1] for i in range(1, Pn)] + [float(Pn)]
    for i in range(1, Pn):
        pts[i] = min(max(pts[i], pts[i - 1]), Pn)
    return np.diff(pts)


def test_degenerate_fits_fall_back_to_the_origin_line():
    """Reading A27: one observation, a spread of Lambda_i below 1e-12 P, or a
    non-increasing fit use the line through the origin and the newest point."""
    lam = np.array([0.8, 1.3, 0.9, 1.0])
    t1 = np.array([1.0, 2.0, 1.2, 1.1])
    t2 = np.array([1.1, 1.9, 1.3, 1.0])
    want = _origin_line(lam, t2)
    # one observation
    assert np.allclose(P.balance_update([lam], [t2]), want, rtol=0, atol=1e-14)
    # two observations with the same coefficients (no spread), and a spread of
    # 1e-15 P, below the threshold
    for eps in (0.0, 1e-15):
        lam2 = lam + eps * np.array([1.0, -1.0, 1.0, -1.0])
        got = P.balance_update([lam, lam2], [t1, t2])
        assert np.allclose(got, _origin_line(lam2, t2), rtol=0, atol=1e-12)
    # a spread above the threshold, but times that fall as the split grows:
    # every fitted slope is negative, so the fallback again
    lamb = np.array([1.0, 1.0, 1.0, 1.0])
    lama = lamb + 0.1 * np.array([1.0, -1.0, 1.0, -1.0])
    ta = np.array([1.0, 1.0, 1.0, 1.0])
    tb = np.array([1.3, 0.7, 1.3, 0.7])  # Upsilon_1 rises while Lambda_1 falls
    got = P.balance_update([lama, lamb], [ta, tb])
    assert np.allclose(got, _origin_line(lamb, tb), rtol=0, atol=1e-12)


def test_spread_above_the_threshold_uses_the_fit():
    """A spread of 1e-9 (above 1e-12 P) at every splitting point: the fit,
    which with two observations is the line through both points, not the
    fallback (which lands 0.2 away on this load)."""
    Pn = 4
    R = lambda s: s + 0.3 * s ** 2  # noqa: E731  work density rising along the curve
    lam0 = np.ones(Pn)
    lam1 = lam0 + 1e-9 * np.array([1.0, 1.0, 1.0, -3.0])  # every Lambda_i moves
    t0, t1 = _times(lam0, R), _times(lam1, R)
    L0, L1 = np.cumsum(lam0), np.cumsum(lam1)
    U0, U1 = np.cumsum(t0) / t0.mean(), np.cumsum(t1) / t1.mean()
    want = [0.0]
    for i in range(1, Pn):
        slope = (U1[i - 1] - U0[i - 1]) / (L1[i - 1] - L0[i - 1])
        want.append(L1[i - 1] + (i - U1[i - 1]) / slope)
    want.append(float(Pn))
    got = np.concatenate([[0.0], np.cumsum(P.balance_update([lam0, lam1], [t0, t1], growth=1.0))])
    assert np.allclose(got, want, rtol=0, atol=1e-9)
    fallback = np.concatenate([[0.0], np.cumsum(_origin_line(lam1, t1))])
    assert np.abs(fallback - want).max() > 0.1


def test_weighted_iteration_converges_on_a_smooth_load():
    Pn = 8
    R = lambda s: s + 0.15 * s ** 2 + 0.3 * np.sin(s)  # noqa: E731  increasing cost along the curve
    lams, ts = [np.ones(Pn)], []
    lb = []
    for _ in range(12):
        t = _times(lams[-1], R)
        ts.append(t)
        lb.append(P.load_balance(t))
        lams.append(P.balance_update(lams, ts, growth=1.5))
    assert lb[0] < 0.8 and lb[-1] > 0.995
    # the total time does not depend on the split
    assert np.allclose([t.sum() for t in ts], ts[0].sum(), rtol=1e-12)


def test_parts_assembled_apart_sum_to_the_whole():
    # substructuring: every part assembles its own elements with duplicated
    # interface nodes; summing the parts at shared nodes gives the whole residual
    import oracle
    c = mg.small_hybrid_case(nx=4, ny=4, seed=3)
    m = c.mesh
    cen, w = P.element_centroids(m.coords, m.conn_offsets, m.conn)
    part, _, _ = P.sfc_partition(cen, w, 5, level=3)
    assert len(np.unique(part)) == 5
    full = oracle.assemble(m, c.u, c.p, c.nu, c.vreman_c)
    acc = np.zeros_like(full)
    for i in range(5):
        sub, fids = mg.submesh(m, np.where(part == i)[0])
        r = oracle.assemble(sub, c.u[fids], None if c.p is None else c.p[fids], c.nu, c.vreman_c)
        np.add.at(acc, fids, r)
    assert np.linalg.norm(acc - full) <= 1e-13 * np.linalg.norm(full)
