"""Plain CPU oracle of the SFC mesh partitioner and of the correction-
coefficient load balancing (Section "Mesh partitioning and load balancing").

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the GPU library.

Partitioner (subsection "Mesh partitioning"): inputs are the element count,
the number of parts P, one location per element (the mean of its node
coordinates) and optional integer weights (by default the number of Gauss
points of the element's type).  Steps, in the paper's order:
  i)   the bounding box of the element locations;
  ii)  a regular grid of 2^L bins per axis inside it;
  iii) each bin weighted by the weights of the elements it holds;
  iv)  a Hilbert curve orders the bins along one dimension;
  v)   the one-dimensional partition: bin b, with weight w_b and weight S_b
       before it along the curve, goes to part i when its midpoint
       S_b + w_b / 2 lies in [T_{i-1}, T_i), where T_i = Lambda_i W / P,
       Lambda_i = lambda_1 + ... + lambda_i (correction coefficients, all 1
       without correction) and W the total weight; every element takes the
       part of its bin.
Readings where the paper is silent: the bin of a coordinate is
floor((c - lo) / (hi - lo) * 2^L), clamped to 2^L - 1 (0 on a flat axis);
the Hilbert curve is Skilling's (AIP Conf. Proc. 707, 2004) transposed-index
construction, bits read from the most significant level down, x before y
before z; the midpoint rule above settles the one-dimensional problem.

Balancing (subsection "Load balancing"): per splitting point i = 1 .. P-1 a
(weighted) linear regression of the observations (Lambda_i^k, Upsilon_i^k),
Upsilon_i^k = (t_1^k + ... + t_i^k) / tbar^k, tbar^k the mean time; the line
y = alpha + beta x is cut with y = i, Lambda_i^{k+1} = (i - alpha) / beta;
lambda_i^{k+1} = Lambda_i^{k+1} - Lambda_{i-1}^{k+1} with Lambda_0 = 0 and
Lambda_P = P.  The weighted form raises each newer observation's weight by
50 %.  Readings: a single observation gives the line through it and the
origin; a regression with beta <= 0 or a degenerate abscissa (a spread of
Lambda_i below 1e-12 P) also falls back to that line through the newest
observation; Lambda^{k+1} is clamped to be
non-decreasing inside [0, P].
"""
from __future__ import annotations

import numpy as np

# Gauss points per element type (node count -> points): the weight model of
# the partitioner (one weight unit per Gauss point).
GAUSS_POINTS = {4: 4, 5: 8, 6: 6, 8: 8}


def element_centroids(coords, conn_offsets, conn):
    """Mean of each element's node coordinates (nodes summed in connectivity
    order, then divided by the node count) and its Gauss-point weight."""
    coords = np.asarray(coords, np.float64)
    off = np.asarray(conn_offsets, np.int64)
    conn = np.asarray(conn, np.int64)
    nn = np.diff(off)
    cen = np.zeros((len(nn), 3))
    wts = np.zeros(len(nn), np.int32)
    for n in np.unique(nn):
        sel = np.where(nn == n)[0]
        acc = np.zeros((len(sel), 3))
        for a in range(n):
            acc = acc + coords[conn[off[sel] + a]]
        cen[sel] = acc / n
        wts[sel] = GAUSS_POINTS[int(n)]
    return cen, wts


def hilbert_index(ix, iy, iz, level):
    """Hilbert curve position of bin (ix, iy, iz) on a 2^level grid (Skilling's
    construction: undo the excess work on the axes level by level, Gray-
    encode, then read the transposed index bit plane by bit plane)."""
    X = [np.array(ix, dtype=np.int64, copy=True), np.array(iy, dtype=np.int64, copy=True),
         np.array(iz, dtype=np.int64, copy=True)]
    top = 1 << (level - 1)
    q = top
    while q > 1:
        low = q - 1
        for i in range(3):
            has = (X[i] & q) != 0
            # bit q set on axis i: flip the low bits of axis 0
            x0_flipped = X[0] ^ low
            # bit q clear: swap the low bits of axes 0 and i
            t = (X[0] ^ X[i]) & low
            x0_swapped = X[0] ^ t
            xi_swapped = X[i] ^ t
            if i == 0:
                X[0] = np.where(has, x0_flipped, X[0])  # swapping axis 0 with itself changes nothing
            else:
                X[0], X[i] = np.where(has, x0_flipped, x0_swapped), np.where(has, X[i], xi_swapped)
        q >>= 1
    # Gray encode
    X[1] = X[1] ^ X[0]
    X[2] = X[2] ^ X[1]
    t = np.zeros_like(X[0])
    q = top
    while q > 1:
        t = np.where((X[2] & q) != 0, t ^ (q - 1), t)
        q >>= 1
    X = [x ^ t for x in X]
    h = np.zeros_like(X[0])
    for b in range(level - 1, -1, -1):
        for i in range(3):
            h = (h << 1) | ((X[i] >> b) & 1)
    return h


def bins(centroids, level):
    """Bin coordinates of each location on the 2^level grid over the
    locations' bounding box (steps i and ii)."""
    c = np.asarray(centroids, np.float64)
    lo, hi = c.min(axis=0), c.max(axis=0)
    nb = 1 << level
    out = np.zeros(c.shape, np.int64)
    for k in range(3):
        ext = hi[k] - lo[k]
        if ext > 0:
            v = np.floor((c[:, k] - lo[k]) / ext * float(nb)).astype(np.int64)
            out[:, k] = np.minimum(v, nb - 1)
    return out


def targets(n_parts, total, lam=None):
    """Cumulative targets T_1 .. T_{P-1}: Lambda_i W / P."""
    lam = np.ones(n_parts) if lam is None else np.asarray(lam, np.float64)
    out = []
    acc = 0.0
    for i in range(n_parts - 1):
        acc = acc + float(lam[i])
        out.append(acc * float(total) / float(n_parts))
    return np.array(out, np.float64)


def sfc_partition(centroids, weights, n_parts, lam=None, level=7):
    """Part of every element (steps i to v).  Returns (part, key, bin_weight)."""
    c = np.asarray(centroids, np.float64)
    n = len(c)
    w = np.ones(n, np.int64) if weights is None else np.asarray(weights, np.int64)
    if n == 0:
        return np.zeros(0, np.int32), np.zeros(0, np.int64), np.zeros(1 << (3 * level), np.int64)
    b = bins(c, level)
    key = hilbert_index(b[:, 0], b[:, 1], b[:, 2], level)
    nbins = 1 << (3 * level)
    binw = np.zeros(nbins, np.int64)
    np.add.at(binw, key, w)
    before = np.concatenate([[0], np.cumsum(binw)[:-1]])
    total = int(binw.sum())
    t2 = 2.0 * targets(n_parts, total, lam)
    mid2 = (2 * before[key] + binw[key]).astype(np.float64)
    part = np.searchsorted(t2, mid2, side="right").astype(np.int32)
    return part, key, binw


def balance_update(lam_hist, t_hist, growth=1.5):
    """New correction coefficients from the observations of iterations
    0 .. K (rows of lam_hist and t_hist, each of length P); growth = 1 is the
    simple regression, 1.5 the weighted one."""
    L = np.atleast_2d(np.asarray(lam_hist, np.float64))
    T = np.atleast_2d(np.asarray(t_hist, np.float64))
    K, P = L.shape
    Lam = np.cumsum(L, axis=1)                      # Lambda_i^k, i = 1..P
    Ups = np.cumsum(T, axis=1) / T.mean(axis=1, keepdims=True)   # Upsilon_i^k
    wk = growth ** np.arange(K)
    new = np.zeros(P + 1)
    new[P] = P
    for i in range(1, P):
        x, y = Lam[:, i - 1], Ups[:, i - 1]
        nxt = None
        if K >= 2:
            sw = wk.sum()
            mx, my = (wk * x).sum() / sw, (wk * y).sum() / sw
            sxx = (wk * (x - mx) ** 2).sum()
            if x.max() - x.min() > 1e-12 * P and sxx > 0:
                beta = (wk * (x - mx) * (y - my)).sum() / sxx
                alpha = my - beta * mx
                if beta > 0:
                    nxt = (i - alpha) / beta
        if nxt is None:
            # line through the origin and the newest observation
            nxt = i * x[-1] / y[-1] if y[-1] > 0 else x[-1]
        new[i] = nxt
    for i in range(1, P):
        new[i] = min(max(new[i], new[i - 1]), P)
    return np.diff(new)


def load_balance(times):
    """Mean over maximum of the per-part times."""
    t = np.asarray(times, np.float64)
    return float(t.mean() / t.max())
