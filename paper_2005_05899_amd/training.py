"""Training data and training of the learned subgrid closure.

Data come from the method itself: decaying turbulence on a periodic cube of
HEX08 elements integrated by this library's fractional-step solver (the plain
method, Vreman closure), box-filtered to coarser grids.  At every Gauss point
of the coarse grid the sample is
  input   x = [G/|G|_F, log(Delta/Delta_ref)]       (G: FE gradient of the filtered velocity)
  target  t = dev(tau) / (Delta^2 |G|_F^2),   tau_ij = filter(u_i u_j) - filter(u_i) filter(u_j)
with Delta the coarse element width.  The network is trained on the GPU by
the library's own kernels (FP32 forward, backward and Adam).

Filter: the discrete top-hat (1/4, 1/2, 1/4) per direction (width 2h) on the
periodic grid, then restriction to every other node; applying the pair twice
gives the 4h level.  Data preparation runs in numpy on the host.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import meshgen

GAUSS_1D = (0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0))  # on [0, 1]


def decaying_turbulence(n: int = 128, nu: float = 0.005, dt: float = 0.004, steps: int = 250,
                        snap_every: int = 25, first_snap: int = 125, seed: int = 7, vreman_c: float = 0.1,
                        rtol: float = 1e-8, log=print):
    """Runs the solver on the periodic n^3 cube; returns snapshots of the
    velocity as [n, n, n, 3] arrays indexed [k, j, i] (z, y, x)."""
    import torch

    from . import lesasm
    case_mesh = meshgen.periodic_hex_cube(n)
    xf = case_mesh.field_coords()
    u0 = meshgen.random_fourier_velocity_peaked(seed=seed)(xf)
    mesh = lesasm.Mesh.from_arrays(case_mesh, vreman_c)
    st = lesasm.Stepper(mesh, nu, dt, rtol=rtol, maxit=4000)
    u = mesh.to_internal(torch.from_numpy(u0).cuda())
    p = torch.zeros(mesh.n_field_nodes, dtype=torch.float64, device="cuda")
    snaps, times = [], []
    t0 = time.time()
    for s in range(1, steps + 1):
        st.step(u, p)
        if s >= first_snap and (s - first_snap) % snap_every == 0:
            uu = mesh.to_user(u).cpu().numpy().reshape(n, n, n, 3)
            snaps.append(uu)
            times.append(s * dt)
            it, res = st.stats()
            log(f"  snapshot t={s * dt:.3f}: u_rms {np.sqrt((uu ** 2).mean()):.4f}, CG {it} it "
                f"(res {res:.1e}), {time.time() - t0:.1f} s")
    st.close()
    mesh.close()
    return snaps, times


def box_filter(f: np.ndarray) -> np.ndarray:
    """(1/4, 1/2, 1/4) along each of the three grid axes (periodic)."""
    for ax in range(3):
        f = 0.25 * np.roll(f, 1, axis=ax) + 0.5 * f + 0.25 * np.roll(f, -1, axis=ax)
    return f


def filter_level(u: np.ndarray, level: int):
    """Filtered velocity and subgrid stress on the grid coarsened 2^level
    times.  Returns (ubar [m,m,m,3], tau [m,m,m,6] in (xx, yy, zz, xy, xz, yz))."""
    prods = np.stack([u[..., 0] * u[..., 0], u[..., 1] * u[..., 1], u[..., 2] * u[..., 2],
                      u[..., 0] * u[..., 1], u[..., 0] * u[..., 2], u[..., 1] * u[..., 2]], axis=-1)
    ub, pb = u, prods
    for _ in range(level):
        ub = box_filter(ub)[::2, ::2, ::2]
        pb = box_filter(pb)[::2, ::2, ::2]
    tau = pb - np.stack([ub[..., 0] * ub[..., 0], ub[..., 1] * ub[..., 1], ub[..., 2] * ub[..., 2],
                         ub[..., 0] * ub[..., 1], ub[..., 0] * ub[..., 2], ub[..., 1] * ub[..., 2]], axis=-1)
    return ub, tau


def gauss_point_fields(f: np.ndarray, h: float):
    """Trilinear interpolation and gradient of a periodic nodal field
    f [m,m,m,c] (indexed z, y, x) at the 8 Gauss points of every cell.
    Returns values [m^3*8, c] and gradients [m^3*8, c, 3] (d/dx, d/dy, d/dz)."""
    corners = {}
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                corners[(dx, dy, dz)] = np.roll(f, (-dz, -dy, -dx), axis=(0, 1, 2))
    vals, grads = [], []
    for gz in GAUSS_1D:
        for gy in GAUSS_1D:
            for gx in GAUSS_1D:
                v = 0.0
                gxv = gyv = gzv = 0.0
                for (dx, dy, dz), c in corners.items():
                    wx = gx if dx else 1 - gx
                    wy = gy if dy else 1 - gy
                    wz = gz if dz else 1 - gz
                    sx = 1.0 if dx else -1.0
                    sy = 1.0 if dy else -1.0
                    sz = 1.0 if dz else -1.0
                    v = v + wx * wy * wz * c
                    gxv = gxv + sx * wy * wz * c
                    gyv = gyv + wx * sy * wz * c
                    gzv = gzv + wx * wy * sz * c
                vals.append(v.reshape(-1, f.shape[-1]))
                grads.append(np.stack([gxv, gyv, gzv], axis=-1).reshape(-1, f.shape[-1], 3) / h)
    return np.concatenate(vals), np.concatenate(grads)


def deviatoric(t6: np.ndarray) -> np.ndarray:
    t = np.array(t6, copy=True)
    tr = t[:, :3].sum(axis=1) / 3.0
    t[:, :3] -= tr[:, None]
    return t


def samples_from_snapshot(u: np.ndarray, levels=(1, 2), length: float = 2 * math.pi, delta_ref: float | None = None):
    """Training samples of one snapshot at the given filter levels.
    Returns dict with x [N,10] f32, t [N,6] f32 (normalised dev tau), G [N,3,3],
    tau [N,6] (deviatoric), delta [N]."""
    n = u.shape[0]
    out = {k: [] for k in ("x", "t", "G", "tau", "delta")}
    if delta_ref is None:
        delta_ref = length / (n // 2)
    for lev in levels:
        m = n >> lev
        h = length / m
        ub, tau = filter_level(u, lev)
        _, G = gauss_point_fields(ub, h)           # G[:, i, j] = du_i/dx_j
        tg, _ = gauss_point_fields(tau, h)
        tg = deviatoric(tg)
        g2 = (G.reshape(-1, 9) ** 2).sum(axis=1)
        keep = g2 > 1e-6 * np.median(g2)
        G, tg, g2 = G[keep], tg[keep], g2[keep]
        x = np.concatenate([G.reshape(-1, 9) / np.sqrt(g2)[:, None],
                            np.full((len(G), 1), math.log(h / delta_ref))], axis=1)
        out["x"].append(x.astype(np.float32))
        out["t"].append((tg / (h * h * g2)[:, None]).astype(np.float32))
        out["G"].append(G)
        out["tau"].append(tg)
        out["delta"].append(np.full(len(G), h))
    return {k: np.concatenate(v) for k, v in out.items()}, delta_ref


# ---- samples on hybrid elements ------------------------------------------------
# The assembly evaluates the closure at the Gauss points of linear TET04, PYR05,
# PEN06 and HEX08 elements with Delta_e = (element volume)^(1/3).  The samples
# below put the filtered fields on such elements: a graded, perturbed hybrid box
# of the benchmark's generator (type mix, splits, grading, perturbation) whose
# core spacing is the filtered grid's, velocity at its nodes interpolated from
# the filtered grid, G the finite-element gradient at each Gauss point, the
# target the filtered subgrid stress at the Gauss point's position.  Reference
# elements and rules as the element definitions of the library's header.

def _gauss_jacobi2():
    """2-point rule for the weight (1 - c)^2 on [0, 1] (from its moments)."""
    mu = [2.0 / ((k + 1) * (k + 2) * (k + 3)) for k in range(4)]
    # monic p2 = c^2 + a c + b orthogonal to 1 and c
    a, b = np.linalg.solve([[mu[1], mu[0]], [mu[2], mu[1]]], [-mu[2], -mu[3]])
    c = np.sort(np.roots([1.0, a, b]).real)
    w = np.linalg.solve([[1.0, 1.0], [c[0], c[1]]], [mu[0], mu[1]])
    return c, w


def reference_rule(t: int):
    """Gauss points xi [g, 3] and weights [g] of element type t."""
    g = 1.0 / math.sqrt(3.0)
    if t == meshgen.TET04:
        a, b = (5 + 3 * math.sqrt(5)) / 20, (5 - math.sqrt(5)) / 20
        xi = np.array([[b, b, b], [a, b, b], [b, a, b], [b, b, a]])
        return xi, np.full(4, 1.0 / 24.0)
    if t == meshgen.PEN06:
        tri = [(1 / 6, 1 / 6), (2 / 3, 1 / 6), (1 / 6, 2 / 3)]
        xi = np.array([[r, s, z] for z in (-g, g) for r, s in tri])
        return xi, np.full(6, 1.0 / 6.0)
    if t == meshgen.HEX08:
        xi = np.array([[x, y, z] for z in (-g, g) for y in (-g, g) for x in (-g, g)])
        return xi, np.ones(8)
    if t == meshgen.PYR05:
        cs, wc = _gauss_jacobi2()
        pts, ws = [], []
        for c, w in zip(cs, wc):
            for bb in (-g, g):
                for aa in (-g, g):
                    pts.append([aa * (1 - c), bb * (1 - c), c])
                    ws.append(w)
        return np.array(pts), np.array(ws)
    raise ValueError(t)


_HEX_NODES = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                       [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], float)
_PYR_BASE = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], float)


def reference_shape(t: int, xi: np.ndarray):
    """Shape functions N [g, n] and reference gradients dN [g, n, 3] at xi."""
    r, s, z = xi[:, 0], xi[:, 1], xi[:, 2]
    one, zero = np.ones_like(r), np.zeros_like(r)
    if t == meshgen.TET04:
        N = np.stack([1 - r - s - z, r, s, z], axis=1)
        d = np.array([[-1, -1, -1], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
        return N, np.broadcast_to(d, (len(r), 4, 3)).copy()
    if t == meshgen.PEN06:
        L = [1 - r - s, r, s]
        dL = [(-one, -one), (one, zero), (zero, one)]
        N, dN = [], []
        for zz, sg in ((1 - z) / 2, -0.5), ((1 + z) / 2, 0.5):
            for k in range(3):
                N.append(L[k] * zz)
                dN.append(np.stack([dL[k][0] * zz, dL[k][1] * zz, L[k] * sg], axis=1))
        return np.stack(N, axis=1), np.stack(dN, axis=1)
    if t == meshgen.HEX08:
        N, dN = [], []
        for a, b, c in _HEX_NODES:
            fx, fy, fz = 1 + a * r, 1 + b * s, 1 + c * z
            N.append(fx * fy * fz / 8)
            dN.append(np.stack([a * fy * fz, b * fx * fz, c * fx * fy], axis=1) / 8)
        return np.stack(N, axis=1), np.stack(dN, axis=1)
    if t == meshgen.PYR05:
        N, dN = [], []
        q = 1 - z
        for a, b in _PYR_BASE:
            A, B = q + a * r, q + b * s
            N.append(A * B / (4 * q))
            dN.append(np.stack([a * B / (4 * q), b * A / (4 * q), -(A + B) / (4 * q) + A * B / (4 * q * q)], axis=1))
        N.append(z)
        dN.append(np.stack([zero, zero, one], axis=1))
        return np.stack(N, axis=1), np.stack(dN, axis=1)
    raise ValueError(t)


def periodic_trilinear(f: np.ndarray, pts: np.ndarray, h: float) -> np.ndarray:
    """Trilinear interpolation of a periodic nodal grid field f [m,m,m,c]
    (indexed z, y, x; node (i,j,k) at (i h, j h, k h)) at points pts [P, 3]."""
    m = f.shape[0]
    q = pts / h
    i0 = np.floor(q).astype(np.int64)
    fr = q - i0
    out = 0.0
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = ((fr[:, 0] if dx else 1 - fr[:, 0]) * (fr[:, 1] if dy else 1 - fr[:, 1])
                     * (fr[:, 2] if dz else 1 - fr[:, 2]))
                v = f[(i0[:, 2] + dz) % m, (i0[:, 1] + dy) % m, (i0[:, 0] + dx) % m]
                out = out + w[:, None] * v
    return out


def hybrid_element_samples(ub: np.ndarray, tau: np.ndarray, length: float, seed: int):
    """Gauss-point samples of the filtered fields ub [m,m,m,3], tau [m,m,m,6]
    (periodic, spacing length/m) on a hybrid box of m x m cells and about m
    graded layers (TET04/PEN06/PYR05/HEX08 = 40/40/5/15 % of the elements,
    perturbed by 10 % of the local spacing with the given seed).  Returns a
    dict with G [N,3,3] (FE gradient of the interpolated velocity), tau [N,6]
    (deviatoric filtered stress at the point), delta [N] (Delta_e of the
    point's element) and etype [N]."""
    m = ub.shape[0]
    h = length / m
    target = int(m ** 3 / (0.4 / 6 + 0.4 / 2 + 0.05 / 6 + 0.15))
    mesh = meshgen.hybrid_box(m, m, meshgen.hybrid_layers(m * m, target), length=(length,) * 3, seed=seed)
    xn = mesh.coords
    un = periodic_trilinear(ub, xn, h)
    out = {k: [] for k in ("G", "tau", "delta", "etype")}
    for t in (meshgen.TET04, meshgen.PYR05, meshgen.PEN06, meshgen.HEX08):
        idx = np.flatnonzero(mesh.types == t)
        if len(idx) == 0:
            continue
        conn = mesh.conn[mesh.conn_offsets[idx][:, None] + np.arange(meshgen.NNODE[t])[None, :]]
        X, U = xn[conn], un[conn]                                   # [E, n, 3]
        xi, w = reference_rule(t)
        N, dN = reference_shape(t, xi)                              # [g, n], [g, n, 3]
        J = np.einsum("ean,gak->egnk", X, dN)                       # J[e,g,i,k] = dx_i/dxi_k
        det = np.linalg.det(J)
        Jinv = np.linalg.inv(J)                                     # [e,g,k,i] = dxi_k/dx_i
        dNx = np.einsum("gak,egkj->egaj", dN, Jinv)                 # dN_a/dx_j
        G = np.einsum("eai,egaj->egij", U, dNx)                     # du_i/dx_j
        pts = np.einsum("ga,eak->egk", N, X).reshape(-1, 3)
        dl = np.cbrt((det * w[None, :]).sum(axis=1))
        out["G"].append(G.reshape(-1, 3, 3))
        out["tau"].append(deviatoric(periodic_trilinear(tau, np.mod(pts, length), h)))
        out["delta"].append(np.repeat(dl, len(w)))
        out["etype"].append(np.full(len(pts), t, np.uint8))
    return {k: np.concatenate(v) for k, v in out.items()}


def network_samples(raw: dict, delta_ref: float):
    """Network inputs x [N,10] and targets t [N,6] (float32) from G, tau and
    delta; points with a negligible gradient are dropped (as at the Gauss
    points of the grid samples)."""
    G, tg, dl = raw["G"], raw["tau"], raw["delta"]
    g2 = (G.reshape(-1, 9) ** 2).sum(axis=1)
    keep = g2 > 1e-6 * np.median(g2)
    out = {k: v[keep] for k, v in raw.items()}
    g2 = g2[keep]
    out["x"] = np.concatenate([out["G"].reshape(-1, 9) / np.sqrt(g2)[:, None],
                               np.log(out["delta"] / delta_ref)[:, None]], axis=1).astype(np.float32)
    out["t"] = (out["tau"] / (out["delta"] ** 2 * g2)[:, None]).astype(np.float32)
    return out


def vreman_tau(G: np.ndarray, delta: np.ndarray, c: float) -> np.ndarray:
    """Vreman's deviatoric model stress -2 nu_t eps(u) at the samples (6 comps)."""
    M = np.einsum("nij,nkj->nik", G, G)
    A = np.trace(M, axis1=1, axis2=2)
    B = (M[:, 0, 0] * M[:, 1, 1] - M[:, 0, 1] ** 2 + M[:, 0, 0] * M[:, 2, 2] - M[:, 0, 2] ** 2
         + M[:, 1, 1] * M[:, 2, 2] - M[:, 1, 2] ** 2)
    nut = np.where((A > 0) & (B > 0), c * delta ** 2 * np.sqrt(np.maximum(B, 0) / np.where(A > 0, A, 1)), 0.0)
    S = G + G.transpose(0, 2, 1)
    t = -nut[:, None] * np.stack([S[:, 0, 0], S[:, 1, 1], S[:, 2, 2], S[:, 0, 1], S[:, 0, 2], S[:, 1, 2]], axis=1)
    return deviatoric(t)


def apriori_errors(params_tau: np.ndarray, data: dict, vreman_c: float = 0.1) -> dict:
    """Relative L2 errors (Frobenius, off-diagonals counted twice) and
    correlation of model stresses against the filtered-DNS stress."""
    w = np.array([1, 1, 1, 2, 2, 2.0])
    true = data["tau"]

    def err(model):
        return float(np.sqrt((w * (model - true) ** 2).sum() / (w * true ** 2).sum()))

    def corr(model):
        a, b = model.ravel(), true.ravel()
        return float(np.corrcoef(a, b)[0, 1])

    tv = vreman_tau(data["G"], data["delta"], vreman_c)
    return {"mlp_rel_err": err(params_tau), "vreman_rel_err": err(tv), "zero_rel_err": 1.0,
            "mlp_corr": corr(params_tau), "vreman_corr": corr(tv)}


def train(x: np.ndarray, t: np.ndarray, steps: int = 3000, batch: int = 8192, lr: float = 1e-3,
          seed: int = 0, log=print, init=None, weights: np.ndarray | None = None):
    """Trains the closure network with the library's GPU kernels.  Batches
    are drawn uniformly, or with probability proportional to `weights`.
    Returns (params float32 [5254], loss history)."""
    import torch

    from . import lesasm
    rng = np.random.default_rng(seed)
    if init is None:
        # He-normal weights, zero biases; order W1, b1, W2, b2, W3, b3
        parts = []
        for fan_in, fan_out in ((10, 64), (64, 64), (64, 6)):
            parts.append(rng.standard_normal((fan_in, fan_out)).ravel() * math.sqrt(2.0 / fan_in))
            parts.append(np.zeros(fan_out))
        init = np.concatenate(parts).astype(np.float32)
    net = lesasm.MLP(init)
    xd = torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
    td = torch.from_numpy(np.ascontiguousarray(t, np.float32)).cuda()
    n = len(x)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    cdf = None
    if weights is not None:  # inverse-CDF draws (the sample count exceeds torch.multinomial's limit)
        cdf = torch.cumsum(torch.from_numpy(np.asarray(weights, np.float64)).cuda(), 0)
        cdf = cdf / cdf[-1]
    for s in range(1, steps + 1):
        if cdf is None:
            idx = torch.randint(0, n, (batch,), device="cuda", generator=gen)
        else:
            r = torch.rand(batch, dtype=torch.float64, device="cuda", generator=gen)
            idx = torch.clamp(torch.searchsorted(cdf, r), max=n - 1)
        xb, tb = xd[idx].contiguous(), td[idx].contiguous()
        lr_s = lr * (0.1 ** (s / steps))  # exponential decay to lr/10
        net.train_step(xb, tb, lr=lr_s, loss=loss)
        if s % max(1, steps // 20) == 0 or s == 1:
            hist.append((s, float(loss.item())))
            log(f"  step {s}: loss {hist[-1][1]:.4e}")
    net.commit()
    params = net.params()
    return params, hist, net


def mesh_delta_ref(mesh) -> float:
    """Width reference of a mesh for the network's width input: the geometric
    mean of its Delta_e.  The network's inputs are then the element's width
    relative to the mesh's typical width (element type and grading), the same
    convention as its training samples (reference: the geometric mean over the
    samples at the 2h filter level), so the trained network carries over to
    meshes of other spacings under the similarity the Delta^2 |G|^2 scaling
    already assumes."""
    w = mesh.filter_width().cpu().numpy()
    return float(np.exp(np.log(w).mean()))


def gathered_samples(snaps, seed0: int, length: float = 2 * math.pi, delta_ref: float | None = None):
    """Grid samples (samples_from_snapshot) and hybrid-element samples of
    every snapshot at filter levels 1 and 2 (a new hybrid box per snapshot and
    level).  delta_ref None: the geometric mean width of the level-1 hybrid
    samples.  Returns (samples dict, delta_ref)."""
    raws, logw = [], {1: [], 2: []}
    for i, u in enumerate(snaps):
        for lev in (1, 2):
            ub, tau = filter_level(u, lev)
            raw = hybrid_element_samples(ub, tau, length, seed=seed0 + 10 * i + lev)
            raw["level"] = np.full(len(raw["delta"]), lev, np.uint8)
            raws.append(raw)
            logw[lev].append(np.log(raw["delta"]))
    level_ref = {lev: float(np.exp(np.concatenate(v).mean())) for lev, v in logw.items()}
    if delta_ref is None:
        delta_ref = level_ref[1]
    hyb = network_samples({k: np.concatenate([r[k] for r in raws]) for k in raws[0]}, delta_ref)
    grid = []
    for u in snaps:
        g, _ = samples_from_snapshot(u, delta_ref=delta_ref)
        g["etype"] = np.full(len(g["delta"]), meshgen.HEX08, np.uint8)
        h1 = length / (u.shape[0] >> 1)  # the grid samples' width is their level's spacing
        g["level"] = np.where(np.abs(g["delta"] - h1) <= 1e-9 * h1, 1, 2).astype(np.uint8)
        grid.append(g)
    keys = ("x", "t", "G", "tau", "delta", "etype", "level")
    out = {k: np.concatenate([hyb[k]] + [g[k] for g in grid]) for k in keys}
    out["hybrid"] = np.concatenate([np.ones(len(hyb["x"]), bool)] + [np.zeros(len(g["x"]), bool) for g in grid])
    # drawing weight (Delta / level width)^4, the level width being the geometric mean Delta_e of the
    # level's hybrid samples: the targets are stresses over Delta^2 |G|^2, so without it the narrow
    # elements (tetrahedra and pyramids, Delta about 0.55 h) would carry larger targets and rule the loss;
    # with it the errors of one level count on the scale of a stress at that level's width
    ref = np.where(out["level"] == 1, level_ref[1], level_ref[2])
    out["w"] = (out["delta"] / ref) ** 4
    return out, delta_ref


def apriori_report(net, test: dict) -> dict:
    """A-priori errors of the trained network (BF16 matrix-core inference)
    and of Vreman on held-out samples: all, the grid samples, the hybrid
    samples and the hybrid samples of each element type."""
    import torch
    y = net.infer_bf16(torch.from_numpy(test["x"]).cuda()).cpu().numpy().astype(np.float64)
    tau_m = (test["delta"] ** 2 * (test["G"].reshape(-1, 9) ** 2).sum(axis=1))[:, None] * deviatoric(y)
    sel = {"all": np.ones(len(y), bool), "grid": ~test["hybrid"], "hybrid": test["hybrid"]}
    for t, name in ((meshgen.TET04, "tet04"), (meshgen.PYR05, "pyr05"), (meshgen.PEN06, "pen06"),
                    (meshgen.HEX08, "hex08")):
        sel[f"hybrid_{name}"] = test["hybrid"] & (test["etype"] == t)
    rep = {}
    for k, m in sel.items():
        if m.any():
            r = apriori_errors(tau_m[m], {kk: test[kk][m] for kk in ("tau", "G", "delta")})
            r["samples"] = int(m.sum())
            rep[k] = r
    return rep


def main():
    ap = argparse.ArgumentParser(description="Generate filtered-DNS data and train the closure network.")
    ap.add_argument("--fine", type=int, default=128)
    ap.add_argument("--steps", type=int, default=250)
    ap.add_argument("--train-steps", type=int, default=3000)
    ap.add_argument("--out", default="closure_weights.npy")
    ap.add_argument("--report", default=None)
    args = ap.parse_args()
    snaps, times = decaying_turbulence(n=args.fine, steps=args.steps)
    data, delta_ref = gathered_samples(snaps[:-1], seed0=1000)
    test, _ = gathered_samples(snaps[-1:], seed0=2000, delta_ref=delta_ref)
    print(f"training samples {len(data['x'])} ({int(data['hybrid'].sum())} on hybrid elements), "
          f"delta_ref {delta_ref:.5f}", flush=True)
    params, hist, net = train(data["x"], data["t"], steps=args.train_steps, weights=data["w"])
    np.save(args.out, params)
    rep = {"a_priori_held_out": apriori_report(net, test), "delta_ref": delta_ref,
           "delta_ref_rule": "geometric mean of Delta_e over the level-1 hybrid samples; on a mesh, the geometric "
                             "mean of its Delta_e (training.mesh_delta_ref)",
           "train_samples": int(len(data["x"])), "train_samples_hybrid": int(data["hybrid"].sum()),
           "test_samples": int(len(test["x"])), "snapshot_times": times, "loss_history": hist}
    print(json.dumps(rep["a_priori_held_out"]), flush=True)
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)


if __name__ == "__main__":
    main()
