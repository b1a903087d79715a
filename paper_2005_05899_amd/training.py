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
          seed: int = 0, log=print, init=None):
    """Trains the closure network with the library's GPU kernels.
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
    for s in range(1, steps + 1):
        idx = torch.randint(0, n, (batch,), device="cuda", generator=gen)
        xb, tb = xd[idx].contiguous(), td[idx].contiguous()
        lr_s = lr * (0.1 ** (s / steps))  # exponential decay to lr/10
        net.train_step(xb, tb, lr=lr_s, loss=loss)
        if s % max(1, steps // 20) == 0 or s == 1:
            hist.append((s, float(loss.item())))
            log(f"  step {s}: loss {hist[-1][1]:.4e}")
    net.commit()
    params = net.params()
    return params, hist, net


def main():
    ap = argparse.ArgumentParser(description="Generate filtered-DNS data and train the closure network.")
    ap.add_argument("--fine", type=int, default=128)
    ap.add_argument("--steps", type=int, default=250)
    ap.add_argument("--train-steps", type=int, default=3000)
    ap.add_argument("--out", default="closure_weights.npy")
    ap.add_argument("--report", default=None)
    args = ap.parse_args()
    snaps, times = decaying_turbulence(n=args.fine, steps=args.steps)
    train_snaps, test_snap = snaps[:-1], snaps[-1]
    datas = []
    delta_ref = None
    for s in train_snaps:
        d, delta_ref = samples_from_snapshot(s, delta_ref=delta_ref)
        datas.append(d)
    data = {k: np.concatenate([d[k] for d in datas]) for k in datas[0]}
    print(f"training samples {len(data['x'])}, delta_ref {delta_ref:.5f}")
    params, hist, net = train(data["x"], data["t"], steps=args.train_steps)
    np.save(args.out, params)
    test, _ = samples_from_snapshot(test_snap, delta_ref=delta_ref)
    import torch
    y = net.infer_bf16(torch.from_numpy(test["x"]).cuda()).cpu().numpy().astype(np.float64)
    tau_m = (test["delta"] ** 2 * (test["G"].reshape(-1, 9) ** 2).sum(axis=1))[:, None] * deviatoric(y)
    rep = apriori_errors(tau_m, test)
    rep.update({"delta_ref": delta_ref, "train_samples": int(len(data["x"])), "test_samples": int(len(test["x"])),
                "snapshot_times": times, "loss_history": hist})
    print(json.dumps(rep))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)


if __name__ == "__main__":
    main()
