"""FP64 reference of the learned subgrid closure (test infrastructure only).

A small multilayer perceptron predicts the subgrid stress at a Gauss point
from the local velocity gradient; it stands in for Vreman's eddy viscosity in
the subgrid term div(tau) of the momentum equation (Section 3.2).  The paper
uses Vreman only; the network, its inputs, outputs and training are project
choices (the readings are listed in the design notes):

  x      = [G / |G|_F (9 values, row-major G_ij = du_i/dx_j), log(Delta / Delta_ref)]
  h1     = relu(x W1 + b1)          W1: 10 x 64
  h2     = relu(h1 W2 + b2)         W2: 64 x 64
  y      = h2 W3 + b3               W3: 64 x 6, components (xx, yy, zz, xy, xz, yz)
  z      = y with the trace removed from (xx, yy, zz)           (deviatoric)
  tau    = Delta^2 |G|_F^2 z                                    (symmetric tensor)

The loss is the mean Frobenius error of z against normalised targets t
(weights 1, 1, 1, 2, 2, 2 on the components); Adam updates the FP32 master
copy on the GPU, and BF16-rounded weights serve inference.  `forward_bf16`
reproduces the rounding points of the GPU inference path: inputs, weights and
hidden activations rounded to BF16, sums in FP32.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 10, 64, 6
COMP_W = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])
SHAPES = {"W1": (N_IN, N_H), "b1": (N_H,), "W2": (N_H, N_H), "b2": (N_H,), "W3": (N_H, N_OUT), "b3": (N_OUT,)}
ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES.values())  # 5254


def init_params(seed: int = 0) -> dict:
    """He-normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for k in ORDER:
        s = SHAPES[k]
        p[k] = rng.standard_normal(s) * np.sqrt(2.0 / s[0]) if k[0] == "W" else np.zeros(s)
    return p


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], np.float64).ravel() for k in ORDER])


def unflatten(v: np.ndarray) -> dict:
    out, o = {}, 0
    for k in ORDER:
        n = int(np.prod(SHAPES[k]))
        out[k] = np.asarray(v[o:o + n], np.float64).reshape(SHAPES[k])
        o += n
    return out


def features(G: np.ndarray, delta: np.ndarray, delta_ref: float):
    """x [N, 10] and |G|_F^2 [N] from gradients G [N, 3, 3] and widths [N]."""
    G = np.asarray(G, np.float64).reshape(-1, 9)
    g2 = (G * G).sum(axis=1)
    gn = np.sqrt(g2)
    x = np.zeros((len(G), N_IN))
    nz = gn > 0
    x[nz, :9] = G[nz] / gn[nz, None]
    x[:, 9] = np.log(np.asarray(delta, np.float64) / delta_ref)
    return x, g2


def deviatoric(y: np.ndarray) -> np.ndarray:
    z = np.array(y, np.float64, copy=True)
    tr = z[:, :3].sum(axis=1) / 3.0
    z[:, :3] -= tr[:, None]
    return z


def forward(p: dict, x: np.ndarray):
    a1 = x @ p["W1"] + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ p["W3"] + p["b3"]
    return y, (x, a1, h1, a2, h2)


def tau(p: dict, G, delta, delta_ref: float) -> np.ndarray:
    """Subgrid stress [N, 6] (xx, yy, zz, xy, xz, yz)."""
    x, g2 = features(G, delta, delta_ref)
    y, _ = forward(p, x)
    return (np.asarray(delta, np.float64) ** 2 * g2)[:, None] * deviatoric(y)


def loss_and_grad(p: dict, x: np.ndarray, t: np.ndarray):
    """L = (1/N) sum_n sum_c w_c (z_nc - t_nc)^2 and dL/dparams."""
    n = len(x)
    y, (x, a1, h1, a2, h2) = forward(p, x)
    z = deviatoric(y)
    r = z - t
    L = float((COMP_W * r * r).sum() / n)
    dz = 2.0 * COMP_W * r / n
    dy = dz.copy()
    dy[:, :3] = dz[:, :3] - dz[:, :3].sum(axis=1, keepdims=True) / 3.0  # trace projection is symmetric
    g = {"W3": h2.T @ dy, "b3": dy.sum(axis=0)}
    dh2 = dy @ p["W3"].T
    da2 = dh2 * (a2 > 0)
    g["W2"] = h1.T @ da2
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ p["W2"].T
    da1 = dh1 * (a1 > 0)
    g["W1"] = x.T @ da1
    g["b1"] = da1.sum(axis=0)
    return L, g


def adam_step(p: dict, g: dict, state: dict, lr: float, step: int, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8) -> None:
    """One Adam update (bias-corrected, step counted from 1), in place."""
    for k in ORDER:
        m = state.setdefault("m_" + k, np.zeros(SHAPES[k]))
        v = state.setdefault("v_" + k, np.zeros(SHAPES[k]))
        m *= b1
        m += (1 - b1) * g[k]
        v *= b2
        v += (1 - b2) * g[k] * g[k]
        mh = m / (1 - b1 ** step)
        vh = v / (1 - b2 ** step)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def bf16_round(a) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(a, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(p: dict, x: np.ndarray) -> np.ndarray:
    """Inference with the GPU's rounding points (BF16 operands, FP32 sums)."""
    q = {k: bf16_round(v) for k, v in p.items() if k[0] == "W"}
    h1 = np.maximum((bf16_round(x).astype(np.float32) @ q["W1"].astype(np.float32)) + p["b1"].astype(np.float32), 0)
    h2 = np.maximum((bf16_round(h1).astype(np.float32) @ q["W2"].astype(np.float32)) + p["b2"].astype(np.float32), 0)
    y = (bf16_round(h2).astype(np.float32) @ q["W3"].astype(np.float32)) + p["b3"].astype(np.float32)
    return y.astype(np.float64)
