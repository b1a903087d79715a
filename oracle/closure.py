"""Residual with the learned subgrid closure and Vreman fallback (test
infrastructure only).

Per element (Section 3.2 momentum residual; the closure replaces Vreman's
stress tau_v = -2 nu_t eps(u) = -nu_t (G + G^T) by the network's tau_m):
  R_v   = the plain residual (oracle_element_residual, all terms)
  D     = int dN_a/dx_j (tau_m - tau_v)_ij dV   (oracle_element_stress_residual)
  R     = R_v + D  if |D|_2 <= tol |R_v|_2, else R_v   (Vreman fallback)
tau_m = Delta^2 |G|_F^2 dev(y(x)), x = [G/|G|_F, log(Delta/Delta_ref)] at each
Gauss point; with bf16=True the network runs at the GPU's rounding points.
"""
from __future__ import annotations

import numpy as np

from . import mlp as _mlp
from . import oracle as _o


def assemble(mesh, u, p, nu, c, params: dict, delta_ref: float, tol: float = 0.05, bf16: bool = True,
             parts: bool = False):
    """Returns (rhs [n_field, 3], use_mlp [n_elems] bool, eps [n_elems]).

    parts=True appends a dict of diagnostics (the residual is unchanged):
    "share" [n_field, 3], the network's own stress term int dN_a/dx_j tau_m
    assembled over the kept elements, and "D", the list of per-element
    stress-difference vectors [n_a, 3] (element order)."""
    coords, types, offs, conn, fn, nf = _o._mesh_args(mesh)
    ne = len(types)
    recs, RV, deltas = [], [], np.zeros(ne)
    for e in range(ne):
        nodes = conn[offs[e]:offs[e + 1]]
        f = nodes if fn is None else fn[nodes]
        R, gp, d = _o.element_residual(int(types[e]), coords[nodes], u[f], None if p is None else p[f], nu, c)
        recs.append(gp)
        RV.append(R)
        deltas[e] = d
    ng = np.array([len(r) for r in recs])
    gp_all = np.concatenate(recs)
    G = gp_all[:, 5:14].reshape(-1, 3, 3)
    dg = np.repeat(deltas, ng)
    x, g2 = _mlp.features(G, dg, delta_ref)
    y = _mlp.forward_bf16(params, x) if bf16 else _mlp.forward(params, x)[0]
    tau_m = (dg ** 2 * g2)[:, None] * _mlp.deviatoric(y)
    S = G + G.transpose(0, 2, 1)
    nut = gp_all[:, 17]
    tau_v = -nut[:, None] * np.stack([S[:, 0, 0], S[:, 1, 1], S[:, 2, 2], S[:, 0, 1], S[:, 0, 2], S[:, 1, 2]], axis=1)
    dtau = tau_m - tau_v
    rhs = np.zeros((nf, 3))
    use = np.zeros(ne, bool)
    eps = np.zeros(ne)
    share = np.zeros((nf, 3)) if parts else None
    d_list = []
    o = 0
    for e in range(ne):
        nodes = conn[offs[e]:offs[e + 1]]
        f = nodes if fn is None else fn[nodes]
        D = _o.element_stress_residual(int(types[e]), coords[nodes], dtau[o:o + ng[e]])
        nr = np.linalg.norm(RV[e])
        eps[e] = np.linalg.norm(D) / nr if nr > 0 else np.inf
        use[e] = np.linalg.norm(D) ** 2 <= tol * tol * nr * nr
        np.add.at(rhs, f, RV[e] + D if use[e] else RV[e])
        if parts:
            d_list.append(D)
            if use[e]:
                np.add.at(share, f, _o.element_stress_residual(int(types[e]), coords[nodes], tau_m[o:o + ng[e]]))
        o += ng[e]
    if parts:
        return rhs, use, eps, {"share": share, "D": d_list}
    return rhs, use, eps
