"""FP64 time step of the fractional-step scheme (test infrastructure only).

Section 3.2 and Algorithm 1: explicit three-stage third-order Runge-Kutta for
the momentum equation, then one pressure Poisson solve that projects the
velocity (incremental pressure projection).  Tableau (Heun's third-order
method): c = (0, 1/3, 2/3), a21 = 1/3, a32 = 2/3, b = (1/4, 0, 3/4).  The
paper names the scheme but not its coefficients; this is the reading used.

  k_s   = M_L^-1 rhs(u_s, p^n)                 (element assembly per stage)
  u*    = u^n + dt (k_1 / 4 + 3 k_3 / 4)
  K dp  = -(1/dt) D u*, projected onto mean-zero right-hand sides
  u^n+1 = u* - dt M_L^-1 G dp,   p^n+1 = p^n + dp

K is the stiffness (Laplacian) matrix int grad N_a . grad N_b, assembled once;
D u = int N_a div u; G p = int N_a grad p.  K is singular (constants) on
periodic and all-Neumann boxes: the solve pins node 0, then shifts dp to zero
mean.  scipy's sparse direct solver serves as the linear-algebra step.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import oracle as _o

RK3_C = (0.0, 1.0 / 3.0, 2.0 / 3.0)
RK3_A = ((), (1.0 / 3.0,), (0.0, 2.0 / 3.0))
RK3_B = (0.25, 0.0, 0.75)


def laplacian(mesh) -> sp.csr_matrix:
    """Global stiffness matrix from element matrices (scatter-add)."""
    coords, types, offs, conn, fn, nf = _o._mesh_args(mesh)
    rows, cols, vals = [], [], []
    for e in range(len(types)):
        nodes = conn[offs[e]:offs[e + 1]]
        Ke = _o.element_laplacian(int(types[e]), coords[nodes])
        f = nodes if fn is None else fn[nodes]
        rows.append(np.repeat(f, len(f)))
        cols.append(np.tile(f, len(f)))
        vals.append(Ke.ravel())
    if not rows:
        return sp.csr_matrix((nf, nf))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nf, nf))


def gradient(mesh, p) -> np.ndarray:
    """(G p)_a = int N_a grad p  (the pressure term of the residual, sign flipped)."""
    nf = mesh.n_field_nodes if mesh.field_node is not None else len(mesh.coords)
    return -_o.assemble(mesh, np.zeros((nf, 3)), p, 0.0, 0.0, terms=_o.TERM_PRES)


def pressure_solve(K: sp.csr_matrix, b: np.ndarray) -> np.ndarray:
    """Mean-zero solution of K x = b - mean(b)."""
    n = K.shape[0]
    b = b - b.mean()
    x = np.zeros(n)
    if n > 1:
        x[1:] = spla.spsolve(K[1:, 1:].tocsc(), b[1:])
    return x - x.mean()


def rk3_momentum(mesh, u, p, nu, c, dt, M=None):
    """The three explicit stages: returns u* (before projection)."""
    if M is None:
        M = _o.lumped_mass(mesh)
    ks, us = [], [u]
    for s in range(3):
        if s:
            us.append(u + dt * sum(a * k for a, k in zip(RK3_A[s], ks)))
        ks.append(_o.assemble(mesh, us[s], p, nu, c) / M[:, None])
    return u + dt * sum(b * k for b, k in zip(RK3_B, ks))


def rk3_step(mesh, u, p, nu, c, dt, K=None, M=None):
    """One full step; returns (u^{n+1}, p^{n+1}, dp)."""
    if M is None:
        M = _o.lumped_mass(mesh)
    if K is None:
        K = laplacian(mesh)
    ustar = rk3_momentum(mesh, u, p, nu, c, dt, M)
    dp = pressure_solve(K, -_o.divergence(mesh, ustar) / dt)
    unew = ustar - dt * gradient(mesh, dp) / M[:, None]
    return unew, p + dp, dp
