"""FP64 Jacobi-preconditioned conjugate gradients (test infrastructure only).

Section 3.2 and Algorithm 1: the pressure Poisson system is solved by CG with
Jacobi diagonal scaling as the preconditioner; Section 3.4 (Code and
Parallelization): each iteration is one sparse matrix-vector product and two
dot products.  The method is the
textbook preconditioned CG (Saad, Iterative Methods for Sparse Linear
Systems, the preconditioned CG algorithm), here with M = diag(K):

  r_0 = b - K x_0,  z_0 = M^-1 r_0,  p_0 = z_0
  per iteration j:  alpha = (r_j . z_j) / (p_j . K p_j)
                    x_j+1 = x_j + alpha p_j,   r_j+1 = r_j - alpha K p_j
                    z_j+1 = M^-1 r_j+1
                    beta  = (r_j+1 . z_j+1) / (r_j . z_j)
                    p_j+1 = z_j+1 + beta p_j

Readings (the paper gives neither): x_0 = 0; the stopping test is
||r_j|| <= rtol ||b|| on the recurrence residual, looked at every
`check_every` iterations and after the last one allowed; for the pressure
system (a Laplacian that is singular on closed boxes, constants in its null
space) the right-hand side is first shifted to zero mean and the solution is
shifted to zero mean at the end (`project`).

Plain numpy; scipy's sparse product serves as the matrix-vector step.
"""
from __future__ import annotations

import numpy as np


def jacobi_pcg(K, b, maxit: int, rtol: float = 0.0, check_every: int = 16, project: bool = True):
    """Returns (x, iterations run, ||r|| / ||b||) for K x = b."""
    b = np.asarray(b, dtype=np.float64)
    if project:
        b = b - b.mean()
    dinv = 1.0 / K.diagonal()
    x = np.zeros_like(b)
    r = b.copy()
    z = dinv * r
    p = z.copy()
    rz = float(r @ z)
    bnorm = float(np.sqrt(b @ b))
    it, res = 0, bnorm
    if bnorm > 0.0:
        for it in range(1, maxit + 1):
            q = K @ p
            alpha = rz / float(p @ q)
            x = x + alpha * p
            r = r - alpha * q
            z = dinv * r
            rz_new = float(r @ z)
            p = z + (rz_new / rz) * p
            rz = rz_new
            if it % check_every == 0 or it == maxit:
                res = float(np.sqrt(r @ r))
                if res <= rtol * bnorm:
                    break
    if project:
        x = x - x.mean()
    return x, it, (res / bnorm if bnorm > 0.0 else 0.0)
