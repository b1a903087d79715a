"""Tolerance of the fused learned closure against the closure oracle, derived
from where the two may differ.

Both sides run the network at the same rounding points (BF16 operands, FP32
sums, forward_bf16 in the oracle), so they differ only where an FP32 sum,
added in another order on the matrix cores, straddles a BF16 rounding
boundary: the rounded value then moves by one BF16 unit in the last place,
2 u with u = 2^-8 the unit roundoff.  Such moves reach the residual only
through the network's own stress term, so per field the bar is

    2 u |S|_2  +  |F|_2  +  base |R|_2

with S the network's stress term int dN_a/dx_j tau_m assembled over the kept
elements, F the stress differences of the elements whose fallback ratio lies
within 2 % of the tolerance (their keep-or-fall-back decision may go either
way), and base the plain assembly's own bar (1e-12 FP64, 1e-5 FP32
contractions).
"""
import numpy as np

U_BF16 = 2.0 ** -8


def closure_bars(mesh, parts, eps, tol, ref, base, rows=None):
    """Per-field bars on |got - ref|_2 (absolute) over the node rows `rows`
    (all if None), from the closure oracle's parts, fallback ratios eps,
    tolerance tol and reference residual ref (rows of the whole mesh)."""
    coords_f = mesh.field_node
    offs, conn = mesh.conn_offsets, mesh.conn
    F = np.zeros_like(ref)
    near = np.flatnonzero((eps > 0.98 * tol) & (eps < 1.02 * tol))
    for e in near:
        nodes = conn[offs[e]:offs[e + 1]]
        f = nodes if coords_f is None else coords_f[nodes]
        np.add.at(F, f, parts["D"][e])
    S = parts["share"]
    if rows is not None:
        S, F, ref = S[rows], F[rows], ref[rows]
    bars = 2 * U_BF16 * np.linalg.norm(S, axis=0) + np.linalg.norm(F, axis=0) + base * np.linalg.norm(ref, axis=0)
    return bars, len(near)
