"""Pins of the CG oracle (Jacobi-preconditioned CG, Section 3.2 / Algorithm 1)
against what the mathematics fixes, none of them re-typing the oracle:

* finite termination: with a preconditioned operator of four distinct
  eigenvalues, the fourth iterate is the exact solution (and the third is not);
* every iterate equals scipy's preconditioned CG, an independent
  implementation of the same textbook method, given M^-1 = diag(K)^-1;
* the error in the energy norm never grows;
* on a singular Neumann Laplacian the projected solution is the
  pseudo-inverse's (minimum-norm, mean-zero) solution;
* the stopping test ends on a checked iteration with the true residual small.

The module under test may be swapped for a planted-mistake copy through
LESASM_CG_ORACLE (used by the mutation tests)."""
import importlib.util
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _load():
    path = os.environ.get("LESASM_CG_ORACLE")
    if not path:
        from oracle import cg
        return cg
    spec = importlib.util.spec_from_file_location("cg_variant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


C = _load()


def _four_eigenvalue_matrix(seed):
    # A = S M S with M = blockdiag((1-c) I + c J) (unit diagonal, so diag(A) =
    # S^2 and diag(A)^-1 A is similar to M): eigenvalues 1-c1, 1+c1(n1-1),
    # 1-c2, 1+c2(n2-1)
    rng = np.random.default_rng(seed)
    blocks = []
    for n, c in ((7, 0.3), (5, -0.15)):
        blocks.append((1 - c) * np.eye(n) + c * np.ones((n, n)))
    M = np.block([[blocks[0], np.zeros((7, 5))], [np.zeros((5, 7)), blocks[1]]])
    s = rng.uniform(0.5, 3.0, 12)
    return sp.csr_matrix(s[:, None] * M * s[None, :]), rng.standard_normal(12)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_four_distinct_eigenvalues_terminate_in_four_iterations(seed):
    A, b = _four_eigenvalue_matrix(seed)
    exact = np.linalg.solve(A.toarray(), b)
    x4, it, _ = C.jacobi_pcg(A, b, 4, project=False)
    assert it == 4
    assert np.abs(x4 - exact).max() <= 1e-11 * np.abs(exact).max()
    x3, _, _ = C.jacobi_pcg(A, b, 3, project=False)
    assert np.abs(x3 - exact).max() > 1e-6 * np.abs(exact).max()


def _variable_poisson(nx, ny, seed):
    # SPD: 2-D five-point operator with random positive edge conductances
    # plus a positive diagonal shift
    rng = np.random.default_rng(seed)
    n = nx * ny
    idx = np.arange(n).reshape(ny, nx)
    rows, cols, vals = [], [], []
    for a, b in ((idx[:, :-1], idx[:, 1:]), (idx[:-1, :], idx[1:, :])):
        a, b = a.ravel(), b.ravel()
        w = rng.uniform(0.1, 10.0, len(a))
        rows += [a, b, a, b]
        cols += [b, a, a, b]
        vals += [-w, -w, w, w]
    K = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return K, rng


def test_iterates_match_scipy_preconditioned_cg():
    K, rng = _variable_poisson(13, 11, 5)
    K = (K + sp.diags(rng.uniform(0.01, 1.0, K.shape[0]))).tocsr()
    b = rng.standard_normal(K.shape[0])
    seen = []
    Minv = spla.LinearOperator(K.shape, matvec=lambda v: v / K.diagonal())
    spla.cg(K, b, x0=np.zeros_like(b), rtol=0.0, atol=0.0, maxiter=40, M=Minv,
            callback=lambda x: seen.append(x.copy()))
    for k in (1, 2, 3, 10, 25, 40):
        x, it, _ = C.jacobi_pcg(K, b, k, project=False)
        assert it == k
        assert np.abs(x - seen[k - 1]).max() <= 1e-10 * np.abs(seen[k - 1]).max(), k


def test_energy_norm_error_never_grows():
    K, rng = _variable_poisson(17, 9, 6)
    K = (K + 0.05 * sp.eye(K.shape[0])).tocsr()
    b = rng.standard_normal(K.shape[0])
    exact = spla.spsolve(K.tocsc(), b)
    errs = []
    for k in range(1, 60):
        x, _, _ = C.jacobi_pcg(K, b, k, project=False)
        e = x - exact
        errs.append(float(e @ (K @ e)))
    assert all(b2 <= b1 * (1 + 1e-12) for b1, b2 in zip(errs, errs[1:]))
    assert errs[-1] < 1e-2 * errs[0]


def test_singular_neumann_laplacian_gives_pseudo_inverse_solution():
    K, rng = _variable_poisson(9, 8, 7)  # rows sum to zero: constants in the null space
    b = rng.standard_normal(K.shape[0]) + 3.0  # not mean-zero: the solve projects it
    x, it, res = C.jacobi_pcg(K, b, 500, rtol=1e-13, check_every=1)
    assert res <= 1e-13
    want = np.linalg.pinv(K.toarray()) @ (b - b.mean())
    assert abs(x.mean()) <= 1e-14 * np.abs(want).max()
    assert np.abs(x - want).max() <= 1e-9 * np.abs(want).max()


def test_stopping_rule_checks_every_few_iterations():
    K, rng = _variable_poisson(20, 20, 8)
    K = (K + 0.02 * sp.eye(K.shape[0])).tocsr()
    b = rng.standard_normal(K.shape[0])
    x, it, res = C.jacobi_pcg(K, b, 10000, rtol=1e-8, check_every=16, project=False)
    assert it % 16 == 0 and res <= 1e-8
    assert np.linalg.norm(b - K @ x) <= 1.01e-8 * np.linalg.norm(b)
    # one check earlier had not yet met the tolerance
    _, _, res_before = C.jacobi_pcg(K, b, it - 16, project=False)
    assert res_before > 1e-8
    # the iteration cap ends the solve on its last iteration
    _, it2, res2 = C.jacobi_pcg(K, b, 21, rtol=1e-8, check_every=16, project=False)
    assert it2 == 21 and res2 > 1e-8
    # a zero right-hand side is solved by zero without iterating
    x0, it0, r0 = C.jacobi_pcg(K, np.zeros(K.shape[0]), 50)
    assert it0 == 0 and r0 == 0.0 and not x0.any()
