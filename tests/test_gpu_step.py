"""GPU fractional-step operators and time step against the FP64 oracle.

Element operators (divergence, gradient, Laplacian) and the three explicit
RK3 stages involve no iterative solve: bar 1e-12.  The pressure solve and the
full step carry the CG tolerance (relative residual 1e-12): bar 1e-9.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_2005_05899_amd import meshgen as mg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


CASES = {
    "hybrid": lambda: mg.small_hybrid_case(nx=6, ny=5, layers=[(mg.PEN06, 2), (mg.TET04, 2), (mg.PYR05, 1), (mg.HEX08, 2)], seed=13),
    "periodic": lambda: mg.periodic_tg_case(8),
}


@pytest.fixture(scope="module", params=list(CASES))
def setup(request, torch_cuda):
    from paper_2005_05899_amd import lesasm
    c = CASES[request.param]()
    m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    perm = m.node_permutation()
    yield c, m, perm
    m.close()


def to_dev(torch, m, a):
    return m.to_internal(torch.from_numpy(np.ascontiguousarray(a)).cuda())


def to_host(m, t):
    return m.to_user(t).cpu().numpy()


def test_divergence_and_gradient(torch_cuda, setup):
    import oracle
    from oracle import step
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c, m, _ = setup
    D = lesasm.divergence(m, to_dev(torch, m, c.u))
    G = lesasm.gradient(m, to_dev(torch, m, c.p))
    torch.cuda.synchronize()
    assert rel(to_host(m, D.reshape(-1, 1))[:, 0], oracle.divergence(c.mesh, c.u)) < 1e-12
    assert rel(to_host(m, G), step.gradient(c.mesh, c.p)) < 1e-12


def test_laplacian_matches_oracle(torch_cuda, setup):
    from oracle import step
    from paper_2005_05899_amd import lesasm
    c, m, perm = setup
    st = lesasm.Stepper(m, c.nu, 1e-3)
    rowptr, col, val = st.laplacian()
    n = m.n_field_nodes
    Kint = sp.csr_matrix((val, col, rowptr), shape=(n, n))
    P = sp.csr_matrix((np.ones(n), (np.arange(n), perm)), shape=(n, n))  # internal <- user
    Kref = P @ step.laplacian(c.mesh) @ P.T
    diff = (Kint - Kref).tocoo()
    assert np.abs(diff.data).max(initial=0) < 1e-13 * np.abs(Kref.data).max()
    st.close()


def test_pressure_solve(torch_cuda, setup):
    from oracle import step
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c, m, _ = setup
    st = lesasm.Stepper(m, c.nu, 1e-3)
    b = np.random.default_rng(3).standard_normal(m.n_field_nodes)
    x = st.pressure_solve(to_dev(torch, m, b.reshape(-1, 1)).reshape(-1))
    torch.cuda.synchronize()
    it, res = st.stats()
    print(f"  CG: {it} iterations, relative residual {res:.2e}", flush=True)
    assert res <= 1e-12
    xref = step.pressure_solve(step.laplacian(c.mesh), b)
    assert rel(to_host(m, x.reshape(-1, 1))[:, 0], xref) < 1e-9
    st.close()


def test_rk3_stages(torch_cuda, setup):
    from oracle import step
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c, m, _ = setup
    dt = 0.05
    st = lesasm.Stepper(m, c.nu, dt)
    us = st.rk3_stages(to_dev(torch, m, c.u), to_dev(torch, m, c.p))
    torch.cuda.synchronize()
    ref = step.rk3_momentum(c.mesh, c.u, c.p, c.nu, c.vreman_c, dt)
    assert rel(to_host(m, us), ref) < 1e-12
    st.close()


def test_full_steps(torch_cuda, setup):
    from oracle import step
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c, m, _ = setup
    dt = 0.02
    st = lesasm.Stepper(m, c.nu, dt)
    u, p = to_dev(torch, m, c.u), to_dev(torch, m, c.p)
    ur, pr = c.u.copy(), c.p.copy()
    K = step.laplacian(c.mesh)
    for _ in range(3):
        st.step(u, p)
        ur, pr, _ = step.rk3_step(c.mesh, ur, pr, c.nu, c.vreman_c, dt, K=K)
    torch.cuda.synchronize()
    assert rel(to_host(m, u), ur) < 1e-9
    assert rel(to_host(m, p.reshape(-1, 1))[:, 0], pr) < 1e-9
    st.close()


SOLVE_SIZES = {  # row counts: below one 64-row slice, one ragged slice, many slices with a ragged tail
    "12_rows": lambda: mg.small_hybrid_case(nx=2, ny=1, layers=[(mg.HEX08, 1)], seed=2),
    "tet_ragged": lambda: mg.small_hybrid_case(nx=4, ny=3, layers=[(mg.TET04, 2), (mg.PYR05, 1)], seed=5),
    "hybrid_many_slices": lambda: mg.small_hybrid_case(
        nx=23, ny=19, layers=[(mg.HEX08, 2), (mg.PEN06, 2), (mg.TET04, 2), (mg.PYR05, 1), (mg.HEX08, 1)], seed=8),
}


@pytest.mark.parametrize("name", list(SOLVE_SIZES))
def test_pressure_solve_row_counts(torch_cuda, name):
    # the CG's SpMV works on 64-row slices padded to their longest row: meshes
    # with fewer rows than a slice, a partial slice and many slices of mixed
    # row lengths with a partial last one
    from oracle import step
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c = SOLVE_SIZES[name]()
    m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    n = m.n_field_nodes
    print(f"  {name}: {n} rows, {n % 64} in the last slice", flush=True)
    st = lesasm.Stepper(m, c.nu, 1e-3)
    b = np.random.default_rng(n).standard_normal(n)
    x = st.pressure_solve(to_dev(torch, m, b.reshape(-1, 1)).reshape(-1))
    torch.cuda.synchronize()
    it, res = st.stats()
    assert res <= 1e-12, (it, res)
    xref = step.pressure_solve(step.laplacian(c.mesh), b)
    assert rel(to_host(m, x.reshape(-1, 1))[:, 0], xref) < 1e-9
    st.close()
    m.close()


@pytest.mark.parametrize("name", list(SOLVE_SIZES))
def test_spmv_rows_vs_oracle_laplacian(torch_cuda, name):
    # the CG's product kernel, row by row against the oracle's K (user order
    # permuted to internal): every row to rounding, relative to the sum of
    # |K_ab p_b| over the row
    from oracle import step
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c = SOLVE_SIZES[name]()
    m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    n = m.n_field_nodes
    st = lesasm.Stepper(m, c.nu, 1e-3)
    lens = np.diff(st.laplacian()[0])
    pad = -(-n // 64) * 64 - n
    slices = np.concatenate([lens, np.zeros(pad, lens.dtype)]).reshape(-1, 64).max(axis=1)
    assert st.sell_entries() == 64 * int(slices.sum())
    K = step.laplacian(c.mesh)
    pu = np.random.default_rng(n + 1).standard_normal(n)
    q = st.spmv(to_dev(torch, m, pu.reshape(-1, 1)).reshape(-1))
    torch.cuda.synchronize()
    got = to_host(m, q.reshape(-1, 1))[:, 0]
    want = K @ pu
    scale = abs(K) @ np.abs(pu)
    assert (np.abs(got - want) <= 1e-14 * scale).all()
    with pytest.raises(ValueError):
        st.spmv(q[:-1])
    st.close()
    m.close()


@pytest.mark.parametrize("name", list(SOLVE_SIZES))
def test_cg_iterates_match_oracle_cg(torch_cuda, name):
    # the GPU's Jacobi-PCG and the oracle's, stopped after the same number of
    # iterations (a tolerance neither reaches): same iterate up to rounding
    from oracle import cg, step
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c = SOLVE_SIZES[name]()
    m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    n = m.n_field_nodes
    K = step.laplacian(c.mesh)
    b = np.random.default_rng(n + 2).standard_normal(n)
    bd = to_dev(torch, m, b.reshape(-1, 1)).reshape(-1)
    for k in ((1, 2, 3, 5) if n < 64 else (1, 4, 17, 40)):
        st = lesasm.Stepper(m, c.nu, 1e-3, rtol=1e-300, maxit=k)
        x = to_host(m, st.pressure_solve(bd).reshape(-1, 1))[:, 0]
        it, res = st.stats()
        want, it_o, res_o = cg.jacobi_pcg(K, b, k, rtol=0.0)
        err = np.abs(x - want).max() / np.abs(want).max()
        print(f"  {name} k={k}: max rel difference {err:.2e}, residual {res:.3e} vs {res_o:.3e}", flush=True)
        assert it == it_o == k
        assert err <= 1e-9
        # relative residuals agree to rounding (an absolute floor once CG has
        # converged to where rounding decides the residual)
        assert abs(res - res_o) <= 1e-9 * res_o + 1e-14
        st.close()
    m.close()
