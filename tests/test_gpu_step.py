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
