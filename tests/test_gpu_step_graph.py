"""The step graph: one whole time step of Algorithm 1 (three Runge-Kutta
stages, divergence, Jacobi-PCG pressure solve, gradient, correction, pressure
update) captured once and replayed, against the eager stepper and the FP64
oracle's step.

Bars: with a CG iteration count fixed on both sides (a tolerance neither
meets) the replay and the eager step run the same kernels on the same data;
only the atomic sums (the node sums of the assembly, the divergence and the
gradient) may differ in order.  Those rounding differences (1e-16 of the
velocity) reach the pressure equation through the divergence of the predicted
velocity, a small difference of large terms for a nearly solenoidal field, so
relative to that right-hand side they are larger by the ratio of |grad u| h to
|div u*|; 30 unconverged CG iterations per step, whose iterates are not a
linear function of the right-hand side, then amplify them by up to the
condition number of the preconditioned Laplacian (about 10^3 on these meshes).
Two eager steps from the same state differ by the same mechanism (printed
beside the replay's difference): on the periodic cube the pressure has been
seen 2e-9 apart after one step.  The bar, 1e-7 relative, stays far below what
a replay that missed or repeated any stage would give (order 1).  With the CG
converged to a relative residual of 1e-12, the oracle's step (direct solve)
bounds the difference by the solve's error: 1e-9, the bar of the eager step's
own test.  Each replay is checked, with eager work and host synchronisations
between replays.
"""
import numpy as np
import pytest

from paper_2005_05899_amd import meshgen as mg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


CASES = {
    "hybrid": lambda: mg.small_hybrid_case(nx=6, ny=5, layers=[(mg.PEN06, 2), (mg.TET04, 2), (mg.PYR05, 1), (mg.HEX08, 2)], seed=13),
    "periodic": lambda: mg.periodic_tg_case(8),
}


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def to_dev(torch, m, a):
    return m.to_internal(torch.from_numpy(np.ascontiguousarray(a)).cuda())


def to_host(m, t):
    return m.to_user(t).cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
def test_replays_match_eager_steps_fixed_iterations(torch_cuda, name):
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c = CASES[name]()
    print(f"  {name}: {c.mesh.n_elems} elements", flush=True)
    m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    dt, iters = 0.02, 30
    st = lesasm.Stepper(m, c.nu, dt, rtol=1e-300, maxit=iters)
    ue, pe = to_dev(torch, m, c.u), to_dev(torch, m, c.p)
    ug, pg = ue.clone(), pe.clone()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = lesasm.StepGraph(st, ug, pg, iters, s)
    for k in range(3):
        g.launch(s)
        s.synchronize()
        it, res, ok = g.stats()
        assert it == iters and not ok and np.isfinite(res)
        u2, p2 = ue.clone(), pe.clone()
        st.step(ue, pe)  # eager steps between the replays
        st.step(u2, p2)  # a second eager step from the same state
        torch.cuda.synchronize()
        assert st.stats()[0] == iters
        pe_h, pg_h = to_host(m, pe.reshape(-1, 1)), to_host(m, pg.reshape(-1, 1))
        du, dp = rel(to_host(m, ug), to_host(m, ue)), rel(pg_h, pe_h)
        ee_u, ee_p = rel(to_host(m, u2), to_host(m, ue)), rel(to_host(m, p2.reshape(-1, 1)), pe_h)
        print(f"  step {k}: replay vs eager u {du:.2e}, p {dp:.2e}; eager vs eager u {ee_u:.2e}, p {ee_p:.2e}",
              flush=True)
        assert du < 1e-7 and dp < 1e-7
        ue.copy_(ug)  # continue both from the replay's state (the spread must not compound)
        pe.copy_(pg)
        torch.cuda.synchronize()  # the copies read ug, pg before the next replay writes them
    g.close()
    st.close()
    m.close()


@pytest.mark.parametrize("name", list(CASES))
def test_converged_replays_match_oracle_step(torch_cuda, name):
    from oracle import step
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c = CASES[name]()
    m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    dt = 0.02
    st = lesasm.Stepper(m, c.nu, dt, rtol=1e-12, maxit=5000)
    u, p = to_dev(torch, m, c.u), to_dev(torch, m, c.p)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = lesasm.StepGraph(st, u, p, 5000, s)
    ur, pr = c.u.copy(), c.p.copy()
    K = step.laplacian(c.mesh)
    for k in range(3):
        g.launch(s)
        ur, pr, _ = step.rk3_step(c.mesh, ur, pr, c.nu, c.vreman_c, dt, K=K)
        it, res, ok = g.stats()
        print(f"  step {k}: {it} CG iterations, relative residual {res:.2e}", flush=True)
        assert ok and res <= 1e-12 and 0 < it < 5000
        assert rel(to_host(m, u), ur) < 1e-9
        assert rel(to_host(m, p.reshape(-1, 1))[:, 0], pr) < 1e-9
    g.close()
    st.close()
    m.close()


def test_unconverged_replay_is_reported(torch_cuda):
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c = CASES["hybrid"]()
    m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    st = lesasm.Stepper(m, c.nu, 0.02, rtol=1e-12, maxit=5000)
    u, p = to_dev(torch, m, c.u), to_dev(torch, m, c.p)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = lesasm.StepGraph(st, u, p, 3, s)
    with pytest.raises(lesasm.LesasmError) as e:
        g.stats()
    assert e.value.code == -5
    g.launch(s)
    it, res, ok = g.stats()
    assert it == 3 and not ok and res > 1e-12
    g.close()
    st.close()
    m.close()


def test_other_buffers_are_rejected(torch_cuda):
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c = CASES["periodic"]()
    m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    st = lesasm.Stepper(m, c.nu, 0.02)
    u, p = to_dev(torch, m, c.u), to_dev(torch, m, c.p)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = lesasm.StepGraph(st, u, p, 50, s)
    with pytest.raises(lesasm.LesasmError) as e:
        g.launch(s, u=u.clone())
    assert e.value.code == -5
    with pytest.raises(lesasm.LesasmError) as e:
        lesasm.StepGraph(st, u, p, 0, s)
    assert e.value.code == -1
    g.close()
    st.close()
    m.close()


def test_destroy_and_recapture_right_after_replays(torch_cuda):
    # graphs destroyed while their replays may still be queued (no host
    # synchronisation in between): destruction waits for the last replay, and a
    # new capture on the same stepper continues from the replayed state
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c = CASES["hybrid"]()
    m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    dt, iters = 0.02, 20
    st = lesasm.Stepper(m, c.nu, dt, rtol=1e-300, maxit=iters)
    ue, pe = to_dev(torch, m, c.u), to_dev(torch, m, c.p)
    ug, pg = ue.clone(), pe.clone()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    for _ in range(3):
        g = lesasm.StepGraph(st, ug, pg, iters, s)
        g.launch(s)
        g.launch(s)
        g.close()
    s.synchronize()
    for _ in range(6):
        st.step(ue, pe)
    torch.cuda.synchronize()
    assert rel(to_host(m, ug), to_host(m, ue)) < 1e-11
    assert rel(to_host(m, pg.reshape(-1, 1)), to_host(m, pe.reshape(-1, 1))) < 1e-11
    st.close()
    m.close()
