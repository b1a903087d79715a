"""The learned closure end to end at small scale: decaying turbulence run by
this library's solver, box-filtered samples, training with the GPU kernels,
and the a-priori gain over the method without it on a held-out snapshot.

Pass criteria: the trained network's subgrid stress is closer to the
filtered-DNS stress than Vreman's (relative L2, Frobenius) and than no model
at all, and correlates better with it.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_trained_closure_beats_vreman_a_priori(torch_cuda):
    from paper_2005_05899_amd import training as tr
    torch = torch_cuda
    snaps, times = tr.decaying_turbulence(n=48, nu=0.01, dt=0.01, steps=60, snap_every=10, first_snap=30)
    assert len(snaps) == 4 and all(np.isfinite(s).all() for s in snaps)
    datas, delta_ref = [], None
    for s in snaps[:-1]:
        d, delta_ref = tr.samples_from_snapshot(s, delta_ref=delta_ref)
        datas.append(d)
    data = {k: np.concatenate([d[k] for d in datas]) for k in datas[0]}
    params, hist, net = tr.train(data["x"], data["t"], steps=800, batch=4096, lr=2e-3)
    assert hist[-1][1] < 0.5 * hist[0][1]
    test, _ = tr.samples_from_snapshot(snaps[-1], delta_ref=delta_ref)
    y = net.infer_bf16(torch.from_numpy(test["x"]).cuda()).cpu().numpy().astype(np.float64)
    tau = (test["delta"] ** 2 * (test["G"].reshape(-1, 9) ** 2).sum(axis=1))[:, None] * tr.deviatoric(y)
    rep = tr.apriori_errors(tau, test)
    print(f"  a-priori on held-out t={times[-1]:.2f}: {rep}", flush=True)
    assert rep["mlp_rel_err"] < rep["vreman_rel_err"]
    assert rep["mlp_rel_err"] < rep["zero_rel_err"]
    assert rep["mlp_corr"] > rep["vreman_corr"]
    net.close()
