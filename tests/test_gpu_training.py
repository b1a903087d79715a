"""The learned closure end to end at small scale: decaying turbulence run by
this library's solver, box-filtered samples (on the filtered grid's own cells
and on the Gauss points of graded, perturbed hybrid boxes at the same
spacing), training with the GPU kernels, and the a-priori gain over the method
without it on a held-out snapshot.

Pass criteria, on all held-out samples, on the grid samples and on the
hybrid-element samples: the trained network's subgrid stress is closer to the
filtered-DNS stress than Vreman's (relative L2, Frobenius) and correlates
better with it; on all samples and on the hybrid ones it is also closer than no
model at all.  (The grid samples of this small case, the 32^3 and 16^3 cells
of three snapshots, are too few for that last margin to be stable; the
committed network, trained on 128^3 data, is 0.74 against no model's 1.00
there.)
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
    snaps, times = tr.decaying_turbulence(n=64, nu=0.01, dt=0.01, steps=60, snap_every=10, first_snap=30)
    assert len(snaps) == 4 and all(np.isfinite(s).all() for s in snaps)
    data, delta_ref = tr.gathered_samples(snaps[:-1], seed0=11)
    assert data["hybrid"].any() and (~data["hybrid"]).any()
    params, hist, net = tr.train(data["x"], data["t"], steps=1500, batch=4096, lr=2e-3, weights=data["w"])
    assert hist[-1][1] < 0.5 * hist[0][1]
    test, _ = tr.gathered_samples(snaps[-1:], seed0=21, delta_ref=delta_ref)
    rep = tr.apriori_report(net, test)
    for k, r in rep.items():
        print(f"  a-priori on held-out t={times[-1]:.2f}, {k}: {r}", flush=True)
    for k in ("all", "grid", "hybrid"):
        assert rep[k]["mlp_rel_err"] < rep[k]["vreman_rel_err"], k
        assert rep[k]["mlp_corr"] > rep[k]["vreman_corr"], k
    for k in ("all", "hybrid"):
        assert rep[k]["mlp_rel_err"] < rep[k]["zero_rel_err"], k
    net.close()
