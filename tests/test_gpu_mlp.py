"""GPU training kernels and matrix-core inference of the learned closure
against the FP64 numpy oracle, and the fused closure inside the assembly.

Bars: FP32 forward/loss 1e-5 relative, gradients 1e-4 (sums of 4096
samples in FP32), Adam 1e-5.  BF16 inference vs the oracle at the same
rounding points: 2e-2 of the output range (a BF16 rounding of a hidden
activation can flip where the FP32 sums differ in order).  Fused closure:
per field, two BF16 units of the network's own stress term, plus the stress
differences of elements within 2 % of the fallback threshold, plus the plain
assembly's bar (tests/closure_bar.py); fallback decisions equal except within
1 % of the threshold.
"""
import numpy as np
import pytest

from oracle import mlp as omlp
from paper_2005_05899_amd import meshgen as mg
from tests.closure_bar import closure_bars

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def net(torch_cuda):
    from paper_2005_05899_amd import lesasm
    p = omlp.init_params(11)
    rng = np.random.default_rng(12)
    for k in p:
        p[k] = p[k] + 0.05 * rng.standard_normal(p[k].shape)
    p32 = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    m = lesasm.MLP(omlp.flatten(p32).astype(np.float32))
    yield m, p32
    m.close()


def samples(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 10)).astype(np.float32)
    t = rng.standard_normal((n, 6)).astype(np.float32)
    t[:, :3] -= t[:, :3].mean(axis=1, keepdims=True)
    return x, t


def test_forward_f32(torch_cuda, net):
    torch = torch_cuda
    m, p = net
    x, _ = samples(3000, 1)
    y = m.forward_f32(torch.from_numpy(x).cuda()).cpu().numpy()
    ref, _ = omlp.forward(p, x.astype(np.float64))
    assert np.abs(y - ref).max() <= 1e-5 * np.abs(ref).max()


def test_loss_and_gradients(torch_cuda, net):
    torch = torch_cuda
    m, p = net
    x, t = samples(4096, 2)
    loss, g = m.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    L, gref = omlp.loss_and_grad(p, x.astype(np.float64), t.astype(np.float64))
    assert abs(loss.item() - L) <= 1e-5 * L
    gg = omlp.unflatten(g.cpu().numpy().astype(np.float64))
    for k in omlp.ORDER:
        assert np.abs(gg[k] - gref[k]).max() <= 1e-4 * np.abs(gref[k]).max(), k


def test_adam_steps(torch_cuda, net):
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    _, p = net
    m = lesasm.MLP(omlp.flatten(p).astype(np.float32))
    x, t = samples(2048, 3)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    pr = {k: v.copy() for k, v in p.items()}
    st = {}
    for s in range(1, 4):
        m.train_step(xd, td, lr=1e-3)
        _, gref = omlp.loss_and_grad(pr, x.astype(np.float64), t.astype(np.float64))
        omlp.adam_step(pr, gref, st, 1e-3, s)
    torch.cuda.synchronize()
    got = omlp.unflatten(m.params().astype(np.float64))
    for k in omlp.ORDER:
        assert np.abs(got[k] - pr[k]).max() <= 1e-5 * max(np.abs(pr[k]).max(), 1e-3), k
    m.close()


def test_bf16_matrix_core_inference(torch_cuda, net):
    torch = torch_cuda
    m, p = net
    for n in (1, 63, 64, 65, 1000, 5000):
        x, _ = samples(n, 4 + n)
        y = m.infer_bf16(torch.from_numpy(x).cuda()).cpu().numpy()
        ref = omlp.forward_bf16(p, x.astype(np.float64))
        err = np.abs(y - ref)
        assert err.max() <= 2e-2 * np.abs(ref).max(), (n, err.max())
        assert np.median(err) <= 1e-5 * np.abs(ref).max(), n


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fused_closure_matches_oracle(torch_cuda, net, precision):
    import oracle
    from oracle import closure
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    _, p0 = net
    c = mg.small_hybrid_case(nx=6, ny=5, layers=[(mg.PEN06, 2), (mg.TET04, 2), (mg.PYR05, 1), (mg.HEX08, 2)], seed=17)
    # last layer scaled so that network and Vreman stresses are comparable and
    # the threshold splits the elements into kept and rejected ones
    p = {k: v.copy() for k, v in p0.items()}
    p["W3"] *= 0.02
    p["b3"] *= 0.02
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    m = lesasm.MLP(omlp.flatten(p).astype(np.float32))
    delta_ref = float(np.median(oracle.filter_width(c.mesh)))
    mesh = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    mesh.precision = precision
    tol = 0.13
    lesasm.set_closure(mesh, m, delta_ref, tol)
    u = mesh.to_internal(torch.from_numpy(c.u).cuda())
    pp = mesh.to_internal(torch.from_numpy(c.p).cuda())
    got = mesh.to_user(mesh.assemble_momentum_rhs(u, pp, c.nu)).cpu().numpy()
    by_type = lesasm.closure_fallbacks_by_type(mesh)
    nfb = sum(by_type.values())
    ref, use, eps, parts = closure.assemble(c.mesh, c.u, c.p, c.nu, c.vreman_c, p, delta_ref, tol, parts=True)
    near_el = (eps > tol * 0.99) & (eps < tol * 1.01)
    near = int(near_el.sum())
    print(f"  {precision}: fallbacks gpu {nfb}, oracle {int((~use).sum())} of {len(use)}, near threshold {near}")
    assert abs(nfb - int((~use).sum())) <= near
    for t in (mg.TET04, mg.PYR05, mg.PEN06, mg.HEX08):  # the same per element type
        of_t = c.mesh.types == t
        assert abs(by_type[t] - int((~use & of_t).sum())) <= int((near_el & of_t).sum()), t
    bars, _ = closure_bars(c.mesh, parts, eps, tol, ref, 1e-12 if precision == "fp64" else 1e-5)
    err = np.linalg.norm(got - ref, axis=0)
    print(f"  {precision}: |got - ref| per field {err}, bars {bars} (relative {bars / np.linalg.norm(ref, axis=0)})")
    assert (err <= bars).all(), (err, bars)
    # every element keeps the network (no keep-or-fall-back decision can
    # differ): the bar is two BF16 units of the network's stress term plus the
    # plain assembly's
    lesasm.set_closure(mesh, m, delta_ref, 1e6)
    got = mesh.to_user(mesh.assemble_momentum_rhs(u, pp, c.nu)).cpu().numpy()
    ref_all, use_all, eps_all, parts_all = closure.assemble(c.mesh, c.u, c.p, c.nu, c.vreman_c, p, delta_ref, 1e6,
                                                            parts=True)
    assert use_all.all() and sum(lesasm.closure_fallbacks_by_type(mesh).values()) == 0
    bars, near_all = closure_bars(c.mesh, parts_all, eps_all, 1e6, ref_all, 1e-12 if precision == "fp64" else 1e-5)
    err = np.linalg.norm(got - ref_all, axis=0)
    print(f"  {precision} all kept: |got - ref| per field {err}, bars {bars} "
          f"(relative {bars / np.linalg.norm(ref_all, axis=0)})")
    assert near_all == 0 and (err <= bars).all(), (err, bars)
    lesasm.set_closure(mesh, None)
    plain = mesh.to_user(mesh.assemble_momentum_rhs(u, pp, c.nu)).cpu().numpy()
    vref = oracle.assemble(c.mesh, c.u, c.p, c.nu, c.vreman_c)
    assert np.linalg.norm(plain - vref) <= (1e-12 if precision == "fp64" else 1e-5) * np.linalg.norm(vref)
    assert 0.2 < use.mean() < 0.8
    mesh.close()
    m.close()


def test_fallback_counts_over_many_workgroups(torch_cuda):
    # the 2.0 M hybrid mesh with the committed network: more chunk workgroups
    # than fallback counter slots; counts add up over assemblies, the query
    # resets them, and a zero tolerance counts every element once
    import json
    import os
    from paper_2005_05899_amd import lesasm, training
    torch = torch_cuda
    case = mg.hybrid_2m_case()
    data = os.path.join(os.path.dirname(lesasm.__file__), "data")
    flat = np.load(os.path.join(data, "closure_weights.npy")).astype(np.float32)
    meta = json.load(open(os.path.join(data, "closure_weights.json")))
    m = lesasm.MLP(flat)
    mesh = lesasm.Mesh.from_arrays(case.mesh, case.vreman_c)
    delta_ref = training.mesh_delta_ref(mesh) if meta.get("delta_ref_rule") else meta["delta_ref"]
    mesh.precision = "fp32"
    u = mesh.to_internal(torch.from_numpy(case.u).cuda())
    p = mesh.to_internal(torch.from_numpy(case.p).cuda())
    lesasm.set_closure(mesh, m, delta_ref, 0.05)
    assert lesasm.closure_fallbacks(mesh) == 0
    mesh.assemble_momentum_rhs(u, p, case.nu)
    one = lesasm.closure_fallbacks(mesh)
    for _ in range(3):
        mesh.assemble_momentum_rhs(u, p, case.nu)
    three = lesasm.closure_fallbacks(mesh)
    print(f"  fallbacks per assembly {one} of {case.mesh.n_elems}", flush=True)
    assert 0 < one < case.mesh.n_elems and three == 3 * one
    assert lesasm.closure_fallbacks(mesh) == 0
    lesasm.set_closure(mesh, m, delta_ref, 0.0)  # zero tolerance: every element falls back
    mesh.assemble_momentum_rhs(u, p, case.nu)
    assert lesasm.closure_fallbacks(mesh) == case.mesh.n_elems
    lesasm.set_closure(mesh, None)
    mesh.close()
    m.close()
