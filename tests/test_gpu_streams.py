"""Calls that share a mesh's state from different streams, graph re-capture
while replays are queued, and the device-memory cap.

* assemblies of one mesh alternating between two streams with no host
  synchronisation: each equals the same assembly made alone (bit for bit: the
  staged scatter sums in a fixed order), so no call overwrote another's
  staging rows
* a batch on one stream and one of its member meshes on another, the same
* the batch's Runge-Kutta graph captured again right after a replay was
  queued (no host synchronisation): the replays equal the eager sequence
* a memory cap below what a mesh needs: LESASM_E_OOM with nothing created and
  the library's bytes back where they were; without the cap the same mesh
  builds
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


def test_alternating_streams_one_mesh(torch_cuda):
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c = mg.small_hybrid_case(nx=24, ny=20, layers=[(mg.PEN06, 3), (mg.TET04, 3), (mg.PYR05, 1), (mg.HEX08, 3)], seed=21)
    m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    u0 = m.to_internal(torch.from_numpy(c.u).cuda())
    p = m.to_internal(torch.from_numpy(c.p).cuda())
    us = [u0 * (1.0 + 0.25 * k) for k in range(8)]
    refs = []
    for u in us:
        refs.append(m.assemble_momentum_rhs(u, p, c.nu))
        torch.cuda.synchronize()
    outs = [torch.full_like(u0, float("nan")) for _ in us]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    print(f"  {c.mesh.n_elems} elements, 8 assemblies over 2 streams", flush=True)
    for k, (u, o) in enumerate(zip(us, outs)):
        with torch.cuda.stream(streams[k % 2]):
            m.assemble_momentum_rhs(u, p, c.nu, out=o)
    torch.cuda.synchronize()
    for k, (o, r) in enumerate(zip(outs, refs)):
        assert torch.equal(o, r), k
    m.close()


def test_batch_and_member_on_two_streams(torch_cuda):
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    cases, meshes, us, ps = [], [], [], []
    for i, (nx, ny) in enumerate([(16, 12), (10, 9), (14, 6)]):
        c = mg.small_hybrid_case(nx=nx, ny=ny, seed=60 + i)
        m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
        cases.append(c)
        meshes.append(m)
        us.append(m.to_internal(torch.from_numpy(c.u).cuda()))
        ps.append(m.to_internal(torch.from_numpy(c.p).cuda()))
    b = lesasm.Batch(meshes)
    nus = [c.nu for c in cases]
    ref_b = b.assemble(us, ps, nus)
    torch.cuda.synchronize()
    ref_m = meshes[0].assemble_momentum_rhs(2.0 * us[0], ps[0], nus[0])
    torch.cuda.synchronize()
    u2 = 2.0 * us[0]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs_b = [torch.full_like(u, float("nan")) for u in us]
    out_m = torch.full_like(us[0], float("nan"))
    torch.cuda.synchronize()
    for _ in range(3):
        with torch.cuda.stream(s1):
            b.assemble(us, ps, nus, outs_b)
        with torch.cuda.stream(s2):
            meshes[0].assemble_momentum_rhs(u2, ps[0], nus[0], out=out_m)
    torch.cuda.synchronize()
    assert torch.equal(out_m, ref_m)
    for o, r in zip(outs_b, ref_b):
        assert torch.equal(o, r)
    b.close()
    for m in meshes:
        m.close()


def test_batch_graph_recaptured_while_replays_queued(torch_cuda):
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    cases, meshes, us, ps = [], [], [], []
    for i, (nx, ny) in enumerate([(8, 6), (6, 5)]):
        c = mg.small_hybrid_case(nx=nx, ny=ny, seed=70 + i)
        m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
        cases.append(c)
        meshes.append(m)
        us.append(m.to_internal(torch.from_numpy(c.u).cuda()))
        ps.append(m.to_internal(torch.from_numpy(c.p).cuda()))
    b = lesasm.Batch(meshes)
    nus = [c.nu for c in cases]
    dt = 0.005
    ug = [u.clone() for u in us]
    ue = [u.clone() for u in us]
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(3):  # capture, replay, capture again at once
        b.rk3_graph(ug, ps, nus, dt, s)
        b.rk3_launch(s)
    s.synchronize()
    for _ in range(3):
        b.rk3_eager(ue, ps, nus, dt)
    torch.cuda.synchronize()
    for g, e in zip(ug, ue):
        assert np.abs(g.cpu().numpy() - e.cpu().numpy()).max() <= 1e-13 * np.abs(e.cpu().numpy()).max()
    b.close()
    for m in meshes:
        m.close()


def test_memory_cap_gives_oom(torch_cuda):
    from paper_2005_05899_amd import lesasm
    import gc
    c = mg.small_hybrid_case(nx=6, ny=5, seed=3)
    gc.collect()
    lesasm.release_deferred()  # objects other tests left to the collector: freed before the baseline
    before = lesasm.memory_in_use()
    lesasm.set_memory_cap(before + 4096)
    try:
        with pytest.raises(lesasm.LesasmError) as e:
            lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
        assert e.value.code == -3 and "memory cap" in str(e.value)
        assert lesasm.memory_in_use() == before
    finally:
        lesasm.set_memory_cap(0)
    m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    assert lesasm.memory_in_use() > before
    m.close()
    assert lesasm.memory_in_use() == before
