"""The assembly's graph cache (LESASM_OPT_GRAPH): repeated calls with the same
buffers replay a captured graph.  Every replay must equal the eager assembly
of the data the buffers hold at that moment, also after in-place changes of
u and p, eager work and synchronisations in between; a new nu, new buffers,
an option change or a closure drop the capture; a caller's own capture still
records the eager launches."""
import numpy as np
import pytest

from paper_2005_05899_amd import meshgen as mg

# The graph cache is taken out of the library: a run of
# test_switching_buffers_retires_captures aborted inside the mesh's
# destruction after several captures and retirements (all its results had
# matched the eager ones), and no cause was found in the cache's code.  These
# tests stay, skipped, with the option they exercise.
pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="assembly graph cache taken out: an abort in mesh destruction after "
                                      "repeated captures, cause not found")]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    return float((a - b).abs().max() / b.abs().max())


@pytest.mark.parametrize("scatter", ["staged", "chunk_atomic", "direct"])
def test_replays_follow_the_data(torch_cuda, scatter):
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c = mg.small_hybrid_case(nx=7, ny=6, layers=[(mg.PEN06, 2), (mg.TET04, 2), (mg.PYR05, 1), (mg.HEX08, 2)], seed=21)
    mesh = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c, scatter=scatter)
    ref = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c, scatter=scatter)
    ref.set_option(lesasm.OPT_GRAPH, 0)
    assert mesh.get_option(lesasm.OPT_GRAPH) == 1 and ref.get_option(lesasm.OPT_GRAPH) == 0
    u = mesh.to_internal(torch.from_numpy(c.u).cuda())
    p = mesh.to_internal(torch.from_numpy(c.p).cuda())
    rhs = torch.empty_like(u)
    scale = 1.0
    for k in range(6):  # eager, capture, then replays
        mesh.assemble_momentum_rhs(u, p, c.nu, out=rhs)
        torch.cuda.synchronize()
        want = ref.assemble_momentum_rhs(u, p, c.nu)
        torch.cuda.synchronize()
        assert _rel(rhs, want) <= 1e-13, k
        # change the data in place (same buffers) and do other work between calls
        u.mul_(1.05)
        p.add_(0.01)
        scale *= 1.05
        junk = torch.randn(1000, device="cuda").sum()
        float(junk)
    # a different nu, then different buffers: captured again
    for nu in (2 * c.nu, 2 * c.nu, 2 * c.nu):
        mesh.assemble_momentum_rhs(u, p, nu, out=rhs)
        assert _rel(rhs, ref.assemble_momentum_rhs(u, p, nu)) <= 1e-13
    rhs2 = torch.empty_like(u)
    for _ in range(3):
        mesh.assemble_momentum_rhs(u, p, c.nu, out=rhs2)
        assert _rel(rhs2, ref.assemble_momentum_rhs(u, p, c.nu)) <= 1e-13
    # an option change drops the capture: FP32 contractions from then on
    mesh.precision = "fp32"
    ref.precision = "fp32"
    for _ in range(3):
        mesh.assemble_momentum_rhs(u, p, c.nu, out=rhs2)
        assert _rel(rhs2, ref.assemble_momentum_rhs(u, p, c.nu)) <= 1e-12
    mesh.close()
    ref.close()


def test_caller_capture_records_the_launches(torch_cuda):
    # with the cache primed, a caller's own graph capture of the call records
    # the kernels (no nested capture); its replays follow the data
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c = mg.small_hybrid_case(nx=5, ny=4, seed=22)
    mesh = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    u = mesh.to_internal(torch.from_numpy(c.u).cuda())
    p = mesh.to_internal(torch.from_numpy(c.p).cuda())
    rhs = torch.empty_like(u)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for _ in range(3):
            mesh.assemble_momentum_rhs(u, p, c.nu, out=rhs)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        mesh.assemble_momentum_rhs(u, p, c.nu, out=rhs)
    mesh.set_option(lesasm.OPT_GRAPH, 0)
    for k in range(4):
        u.mul_(0.9)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        want = mesh.assemble_momentum_rhs(u, p, c.nu)
        assert _rel(rhs, want) <= 1e-13, k
    del g
    mesh.close()


def test_closure_and_profiling_run_eagerly(torch_cuda):
    from oracle import mlp as omlp
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c = mg.small_hybrid_case(nx=5, ny=4, seed=23)
    mesh = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    u = mesh.to_internal(torch.from_numpy(c.u).cuda())
    p = mesh.to_internal(torch.from_numpy(c.p).cuda())
    rhs = torch.empty_like(u)
    mesh.set_option(lesasm.OPT_PROFILE, 1)
    mesh.kernel_times(reset=True)
    for _ in range(3):
        mesh.assemble_momentum_rhs(u, p, c.nu, out=rhs)
    kt = mesh.kernel_times(reset=True)
    assert max(n for _, n in kt.values()) == 3  # every call's kernels were timed: no replay
    mesh.set_option(lesasm.OPT_PROFILE, 0)
    net = lesasm.MLP(omlp.flatten(omlp.init_params(3)).astype(np.float32))
    lesasm.set_closure(mesh, net, 0.1, 0.05)
    outs = []
    for _ in range(3):
        mesh.assemble_momentum_rhs(u, p, c.nu, out=rhs)
        outs.append(rhs.clone())
    # the fallback count is kept per call (eager launches): three assemblies
    assert lesasm.closure_fallbacks(mesh) % 3 == 0
    assert _rel(outs[2], outs[0]) <= 1e-6
    lesasm.set_closure(mesh, None)
    net.close()
    mesh.close()


def test_switching_buffers_retires_captures(torch_cuda):
    # captures are made and dropped as the output buffer changes, without
    # waiting for the caller: every result equals the eager one
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c = mg.small_hybrid_case(nx=6, ny=5, seed=24)
    mesh = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    ref = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    ref.set_option(lesasm.OPT_GRAPH, 0)
    u = mesh.to_internal(torch.from_numpy(c.u).cuda())
    p = mesh.to_internal(torch.from_numpy(c.p).cuda())
    bufs = [torch.empty_like(u), torch.empty_like(u)]
    outs = []
    for k, b in enumerate([0, 0, 0, 1, 1, 1, 0, 0, 1, 0, 0, 0]):
        u.add_(0.001 * k)
        mesh.assemble_momentum_rhs(u, p, c.nu, out=bufs[b])
        outs.append((bufs[b].clone(), ref.assemble_momentum_rhs(u, p, c.nu)))
    torch.cuda.synchronize()
    for k, (got, want) in enumerate(outs):
        assert _rel(got, want) <= 1e-13, k
    mesh.close()
    ref.close()
