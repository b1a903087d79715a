"""GPU path against the FP64 oracle (needs an MI355X and the built library).

Bars: FP64 per field (velocity component) relative L2 and relative max error
<= 1e-12; FP32 contractions <= 1e-5.  Integer/index work (permutations) is
bit-exact.  Colour scatter is bitwise reproducible run to run.
"""
import numpy as np
import pytest

from paper_2005_05899_amd import meshgen as mg

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def field_errors(got, ref):
    """Per component: (relative L2, relative max) of got vs ref."""
    out = []
    for i in range(ref.shape[1]):
        d = got[:, i] - ref[:, i]
        n2 = np.linalg.norm(ref[:, i])
        nm = np.abs(ref[:, i]).max()
        out.append((np.linalg.norm(d) / n2 if n2 else np.linalg.norm(d),
                    np.abs(d).max() / nm if nm else np.abs(d).max()))
    return out


def assert_close(got, ref, tol, what=""):
    assert np.isfinite(got).all(), (what, "non-finite output: a node left unwritten or a NaN")
    errs = field_errors(got, ref)
    worst = max(max(e) for e in errs)
    print(f"  {what}: worst per-field error {worst:.3e}", flush=True)
    assert worst <= tol, (what, errs)


def run_gpu(torch, case, colour=False, keep_order=False, precision="fp64", with_p=True, mesh=None, scatter=None,
            chunk=None):
    from paper_2005_05899_amd import lesasm
    m = mesh or lesasm.Mesh.from_arrays(case.mesh, case.vreman_c, colour=colour, keep_order=keep_order,
                                        scatter=scatter)
    if chunk is not None:
        m.set_option(lesasm.OPT_CHUNK, chunk)
    m.precision = precision
    u = m.to_internal(torch.from_numpy(case.u).cuda())
    p = m.to_internal(torch.from_numpy(case.p).cuda()) if (with_p and case.p is not None) else None
    # NaN-filled output: every scatter mode must write every node
    rhs = m.to_user(m.assemble_momentum_rhs(u, p, case.nu, out=torch.full_like(u, float("nan"))))
    torch.cuda.synchronize()
    return rhs.cpu().numpy(), m


@pytest.fixture(scope="module")
def periodic():
    import oracle
    c = mg.periodic_tg_case(16)
    return c, oracle.assemble(c.mesh, c.u, c.p, c.nu, c.vreman_c)


@pytest.fixture(scope="module")
def small():
    import oracle
    c = mg.small_hybrid_case(nx=7, ny=5, layers=[(mg.PEN06, 3), (mg.TET04, 3), (mg.PYR05, 2), (mg.HEX08, 3)], seed=11)
    return c, oracle.assemble(c.mesh, c.u, c.p, c.nu, c.vreman_c)


@pytest.mark.parametrize("scatter", ["staged", "chunk_atomic", "colour", "direct"])
def test_periodic_cube_fp64(torch_cuda, periodic, scatter):
    c, ref = periodic
    got, m = run_gpu(torch_cuda, c, scatter=scatter)
    assert_close(got, ref, TOL64, f"periodic 16^3 HEX08 fp64 {scatter}")
    m.close()


@pytest.mark.parametrize("scatter", ["staged", "chunk_atomic", "colour", "direct"])
@pytest.mark.parametrize("keep", [False, True])
def test_small_hybrid_fp64(torch_cuda, small, scatter, keep):
    c, ref = small
    got, m = run_gpu(torch_cuda, c, scatter=scatter, keep_order=keep)
    assert_close(got, ref, TOL64, f"small hybrid ({c.mesh.n_elems} el) scatter={scatter} keep={keep}")
    if scatter == "colour":
        assert all(v > 0 for t, v in m.n_colours.items() if m.n_per_type[t] > 0)
    m.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("scatter", ["staged", "chunk_atomic"])
@pytest.mark.parametrize("chunk", [32, 100, 1024, 4096, 0])
def test_chunk_sizes(torch_cuda, small, periodic, chunk, scatter, precision):
    """Many small chunks (ragged last chunks), chunks longer than a workgroup
    (FP32: 512-thread workgroups, several elements per thread), one chunk per
    type, and the per-type default; the periodic cube exercises separate
    geometry and field node lists."""
    tol = TOL64 if precision == "fp64" else TOL32
    for c, ref in (small, periodic):
        got, m = run_gpu(torch_cuda, c, chunk=chunk, scatter=scatter, precision=precision)
        assert_close(got, ref, tol, f"{c.name} {scatter} chunk={chunk} {precision}")
        m.close()


@pytest.mark.parametrize("chunk", [32, 1024])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("persist", [0, 1, 3])
def test_persistent_chunk_loop(torch_cuda, small, periodic, persist, precision, chunk):
    """Workgroups looping over chunks: one workgroup per chunk (0), as many as
    the GPU holds (1), and three workgroups that each process many chunks (3),
    with short chunks so that every workgroup loops, and with chunks longer
    than a workgroup (FP32 in 512-thread workgroups)."""
    from paper_2005_05899_amd import lesasm
    tol = TOL64 if precision == "fp64" else TOL32
    for c, ref in (small, periodic):
        m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
        m.set_option(lesasm.OPT_PERSISTENT, persist)
        got, m = run_gpu(torch_cuda, c, chunk=chunk, mesh=m, precision=precision)
        assert_close(got, ref, tol, f"{c.name} persist={persist} chunk={chunk} {precision}")
        m.close()


def test_staged_scatter_overwrites_every_node(torch_cuda, small):
    """No zero-fill in the staged scatter: every node is stored exactly once,
    so a NaN-filled output buffer must come back fully overwritten."""
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c, ref = small
    m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    u = m.to_internal(torch.from_numpy(c.u).cuda())
    p = m.to_internal(torch.from_numpy(c.p).cuda())
    out = torch.full_like(u, float("nan"))
    got = m.to_user(m.assemble_momentum_rhs(u, p, c.nu, out=out)).cpu().numpy()
    assert np.isfinite(got).all()
    assert_close(got, ref, TOL64, "staged, NaN-filled output")
    m.close()


def test_small_hybrid_without_pressure(torch_cuda, small):
    import oracle
    c, _ = small
    ref = oracle.assemble(c.mesh, c.u, None, c.nu, c.vreman_c)
    got, m = run_gpu(torch_cuda, c, with_p=False)
    assert_close(got, ref, TOL64, "small hybrid, p = NULL")
    m.close()


def test_colour_scatter_is_bitwise_reproducible(torch_cuda, small):
    c, ref = small
    a, m = run_gpu(torch_cuda, c, colour=True)
    b, _ = run_gpu(torch_cuda, c, mesh=m)
    assert np.array_equal(a, b)
    at, m2 = run_gpu(torch_cuda, c)
    assert_close(at, a, 1e-13, "atomic vs colour")
    m.close()
    m2.close()


@pytest.mark.parametrize("t", [mg.TET04, mg.PYR05, mg.PEN06, mg.HEX08])
def test_single_type_meshes(torch_cuda, t):
    """One type at a time, element counts that leave ragged tails."""
    import oracle
    c = mg.small_hybrid_case(nx=3, ny=2, layers=[(t, 2)], seed=20 + t)
    ref = oracle.assemble(c.mesh, c.u, c.p, c.nu, c.vreman_c)
    got, m = run_gpu(torch_cuda, c)
    assert_close(got, ref, TOL64, f"{mg.TYPE_NAME[t]} x {c.mesh.n_elems}")
    m.close()


def test_single_element(torch_cuda):
    """One element per type with random nodal data (a one-cell box spans a whole
    period of the Fourier fields, which would make them constant)."""
    import oracle
    for t in (mg.TET04, mg.PYR05, mg.PEN06, mg.HEX08):
        c = mg.small_hybrid_case(nx=1, ny=1, layers=[(t, 1)], seed=30 + t)
        one = mg.Mesh(c.mesh.coords, c.mesh.types[:1], c.mesh.conn_offsets[:2], c.mesh.conn[:t])
        rng = np.random.default_rng(t)
        u = rng.standard_normal((one.n_nodes, 3))
        p = rng.standard_normal(one.n_nodes)
        case = mg.Case("one", one, u, p, 0.3, 0.1)
        ref = oracle.assemble(one, u, p, 0.3, 0.1)
        got, m = run_gpu(torch_cuda, case)
        assert_close(got, ref, TOL64, f"single {mg.TYPE_NAME[t]}")
        m.close()


def test_empty_mesh(torch_cuda):
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    coords = np.random.default_rng(0).standard_normal((5, 3))
    m = lesasm.Mesh(coords, np.zeros(0, np.uint8), np.zeros(1, np.int64), np.zeros(0, np.int32))
    u = torch.ones((5, 3), dtype=torch.float64, device="cuda")
    rhs = m.assemble_momentum_rhs(u, None, 0.1)
    torch.cuda.synchronize()
    assert (rhs.cpu().numpy() == 0).all()
    m.close()


def test_check_reports_clean_stream(torch_cuda, small):
    """lesasm_check waits for the stream and returns OK after good work."""
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c, _ = small
    m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    u = m.to_internal(torch.from_numpy(c.u).cuda())
    m.assemble_momentum_rhs(u, None, c.nu)
    lesasm.check_stream()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        m.assemble_momentum_rhs(u, None, c.nu)
    lesasm.check_stream(s.cuda_stream)
    m.close()


def test_lumped_mass_and_filter_width(torch_cuda, small):
    import oracle
    torch = torch_cuda
    c, _ = small
    from paper_2005_05899_amd import lesasm
    m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    M = m.to_user(m.lumped_mass().reshape(-1, 1)).cpu().numpy()[:, 0]
    Mref = oracle.lumped_mass(c.mesh)
    assert np.abs(M - Mref).max() <= 1e-13 * Mref.max()
    d = m.filter_width().cpu().numpy()
    dref = oracle.filter_width(c.mesh)[m.element_permutation()]
    assert np.abs(d - dref).max() <= 1e-14 * dref.max()
    m.close()


def test_permutations_roundtrip_bit_exact(torch_cuda, small):
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c, _ = small
    m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    perm = m.node_permutation()
    assert np.array_equal(np.sort(perm), np.arange(m.n_field_nodes))
    x = torch.from_numpy(np.random.default_rng(1).standard_normal((m.n_field_nodes, 5))).cuda()
    xi = m.to_internal(x)
    assert torch.equal(xi.cpu(), x.cpu()[torch.from_numpy(perm).long()])
    assert torch.equal(m.to_user(xi), x)
    m.close()


def test_increment_mode(torch_cuda, small):
    import oracle
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c, ref = small
    m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    m.set_option(lesasm.OPT_RHS_MODE, lesasm.RHS_INCREMENT)
    u = m.to_internal(torch.from_numpy(c.u).cuda())
    p = m.to_internal(torch.from_numpy(c.p).cuda())
    dt = 1e-3
    inc = m.to_user(m.assemble_momentum_rhs(u, p, c.nu, dt)).cpu().numpy()
    expect = dt * ref / oracle.lumped_mass(c.mesh)[:, None]
    assert_close(inc, expect, TOL64, "increment dt M^-1 R")
    m.close()


def test_nonfinite_check(torch_cuda, small):
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c, _ = small
    m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    m.set_option(lesasm.OPT_CHECK_FINITE, 1)
    u = torch.from_numpy(c.u).cuda().contiguous()
    m.assemble_momentum_rhs(u, None, c.nu)
    u[3, 1] = float("nan")
    with pytest.raises(lesasm.LesasmError) as ei:
        m.assemble_momentum_rhs(u, None, c.nu)
    assert ei.value.code == lesasm.E_NONFINITE
    m.close()


def test_inverted_element_is_reported(torch_cuda):
    from paper_2005_05899_amd import lesasm
    m = mg.uniform_hex_box((3, 1, 1))
    conn = m.conn.copy()
    o = m.conn_offsets[2]
    conn[o:o + 8] = np.concatenate([m.conn[o + 4:o + 8], m.conn[o:o + 4]])
    with pytest.raises(lesasm.LesasmError) as ei:
        lesasm.Mesh(m.coords, m.types, m.conn_offsets, conn)
    assert ei.value.code == lesasm.E_INVERTED_ELEMENT and "element 2 " in str(ei.value)


@pytest.mark.parametrize("precision,tol", [("fp32", TOL32)])
def test_small_hybrid_fp32(torch_cuda, small, precision, tol):
    c, ref = small
    got, m = run_gpu(torch_cuda, c, precision=precision)
    assert_close(got, ref, tol, "small hybrid fp32 contractions")
    m.close()


def test_periodic_cube_fp32(torch_cuda, periodic):
    c, ref = periodic
    got, m = run_gpu(torch_cuda, c, precision="fp32")
    assert_close(got, ref, TOL32, "periodic 16^3 fp32 contractions")
    m.close()


@pytest.fixture(scope="module")
def hybrid2m():
    import oracle
    c = mg.hybrid_2m_case()
    return c, oracle.assemble(c.mesh, c.u, c.p, c.nu, c.vreman_c)


def test_hybrid_2m_fp64_full(torch_cuda, hybrid2m):
    """The benchmark's 2.0 M sub-record workload (2.0 M hybrid elements) in the
    benchmark's launch configuration, every node compared with the oracle."""
    c, ref = hybrid2m
    got, m = run_gpu(torch_cuda, c)
    assert_close(got, ref, TOL64, "2M hybrid fp64 staged scatter")
    m.close()


def test_hybrid_2m_fp32_full(torch_cuda, hybrid2m):
    c, ref = hybrid2m
    got, m = run_gpu(torch_cuda, c, precision="fp32")
    assert_close(got, ref, TOL32, "2M hybrid fp32 contractions")
    m.close()


@pytest.mark.parametrize("scatter", ["chunk_atomic", "colour", "direct"])
def test_hybrid_2m_other_scatters(torch_cuda, hybrid2m, scatter):
    c, ref = hybrid2m
    got, m = run_gpu(torch_cuda, c, scatter=scatter)
    assert_close(got, ref, TOL64, f"2M hybrid fp64 {scatter}")
    m.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_captured_assembly_replays(torch_cuda, small, precision):
    # one assembly (fork to the side streams, four element kernels, join,
    # gather) captured in a HIP graph; every replay, with eager work in
    # between, must equal the eager result and match the oracle
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c, ref = small
    m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    m.precision = precision
    u = m.to_internal(torch.from_numpy(c.u).cuda())
    p = m.to_internal(torch.from_numpy(c.p).cuda())
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        eager = m.assemble_momentum_rhs(u, p, c.nu).clone()
        out = torch.empty_like(u)
        m.assemble_momentum_rhs(u, p, c.nu, out=out)  # warm the stream
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        m.assemble_momentum_rhs(u, p, c.nu, out=out)
    torch.cuda.synchronize()
    for rep in range(4):
        out.fill_(float("nan"))
        other = m.assemble_momentum_rhs(u * 0.5, p, c.nu)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        diff = float((out - eager).abs().max() / eager.abs().max())
        assert diff <= (1e-14 if precision == "fp64" else 1e-6), (rep, diff)
        assert torch.isfinite(other).all()
    assert_close(m.to_user(out).cpu().numpy(), ref, TOL64 if precision == "fp64" else TOL32, f"graph {precision}")
    del g
    m.close()
