"""GPU wall model (boundary assembly) against the oracle, element by element
on seeded inputs: triangles (prism and tetrahedron walls), quads (hexahedron
walls), the 2.0 M-element hybrid box, and the error paths."""
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


def _run(torch, mesh_arrays, u, nu, faces, vreman_c=0.1):
    from paper_2005_05899_amd import lesasm
    m = lesasm.Mesh.from_arrays(mesh_arrays, vreman_c)
    m.set_wall(*faces)
    ui = m.to_internal(torch.from_numpy(u).cuda())
    out = torch.zeros_like(ui)
    m.assemble_wall(ui, nu, out)
    got = m.to_user(out).cpu().numpy()
    m.close()
    return got


def _compare(got, ref, tol=1e-12):
    for i in range(3):
        n = np.linalg.norm(ref[:, i])
        if n == 0:
            assert np.abs(got[:, i]).max() < 1e-300
            continue
        assert np.linalg.norm(got[:, i] - ref[:, i]) / n < tol, i


@pytest.mark.parametrize("layers", [[(mg.PEN06, 2), (mg.HEX08, 1)], [(mg.TET04, 2), (mg.PYR05, 1), (mg.HEX08, 1)],
                                    [(mg.HEX08, 3)], [(mg.PYR05, 1), (mg.HEX08, 2)]])
def test_wall_matches_oracle_small(torch_cuda, layers):
    import oracle
    mesh = mg.hybrid_box(5, 4, layers, seed=21)
    xf = mesh.field_coords()
    u = mg.random_fourier_velocity(n_modes=64, kmax=4, seed=31)(xf)
    faces = mg.wall_faces(mesh)
    assert len(faces[2]) > 0
    ref, *_ = oracle.wall_assemble(mesh, u, 1e-3, *faces)
    got = _run(torch_cuda, mesh, u, 1e-3, faces)
    _compare(got, ref)


def test_wall_on_a_periodic_field_map(torch_cuda):
    # a periodic map in x and y (field nodes folded), wall at z = 0
    import oracle
    mesh = mg.hybrid_box(4, 4, [(mg.PEN06, 2), (mg.HEX08, 1)], seed=5)
    c = mesh.coords
    lx, ly = c[:, 0].max(), c[:, 1].max()
    key = np.stack([np.where(np.isclose(c[:, 0], lx), 0.0, c[:, 0]), np.where(np.isclose(c[:, 1], ly), 0.0, c[:, 1]),
                    c[:, 2]], axis=1).round(9)
    _, fmap = np.unique(key, axis=0, return_inverse=True)
    folded = mg.Mesh(mesh.coords, mesh.types, mesh.conn_offsets, mesh.conn, fmap.astype(np.int32).ravel(),
                     int(fmap.max()) + 1)
    u = np.random.default_rng(2).uniform(-1, 1, (folded.n_field_nodes, 3))
    faces = mg.wall_faces(folded)
    ref, *_ = oracle.wall_assemble(folded, u, 2e-3, *faces)
    got = _run(torch_cuda, folded, u, 2e-3, faces)
    _compare(got, ref)


def test_wall_hybrid_2m_full(torch_cuda):
    import oracle
    case = mg.hybrid_2m_case()
    faces = mg.wall_faces(case.mesh)
    assert len(faces[2]) == 2 * 95 * 95
    ref, *_ = oracle.wall_assemble(case.mesh, case.u, case.nu, *faces)
    got = _run(torch_cuda, case.mesh, case.u, case.nu, faces)
    _compare(got, ref)


def test_wall_errors_and_empty(torch_cuda):
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    mesh = mg.hybrid_box(3, 3, [(mg.HEX08, 2)], seed=1)
    m = lesasm.Mesh.from_arrays(mesh, 0.1)
    u = torch.ones((m.n_field_nodes, 3), dtype=torch.float64, device="cuda")
    out = torch.zeros_like(u)
    m.assemble_wall(u, 1e-3, out)  # no wall: no-op
    assert float(out.abs().max()) == 0.0
    with pytest.raises(lesasm.LesasmError):
        m.set_wall(np.array([0, 5]), np.arange(5, dtype=np.int32), np.array([0]))
    with pytest.raises(lesasm.LesasmError):
        m.set_wall(np.array([0, 4]), np.array([0, 1, 2, 10 ** 6], np.int32), np.array([0]))
    with pytest.raises(lesasm.LesasmError):
        m.set_wall(np.array([0, 4]), np.array([0, 1, 2, 3], np.int32), np.array([10 ** 6]))
    faces = mg.wall_faces(mesh)
    m.set_wall(*faces)
    with pytest.raises(lesasm.LesasmError):
        m.assemble_wall(u, 0.0, out)
    m.set_wall(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int64))  # removes the wall
    m.assemble_wall(u, 1e-3, out)
    assert float(out.abs().max()) == 0.0
    m.close()
