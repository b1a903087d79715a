"""Checkpoint and resume of (u, p, step, t, seeds) on the CPU: bit-exact round
trip, refusal of another mesh, of a truncated or foreign file, and of
ill-shaped fields; nothing is unpickled."""
import numpy as np
import pytest

from paper_2005_05899_amd import checkpoint as ck
from paper_2005_05899_amd import meshgen as mg


def test_round_trip_is_exact(tmp_path):
    c = mg.small_hybrid_case(nx=4, ny=3, seed=5)
    path = str(tmp_path / "state.npz")
    ck.save(path, c.mesh, c.u, c.p, 17, 0.125, {"seed_u": 3, "seed_mesh": 2})
    u, p, step, t, seeds = ck.load(path, c.mesh)
    assert np.array_equal(u, c.u) and np.array_equal(p, c.p)
    assert (step, t, seeds) == (17, 0.125, {"seed_u": 3, "seed_mesh": 2})


def test_another_mesh_is_refused(tmp_path):
    a = mg.small_hybrid_case(nx=4, ny=3, seed=5)
    b = mg.small_hybrid_case(nx=4, ny=3, seed=6)  # same sizes, other perturbation: same connectivity
    c = mg.small_hybrid_case(nx=5, ny=3, seed=5)
    path = str(tmp_path / "state.npz")
    ck.save(path, a.mesh, a.u, a.p, 1, 0.0)
    ck.load(path, b.mesh)  # node positions are not part of the signature, the topology is
    with pytest.raises(ValueError, match="another mesh"):
        ck.load(path, c.mesh)
    periodic = mg.periodic_tg_case(4)
    ck.save(path, periodic.mesh, periodic.u, periodic.p, 2, 1.0)
    assert ck.load(path, periodic.mesh)[2] == 2
    with pytest.raises(ValueError, match="another mesh"):
        ck.load(path, mg.periodic_hex_cube(5))


def test_bad_files_and_shapes(tmp_path):
    c = mg.small_hybrid_case(nx=4, ny=3, seed=5)
    with pytest.raises(ValueError):
        ck.save(str(tmp_path / "x.npz"), c.mesh, c.u[:, :2], c.p, 0, 0.0)
    with pytest.raises(ValueError):
        ck.save(str(tmp_path / "x.npz"), c.mesh, c.u, c.p[:-1], 0, 0.0)
    foreign = str(tmp_path / "foreign.npz")
    np.savez(foreign, u=c.u, p=c.p, meta=np.frombuffer(b'{"format": "other"}', np.uint8))
    with pytest.raises(ValueError, match="unknown format"):
        ck.load(foreign, c.mesh)
    pickled = str(tmp_path / "pickled.npz")
    np.savez(pickled, u=c.u, p=c.p, meta=np.array([{"format": ck.FORMAT}], dtype=object))
    with pytest.raises(ValueError):  # an object array would need unpickling: refused by numpy
        ck.load(pickled, c.mesh)
