"""Stored oracle values (tests/golden/, written by make_golden.py from the
oracle alone): the oracle must keep reproducing them (no silent drift of the
oracle or of the seeded input generators), and the GPU library must match
them at the FP64 parity bar."""
import os

import numpy as np
import pytest

import oracle
from paper_2005_05899_amd import meshgen

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    return np.loadtxt(os.path.join(HERE, name))


def _small():
    return meshgen.small_hybrid_case(nx=3, ny=2, seed=7)


def _tg():
    return meshgen.periodic_tg_case(16)


def _tg_norms():
    with open(os.path.join(HERE, "tg16_rhs_sample.txt")) as f:
        for line in f:
            if "column 2-norms" in line:
                return np.array([float(v) for v in line.split(":")[1].split()])
    raise AssertionError("norm line missing")


def test_oracle_reproduces_small_hybrid_golden():
    c = _small()
    got = oracle.assemble(c.mesh, c.u, c.p, c.nu, c.vreman_c)
    ref = _load("small_hybrid_rhs.txt")
    assert got.shape == ref.shape
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_oracle_reproduces_tg16_golden():
    t = _tg()
    got = oracle.assemble(t.mesh, t.u, t.p, t.nu, t.vreman_c)
    rows = _load("tg16_rhs_sample.txt")
    idx = rows[:, 0].astype(int)
    np.testing.assert_allclose(got[idx], rows[:, 1:], rtol=0, atol=1e-13 * np.abs(got).max())
    np.testing.assert_allclose(np.linalg.norm(got, axis=0), _tg_norms(), rtol=1e-13)


@pytest.mark.gpu
def test_gpu_matches_small_hybrid_golden():
    import torch
    from paper_2005_05899_amd import lesasm
    c = _small()
    mesh = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    u = mesh.to_internal(torch.from_numpy(c.u).cuda())
    p = mesh.to_internal(torch.from_numpy(c.p).cuda())
    got = mesh.to_user(mesh.assemble_momentum_rhs(u, p, c.nu)).cpu().numpy()
    mesh.close()
    ref = _load("small_hybrid_rhs.txt")
    for i in range(3):
        err = np.linalg.norm(got[:, i] - ref[:, i]) / np.linalg.norm(ref[:, i])
        assert err < 1e-12, (i, err)


@pytest.mark.gpu
def test_gpu_matches_tg16_golden():
    import torch
    from paper_2005_05899_amd import lesasm
    t = _tg()
    mesh = lesasm.Mesh.from_arrays(t.mesh, t.vreman_c)
    u = mesh.to_internal(torch.from_numpy(t.u).cuda())
    p = mesh.to_internal(torch.from_numpy(t.p).cuda())
    got = mesh.to_user(mesh.assemble_momentum_rhs(u, p, t.nu)).cpu().numpy()
    mesh.close()
    rows = _load("tg16_rhs_sample.txt")
    idx = rows[:, 0].astype(int)
    scale = np.abs(rows[:, 1:]).max()
    assert np.abs(got[idx] - rows[:, 1:]).max() < 1e-12 * scale
    np.testing.assert_allclose(np.linalg.norm(got, axis=0), _tg_norms(), rtol=1e-12)
