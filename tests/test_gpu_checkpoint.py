"""Checkpoint and resume through the device: a state saved from internal-order
device tensors after a time step and loaded back into them is bit for bit the
state that was saved, and the step and time come back."""
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


def test_save_and_resume_through_the_device(torch_cuda, tmp_path):
    from paper_2005_05899_amd import checkpoint as ck
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    c = mg.small_hybrid_case(nx=6, ny=5, seed=9)
    m = lesasm.Mesh.from_arrays(c.mesh, c.vreman_c)
    st = lesasm.Stepper(m, c.nu, 0.01)
    u = m.to_internal(torch.from_numpy(c.u).cuda())
    p = m.to_internal(torch.from_numpy(c.p).cuda())
    st.step(u, p)
    torch.cuda.synchronize()
    path = str(tmp_path / "state.npz")
    ck.save_device(path, c.mesh, m, u, p, 1, 0.01, {"seed": 9})
    u2, p2, step, t, seeds = ck.load_device(path, c.mesh, m)
    torch.cuda.synchronize()
    assert torch.equal(u2, u) and torch.equal(p2, p)
    assert (step, t, seeds) == (1, 0.01, {"seed": 9})
    st.step(u2, p2)  # the run goes on from the loaded state
    torch.cuda.synchronize()
    assert torch.isfinite(u2).all() and not torch.equal(u2, u)
    st.close()
    m.close()
