"""The loss gradient of the learned closure without device allocation
(lesasm_mlp_loss_grad_noalloc) against the allocating call
(lesasm_mlp_loss_grad) through the C ABI.

Both run the same kernels in the same fixed summation order, so the bar is
bit-for-bit equality of the loss and of all 5254 gradient entries.  Two
no-allocation calls in a row, the first at the 8192-sample maximum and the
second smaller (3001, a ragged block), so the second runs on an area that
still holds the first call's values; the library's counted device bytes must
not move during them.  One sample over the maximum is refused before any
launch.
"""
import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu

MAX_SAMPLES = 8192


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def samples(torch, n, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 10)).astype(np.float32)
    t = rng.standard_normal((n, 6)).astype(np.float32)
    t[:, :3] -= t[:, :3].mean(axis=1, keepdims=True)
    return torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()


def test_noalloc_loss_grad_equals_allocating_call(torch_cuda):
    from paper_2005_05899_amd import lesasm
    torch = torch_cuda
    p = omlp.init_params(31)
    rng = np.random.default_rng(32)
    for k in p:
        p[k] = p[k] + 0.05 * rng.standard_normal(p[k].shape)
    net = lesasm.MLP(omlp.flatten(p).astype(np.float32))
    sizes = (MAX_SAMPLES, 3001)
    inputs = [samples(torch, n, 40 + i) for i, n in enumerate(sizes)]
    outs = [(torch.full((lesasm.MLP_PARAMS,), float("nan"), device="cuda"),
             torch.full((1,), float("nan"), device="cuda")) for _ in sizes]
    torch.cuda.synchronize()
    held = lesasm.memory_in_use()  # (no call below creates or closes a library object)
    for n, (x, t), (g, loss) in zip(sizes, inputs, outs):
        print(f"  noalloc loss_grad, {n} samples", flush=True)
        net.loss_grad_noalloc(x, t, g, loss)
    torch.cuda.synchronize()
    assert lesasm.memory_in_use() == held
    for n, (x, t), (g, loss) in zip(sizes, inputs, outs):
        ref_loss, ref_g = net.loss_grad(x, t)
        torch.cuda.synchronize()
        assert torch.isfinite(g).all() and torch.isfinite(loss).all()
        assert torch.equal(loss, ref_loss), n
        assert torch.equal(g, ref_g), n
    with pytest.raises(lesasm.LesasmError) as e:
        x, t = samples(torch, MAX_SAMPLES + 1, 50)
        net.loss_grad_noalloc(x, t, outs[0][0], outs[0][1])
    assert e.value.code == lesasm.E_INVALID_ARG
    torch.cuda.synchronize()
    net.close()
