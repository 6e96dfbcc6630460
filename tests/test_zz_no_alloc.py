"""The allocation-free forward pass of the surrogate (fps_sur_forward_noalloc)
against the handle-based forward pass (fps_sur_forward) through the C-ABI:
the same kernels on the same parameters, so the outputs must be identical bit
for bit, on two calls in a row (the second with a smaller input, which reuses
the static scratch the first one filled), and a call beyond the scratch's
capacity is refused before any device work."""
import numpy as np
import pytest
import torch

from paper_1908_05232_amd import fps, surrogate as SG
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _inputs(seed, n, H, W):
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = torch.zeros(n, H, W, 16)
    x[..., :6] = torch.rand(n, H, W, 6, generator=g) * 2 - 1
    return x.bfloat16().cuda().contiguous()


def test_forward_noalloc_equals_forward():
    params = torch.tensor(SG.init_params(3)).cuda()
    # trained-looking biases: non-zero, so the bias path is exercised too
    params += 0.01 * torch.randn(params.shape, generator=torch.Generator(device="cpu").manual_seed(4)).cuda()
    for call, (n, H, W) in enumerate(((2, 256, 256), (1, 48, 96))):
        x = _inputs(10 + call, n, H, W)
        sur = fps.Surrogate(n, H, W)
        sur.set_params(params)
        ref = sur.forward(x).clone()
        y = torch.full((n, H, W, 4), float("nan"), device="cuda")
        fps.sur_forward_noalloc(params, x, y)
        torch.cuda.synchronize()
        diff = float((y - ref).abs().max())
        say(f"call {call + 1}: {n} x {H} x {W}, max|y - y_handle| = {diff:.3e}, max|y| = {float(ref.abs().max()):.3e}")
        assert torch.equal(y, ref)
        sur.close()
    # beyond the 131,072 pixels of the static scratch: refused, output untouched
    x = _inputs(20, 3, 256, 256)
    y = torch.zeros(3, 256, 256, 4, device="cuda")
    with pytest.raises(fps.FpsError) as err:
        fps.sur_forward_noalloc(params, x, y)
    assert err.value.code == fps.FPS_E_CAPACITY
    torch.cuda.synchronize()
    assert float(y.abs().max()) == 0.0
