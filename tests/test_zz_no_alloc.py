"""The allocation-free CNN forward (pngf_model_forward_noalloc: device
pointers in and out, scratch in the library's file-scope device array)
against pngf_model_forward on the same parameters and inputs: the same
kernels and arithmetic, so the outputs are bit-identical.  Two calls in a
row, the second with a smaller input, then a call past the size limit."""
import numpy as np
import pytest

import paper_2501_18054_amd as P
from gpu_util import say

pytestmark = pytest.mark.gpu


def _ref_and_noalloc(H, W, N, seed):
    import torch
    rng = np.random.default_rng(seed)
    m = P.Model(H, W, max_batch=N, seed=seed)
    params = m.get_params() + rng.normal(0.0, 0.01, m.num_params).astype(np.float32)
    m.set_params(params)
    X = rng.normal(0.0, 1.0, (N, 7, H, W)).astype(np.float32)
    want = m.forward(X)
    m.close()
    dp = torch.from_numpy(params).cuda()
    dX = torch.from_numpy(X).cuda()
    dY = torch.full((N, 1, H, W), float("nan"), dtype=torch.float32, device="cuda")
    P.model_forward_noalloc(dp, dX, dY)
    torch.cuda.synchronize()
    return want, dY.cpu().numpy()


def test_noalloc_forward_equals_model_forward():
    say("no-alloc forward: 4 x 40x40, then 1 x 24x20")
    want, got = _ref_and_noalloc(40, 40, 4, 11)
    assert np.array_equal(want, got)
    # second call, smaller input: the scratch keeps the first call's
    # contents, which must not leak into this one
    want, got = _ref_and_noalloc(24, 20, 1, 12)
    assert np.array_equal(want, got)


def test_noalloc_forward_rejects_oversize():
    import torch
    say("no-alloc forward: size limit")
    m = P.Model(8, 8, max_batch=1, seed=1)
    dp = torch.from_numpy(m.get_params()).cuda()
    m.close()
    dX = torch.zeros((1, 7, 129, 128), dtype=torch.float32, device="cuda")
    dY = torch.zeros((1, 1, 129, 128), dtype=torch.float32, device="cuda")
    with pytest.raises(P.PngfError) as e:
        P.model_forward_noalloc(dp, dX, dY)
    assert e.value.code == -1
    with pytest.raises(P.PngfError):
        P.model_forward_noalloc(dp[:-1].contiguous(), dX[:, :, :8, :8].contiguous(),
                                dY[:, :, :8, :8].contiguous())
