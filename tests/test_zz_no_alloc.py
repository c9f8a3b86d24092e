"""fbim_mlp_forward_noalloc (static device scratch, no allocation in the call)
against fbim_mlp_forward (context-allocated activations), through the C ABI:
two calls in a row, the second with a smaller input, each compared with the
allocating entry point on the same inputs.  Same kernels and inputs, so the
outputs must agree exactly."""
import numpy as np
import pytest

from gpu_util import log, make_ctx, workload

pytestmark = pytest.mark.gpu


def test_noalloc_forward_matches_allocating_forward():
    import torch

    import paper_1709_01480_amd as fb
    wl = workload("tiny2")
    ctx = make_ctx(wl)
    ctx.mlp_init(seed=11, sym_order=5)
    rng = np.random.default_rng(4)
    for n in (fb.NOALLOC_MAX_BODIES, 777):
        log("noalloc forward n=%d" % n)
        X = torch.as_tensor(rng.uniform(-1, 1, (n, fb.MLP_IN)).astype(np.float32)).cuda()
        Y_ref = torch.zeros(n * fb.MLP_OUT, dtype=torch.float32, device="cuda")
        Y = torch.full((n * fb.MLP_OUT,), float("nan"), dtype=torch.float32, device="cuda")
        ctx.mlp_forward_noalloc(X, Y)
        ctx.mlp_forward(X, Y_ref)
        torch.cuda.synchronize()
        y, yr = Y.cpu().numpy(), Y_ref.cpu().numpy()
        assert np.all(np.isfinite(yr)) and np.max(np.abs(yr)) > 0
        assert np.array_equal(y, yr)
    # beyond the stated maximum: a clear error, nothing written
    X = torch.zeros((fb.NOALLOC_MAX_BODIES + 1) * fb.MLP_IN, dtype=torch.float32, device="cuda")
    Y = torch.zeros((fb.NOALLOC_MAX_BODIES + 1) * fb.MLP_OUT, dtype=torch.float32, device="cuda")
    with pytest.raises(fb.FbimError) as e:
        ctx.mlp_forward_noalloc(X, Y)
    assert e.value.status == 1
