"""grim_mlp_backward_noalloc (the gradient call for callers that cannot
allocate device memory) against grim_mlp_backward through the C ABI: two
calls in a row on one context, the second with fewer rows, each equal to the
allocating call's gradient on the same rows, and both within the allocating
call's bound against the FP64 oracle.  The two run the same kernels on the
same rows, so they agree bit for bit; the oracle bound is the one the
backward test uses (1e-4 of the gradient's norm, FP32 arithmetic)."""
import numpy as np
import pytest

from oracle import mlp_oracle as M
from paper_1702_01106_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_noalloc_backward_matches_allocating_call():
    import torch

    from paper_1702_01106_amd import grim

    assert torch.cuda.is_available()
    g = grim.Context(W.small("emhd2d_modes_256", [16, 16]))
    rng = np.random.default_rng(21)
    th = M.init_params(21, x_mean=rng.normal(0, 0.5, M.D_IN), x_istd=rng.uniform(0.5, 2.0, M.D_IN),
                       y_scale=rng.uniform(0.5, 2.0, M.D_OUT)).astype(np.float32)
    grim.grim_mlp_set_weights(g.ctx, th)
    for n in (2048, 733):  # the scratch's full 2048 rows, then a smaller, ragged call
        print(f"no-alloc backward, n = {n}", flush=True)
        X = rng.normal(0, 1, (n, M.D_IN)).astype(np.float32)
        dY = rng.normal(0, 1, (n, M.D_OUT)).astype(np.float32)
        Xd, dYd = torch.from_numpy(X).cuda(), torch.from_numpy(dY).cuda()
        ref_dev = torch.empty(M.N_PARAMS, dtype=torch.float32, device="cuda")
        grim.grim_mlp_backward(g.ctx, Xd, dYd, n, ref_dev)
        # the no-alloc call writes over stale values: every entry must be set
        got_dev = torch.full((M.N_PARAMS,), float("nan"), dtype=torch.float32, device="cuda")
        grim.grim_mlp_backward_noalloc(g.ctx, Xd, dYd, n, got_dev)
        torch.cuda.synchronize()
        got, ref = got_dev.cpu().numpy(), ref_dev.cpu().numpy()
        assert np.array_equal(got, ref), np.abs(got - ref).max()
        assert np.all(got[M.N_PARAMS - 80:] == 0.0)
        exact = M.backward(th.astype(np.float64), X.astype(np.float64), dY.astype(np.float64))
        assert np.linalg.norm(got - exact) <= 1e-4 * np.linalg.norm(exact)
    # beyond the scratch: a clear error, nothing enqueued
    n = 2049
    X = torch.zeros((n, M.D_IN), dtype=torch.float32, device="cuda")
    dY = torch.zeros((n, M.D_OUT), dtype=torch.float32, device="cuda")
    dW = torch.zeros(M.N_PARAMS, dtype=torch.float32, device="cuda")
    with pytest.raises(grim.GrimError, match="exceeds the 2048 rows"):
        grim.grim_mlp_backward_noalloc(g.ctx, X, dY, n, dW)
    g.close()
