"""The allocation-free curvature evaluation (mf_mlp_eval_noalloc) against mf_mlp_eval.

Both run the same canonicalisation and matrix-core kernels, so the curvature of every
stencil must agree exactly. Two calls in a row, the second with fewer stencils (its
padding rows then hold the first call's values, which the entry point must clear), and
a call beyond the array's capacity, which must be refused without touching the GPU.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_noalloc_eval_matches_allocating_eval():
    import torch

    from paper_1908_04262_amd import CurvatureNet, MifoamError, generate_stencils
    net = CurvatureNet(5)
    rng = np.random.default_rng(3)
    theta = net.params() + rng.normal(size=net.nparam).astype(np.float32) * 0.05
    theta[125 * 64:128 * 64] = 0.0
    net.set_params(theta)
    for n in (5000, 301):
        _say(f"noalloc eval: {n} stencils")
        X, _ = generate_stencils(11, 7 * n, n)
        want = net.eval(X)
        Xd = torch.from_numpy(X).to("cuda:0")
        kd = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda:0")
        net.eval_noalloc(Xd, kd)
        torch.cuda.synchronize()
        got = kd.cpu().numpy()
        assert np.isfinite(got).all()
        assert np.array_equal(got, want), np.abs(got - want).max()
    big = torch.zeros((8193, 125), dtype=torch.float32, device="cuda:0")
    kb = torch.zeros(8193, dtype=torch.float32, device="cuda:0")
    with pytest.raises(MifoamError, match="MF_EINVAL.*at most 8192"):
        net.eval_noalloc(big, kb)
    net.close()
