"""The allocation-free forward pass of the distilled synthesis network
(lic_distill_forward_noalloc) against lic_distill_forward.

Both run the same kernels on the same packed weights; only where the hidden
activations live differs (the library's fixed per-device workspace instead of
the handle's buffers), so the outputs must be identical bit for bit.  Two
calls in a row, the second smaller, check that nothing of the first call's
workspace contents leaks into the second.  A call larger than the workspace
is refused on the host with LIC_E_BUDGET before anything is launched.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
M, F = 192, 64


def _sym(rng, n, hy, wy):
    return np.clip(np.rint(rng.laplace(0.0, 2.0, (n, hy, wy, M))), -64, 64).astype(np.int8)


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_forward_equals_forward(precision):
    import torch
    from paper_2208_01641_amd import Distill
    assert torch.cuda.is_available()
    P = synth.distill_params(M, F, seed=2209)
    rng = np.random.default_rng(55 + precision)
    mu = torch.from_numpy(rng.uniform(-0.5, 0.5, M).astype(np.float32)).cuda()
    d = Distill(P, M, F, precision=precision, max_batch=2, max_hy=48, max_wy=80, train=False)
    # a full 720p latent grid, then a smaller batch of two ragged crops
    for n, hy, wy, H, W in [(1, 48, 80, 720, 1280), (2, 7, 11, 100, 171)]:
        print(f"noalloc forward: precision {precision}, n {n}, latents {hy}x{wy}, crop {H}x{W}", flush=True)
        sym = torch.from_numpy(_sym(rng, n, hy, wy)).cuda()
        outs = []
        for fn in (d.forward, d.forward_noalloc):
            pre = torch.full((n, 3, 16 * hy, 16 * wy), float("nan"), device="cuda")
            xh = torch.full((n, 3, H, W), float("nan"), device="cuda")
            fn(sym, mu=mu, pre=pre, x_hat=xh)
            outs.append((pre.cpu(), xh.cpu()))
        (p0, x0), (p1, x1) = outs
        assert torch.isfinite(p0).all() and torch.isfinite(x0).all()
        assert torch.equal(p0, p1), f"pre-clamp output differs at n={n} {hy}x{wy}"
        assert torch.equal(x0, x1), f"image differs at n={n} {hy}x{wy}"
    d.close()


def test_noalloc_forward_rejects_calls_beyond_the_workspace():
    import torch
    from paper_2208_01641_amd import Distill, LicError
    P = synth.distill_params(M, F, seed=2209)
    d = Distill(P, M, F, precision=0, max_batch=2, max_hy=48, max_wy=80, train=False)
    # two 720p latent grids in FP32: 2 * 80 * 48 * 80 * 64 bytes > 32 MiB
    sym = torch.zeros((2, 48, 80, M), dtype=torch.int8, device="cuda")
    pre = torch.empty((2, 3, 768, 1280), device="cuda")
    with pytest.raises(LicError) as e:
        d.forward_noalloc(sym, pre=pre)
    assert e.value.code == -6 and "workspace" in str(e.value)
    d.close()
