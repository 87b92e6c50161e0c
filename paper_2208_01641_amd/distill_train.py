"""Training driver of the distilled synthesis network (host loop only).

Data set: latents and reconstructions of the full decoder.  Each image goes
through the codec's own kernels, g_a with its quantiser (symbols y_hat) and
then g_s (the reconstruction x_hat), layer by layer through the C ABI; the
pairs (y_hat, x_hat) stay on the device.  Training: lic_distill_step on
random batches (forward, MSE, backward, AdamW, all in the library).  The
judge threshold for the decoder's sampled fallback is calibrated on held-out
pairs.
"""
from __future__ import annotations

import math

import numpy as np

from .codec import Codec
from .distill import Distill


def build_pairs(codec: Codec, images, batch: int = 64):
    """images: float32 device tensor [count, 3, H, W] (H, W multiples of 64)
    -> (symbols int8 [count, H/16, W/16, M], reconstructions [count, 3, H, W]),
    both from the full FP32 codec path."""
    import torch

    count, _, H, W = images.shape
    assert H % 64 == 0 and W % 64 == 0
    N, M = codec.N, codec.M
    hy, wy = H // 16, W // 16
    sym = torch.empty((count, hy, wy, M), dtype=torch.int8, device=images.device)
    rec = torch.empty((count, 3, H, W), dtype=torch.float32, device=images.device)
    a = torch.empty((batch, H // 2, W // 2, N), device=images.device)
    b = torch.empty((batch, H // 4, W // 4, N), device=images.device)
    y = torch.empty((batch, hy, wy, M), device=images.device)
    for s in range(0, count, batch):
        n = min(batch, count - s)
        x = images[s:s + n].contiguous()
        codec.run_layer("GA0", n, H, W, x, a)
        codec.run_layer("GA1", n, H, W, a, b)
        c = torch.empty((n, H // 8, W // 8, N), device=images.device)
        codec.run_layer("GA2", n, H, W, b, c)
        codec.run_layer("GA3", n, H, W, c, y, sym[s:s + n])
        codec.run_layer("GS0", n, H, W, sym[s:s + n], c)
        codec.run_layer("GS1", n, H, W, c, b)
        codec.run_layer("GS2", n, H, W, b, a)
        codec.run_layer("GS3", n, H, W, a, rec[s:s + n])
    return sym, rec


def train(net: Distill, sym, target, steps: int, batch: int = 32, seed: int = 0, mu=None):
    """steps AdamW steps on random batches (without replacement inside an
    epoch); returns the per-step losses (numpy)."""
    import torch

    count = sym.shape[0]
    rng = np.random.default_rng(seed)
    losses = torch.zeros(steps, dtype=torch.float32, device=sym.device)
    perm, pos = rng.permutation(count), 0
    for s in range(steps):
        if pos + batch > count:
            perm, pos = rng.permutation(count), 0
        net.step(sym, target, perm[pos:pos + batch], mu=mu, loss_out=losses[s:s + 1])
        pos += batch
    net.sync()
    return losses.cpu().numpy()


def psnr(a, b) -> float:
    mse = float(((a.double() - b.double()) ** 2).mean())
    return float("inf") if mse == 0 else 10.0 * math.log10(1.0 / mse)


def evaluate(net: Distill, sym, rec_full, source, batch: int = 32):
    """Per sample: fidelity PSNR(x_hat_full, x_hat_distilled) and quality gap
    PSNR(x, x_hat_full) - PSNR(x, x_hat_distilled)."""
    import torch

    count, _, H, W = rec_full.shape
    out = torch.empty((batch, 3, H, W), device=sym.device)
    fid, gap = [], []
    for s in range(0, count, batch):
        n = min(batch, count - s)
        net.forward(sym[s:s + n].contiguous(), x_hat=out[:n])
        for i in range(n):
            xf, xd, x = rec_full[s + i], out[i], source[s + i]
            fid.append(psnr(xf, xd))
            gap.append(psnr(x, xf) - psnr(x, xd))
    return np.array(fid), np.array(gap)


def judge_threshold(fidelity, gap, max_gap_db: float = 0.1) -> float:
    """Smallest fidelity threshold T such that every held-out sample with
    fidelity >= T loses at most max_gap_db against the full g_s; +inf when
    no threshold admits any sample."""
    order = np.argsort(-np.asarray(fidelity))
    best = float("inf")
    for i in order:                       # admit samples from the most faithful down
        if gap[i] > max_gap_db:
            break
        best = float(fidelity[i])
    return best
