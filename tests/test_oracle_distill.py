"""Pins of the oracle's distilled synthesis network: backward pass and AdamW."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
import synth

rng = np.random.default_rng(11)


def _tiny(M=4, Fc=3):
    P = synth.distill_params(M, Fc, seed=5)
    return {k: np.asarray(v, np.float64) for k, v in P.items()}


def test_shapes_upsample_16x():
    P = _tiny()
    out, acts = oracle.distill_forward(P, rng.standard_normal((2, 4, 2, 3)))
    assert out.shape == (2, 3, 32, 48)
    assert [a.shape for a in acts[0]] == [(4, 2, 3), (3, 4, 6), (3, 8, 12), (3, 32, 48)]


def test_gradients_match_central_differences():
    P = _tiny()
    y = rng.standard_normal((2, 4, 2, 2))
    tgt = rng.uniform(0, 1, (2, 3, 32, 32))
    loss, g = oracle.distill_loss_and_grads(P, y, tgt)
    h = 1e-6
    for name in P:
        flat = P[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = oracle.distill_loss_and_grads(P, y, tgt)[0]
            flat[idx] = old - h
            lm = oracle.distill_loss_and_grads(P, y, tgt)[0]
            flat[idx] = old
            num = (lp - lm) / (2 * h)
            assert g[name].reshape(-1)[idx] == pytest.approx(num, rel=1e-5, abs=1e-10), (name, idx)


def test_gradients_match_torch_autograd():
    P = _tiny(M=5, Fc=4)
    y = rng.standard_normal((3, 5, 3, 2))
    tgt = rng.uniform(0, 1, (3, 3, 48, 32))
    loss, g = oracle.distill_loss_and_grads(P, y, tgt)
    T = {k: torch.tensor(v, requires_grad=True) for k, v in P.items()}
    h = torch.tensor(y)
    h = F.relu(F.conv_transpose2d(h, T["t1.w"], T["t1.b"], stride=2, padding=2, output_padding=1))
    h = F.relu(F.conv_transpose2d(h, T["t2.w"], T["t2.b"], stride=2, padding=2, output_padding=1))
    out = F.conv_transpose2d(h, T["t3.w"], T["t3.b"], stride=4, padding=2)
    ref = torch.mean((out - torch.tensor(tgt)) ** 2)
    ref.backward()
    assert loss == pytest.approx(ref.item(), rel=1e-12)
    for k in P:
        np.testing.assert_allclose(g[k], T[k].grad.numpy(), rtol=1e-10, atol=1e-14)


def test_dgrad_is_adjoint_of_deconv():
    x = rng.standard_normal((4, 5, 6))
    w = rng.standard_normal((4, 3, 8, 8))
    gy = rng.standard_normal((3, 20, 24))
    lhs = np.sum(oracle.deconv2d(x, w, None, 4, 2, 0) * gy)
    rhs = np.sum(x * oracle.deconv2d_dgrad(gy, w, 4, 2, 5, 6))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_adamw_first_step_closed_form_and_decay():
    w0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    w = w0.copy(); m = np.zeros(50); v = np.zeros(50)
    oracle.adamw_step(w, m, v, g, 1, lr=1e-3, wd=0.01)
    np.testing.assert_allclose(w, w0 * (1 - 1e-3 * 0.01) - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # zero gradient: only the decoupled decay acts
    w = w0.copy(); m = np.zeros(50); v = np.zeros(50)
    oracle.adamw_step(w, m, v, np.zeros(50), 1, lr=1e-2, wd=0.1)
    np.testing.assert_allclose(w, w0 * (1 - 1e-3), rtol=1e-15)
    # second step against torch.optim.AdamW
    wt = torch.tensor(w0, requires_grad=True)
    opt = torch.optim.AdamW([wt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.01)
    w = w0.copy(); m = np.zeros(50); v = np.zeros(50)
    for t, gg in enumerate((g, 0.5 * g + 0.1), start=1):
        wt.grad = torch.tensor(gg)
        opt.step()
        oracle.adamw_step(w, m, v, gg, t)
    np.testing.assert_allclose(w, wt.detach().numpy(), rtol=1e-12)
