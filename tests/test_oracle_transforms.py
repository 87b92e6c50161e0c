"""Pins of the oracle's neural-transform primitives (CPU only).

Each check is independent of the oracle's own formula: brute force written
differently (explicit padding, scatter form), closed forms, the adjoint
identity, and the textbook routines of torch in float64.
"""
import itertools

import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
import synth

rng = np.random.default_rng(7)


def brute_conv(x, w, b, s, p):
    """Correlation on an explicitly zero-padded copy (pure Python loops)."""
    C, H, W = x.shape
    Co, _, k, _ = w.shape
    xp = np.zeros((C, H + 2 * p, W + 2 * p))
    xp[:, p:p + H, p:p + W] = x
    Ho, Wo = (H + 2 * p - k) // s + 1, (W + 2 * p - k) // s + 1
    out = np.zeros((Co, Ho, Wo))
    for o, i, j in itertools.product(range(Co), range(Ho), range(Wo)):
        acc = b[o]
        for c in range(C):
            for u in range(k):
                for v in range(k):
                    acc += w[o, c, u, v] * xp[c, s * i + u, s * j + v]
        out[o, i, j] = acc
    return out


def brute_deconv_scatter(x, w, b, s, p, op):
    """Transposed convolution as a scatter of every input pixel, then crop."""
    C, H, W = x.shape
    _, Co, k, _ = w.shape
    Hf, Wf = (H - 1) * s + k, (W - 1) * s + k
    full = np.zeros((Co, Hf + op, Wf + op))
    for c, r, q in itertools.product(range(C), range(H), range(W)):
        full[:, s * r:s * r + k, s * q:s * q + k] += x[c, r, q] * w[c]
    Ho, Wo = (H - 1) * s - 2 * p + k + op, (W - 1) * s - 2 * p + k + op
    return full[:, p:p + Ho, p:p + Wo] + b[:, None, None]


@pytest.mark.parametrize("k,s,p", [(5, 2, 2), (3, 1, 1), (5, 1, 2)])
def test_conv_matches_bruteforce_8x8(k, s, p):
    x = rng.standard_normal((3, 8, 8))
    w = rng.standard_normal((4, 3, k, k))
    b = rng.standard_normal(4)
    np.testing.assert_allclose(oracle.conv2d(x, w, b, s, p), brute_conv(x, w, b, s, p), rtol=1e-12, atol=1e-12)


def test_conv_point_equals_full():
    x = rng.standard_normal((5, 9, 7))
    w = rng.standard_normal((6, 5, 5, 5))
    b = rng.standard_normal(6)
    full = oracle.conv2d(x, w, b, 2, 2)
    for o, i, j in [(0, 0, 0), (5, 4, 3), (2, 1, 2), (3, 4, 0)]:
        assert oracle.conv2d_at(x, w, b, 2, 2, o, i, j) == full[o, i, j]


def test_conv_delta_kernel_is_strided_shift():
    x = rng.standard_normal((2, 12, 10))
    w = np.zeros((2, 2, 5, 5))
    w[0, 0, 2, 2] = 1.0          # centre tap: out = x[2i, 2j]
    w[1, 1, 0, 0] = 1.0          # corner tap: out = x[2i-2, 2j-2] (zero outside)
    out = oracle.conv2d(x, w, np.zeros(2), 2, 2)
    np.testing.assert_array_equal(out[0], x[0, ::2, ::2])
    ref = np.zeros_like(out[1])
    ref[1:, 1:] = x[1, 0:-2:2, 0:-2:2][: ref.shape[0] - 1, : ref.shape[1] - 1]
    np.testing.assert_array_equal(out[1], ref)


def test_conv_all_ones_gives_box_sums():
    x = rng.uniform(size=(1, 6, 6))
    out = oracle.conv2d(x, np.ones((1, 1, 3, 3)), np.zeros(1), 1, 1)
    xp = np.pad(x[0], 1)
    for i, j in itertools.product(range(6), range(6)):
        assert out[0, i, j] == pytest.approx(xp[i:i + 3, j:j + 3].sum(), abs=1e-13)


def test_conv_matches_torch_float64():
    x = rng.standard_normal((7, 19, 23))
    w = rng.standard_normal((5, 7, 5, 5))
    b = rng.standard_normal(5)
    ref = F.conv2d(torch.from_numpy(x)[None], torch.from_numpy(w), torch.from_numpy(b), stride=2, padding=2)[0]
    np.testing.assert_allclose(oracle.conv2d(x, w, b, 2, 2), ref.numpy(), rtol=1e-12, atol=1e-12)


def test_deconv_matches_scatter_bruteforce():
    x = rng.standard_normal((3, 5, 4))
    w = rng.standard_normal((3, 2, 5, 5))
    b = rng.standard_normal(2)
    out = oracle.deconv2d(x, w, b, 2, 2, 1)
    assert out.shape == (2, 10, 8)
    np.testing.assert_allclose(out, brute_deconv_scatter(x, w, b, 2, 2, 1), rtol=1e-12, atol=1e-12)


def test_deconv_matches_torch_float64():
    x = rng.standard_normal((6, 7, 9))
    w = rng.standard_normal((6, 4, 5, 5))
    b = rng.standard_normal(4)
    ref = F.conv_transpose2d(torch.from_numpy(x)[None], torch.from_numpy(w), torch.from_numpy(b),
                             stride=2, padding=2, output_padding=1)[0]
    np.testing.assert_allclose(oracle.deconv2d(x, w, b, 2, 2, 1), ref.numpy(), rtol=1e-12, atol=1e-12)


def test_deconv_is_adjoint_of_conv():
    # <conv(x), g> = <x, T(g)> with zero bias, the same weights, k, s, p.
    x = rng.standard_normal((3, 16, 12))
    w = rng.standard_normal((4, 3, 5, 5))          # conv: 3 -> 4
    g = rng.standard_normal((4, 8, 6))
    lhs = np.sum(oracle.conv2d(x, w, None, 2, 2) * g)
    rhs = np.sum(x * oracle.deconv2d(g, w, None, 2, 2, 1))   # deconv weights [C_in=4, C_out=3]
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_deconv_point_equals_full():
    x = rng.standard_normal((4, 5, 6))
    w = rng.standard_normal((4, 3, 5, 5))
    b = rng.standard_normal(3)
    full = oracle.deconv2d(x, w, b, 2, 2, 1)
    for o, i, j in [(0, 0, 0), (2, 9, 11), (1, 4, 7), (0, 3, 0)]:
        assert oracle.deconv2d_at(x, w, b, 2, 2, o, i, j) == full[o, i, j]


# ---------------------------------------------------------------- GDN -----
def test_gdn_closed_form_gamma_zero():
    x = rng.standard_normal((4, 3, 3))
    beta = np.array([1.0, 2.0, 4.0, 0.25])
    out = oracle.gdn(x, beta, np.zeros((4, 4)))
    np.testing.assert_allclose(out, x / np.sqrt(beta)[:, None, None], rtol=1e-15)
    out = oracle.gdn(x, beta, np.zeros((4, 4)), inverse=True)
    np.testing.assert_allclose(out, x * np.sqrt(beta)[:, None, None], rtol=1e-15)


def test_gdn_single_channel():
    x = rng.standard_normal((1, 5, 5))
    out = oracle.gdn(x, np.array([0.7]), np.array([[0.3]]))
    np.testing.assert_allclose(out, x / np.sqrt(0.7 + 0.3 * x * x), rtol=1e-15)


def test_gdn_times_igdn_is_square_and_odd():
    x = rng.standard_normal((6, 4, 4))
    beta = rng.uniform(0.5, 2.0, 6)
    gamma = rng.uniform(0.0, 0.2, (6, 6))
    g = oracle.gdn(x, beta, gamma)
    ig = oracle.gdn(x, beta, gamma, inverse=True)
    np.testing.assert_allclose(g * ig, x * x, rtol=1e-13)
    np.testing.assert_allclose(oracle.gdn(-x, beta, gamma), -g, rtol=0, atol=0)


def test_gdn_bounded_for_diagonal_gamma():
    x = 100.0 * rng.standard_normal((3, 6, 6))
    gamma = np.diag([0.1, 0.5, 2.0])
    g = oracle.gdn(x, np.ones(3), gamma)
    assert np.all(np.abs(g) < 1.0 / np.sqrt(np.diag(gamma))[:, None, None])


def test_gdn_couples_channels_with_dense_gamma():
    # element (i, j) of gamma must weigh channel j's square in channel i's norm
    x = np.zeros((3, 1, 1)); x[0] = 1.0; x[2] = 2.0
    gamma = np.zeros((3, 3)); gamma[0, 2] = 0.5
    g = oracle.gdn(x, np.ones(3), gamma)
    assert g[0, 0, 0] == pytest.approx(1.0 / np.sqrt(1.0 + 0.5 * 4.0))
    assert g[2, 0, 0] == pytest.approx(2.0)


# --------------------------------------------------- whole transforms -----
def _torch_gdn(h, beta, gamma, inverse):
    n = F.conv2d(h * h, torch.from_numpy(np.asarray(gamma, np.float64))[:, :, None, None],
                 torch.from_numpy(np.asarray(beta, np.float64)))
    return h * torch.sqrt(n) if inverse else h / torch.sqrt(n)


def test_transforms_match_torch_float64():
    """g_a, h_a, h_s and g_s against the same layers built from torch's routines."""
    N, M = 16, 24
    P = synth.model_params(1, N, M, gamma="dense")
    m = oracle.Model(P, 1, N, M)
    T = {k: torch.from_numpy(np.asarray(v, np.float64)) for k, v in P.items()}
    x = synth.frame_sinusoid(64, 64)
    xt = torch.from_numpy(x.astype(np.float64))[None]
    h = xt
    for i in range(4):
        h = F.conv2d(h, T[f"ga{i}.w"], T[f"ga{i}.b"], stride=2, padding=2)
        if i < 3:
            h = _torch_gdn(h, P[f"ga{i}.beta"], P[f"ga{i}.gamma"], False)
    y = m.g_a(oracle.pad64(x))
    np.testing.assert_allclose(y, h[0].numpy(), rtol=1e-11, atol=1e-12)
    z_ref = F.conv2d(F.relu(F.conv2d(F.relu(F.conv2d(h.abs(), T["ha0.w"], T["ha0.b"], padding=1)),
                                     T["ha1.w"], T["ha1.b"], stride=2, padding=2)),
                     T["ha2.w"], T["ha2.b"], stride=2, padding=2)
    np.testing.assert_allclose(m.h_a(y), z_ref[0].numpy(), rtol=1e-11, atol=1e-12)
    zt = torch.round(z_ref)
    v_ref = F.conv2d(F.relu(F.conv_transpose2d(F.relu(F.conv_transpose2d(
        zt, T["hs0.w"], T["hs0.b"], stride=2, padding=2, output_padding=1)),
        T["hs1.w"], T["hs1.b"], stride=2, padding=2, output_padding=1)), T["hs2.w"], T["hs2.b"], padding=1)
    np.testing.assert_allclose(m.h_s(zt[0].numpy()), v_ref[0].numpy(), rtol=1e-11, atol=1e-12)
    yh = torch.round(h)
    g = yh
    for i in range(4):
        g = F.conv_transpose2d(g, T[f"gs{i}.w"], T[f"gs{i}.b"], stride=2, padding=2, output_padding=1)
        if i < 3:
            g = _torch_gdn(g, P[f"gs{i}.beta"], P[f"gs{i}.gamma"], True)
    np.testing.assert_allclose(m.g_s(yh[0].numpy()), g[0].numpy(), rtol=1e-11, atol=1e-12)
