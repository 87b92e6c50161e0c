"""Pins of the oracle's 1DN normalisation (implementation C of Section IV.C,
read as y_i = x_i / (beta_i + sum_j gamma_ij |x_j|) and x_i * (...) for the
inverse; the paper prints no formula) and of the codec built with it.

Fixed by closed forms (gamma = 0, one channel), a two-channel example worked
by hand, identities (forward times inverse is x^2, odd symmetry, the bound
1/gamma_ii), torch float64 routines, and the codec's own round trip.
"""
import numpy as np
import pytest

import oracle
import synth

rng = np.random.default_rng(1741)


def test_gamma_zero_is_division_by_beta():
    x = rng.standard_normal((5, 3, 4))
    b = rng.uniform(0.5, 2.0, 5)
    g = np.zeros((5, 5))
    np.testing.assert_allclose(oracle.gdn1(x, b, g), x / b[:, None, None], rtol=1e-15)
    np.testing.assert_allclose(oracle.gdn1(x, b, g, inverse=True), x * b[:, None, None], rtol=1e-15)


@pytest.mark.parametrize("v", [-3.0, -0.5, 0.0, 0.25, 7.0])
def test_one_channel_closed_form(v):
    beta, gamma = 0.7, 0.3
    got = oracle.gdn1(np.array([[[v]]]), np.array([beta]), np.array([[gamma]]))[0, 0, 0]
    assert got == pytest.approx(v / (beta + gamma * abs(v)), rel=1e-15)
    inv = oracle.gdn1(np.array([[[v]]]), np.array([beta]), np.array([[gamma]]), inverse=True)[0, 0, 0]
    assert inv == pytest.approx(v * (beta + gamma * abs(v)), rel=1e-15)


def test_two_channels_by_hand():
    # n0 = 1 + 0.1*|1| + 0.2*|-2| = 1.5,  n1 = 0.5 + 0.3*|1| + 0.4*|-2| = 1.6
    x = np.array([1.0, -2.0]).reshape(2, 1, 1)
    beta = np.array([1.0, 0.5])
    gamma = np.array([[0.1, 0.2], [0.3, 0.4]])
    np.testing.assert_allclose(oracle.gdn1(x, beta, gamma).ravel(), [1.0 / 1.5, -2.0 / 1.6], rtol=1e-15)
    np.testing.assert_allclose(oracle.gdn1(x, beta, gamma, inverse=True).ravel(), [1.5, -3.2], rtol=1e-15)
    # GDN on the same input differs (squares and a root): n0 = 1.9, n1 = 2.4
    np.testing.assert_allclose(oracle.gdn(x, beta, gamma).ravel(), [1 / np.sqrt(1.9), -2 / np.sqrt(2.4)],
                               rtol=1e-15)


def test_forward_times_inverse_is_square_and_odd():
    x = rng.standard_normal((6, 5, 7))
    b = rng.uniform(0.5, 1.5, 6)
    g = rng.uniform(0.0, 0.2, (6, 6))
    f = oracle.gdn1(x, b, g)
    i = oracle.gdn1(x, b, g, inverse=True)
    np.testing.assert_allclose(f * i, x * x, rtol=1e-13, atol=1e-300)
    np.testing.assert_allclose(oracle.gdn1(-x, b, g), -f, rtol=0, atol=0)


def test_bound_with_diagonal_gamma():
    x = 1e3 * rng.standard_normal((4, 8, 8))
    g = np.diag([0.1, 0.2, 0.5, 1.0])
    y = oracle.gdn1(x, np.ones(4), g)
    assert np.all(np.abs(y) < 1.0 / np.diag(g)[:, None, None])


def test_against_torch_float64():
    torch = pytest.importorskip("torch")
    x = rng.standard_normal((16, 9, 11))
    b = rng.uniform(0.5, 1.5, 16)
    g = 0.1 * np.eye(16) + 0.01 * rng.uniform(0, 1, (16, 16))
    xt = torch.from_numpy(x)[None]
    n = torch.nn.functional.conv2d(xt.abs(), torch.from_numpy(g)[:, :, None, None], torch.from_numpy(b))[0]
    np.testing.assert_allclose(oracle.gdn1(x, b, g), (xt[0] / n).numpy(), rtol=1e-13)
    np.testing.assert_allclose(oracle.gdn1(x, b, g, inverse=True), (xt[0] * n).numpy(), rtol=1e-13)


def test_codec_with_1dn_round_trip_and_container_flag():
    H, W = 64, 128
    P = synth.model_params(1, 16, 24, gamma="dense")
    blob = synth.weight_blob(P, 1, 16, 24)
    m = oracle.Model(P, 1, 16, 24, blob, norm=1)
    x = synth.frame_sinusoid(H, W, t=3)
    bits, inter = m.encode(x, S=2)
    hdr = oracle.parse_container(bits)
    assert hdr["norm"] == 1 and hdr["hs_out"] == 1
    assert bits[6] == 0b11                          # flags byte: exp output, 1DN
    xr, d = m.decode(bits)
    assert np.array_equal(d["yhat"], inter["yhat"])
    np.testing.assert_allclose(xr, np.clip(m.g_s(inter["yhat"]), 0, 1)[:, :H, :W], rtol=0, atol=0)
    # the transforms use 1DN: the first analysis layer equals conv + gdn1
    h0 = oracle.gdn1(oracle.conv2d(oracle.pad64(x), P["ga0.w"], P["ga0.b"], 2, 2), P["ga0.beta"], P["ga0.gamma"])
    np.testing.assert_array_equal(inter["ga"][0], h0)
    # a GDN decoder refuses the 1DN stream (same weights, other normalisation)
    with pytest.raises(ValueError):
        oracle.Model(P, 1, 16, 24, blob, norm=0).decode(bits)
