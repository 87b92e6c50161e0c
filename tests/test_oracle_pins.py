"""Further pins of the oracle (CPU only): the channel offset of the
factorized tables, the per-point convolution wrappers that the full-size GPU
tests use as their reference, and the bitstream container's byte layout.

Each check is fixed by something other than the oracle's own formula: the
logistic closed form of the factorized density, the full convolutions (which
are pinned against brute force in test_oracle_transforms.py), and bytes
written out by hand from the container layout.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _softplus(x):
    return math.log1p(math.exp(x))


def _logistic_params(seed):
    """Density parameters with every factor a_k = 0, so the cumulative is
    sigmoid(alpha x + beta) with alpha, beta from the products of the
    (softplus'd) matrices and biases."""
    prm = synth.density_params(1, np.random.default_rng(seed))[0].copy()
    prm[[6, 7, 8, 21, 22, 23, 36, 37, 38]] = 0.0
    H1 = np.array([_softplus(v) for v in prm[0:3]]).reshape(3, 1); b1 = prm[3:6]
    H2 = np.array([_softplus(v) for v in prm[9:18]]).reshape(3, 3); b2 = prm[18:21]
    H3 = np.array([_softplus(v) for v in prm[24:33]]).reshape(3, 3); b3 = prm[33:36]
    H4 = np.array([_softplus(v) for v in prm[39:42]]).reshape(1, 3); b4 = prm[42:43]
    alpha = (H4 @ H3 @ H2 @ H1)[0, 0]
    beta = (H4 @ (H3 @ (H2 @ b1 + b2) + b3) + b4)[0]
    return prm, alpha, beta


def _sig(u):
    return 1.0 / (1.0 + math.exp(-u))


@pytest.mark.parametrize("seed,mu", [(5, 0.37), (6, -1.25), (7, 2.5)])
def test_factorized_pmf_offset_against_logistic_closed_form(seed, mu):
    """p_j = c(j + 1/2 + mu) - c(j - 1/2 + mu) with c the logistic; the
    edge bins take the tails.  A flipped or dropped offset fails here."""
    prm, alpha, beta = _logistic_params(seed)
    p = oracle.pmf_factorized(prm, mu)
    c = lambda x: _sig(alpha * x + beta)
    for a, j in enumerate(range(-64, 65)):
        hi = 1.0 if j == 64 else c(j + 0.5 + mu)
        lo = 0.0 if j == -64 else c(j - 0.5 + mu)
        assert p[a] == pytest.approx(hi - lo, rel=1e-10, abs=1e-16), j
    # the mass sits around the symbol nearest to (median - mu)
    med = -beta / alpha
    assert abs(int(np.argmax(p)) - 64 - (med - mu)) <= 1.0


@pytest.mark.parametrize("seed", [5, 6, 7, 8])
def test_factorized_pmf_at_the_median_is_symmetric_with_mode_zero(seed):
    """A logistic is symmetric about its median, so with mu = median the
    probabilities of j and -j agree and symbol 0 is the most probable."""
    prm, alpha, beta = _logistic_params(seed)
    m = oracle.density_median(prm)
    assert m == pytest.approx(-beta / alpha, abs=1e-12)
    p = oracle.pmf_factorized(prm, m)
    np.testing.assert_allclose(p, p[::-1], rtol=1e-9, atol=1e-15)
    assert int(np.argmax(p)) == 64
    # and away from the median the symmetry breaks
    q = oracle.pmf_factorized(prm, m + 0.3)
    assert np.max(np.abs(q - q[::-1])) > 1e-3


def test_factorized_tables_of_the_model_use_the_float32_medians():
    """Model tables are the quantised pmf at the float32-rounded median."""
    P = synth.model_params(1, 16, 24)
    m = oracle.Model(P, 1, 16, 24)
    dens = P["eb.density"]
    for c in (0, 7, 15):
        mu32 = np.float32(oracle.density_median(dens[c]))
        assert m.medians[c] == mu32
        np.testing.assert_array_equal(m.freq_fact[c], oracle.quantize_pmf(oracle.pmf_factorized(dens[c], float(mu32))))


rng = np.random.default_rng(11)


@pytest.mark.parametrize("k,s,p", [(5, 2, 2), (3, 1, 1)])
def test_conv_points_equal_the_full_convolution(k, s, p):
    """conv2d_points (the reference of the sampled full-size GPU checks)
    equals the full convolution at every output position of a small input,
    corners and edges included."""
    x = rng.standard_normal((6, 13, 11))
    w = rng.standard_normal((5, 6, k, k))
    b = rng.standard_normal(5)
    full = oracle.conv2d(x, w, b, s, p)
    Ho, Wo = full.shape[1:]
    pts = [(i, j) for i in range(Ho) for j in range(Wo)]
    got = oracle.conv2d_points(x, w, b, s, p, pts)
    np.testing.assert_array_equal(got, full.reshape(full.shape[0], -1).T)


def test_deconv_points_equal_the_full_transposed_convolution():
    """deconv2d_points equals the full transposed convolution (stride 2,
    pad 2, output padding 1) at every output position, all four sub-pixel
    phases and the last row / column that only the output padding adds."""
    x = rng.standard_normal((4, 7, 9))
    w = rng.standard_normal((4, 3, 5, 5))
    b = rng.standard_normal(3)
    full = oracle.deconv2d(x, w, b, 2, 2, 1)
    assert full.shape == (3, 14, 18)
    Ho, Wo = full.shape[1:]
    pts = [(i, j) for i in range(Ho) for j in range(Wo)]
    got = oracle.deconv2d_points(x, w, b, 2, 2, pts)
    np.testing.assert_array_equal(got, full.reshape(full.shape[0], -1).T)


def test_points_at_random_positions_of_a_larger_input():
    x = rng.standard_normal((16, 40, 56))
    w = rng.standard_normal((16, 16, 5, 5))
    b = rng.standard_normal(16)
    full = oracle.conv2d(x, w, b, 2, 2)
    pts = np.stack([rng.integers(0, full.shape[1], 64), rng.integers(0, full.shape[2], 64)], 1)
    pts[:4] = [(0, 0), (0, full.shape[2] - 1), (full.shape[1] - 1, 0), (full.shape[1] - 1, full.shape[2] - 1)]
    np.testing.assert_array_equal(oracle.conv2d_points(x, w, b, 2, 2, pts), full[:, pts[:, 0], pts[:, 1]].T)
    wt = rng.standard_normal((16, 8, 5, 5))
    fd = oracle.deconv2d(x, wt, b[:8], 2, 2, 1)
    pts = np.stack([rng.integers(0, fd.shape[1], 64), rng.integers(0, fd.shape[2], 64)], 1)
    pts[:4] = [(0, 0), (0, fd.shape[2] - 1), (fd.shape[1] - 1, 0), (fd.shape[1] - 1, fd.shape[2] - 1)]
    np.testing.assert_array_equal(oracle.deconv2d_points(x, wt, b[:8], 2, 2, pts), fd[:, pts[:, 0], pts[:, 1]].T)


def test_container_bytes_written_by_hand():
    with open(os.path.join(GOLDEN, "lics_header.json")) as fh:
        cases = json.load(fh)["cases"]
    for case in cases:
        f = case["fields"]
        z = bytes.fromhex(case["z_hex"]) if case["z_hex"] is not None else None
        ys = [bytes.fromhex(y) for y in case["y_hex"]]
        bits = oracle.pack_container(f["kind"], f["hs_out"], f["S"], f["H"], f["W"], f["N"], f["M"],
                                     f["model_id"], z, ys)
        assert bits == bytes.fromhex(case["bytes_hex"].replace(" ", "")), case["name"]
        h = oracle.parse_container(bits)
        assert all(h[k] == v for k, v in f.items())
