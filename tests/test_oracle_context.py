"""Pins of the context-model oracle (kind 2: mean-scale hyperprior with a
checkerboard context model, the parallel context prediction that Sections II
and VII name as the next step).  CPU only.

What fixes each part independently of the oracle's own code:
  * the mask and the anchor set: which latents a non-anchor's context depends
    on, found by perturbing every input element one at a time;
  * the context convolution: explicit loops over the taps of the window;
  * the 1 x 1 layers: the oracle's C convolution with 1 x 1 kernels;
  * the two passes and the output channel order: weights for which the
    entropy parameters reduce to psi itself (means first, scales second), so
    the codec's decisions become the plain quantiser and scale index;
  * causality: the decoder, which sees the anchors only after pass 1,
    reproduces the encoder's y_hat exactly; y at a non-anchor changes only
    its own symbol;
  * the rate: the stream lengths match the ideal code length of the tables.
"""
import numpy as np
import pytest

import oracle
import synth

N, M = 128, 192


@pytest.fixture(scope="module")
def ctx_model():
    P = synth.model_params(2, N, M)
    return oracle.Model(P, 2, N, M, synth.weight_blob(P, 2, N, M))


def test_mask_and_anchor_set():
    m = oracle.context_mask(5)
    assert m.sum() == 12 and not m[2, 2]
    A = oracle.checkerboard(4, 6)
    assert A.sum() == 12 and A[0, 0] and not A[0, 1] and A[1, 1]


def test_context_depends_on_exactly_the_anchors_of_the_window():
    rng = np.random.default_rng(5)
    C, H, W = 2, 7, 8
    yhat = rng.standard_normal((C, H, W))
    w = rng.standard_normal((3, C, 5, 5))
    b = rng.standard_normal(3)
    base = oracle.context(yhat, w, b)
    A = oracle.checkerboard(H, W)
    assert np.all(base[:, A] == 0.0)              # anchors have an empty context
    r0, c0 = 3, 4                                 # a non-anchor
    assert not A[r0, c0]
    dep = np.zeros((H, W), bool)
    for r in range(H):
        for c in range(W):
            for ch in range(C):
                y2 = yhat.copy()
                y2[ch, r, c] += 1.0
                if not np.array_equal(oracle.context(y2, w, b)[:, r0, c0], base[:, r0, c0]):
                    dep[r, c] = True
    want = np.zeros((H, W), bool)
    for r in range(H):
        for c in range(W):
            want[r, c] = abs(r - r0) <= 2 and abs(c - c0) <= 2 and (r + c) % 2 == 0
    assert want.sum() == 12
    assert np.array_equal(dep, want)
    # weights at masked taps are ignored
    w2 = w.copy()
    w2[:, :, ~oracle.context_mask(5)] += 7.0
    assert np.array_equal(oracle.context(yhat, w2, b), base)


def test_context_brute_force():
    rng = np.random.default_rng(6)
    C, H, W, Co = 3, 6, 6, 4
    yhat = rng.standard_normal((C, H, W))
    w = rng.standard_normal((Co, C, 5, 5))
    b = rng.standard_normal(Co)
    got = oracle.context(yhat, w, b)
    for r in range(H):
        for c in range(W):
            if (r + c) % 2 == 0:
                continue
            acc = b.copy()
            for dy in range(-2, 3):
                for dx in range(-2, 3):
                    if (dy + dx) % 2 == 0 or not (0 <= r + dy < H and 0 <= c + dx < W):
                        continue
                    acc += w[:, :, dy + 2, dx + 2] @ yhat[:, r + dy, c + dx]
            assert np.allclose(got[:, r, c], acc, rtol=1e-13, atol=1e-13)


def test_conv1x1_is_a_1x1_convolution():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((6, 5, 7))
    w = rng.standard_normal((4, 6, 1, 1))
    b = rng.standard_normal(4)
    assert np.allclose(oracle.conv1x1(x, w, b), oracle.conv2d(x, w, b, 1, 0), rtol=1e-13, atol=1e-13)


def _identity_parameters(M, E1, E2):
    """Entropy-parameter weights whose output is psi itself: layer 1 keeps
    ReLU(psi_j) and ReLU(-psi_j) in rows 2j and 2j + 1, layer 2 passes both
    on, layer 3 takes their difference.  The context columns of layer 1 are
    zero.  Needs E1, E2 >= 4M."""
    assert E1 >= 4 * M and E2 >= 4 * M
    w0 = np.zeros((E1, 4 * M, 1, 1))
    w1 = np.zeros((E2, E1, 1, 1))
    w2 = np.zeros((2 * M, E2, 1, 1))
    for j in range(2 * M):
        w0[2 * j, j] = 1.0
        w0[2 * j + 1, j] = -1.0
        w1[2 * j, 2 * j] = 1.0
        w1[2 * j + 1, 2 * j + 1] = 1.0
        w2[j, 2 * j] = 1.0
        w2[j, 2 * j + 1] = -1.0
    return {"ep0.w": w0, "ep1.w": w1, "ep2.w": w2,
            "ep0.b": np.zeros(E1), "ep1.b": np.zeros(E2), "ep2.b": np.zeros(2 * M)}


def test_entropy_parameters_reduce_to_psi():
    """With small widths the identity construction fits: the means are the
    first half of psi, the scales the second, in both passes, and the codec's
    decisions are the plain quantiser around psi's means and the scale index
    of psi's scales."""
    Ms = 4
    E1 = E2 = 4 * Ms
    rng = np.random.default_rng(8)
    Q = _identity_parameters(Ms, E1, E2)
    Q["cx.w"] = rng.standard_normal((2 * Ms, Ms, 5, 5))
    Q["cx.b"] = rng.standard_normal(2 * Ms)
    psi = rng.standard_normal((2 * Ms, 6, 8))
    ctx = rng.standard_normal((2 * Ms, 6, 8))
    mu, s = oracle.entropy_parameters(Q, psi, ctx)
    assert np.array_equal(mu, psi[:Ms]) and np.array_equal(s, psi[Ms:])
    # the passes of a model with these weights
    m = oracle.Model.__new__(oracle.Model)
    m.P, m.hs_out, m.t = Q, 1, oracle.scale_table()
    y = 3.0 * rng.standard_normal((Ms, 6, 8))
    r = m.checkerboard_passes(psi, y=y)
    sym, _ = oracle.quantize(y, psi[:Ms])
    assert np.array_equal(r["sym"], sym)
    assert np.array_equal(r["idx"], oracle.scale_index(np.exp(psi[Ms:])))
    assert np.array_equal(r["yhat"], sym + psi[:Ms])


def test_non_anchor_y_changes_only_its_own_symbol(ctx_model):
    rng = np.random.default_rng(9)
    psi = rng.standard_normal((2 * M, 4, 6))
    y = 2.0 * rng.standard_normal((M, 4, 6))
    a = ctx_model.checkerboard_passes(psi, y=y)
    y2 = y.copy()
    y2[:, 1, 2] += 5.0                      # (1, 2) is a non-anchor
    b = ctx_model.checkerboard_passes(psi, y=y2)
    assert np.array_equal(a["mu"], b["mu"]) and np.array_equal(a["idx"], b["idx"])
    d = a["sym"] != b["sym"]
    assert d[:, 1, 2].any() and d.sum() == d[:, 1, 2].sum()
    # y at an anchor moves the non-anchor parameters of its neighbours only
    y3 = y.copy()
    y3[:, 2, 2] += 5.0
    c = ctx_model.checkerboard_passes(psi, y=y3)
    A = oracle.checkerboard(4, 6)
    assert np.array_equal(a["mu"][:, A], c["mu"][:, A])
    moved = np.any(a["mu"] != c["mu"], axis=0)
    assert moved[2, 1] and moved[1, 2] and not moved[2, 2] and not moved[0, 5]


def test_context_codec_round_trip_ragged(ctx_model):
    x = synth.frame_sinusoid(100, 150)
    bits, enc = ctx_model.encode(x, S=3)
    hdr = oracle.parse_container(bits)
    assert hdr["kind"] == 2 and len(hdr["y"]) == 6 and hdr["S"] == 3
    xr, dec = ctx_model.decode(bits)
    assert xr.shape == (3, 100, 150)
    assert np.array_equal(dec["yhat"], enc["yhat"])
    assert np.array_equal(dec["idx"], enc["idx"])
    assert np.array_equal(dec["mu"], enc["mu"])
    assert np.array_equal(xr, np.clip(ctx_model.g_s(enc["yhat"]), 0, 1)[:, :100, :150])
    # y_hat is the quantised y around the means
    assert np.array_equal(enc["sym_y"], np.clip(np.rint(enc["y"] - enc["mu"]), -64, 64))


def test_context_rate_close_to_model_entropy(ctx_model):
    x = synth.frame_sinusoid(128, 128)
    bits, enc = ctx_model.encode(x, S=1)
    hdr = oracle.parse_container(bits)
    A = oracle.checkerboard(8, 8)
    for part, sel in ((0, A), (1, ~A)):
        sym = enc["sym_y"][:, sel].ravel() + 64
        tab = enc["idx"][:, sel].ravel()
        ideal = -np.sum(np.log2(ctx_model.freq_gauss[tab, sym] / 65536.0))
        assert len(hdr["y"][part]) * 8 == pytest.approx(ideal, rel=0.01, abs=64)


def test_context_interleaved_coder_round_trip():
    P = synth.model_params(2, N, M)
    m = oracle.Model(P, 2, N, M, synth.weight_blob(P, 2, N, M), lanes=8, hs_out=0)
    x = synth.frame_sinusoid(64, 128)
    bits, enc = m.encode(x, S=2)
    xr, dec = m.decode(bits)
    assert np.array_equal(dec["yhat"], enc["yhat"])
    hdr = oracle.parse_container(bits)
    assert hdr["lanes"] == 8 and hdr["hs_out"] == 0 and len(hdr["y"]) == 4
