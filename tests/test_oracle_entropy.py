"""Pins of the oracle's quantiser, tables and rANS coder (CPU only)."""
import json
import math
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st
from scipy.stats import norm

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ quantiser ---
def test_rne_table():
    v = np.array([0.5, -0.5, 1.5, 2.5, -1.5, -2.5, 0.49999999999999994, 2.5000000000000004, 3.7, -3.7])
    assert oracle.rne(v).tolist() == [0.0, -0.0, 2.0, 2.0, -2.0, -2.0, 0.0, 3.0, 4.0, -4.0]


def test_quantize_clamps_and_offsets():
    sym, vh = oracle.quantize(np.array([100.0, -100.0, 1.2, 0.5]), 0.25)
    assert sym.tolist() == [64, -64, 1, 0]
    assert vh.tolist() == [64.25, -63.75, 1.25, 0.25]


def test_quantize_f32_takes_the_decision_in_single_precision():
    # 0.5 + 2^-25 is not representable in float32: it rounds to 0.5 (a tie -> 0)
    v = np.float64(0.5) + 2.0 ** -25
    assert oracle.quantize(v, 0.0)[0] == 1
    assert oracle.quantize_f32(np.float32(v), np.float32(0.0)) == 0


# --------------------------------------------------------- scale table ---
def test_scale_table_endpoints_and_ratio():
    t = oracle.scale_table()
    assert t[0] == 0.11 and t[63] == 256.0
    r = t[1:] / t[:-1]
    assert np.max(np.abs(r - r[1])) < 1e-13
    assert r[1] == pytest.approx(math.exp((math.log(256) - math.log(0.11)) / 63), rel=1e-15)


def test_scale_index_of_table_entries_and_monotone():
    t = oracle.scale_table()
    assert oracle.scale_index(t).tolist() == list(range(64))
    s = np.sort(np.random.default_rng(1).uniform(0.0, 400.0, 5000))
    idx = oracle.scale_index(s)
    assert np.all(np.diff(idx) >= 0)
    assert oracle.scale_index(np.array([0.0, -1.0, 0.05]), t).tolist() == [0, 0, 0]
    assert oracle.scale_index(np.array([1e9]), t).tolist() == [63]
    # just above t_k selects k + 1
    assert oracle.scale_index(t[:63] * (1 + 1e-12)).tolist() == list(range(1, 64))


def test_scale_index_f32_agrees_with_fp64_away_from_boundaries():
    rng = np.random.default_rng(3)
    v = rng.uniform(-4.0, 6.5, 20000).astype(np.float32)
    t = oracle.scale_table()
    i64 = oracle.scale_index(np.exp(v.astype(np.float64)), t)
    i32 = oracle.scale_index_f32(v, 1)
    lt = np.log(t[:63])
    near = np.min(np.abs(v[:, None].astype(np.float64) - lt[None, :]), axis=1) < 1e-6
    assert np.array_equal(i64[~near], i32[~near])
    r = rng.uniform(-1.0, 300.0, 20000).astype(np.float32)
    assert np.array_equal(oracle.scale_index_f32(r, 0)[r > 1], oracle.scale_index(r.astype(np.float64), t)[r > 1])


# --------------------------------------------------------------- tables ---
def _check_freq(f, p):
    assert f.sum() == 1 << 16
    assert f.min() >= 1
    dev = np.abs(f.astype(np.float64) - 65536.0 * p)
    mode = int(np.argmax(p))
    assert np.all(np.delete(dev, mode) <= 129)
    assert dev[mode] <= 2 * 129


def test_gaussian_pmf_matches_scipy_and_tables_are_valid():
    t = oracle.scale_table()
    j = np.arange(-64, 65)
    for k in (0, 5, 20, 40, 63):
        p = oracle.pmf_gaussian(t[k])
        ref = norm.cdf((j + 0.5) / t[k]) - norm.cdf((j - 0.5) / t[k])
        ref[0] = norm.cdf(-63.5 / t[k])
        ref[-1] = norm.sf(63.5 / t[k])
        np.testing.assert_allclose(p, ref, rtol=1e-9, atol=1e-15)
        assert p.sum() == pytest.approx(1.0, abs=1e-12)
        _check_freq(oracle.quantize_pmf(p), p)


def test_quantize_pmf_remainder_goes_to_mode():
    p = np.zeros(129); p[10] = 0.5; p[20] = 0.5
    f = oracle.quantize_pmf(p)
    assert f.sum() == 65536
    assert f[10] == 1 + 32703 + (65536 - 129 - 2 * 32703)   # tie: lowest index takes the remainder
    assert f[20] == 1 + 32703
    p = np.full(129, 1.0 / 129)
    f = oracle.quantize_pmf(p)
    assert f.sum() == 65536 and f[0] == f.max()


def _softplus(x):
    return math.log1p(math.exp(x))


def test_factorized_density_reduces_to_logistic_without_nonlinearity():
    """With all factors a_k = 0 the network is affine: c(x) = sigmoid(alpha x + beta)."""
    rng = np.random.default_rng(5)
    prm = synth.density_params(1, rng)[0].copy()
    # zero the factor entries (positions of a1, a2, a3 in the layout)
    a_pos = [6, 7, 8, 21, 22, 23, 36, 37, 38]
    prm[a_pos] = 0.0
    H1 = np.array([_softplus(v) for v in prm[0:3]]).reshape(3, 1); b1 = prm[3:6]
    H2 = np.array([_softplus(v) for v in prm[9:18]]).reshape(3, 3); b2 = prm[18:21]
    H3 = np.array([_softplus(v) for v in prm[24:33]]).reshape(3, 3); b3 = prm[33:36]
    H4 = np.array([_softplus(v) for v in prm[39:42]]).reshape(1, 3); b4 = prm[42:43]
    alpha = (H4 @ H3 @ H2 @ H1)[0, 0]
    beta = (H4 @ (H3 @ (H2 @ b1 + b2) + b3) + b4)[0]
    for x in (-7.0, -1.3, 0.0, 0.4, 3.9):
        assert oracle.density_logit(prm, x) == pytest.approx(alpha * x + beta, rel=1e-12, abs=1e-12)
        assert oracle.density_cdf(prm, x) == pytest.approx(1.0 / (1.0 + math.exp(-(alpha * x + beta))), rel=1e-12)
    assert oracle.density_median(prm) == pytest.approx(-beta / alpha, abs=1e-12)


def test_factorized_density_is_monotone_and_median_halves_it():
    P = synth.model_params(1, 16, 24)
    dens = P["eb.density"]
    xs = np.linspace(-20, 20, 801)
    for c in range(dens.shape[0]):
        cdf = np.array([oracle.density_cdf(dens[c], x) for x in xs])
        assert np.all(np.diff(cdf) > 0)
        m = oracle.density_median(dens[c])
        assert oracle.density_cdf(dens[c], m) == pytest.approx(0.5, abs=1e-12)
        p = oracle.pmf_factorized(dens[c], np.float32(m))
        assert p.sum() == pytest.approx(1.0, abs=1e-12)
        assert np.all(p >= 0)          # differences of a monotone cumulative
        _check_freq(oracle.quantize_pmf(p), p)


# ----------------------------------------------------------------- rANS ---
def _peak_table():
    f = np.ones(129, np.uint32)
    f[64] = 65536 - 128
    return f[None, :]


def test_rans_hand_worked_examples():
    with open(os.path.join(GOLDEN, "rans_hand.json")) as fh:
        cases = json.load(fh)["cases"]
    freq = _peak_table()
    for case in cases:
        syms = np.array(case["symbols"], np.int32)
        data = oracle.rans_encode(syms, np.zeros_like(syms), freq)
        assert data.hex() == case["bytes_hex"], case["name"]
        assert oracle.rans_decode(data, np.zeros_like(syms), freq, len(syms)).tolist() == case["symbols"]


def _random_table(draw_seed):
    rng = np.random.default_rng(draw_seed)
    w = rng.exponential(1.0, 129) ** 3
    return oracle.quantize_pmf(w / w.sum())


@settings(max_examples=60, deadline=None)
@given(st.integers(0, 2 ** 31), st.integers(0, 3000), st.integers(1, 4))
def test_rans_round_trip_and_length_bound(seed, n, ntab):
    rng = np.random.default_rng(seed)
    freq = np.stack([_random_table(seed + k) for k in range(ntab)])
    tab = rng.integers(0, ntab, n).astype(np.int32)
    # draw symbols from the tables themselves, plus some rare ones
    sym = np.empty(n, np.int32)
    for i in range(n):
        p = freq[tab[i]] / 65536.0
        sym[i] = rng.choice(129, p=p) if rng.uniform() < 0.95 else rng.integers(0, 129)
    data = oracle.rans_encode(sym, tab, freq)
    out = oracle.rans_decode(data, tab, freq, n)
    assert np.array_equal(out, sym)
    bits = -np.sum(np.log2(freq[tab, sym] / 65536.0)) if n else 0.0
    assert len(data) <= math.ceil(bits / 8) + 4 + 2
    assert len(data) >= 4


def test_rans_edge_cases():
    freq = _peak_table()
    # zero symbols: only the flushed initial state L
    data = oracle.rans_encode(np.zeros(0, np.int32), np.zeros(0, np.int32), freq)
    assert data == bytes([0, 0, 0x80, 0])
    assert oracle.rans_decode(data, np.zeros(0, np.int32), freq, 0).size == 0
    # long run of f = 1 symbols and of the f = 65408 symbol
    for s in (0, 128, 64):
        syms = np.full(5000, s, np.int32)
        data = oracle.rans_encode(syms, np.zeros_like(syms), freq)
        assert np.array_equal(oracle.rans_decode(data, np.zeros_like(syms), freq, 5000), syms)
        if s != 64:
            assert len(data) == pytest.approx(5000 * 2, abs=8)


def test_rans_rejects_truncated_and_extended_streams():
    freq = np.stack([_random_table(11)])
    rng = np.random.default_rng(2)
    sym = rng.integers(0, 129, 500).astype(np.int32)
    tab = np.zeros(500, np.int32)
    data = oracle.rans_encode(sym, tab, freq)
    with pytest.raises(ValueError):
        oracle.rans_decode(data[:-3], tab, freq, 500)
    with pytest.raises(ValueError):
        oracle.rans_decode(data + b"\x00", tab, freq, 500)


# ------------------------------------------------------------ container ---
def test_container_round_trip_and_validation():
    ys = [b"\x01\x02\x03", b"", b"\xff" * 7]
    bits = oracle.pack_container(1, 1, 3, 720, 1280, 128, 192, 0xDEADBEEF, b"zz", ys)
    assert len(bits) == 20 + 4 + 12 + 2 + 10
    h = oracle.parse_container(bits)
    assert (h["kind"], h["hs_out"], h["S"], h["H"], h["W"], h["N"], h["M"], h["model_id"]) == \
        (1, 1, 3, 720, 1280, 128, 192, 0xDEADBEEF)
    assert h["z"] == b"zz" and h["y"] == ys
    with pytest.raises(ValueError):
        oracle.parse_container(bits[:-1])
    with pytest.raises(ValueError):
        oracle.parse_container(b"LICX" + bits[4:])


def test_fnv1a_reference_values():
    # published FNV-1a 32-bit test vectors
    assert oracle.fnv1a32(b"") == 0x811C9DC5
    assert oracle.fnv1a32(b"a") == 0xE40C292C
    assert oracle.fnv1a32(b"foobar") == 0xBF9CF968
