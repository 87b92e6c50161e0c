"""Pins of the oracle's interleaved word-wise rANS (K states sharing one
stream; the faster entropy coding of Sections II and VII, after Giesen's
interleaved rANS).

Fixed by two streams worked out by hand from the definition
(tests/golden/rans_ileave_hand.json), by a pure-Python construction of the
same stream from K independent single-state coders whose words are merged by
the step that produced them (a different formulation of the interleaving),
by round trips and a length bound under hypothesis, and by edge cases.
"""
import json
import math
import os

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table(head):
    f = np.zeros(129, np.uint32)
    f[:len(head)] = head
    return f[None, :]


def test_hand_worked_streams():
    with open(os.path.join(GOLDEN, "rans_ileave_hand.json")) as fh:
        cases = json.load(fh)["cases"]
    for c in cases:
        freq = _table(c["freq_head"])
        sym = np.array(c["sym"], np.int32)
        tab = np.zeros_like(sym)
        got = oracle.rans_ileave_encode(sym, tab, freq, K=c["K"])
        assert got == bytes.fromhex(c["bytes_hex"].replace(" ", "")), c["name"]
        np.testing.assert_array_equal(oracle.rans_ileave_decode(got, tab, freq, len(sym), K=c["K"]), sym)


def _merged_reference(sym, tab, freq, K):
    """K single-state word coders, one per lane, each run over its own
    symbols in reverse; every pushed word is tagged with the position i of
    the symbol whose encoding pushed it.  The shared stream is the final
    states, then all words ordered by increasing i (the order in which the
    decoder, running forward, reads them)."""
    L = 1 << 16
    tagged = []
    finals = []
    for j in range(K):
        x = L
        for i in range(len(sym) - 1 - ((len(sym) - 1 - j) % K) if len(sym) > j else -1, -1, -K):
            f = int(freq[tab[i], sym[i]])
            s = int(sum(int(v) for v in freq[tab[i], :sym[i]]))
            if x >= f * 65536:
                tagged.append((i, x & 0xFFFF))
                x >>= 16
            x = (x // f) * 65536 + x % f + s
        finals.append(x)
    out = b"".join(int(v).to_bytes(4, "little") for v in finals)
    for _, w in sorted(tagged):
        out += int(w).to_bytes(2, "little")
    return out


def _random_tables(rng, ntab):
    p = rng.dirichlet(np.full(129, 0.3), size=ntab)
    return np.stack([oracle.quantize_pmf(pi) for pi in p])


@pytest.mark.parametrize("K", [1, 2, 3, 8])
def test_equals_lanes_merged_by_step(K):
    rng = np.random.default_rng(40 + K)
    freq = _random_tables(rng, 3)
    for n in (0, 1, K - 1, K, 5 * K + 3, 300):
        n = max(n, 0)
        tab = rng.integers(0, 3, n).astype(np.int32)
        cdf = np.cumsum(freq, axis=1)
        sym = np.array([np.searchsorted(cdf[t], rng.integers(0, 1 << 16), side="right") for t in tab], np.int32)
        assert oracle.rans_ileave_encode(sym, tab, freq, K=K) == _merged_reference(sym, tab, freq, K), (K, n)


@settings(max_examples=60, deadline=None)
@given(st.integers(1, 8), st.integers(0, 2000), st.integers(0, 2 ** 32 - 1))
def test_round_trip_and_length(K, n, seed):
    rng = np.random.default_rng(seed)
    freq = _random_tables(rng, 4)
    tab = rng.integers(0, 4, n).astype(np.int32)
    cdf = np.cumsum(freq, axis=1)
    sym = np.array([np.searchsorted(cdf[t], rng.integers(0, 1 << 16), side="right") for t in tab], np.int32)
    data = oracle.rans_ileave_encode(sym, tab, freq, K=K)
    np.testing.assert_array_equal(oracle.rans_ileave_decode(data, tab, freq, n, K=K), sym)
    bits = float(sum(-math.log2(freq[t, s] / 65536.0) for t, s in zip(tab, sym)))
    # K states of 4 bytes, the information in 16-bit words, at most one
    # partly filled word per state
    assert len(data) <= 4 * K + 2 * (math.ceil(bits / 16) + K)
    assert (len(data) - 4 * K) % 2 == 0


def test_edge_cases_and_corruption():
    freq = np.stack([oracle.quantize_pmf(np.full(129, 1 / 129)),
                     oracle.quantize_pmf(np.r_[np.full(64, 1e-9), 1.0, np.full(64, 1e-9)])])
    assert freq[1, 64] == 65536 - 128 and freq[1, 0] == 1
    assert oracle.rans_ileave_encode([], [], freq) == (1 << 16).to_bytes(4, "little") * 8
    assert oracle.rans_ileave_decode((1 << 16).to_bytes(4, "little") * 8, [], freq, 0).size == 0
    sym = np.array([0, 64, 128, 64, 64, 0, 1, 127] * 5, np.int32)
    tab = np.ones_like(sym)
    data = oracle.rans_ileave_encode(sym, tab, freq)
    np.testing.assert_array_equal(oracle.rans_ileave_decode(data, tab, freq, sym.size), sym)
    with pytest.raises(ValueError):
        oracle.rans_ileave_decode(data[:-2], tab, freq, sym.size)
    with pytest.raises(ValueError):
        oracle.rans_ileave_decode(data + b"\0\0", tab, freq, sym.size)
    with pytest.raises(ValueError):
        oracle.rans_ileave_decode(data[:20], tab, freq, sym.size)
