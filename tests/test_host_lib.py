"""Host side of the HIP library on the CPU: exported symbols, entropy tables,
rANS bytes and the model id, all against the oracle (no GPU calls)."""
import os
import re

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2208_01641_amd import _lib
    return _lib


def test_library_exports_every_declared_symbol(L):
    with open(os.path.join(ROOT, "include", "lic.h")) as fh:
        text = fh.read()
    # function declarations: "<type> name(" at the start of a line
    names = set(re.findall(r"^[A-Za-z_][\w \*]*?\b(codec_\w+|lic_\w+)\s*\(", text, re.M))
    assert len(names) >= 16, names
    for n in sorted(names):
        assert hasattr(L.lib, n), f"liblic.so does not export {n}"
    assert set(L.SIGNATURES) == names


def test_fnv1a_matches_oracle():
    from paper_2208_01641_amd import fnv1a
    for data in (b"", b"a", b"foobar", bytes(range(256)) * 3):
        assert fnv1a(data) == oracle.fnv1a32(data)


@pytest.mark.parametrize("kind,N,M", [(1, 128, 192), (0, 128, 192), (1, 192, 320)])
def test_library_tables_equal_oracle_tables(L, kind, N, M):
    import ctypes
    P = synth.model_params(kind, N, M)
    blob = synth.weight_blob(P, kind, N, M)
    m = oracle.Model(P, kind, N, M, blob)
    buf = ctypes.create_string_buffer(blob, len(blob))
    C = M if kind == 0 else N
    f = np.zeros(C * 129, np.uint32)
    mu = np.zeros(C, np.float32)
    n = L.lib.lic_blob_tables(buf, len(blob), 0, f.ctypes.data, f.size, mu.ctypes.data, mu.size)
    assert n == C * 129
    assert np.array_equal(mu, m.medians)
    assert np.array_equal(f.reshape(C, 129), m.freq_fact)
    if kind == 1:
        g = np.zeros(64 * 129, np.uint32)
        assert L.lib.lic_blob_tables(buf, len(blob), 1, g.ctypes.data, g.size, None, 0) == 64 * 129
        assert np.array_equal(g.reshape(64, 129), m.freq_gauss)
    # too small a buffer is reported, not overrun
    small = np.zeros(10, np.uint32)
    assert L.lib.lic_blob_tables(buf, len(blob), 0, small.ctypes.data, small.size, None, 0) == L.LIC_E_SMALLBUF


def _tables(seed, ntab):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(ntab):
        w = rng.exponential(1.0, 129) ** 4
        out.append(oracle.quantize_pmf(w / w.sum()))
    return np.stack(out)


@settings(max_examples=40, deadline=None)
@given(st.integers(0, 2 ** 31), st.integers(0, 5000), st.integers(1, 64))
def test_library_rans_bytes_equal_oracle(seed, n, ntab):
    from paper_2208_01641_amd import rans_decode, rans_encode
    freq = _tables(seed, ntab)
    rng = np.random.default_rng(seed + 1)
    tab = rng.integers(0, ntab, n).astype(np.uint8)
    sym = np.array([rng.choice(129, p=freq[t] / 65536.0) for t in tab], np.uint8)
    lib_bytes = rans_encode(sym, tab, freq)
    assert lib_bytes == oracle.rans_encode(sym.astype(np.int32), tab.astype(np.int32), freq)
    assert np.array_equal(rans_decode(lib_bytes, tab, freq, n), sym)


def test_library_rans_hand_example_and_errors(L):
    from paper_2208_01641_amd import LicError, rans_decode, rans_encode
    f = np.ones(129, np.uint32)
    f[64] = 65536 - 128
    assert rans_encode(np.array([64, 0], np.uint8), np.zeros(2, np.uint8), f[None]).hex() == "404080000000"
    data = rans_encode(np.arange(129, dtype=np.uint8), np.zeros(129, np.uint8), f[None])
    with pytest.raises(LicError):
        rans_decode(data[:-1], np.zeros(129, np.uint8), f[None], 129)
    with pytest.raises(LicError):
        rans_decode(data + b"\x01", np.zeros(129, np.uint8), f[None], 129)
    bad = f.copy()
    bad[0] = 2                     # does not sum to 2^16
    with pytest.raises(LicError):
        rans_encode(np.zeros(3, np.uint8), np.zeros(3, np.uint8), bad[None])


@settings(max_examples=40, deadline=None)
@given(st.integers(0, 2 ** 31), st.integers(0, 3000), st.integers(1, 64), st.sampled_from([2, 4, 8, 16, 32]))
def test_library_interleaved_rans_bytes_equal_oracle(seed, n, ntab, lanes):
    from paper_2208_01641_amd import rans_ileave_decode, rans_ileave_encode
    freq = _tables(seed, ntab)
    rng = np.random.default_rng(seed + 2)
    tab = rng.integers(0, ntab, n).astype(np.uint8)
    sym = np.array([rng.choice(129, p=freq[t] / 65536.0) for t in tab], np.uint8)
    lib_bytes = rans_ileave_encode(sym, tab, freq, lanes)
    assert lib_bytes == oracle.rans_ileave_encode(sym.astype(np.int32), tab.astype(np.int32), freq, K=lanes)
    assert len(lib_bytes) <= 2 * n + 4 * lanes
    assert np.array_equal(rans_ileave_decode(lib_bytes, tab, freq, n, lanes), sym)


def test_library_interleaved_rans_golden_and_errors(L):
    """The hand-worked streams of the interleaved coder, the unchecked (room
    for a whole group) and checked paths on long and short streams, and
    rejection of truncated, extended and mis-laned streams."""
    import json
    from paper_2208_01641_amd import LicError, rans_ileave_decode, rans_ileave_encode
    with open(os.path.join(ROOT, "tests", "golden", "rans_ileave_hand.json")) as fh:
        cases = json.load(fh)["cases"]
    for c in cases:
        f = np.zeros(129, np.uint32)
        f[:len(c["freq_head"])] = c["freq_head"]
        sym = np.array(c["sym"], np.uint8)
        got = rans_ileave_encode(sym, np.zeros_like(sym), f[None], c["K"])
        assert got == bytes.fromhex(c["bytes_hex"].replace(" ", "")), c["name"]
    f = np.ones(129, np.uint32)
    f[64] = 65536 - 128
    rng = np.random.default_rng(3)
    sym = rng.integers(0, 129, 1001).astype(np.uint8)      # mostly f = 1: a word per symbol
    tab = np.zeros_like(sym)
    data = rans_ileave_encode(sym, tab, f[None], 8)
    assert np.array_equal(rans_ileave_decode(data, tab, f[None], sym.size, 8), sym)
    for bad in (data[:-2], data + b"\x00\x00", data[:-1]):
        with pytest.raises(LicError):
            rans_ileave_decode(bad, tab, f[None], sym.size, 8)
    with pytest.raises(LicError):
        rans_ileave_decode(data, tab, f[None], sym.size, 4)
    with pytest.raises(LicError):
        rans_ileave_encode(sym, tab, f[None], 3)
    # empty input: the K initial states alone
    assert rans_ileave_encode(np.zeros(0, np.uint8), np.zeros(0, np.uint8), f[None], 4) == bytes.fromhex("00000100" * 4)
