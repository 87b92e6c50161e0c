"""Whole-oracle pins: the codec round trip (CPU only)."""
import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module")
def fact_model():
    P = synth.model_params(0, 128, 192)
    return oracle.Model(P, 0, 128, 192, synth.weight_blob(P, 0, 128, 192))


@pytest.fixture(scope="module")
def hyper_model():
    P = synth.model_params(1, 128, 192)
    return oracle.Model(P, 1, 128, 192, synth.weight_blob(P, 1, 128, 192))


def test_factorized_round_trip_cfg1(fact_model):
    x = synth.image_1f(128, 128)
    bits, enc = fact_model.encode(x, S=3)
    xr, dec = fact_model.decode(bits)
    assert np.array_equal(dec["yhat"], enc["yhat"])
    direct = np.clip(fact_model.g_s(enc["yhat"]), 0, 1)[:, :128, :128]
    assert np.array_equal(xr, direct)
    assert xr.shape == (3, 128, 128) and xr.min() >= 0 and xr.max() <= 1
    # the y offsets are the channel medians: mean of (y - mu) is small next to y's spread
    d = enc["y"] - fact_model.medians[:, None, None]
    assert np.all(np.abs(enc["sym_y"]) <= 64)
    assert np.array_equal(enc["sym_y"], np.clip(np.rint(d), -64, 64))


def test_hyperprior_round_trip_ragged_size(hyper_model):
    # 100 x 150 is padded to 128 x 192; the crop must restore the original size
    x = synth.frame_sinusoid(100, 150)
    bits, enc = hyper_model.encode(x, S=2)
    hdr = oracle.parse_container(bits)
    assert (hdr["H"], hdr["W"], hdr["S"], hdr["hs_out"]) == (100, 150, 2, 1)
    assert hdr["model_id"] == hyper_model.model_id
    xr, dec = hyper_model.decode(bits)
    assert xr.shape == (3, 100, 150)
    assert np.array_equal(dec["sym_z"], enc["sym_z"])
    assert np.array_equal(dec["idx"], enc["idx"])
    assert np.array_equal(dec["yhat"], enc["yhat"])
    assert enc["y"].shape == (192, 8, 12) and enc["z"].shape == (128, 2, 3)


def test_hyperprior_rate_close_to_model_entropy(hyper_model):
    x = synth.frame_sinusoid(128, 128)
    bits, enc = hyper_model.encode(x, S=1)
    sym = np.transpose(enc["sym_y"], (1, 2, 0)).ravel() + 64
    tab = np.transpose(enc["idx"], (1, 2, 0)).ravel()
    ybits = -np.sum(np.log2(hyper_model.freq_gauss[tab, sym] / 65536.0))
    hdr = oracle.parse_container(bits)
    assert len(hdr["y"][0]) * 8 == pytest.approx(ybits, rel=0.01, abs=64)


def test_relu_output_mode_round_trip():
    P = synth.model_params(1, 128, 192)
    m = oracle.Model(P, 1, 128, 192, synth.weight_blob(P, 1, 128, 192), hs_out=0)
    x = synth.frame_sinusoid(64, 64)
    bits, enc = m.encode(x)
    xr, dec = m.decode(bits)
    assert np.array_equal(dec["yhat"], enc["yhat"])
    assert oracle.parse_container(bits)["hs_out"] == 0


def test_decode_rejects_other_model(hyper_model):
    x = synth.frame_sinusoid(64, 64)
    bits, _ = hyper_model.encode(x)
    P = synth.model_params(1, 128, 192, seed=99)
    other = oracle.Model(P, 1, 128, 192, synth.weight_blob(P, 1, 128, 192))
    with pytest.raises(ValueError):
        other.decode(bits)


@pytest.mark.parametrize("kind,lanes", [(1, 8), (0, 4)])
def test_interleaved_coder_round_trip_and_flag(kind, lanes):
    """With the interleaved coder the codec round trip is unchanged: the same
    symbols, the same rate up to the coders' per-stream overhead, and the
    coder recorded in flag bits 2..4 of the container."""
    P = synth.model_params(kind, 128, 192)
    blob = synth.weight_blob(P, kind, 128, 192)
    byte = oracle.Model(P, kind, 128, 192, blob)
    il = oracle.Model(P, kind, 128, 192, blob, lanes=lanes)
    x = synth.frame_sinusoid(96, 160)
    b0, e0 = byte.encode(x, S=2)
    b1, e1 = il.encode(x, S=2)
    assert np.array_equal(e0["sym_y"], e1["sym_y"])
    hdr = oracle.parse_container(b1)
    assert hdr["lanes"] == lanes and oracle.parse_container(b0)["lanes"] == 0
    assert b1[6] >> 2 == lanes.bit_length() - 1
    xr, dec = il.decode(b1)
    assert np.array_equal(dec["yhat"], e0["yhat"])
    # each stream pays at most 4 lanes + 1 bytes of states beyond the byte-wise coder's
    nstreams = 2 + (1 if kind == 1 else 0)
    assert abs(len(b1) - len(b0)) <= nstreams * (4 * lanes + 8) + len(b0) // 50
    with pytest.raises(ValueError):
        byte.decode(b1)
    with pytest.raises(ValueError):
        il.decode(b0)
    bad = bytearray(b1)
    bad[6] |= 0x80            # an undefined flag bit
    with pytest.raises(ValueError):
        oracle.parse_container(bytes(bad))
