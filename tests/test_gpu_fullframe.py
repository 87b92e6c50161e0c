"""Whole-tensor parity of one full 3x720x1280 frame in the FP32 form.

Every layer of g_a, h_a, h_s and g_s is run on the GPU through the C ABI in
the launch configuration the pipeline uses for a 720p frame (the whole-frame
split-FP32 GDN kernels, the halo-tile output layer, the split-K hyper
kernels), and every output element is compared with the FP64 oracle applied
to the GPU's own input of that layer (stage by stage, so a symbol flip
upstream never propagates into a comparison).  Integer outputs are checked
over the whole tensor against the FP64 decision (mismatches only inside the
rounding band) and against the float32 decision (bit for bit).  The codec's
own 720p bitstream must equal, byte for byte, the oracle's rANS coder run on
the GPU's symbols and scale indices, and the zero-copy toggle must not change
a byte or a pixel.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import boundary_mismatches, chw, index_mismatches, layer_out_shape, make_codec, rel_err

pytestmark = pytest.mark.gpu

H, W, N, M, S = 720, 1280, 128, 192, 8


@pytest.fixture(scope="module")
def run720():
    import torch
    assert torch.cuda.is_available()
    c, m = make_codec(1, N, M, gamma="dense", max_h=H, max_w=W, max_in_flight=2, y_slices=S, entropy_threads=8)
    x = synth.frame_sinusoid(H, W, t=23)
    xd = torch.from_numpy(x)[None].cuda()
    o = {"x": x, "xd": xd}

    def run(L, inp, dtype=None, aux_dtype=None):
        out = torch.empty((1,) + layer_out_shape(L, H, W, N, M), device="cuda", dtype=dtype or torch.float32)
        a = None if aux_dtype is None else torch.empty(out.shape, device="cuda", dtype=aux_dtype)
        c.run_layer(L, 1, H, W, inp, out, a)
        return out, a

    o["GA0"], _ = run("GA0", xd)
    o["GA1"], _ = run("GA1", o["GA0"])
    o["GA2"], _ = run("GA2", o["GA1"])
    o["GA3"], o["sym_y"] = run("GA3", o["GA2"], aux_dtype=torch.int8)
    o["HA0"], _ = run("HA0", o["GA3"])
    o["HA1"], _ = run("HA1", o["HA0"])
    o["HA2"], o["sym_z"] = run("HA2", o["HA1"], aux_dtype=torch.int8)
    o["HS0"], _ = run("HS0", o["sym_z"])
    o["HS1"], _ = run("HS1", o["HS0"])
    o["idx"], o["v"] = run("HS2", o["HS1"], dtype=torch.uint8, aux_dtype=torch.float32)
    o["GS0"], _ = run("GS0", o["sym_y"])
    o["GS1"], _ = run("GS1", o["GS0"])
    o["GS2"], _ = run("GS2", o["GS1"])
    img = torch.empty((1, 3, H, W), device="cuda")
    pre = torch.empty((1, 3, 768, 1280), device="cuda")
    c.run_layer("GS3", 1, H, W, o["GS2"], img, pre)
    o["img"], o["pre"] = img, pre
    torch.cuda.synchronize()
    yield c, m, o
    c.close()


def _chw_int(t):
    return np.transpose(t[0].cpu().numpy(), (2, 0, 1)).astype(np.int32)


# layer: (input key, weight prefix, kind, stride, post)
LAYERS = {
    "GA1": ("GA0", "ga1", "conv", 2, "gdn"), "GA2": ("GA1", "ga2", "conv", 2, "gdn"),
    "HA1": ("HA0", "ha1", "conv", 2, "relu"),
    "HS1": ("HS0", "hs1", "deconv", 2, "relu"),
    "GS1": ("GS0", "gs1", "deconv", 2, "igdn"), "GS2": ("GS1", "gs2", "deconv", 2, "igdn"),
}


def _post(m, pre, ref, post):
    if post == "gdn":
        return oracle.gdn(ref, m.P[pre + ".beta"], m.P[pre + ".gamma"])
    if post == "igdn":
        return oracle.gdn(ref, m.P[pre + ".beta"], m.P[pre + ".gamma"], inverse=True)
    if post == "relu":
        return oracle.relu(ref)
    return ref


@pytest.mark.parametrize("layer", list(LAYERS))
def test_layer_whole_tensor(run720, layer):
    c, m, o = run720
    src, pre, kind, s, post = LAYERS[layer]
    x = chw(o[src])
    if kind == "conv":
        ref = oracle.conv2d(x, m.P[pre + ".w"], m.P[pre + ".b"], s, 2)
    else:
        ref = oracle.deconv2d(x, m.P[pre + ".w"], m.P[pre + ".b"], s, 2, 1)
    ref = _post(m, pre, ref, post)
    got = chw(o[layer])
    assert got.shape == ref.shape
    err = rel_err(got, ref)
    print(f"{layer}: {ref.size} elements, max error / max |ref| = {err:.2e}")
    assert err <= 1e-4


def test_image_layer_whole_tensor(run720):
    c, m, o = run720
    P = m.P
    ref = oracle.gdn(oracle.conv2d(oracle.pad64(o["x"]), P["ga0.w"], P["ga0.b"], 2, 2), P["ga0.beta"], P["ga0.gamma"])
    err = rel_err(chw(o["GA0"]), ref)
    print(f"GA0: max error / max |ref| = {err:.2e}")
    assert err <= 1e-4


def test_latents_and_symbols_whole_tensor(run720):
    """y within 1e-4 of FP64 on the GPU's GA2 output; every symbol equals the
    FP64 quantiser except inside the 1e-3 band around a half-integer, and
    equals the float32 decision on the GPU's own y bit for bit."""
    c, m, o = run720
    yref = oracle.conv2d(chw(o["GA2"]), m.P["ga3.w"], m.P["ga3.b"], 2, 2)
    y = chw(o["GA3"])
    assert rel_err(y, yref) <= 1e-4
    sy = _chw_int(o["sym_y"])
    n, ok = boundary_mismatches(sy, yref, 0.0)
    print(f"y symbols: {sy.size}, {n} differ from the FP64 quantiser (all inside the band: {ok})")
    assert ok
    assert np.array_equal(sy, oracle.quantize_f32(y.astype(np.float32), np.float32(0)))


def test_hyper_analysis_whole_tensor(run720):
    c, m, o = run720
    P = m.P
    ref = oracle.relu(oracle.conv2d(np.abs(chw(o["GA3"])), P["ha0.w"], P["ha0.b"], 1, 1))
    assert rel_err(chw(o["HA0"]), ref) <= 1e-4
    zref = oracle.conv2d(chw(o["HA1"]), P["ha2.w"], P["ha2.b"], 2, 2)
    z = chw(o["HA2"])
    assert rel_err(z, zref) <= 1e-4
    sz = _chw_int(o["sym_z"])
    mu = m.medians[:, None, None]
    n, ok = boundary_mismatches(sz, zref, mu.astype(np.float64))
    print(f"z symbols: {sz.size}, {n} differ from the FP64 quantiser (all inside the band: {ok})")
    assert ok
    assert np.array_equal(sz, oracle.quantize_f32(z.astype(np.float32), mu))


def test_hyper_synthesis_and_index_whole_tensor(run720):
    c, m, o = run720
    P = m.P
    zhat = _chw_int(o["sym_z"]).astype(np.float64) + m.medians[:, None, None].astype(np.float64)
    ref = oracle.relu(oracle.deconv2d(zhat, P["hs0.w"], P["hs0.b"], 2, 2, 1))
    assert rel_err(chw(o["HS0"]), ref) <= 1e-4
    vref = oracle.conv2d(chw(o["HS1"]), P["hs2.w"], P["hs2.b"], 1, 1)
    v = chw(o["v"])
    assert rel_err(v, vref) <= 1e-4
    idx = _chw_int(o["idx"])
    n, ok = index_mismatches(idx, oracle.scales_from_hs(vref, 1), m.t)
    print(f"scale indices: {idx.size}, {n} differ from FP64 (all inside the band: {ok})")
    assert ok
    assert np.array_equal(idx, oracle.scale_index_f32(v.astype(np.float32), 1))


def test_first_synthesis_layer_whole_tensor(run720):
    c, m, o = run720
    P = m.P
    yhat = _chw_int(o["sym_y"]).astype(np.float64)
    ref = oracle.gdn(oracle.deconv2d(yhat, P["gs0.w"], P["gs0.b"], 2, 2, 1), P["gs0.beta"], P["gs0.gamma"],
                     inverse=True)
    err = rel_err(chw(o["GS0"]), ref)
    print(f"GS0: max error / max |ref| = {err:.2e}")
    assert err <= 1e-4


def test_output_layer_whole_tensor(run720):
    c, m, o = run720
    ref = oracle.deconv2d(chw(o["GS2"]), m.P["gs3.w"], m.P["gs3.b"], 2, 2, 1)      # 3 x 768 x 1280
    pre = o["pre"][0].cpu().numpy().astype(np.float64)
    err = rel_err(pre, ref)
    print(f"GS3 (before the clamp): max error / max |ref| = {err:.2e}")
    assert err <= 1e-4
    img = o["img"][0].cpu().numpy().astype(np.float64)
    assert img.shape == (3, H, W)
    assert np.max(np.abs(img - np.clip(ref, 0, 1)[:, :H, :W])) <= 1e-3


def test_bitstream_equals_oracle_coder_at_720p(run720):
    """The pipelined encoder's 720p bitstream equals the oracle's rANS coder
    and container on the GPU's symbols and indices; the pipelined decoder
    reproduces the layer-by-layer synthesis bit for bit."""
    import torch
    c, m, o = run720
    bits = c.encode(o["xd"])[0]
    sy = o["sym_y"][0].cpu().numpy().astype(np.int32)        # Hy x Wy x M (coding order)
    sz = o["sym_z"][0].cpu().numpy().astype(np.int32)
    idx = o["idx"][0].cpu().numpy().astype(np.int32)
    zb = oracle.rans_encode(sz.ravel() + 64, np.broadcast_to(np.arange(N, dtype=np.int32), sz.shape).ravel(),
                            m.freq_fact)
    ys = [oracle.rans_encode(sy[a:b].ravel() + 64, idx[a:b].ravel(), m.freq_gauss) for a, b in m.slice_rows(48, S)]
    ref = oracle.pack_container(1, 1, S, H, W, N, M, m.model_id, zb, ys)
    print(f"720p bitstream: {len(bits)} bytes")
    assert bits == ref
    xh = torch.empty((1, 3, H, W), device="cuda")
    assert c.decode([bits], xh) == (H, W)
    assert torch.equal(xh, o["img"])


def test_zero_copy_toggle_changes_nothing():
    """Symbols and indices through mapped host memory (zero_copy=1) or through
    device buffers and asynchronous copies (zero_copy=0): identical bytes and
    pixels, for single frames and for a pipelined batch of frames."""
    import torch
    frames = torch.from_numpy(np.stack([synth.frame_sinusoid(H, W, t=t) for t in range(4)])).cuda()
    res = {}
    for zc in (1, 0):
        c, _ = make_codec(1, N, M, max_h=H, max_w=W, y_slices=S, entropy_threads=8, max_in_flight=3, zero_copy=zc)
        bits = c.encode(frames)
        out = torch.empty_like(frames)
        c.decode(bits, out)
        out2 = torch.empty_like(frames)
        bits2 = c.encode_decode(frames, out2)
        assert bits2 == bits and torch.equal(out2, out)
        res[zc] = (bits, out)
        c.close()
    assert res[0][0] == res[1][0]
    assert torch.equal(res[0][1], res[1][1])
