"""Parity at the full 3x720x1280 frame size, in the launch configuration the
pipeline and the benchmark use (one frame per launch).

The oracle cannot run whole 720p transforms quickly, so every layer is
checked on sampled output pixels (all channels of each sampled pixel, from
the GPU's own input to that layer, corners and edges included), plus the
integer outputs (symbols, scale indices) over the whole tensor against the
same decision taken in float32 on the GPU's values.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import chw, layer_out_shape, make_codec

pytestmark = pytest.mark.gpu

H, W = 720, 1280
NPTS = 40


def _points(Hout, Wout, rng):
    edge = [(0, 0), (0, Wout - 1), (Hout - 1, 0), (Hout - 1, Wout - 1), (Hout // 2, 0), (0, Wout // 2)]
    rnd = [(int(rng.integers(Hout)), int(rng.integers(Wout))) for _ in range(NPTS - len(edge))]
    return edge + rnd


def _gather(t, pts):
    a = t[0].cpu().numpy().astype(np.float64)          # Hout x Wout x C
    return np.stack([a[i, j] for i, j in pts])


def _rel(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


@pytest.fixture(scope="module")
def run720():
    import torch
    assert torch.cuda.is_available()
    c, m = make_codec(1, 128, 192, gamma="dense", max_h=H, max_w=W, max_in_flight=1)
    x = synth.frame_sinusoid(H, W, t=11)
    xd = torch.from_numpy(x)[None].cuda()
    outs = {"x": x}

    def run(L, inp, dtype=None, aux_dtype=None):
        o = torch.empty((1,) + layer_out_shape(L, H, W, 128, 192), device="cuda", dtype=dtype or torch.float32)
        a = None if aux_dtype is None else torch.empty(o.shape, device="cuda", dtype=aux_dtype)
        c.run_layer(L, 1, H, W, inp, o, a)
        return o, a

    outs["GA0"], _ = run("GA0", xd)
    outs["GA1"], _ = run("GA1", outs["GA0"])
    outs["GA2"], _ = run("GA2", outs["GA1"])
    outs["GA3"], outs["sym_y"] = run("GA3", outs["GA2"], aux_dtype=torch.int8)
    outs["HA0"], _ = run("HA0", outs["GA3"])
    outs["HA1"], _ = run("HA1", outs["HA0"])
    outs["HA2"], outs["sym_z"] = run("HA2", outs["HA1"], aux_dtype=torch.int8)
    outs["HS0"], _ = run("HS0", outs["sym_z"])
    outs["HS1"], _ = run("HS1", outs["HS0"])
    outs["idx"], outs["v"] = run("HS2", outs["HS1"], dtype=torch.uint8, aux_dtype=torch.float32)
    outs["GS0"], _ = run("GS0", outs["sym_y"])
    outs["GS1"], _ = run("GS1", outs["GS0"])
    outs["GS2"], _ = run("GS2", outs["GS1"])
    img = torch.empty((1, 3, H, W), device="cuda")
    pre = torch.empty((1, 3, 768, 1280), device="cuda")
    c.run_layer("GS3", 1, H, W, outs["GS2"], img, pre)
    outs["img"], outs["pre"] = img, pre
    yield c, m, outs
    c.close()


CONV = {  # layer: (input key, weight prefix, stride, pad, post)
    "GA1": ("GA0", "ga1", 2, 2, "gdn"), "GA2": ("GA1", "ga2", 2, 2, "gdn"), "GA3": ("GA2", "ga3", 2, 2, ""),
    "HA1": ("HA0", "ha1", 2, 2, "relu"), "HA2": ("HA1", "ha2", 2, 2, ""),
}
DECONV = {"HS1": ("HS0", "hs1", "relu"), "GS1": ("GS0", "gs1", "igdn"), "GS2": ("GS1", "gs2", "igdn")}


@pytest.mark.parametrize("layer", list(CONV))
def test_conv_layers_sampled(run720, layer):
    c, m, o = run720
    src, pre, s, p, post = CONV[layer]
    x = chw(o[src])
    out = o[layer]
    pts = _points(out.shape[1], out.shape[2], np.random.default_rng(sum(map(ord, layer))))
    ref = oracle.conv2d_points(x, m.P[pre + ".w"], m.P[pre + ".b"], s, p, pts)     # npts x Co
    if post == "gdn":
        ref = oracle.gdn(ref.T, m.P[pre + ".beta"], m.P[pre + ".gamma"]).T
    elif post == "relu":
        ref = np.maximum(ref, 0.0)
    err = _rel(_gather(out, pts), ref)
    print(f"{layer}: max error / max |ref| = {err:.2e}")
    assert err < 1e-4


@pytest.mark.parametrize("layer", list(DECONV))
def test_deconv_layers_sampled(run720, layer):
    c, m, o = run720
    src, pre, post = DECONV[layer]
    x = chw(o[src])
    out = o[layer]
    pts = _points(out.shape[1], out.shape[2], np.random.default_rng(7 * sum(map(ord, layer))))
    ref = oracle.deconv2d_points(x, m.P[pre + ".w"], m.P[pre + ".b"], 2, 2, pts)
    if post == "igdn":
        ref = oracle.gdn(ref.T, m.P[pre + ".beta"], m.P[pre + ".gamma"], inverse=True).T
    else:
        ref = np.maximum(ref, 0.0)
    err = _rel(_gather(out, pts), ref)
    print(f"{layer}: max error / max |ref| = {err:.2e}")
    assert err < 1e-4


def test_first_layers_sampled(run720):
    c, m, o = run720
    P = m.P
    xp = oracle.pad64(o["x"])
    pts = _points(384, 640, np.random.default_rng(1))
    ref = oracle.gdn(oracle.conv2d_points(xp, P["ga0.w"], P["ga0.b"], 2, 2, pts).T, P["ga0.beta"], P["ga0.gamma"]).T
    assert _rel(_gather(o["GA0"], pts), ref) < 1e-4
    pts = _points(48, 80, np.random.default_rng(2))
    ref = np.maximum(oracle.conv2d_points(np.abs(chw(o["GA3"])), P["ha0.w"], P["ha0.b"], 1, 1, pts), 0)
    assert _rel(_gather(o["HA0"], pts), ref) < 1e-4
    zhat = np.transpose(o["sym_z"][0].cpu().numpy(), (2, 0, 1)).astype(np.float64) + \
        m.medians[:, None, None].astype(np.float64)
    pts = _points(24, 40, np.random.default_rng(3))
    ref = np.maximum(oracle.deconv2d_points(zhat, P["hs0.w"], P["hs0.b"], 2, 2, pts), 0)
    assert _rel(_gather(o["HS0"], pts), ref) < 1e-4
    pts = _points(48, 80, np.random.default_rng(4))
    ref = oracle.conv2d_points(chw(o["HS1"]), P["hs2.w"], P["hs2.b"], 1, 1, pts)
    assert _rel(_gather(o["v"], pts), ref) < 1e-4
    yhat = np.transpose(o["sym_y"][0].cpu().numpy(), (2, 0, 1)).astype(np.float64)
    pts = _points(96, 160, np.random.default_rng(5))
    ref = oracle.gdn(oracle.deconv2d_points(yhat, P["gs0.w"], P["gs0.b"], 2, 2, pts).T,
                     P["gs0.beta"], P["gs0.gamma"], inverse=True).T
    assert _rel(_gather(o["GS0"], pts), ref) < 1e-4


def test_output_image_sampled(run720):
    c, m, o = run720
    pts = _points(768, 1280, np.random.default_rng(6))
    ref = oracle.deconv2d_points(chw(o["GS2"]), m.P["gs3.w"], m.P["gs3.b"], 2, 2, pts)      # npts x 3
    pre = o["pre"][0].cpu().numpy()
    got = np.stack([pre[:, i, j] for i, j in pts])
    assert _rel(got, ref) < 1e-4
    img = o["img"][0].cpu().numpy()
    for q, (i, j) in enumerate(pts):
        if i < H and j < W:
            assert np.max(np.abs(img[:, i, j] - np.clip(ref[q], 0, 1))) <= 1e-3
    assert img.shape == (3, H, W)


def test_integer_outputs_whole_tensor(run720):
    c, m, o = run720
    y = np.transpose(o["GA3"][0].cpu().numpy(), (2, 0, 1))
    sy = np.transpose(o["sym_y"][0].cpu().numpy(), (2, 0, 1)).astype(np.int32)
    assert np.array_equal(sy, oracle.quantize_f32(y, np.float32(0)))
    z = np.transpose(o["HA2"][0].cpu().numpy(), (2, 0, 1))
    sz = np.transpose(o["sym_z"][0].cpu().numpy(), (2, 0, 1)).astype(np.int32)
    assert np.array_equal(sz, oracle.quantize_f32(z, m.medians[:, None, None]))
    v = np.transpose(o["v"][0].cpu().numpy(), (2, 0, 1))
    idx = np.transpose(o["idx"][0].cpu().numpy(), (2, 0, 1)).astype(np.int32)
    assert np.array_equal(idx, oracle.scale_index_f32(v, 1))
