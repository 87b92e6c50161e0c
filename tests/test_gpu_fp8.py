"""OCP e4m3 precision form of the analysis / synthesis transforms.

The GEMM operands are e4m3: weights w8 = e4m3(w / s_row) with one FP32 scale
per output row (s_row = max |w| of the row / 448), activations between layers
stored as e4m3(8 x value), y_hat converted in the loader; the image layer
runs on bf16 operands and stores e4m3 activations, and so does the output
layer, whose input the last GDN layer of g_s (GS2) stores in bf16.
Products of e4m3 values are exact in FP32, so the oracle runs in FP64 on the
same dequantised operands: what remains is FP32 accumulation (float outputs
within 1e-4) and, for layers that store e4m3 activations, one e4m3 rounding
of the output (within 2^-4 of max |ref|, half an e4m3 step).  Codec level:
the bitstream is bit-exact given the GPU's symbols and indices, and the
reconstruction's PSNR is within 0.1 dB of the FP64 codec's.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import chw, layer_out_shape, make_codec, rel_err
from test_gpu_codec import _expected_stream
from test_gpu_precision import BF16_OUT_TOL, bf16, chw_any

pytestmark = pytest.mark.gpu

Q = 8.0                         # activation scale of the e4m3 form
FP8_OUT_TOL = 2.0 ** -4 + 1e-4


def e4m3(a):
    """Nearest OCP e4m3 value (ties to even), saturated at +-448, as float64."""
    a = np.asarray(a, np.float64)
    x = np.minimum(np.abs(a), 448.0)
    _, ex = np.frexp(x)
    e = np.maximum(ex - 1, -6)
    q = np.ldexp(1.0, e - 3)
    return np.sign(a) * np.minimum(np.round(x / q) * q, 448.0)


def e4m3_decode(b):
    """Values of e4m3 codes (uint8 array)."""
    b = np.asarray(b, np.uint8).astype(np.int64)
    s = np.where(b & 0x80, -1.0, 1.0)
    e = (b >> 3) & 15
    m = b & 7
    v = np.where(e == 0, m * 2.0 ** -9, (1.0 + m / 8.0) * np.ldexp(1.0, e - 7))
    return s * v


def w_fp8(w, kind):
    """Dequantised e4m3 weights with the library's per-row scales.
    kind: "conv" [co, ci, k, k], "deconv" [ci, co, k, k] (row = output
    channel), "rows" [ci, 3, 5, 5] (row = (u % 2, v % 2, output channel))."""
    w = np.asarray(w, np.float32)
    a = np.abs(w.astype(np.float64))
    if kind == "conv":
        amax = a.max(axis=(1, 2, 3))[:, None, None, None]
    elif kind == "deconv":
        amax = a.max(axis=(0, 2, 3))[None, :, None, None]
    else:
        k = w.shape[2]
        par = (np.arange(k) % 2)
        amax = np.zeros_like(a)
        for py in (0, 1):
            for px in (0, 1):
                sel = np.ix_(np.arange(w.shape[0]), np.arange(3), par == py, par == px)
                mx = a[sel].max(axis=(0, 2, 3))
                amax[sel] = mx[None, :, None, None]
    s = np.where(amax > 0, (amax / 448.0).astype(np.float32), np.float32(1.0)).astype(np.float32)
    q = (w / s).astype(np.float32)
    return e4m3(q) * s.astype(np.float64)


def act(t):
    """An e4m3 activation tensor [1, H, W, C] (uint8) as CHW values."""
    return np.transpose(e4m3_decode(t[0].cpu().numpy()) / Q, (2, 0, 1))


# (N, M, H, W): both channel widths of the transforms, ragged sizes included
CASES = [(128, 192, 128, 192), (128, 192, 200, 328), (192, 320, 136, 200)]

@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("N,M,H,W", CASES)
def test_fp8_analysis_layers(torch_dev, N, M, H, W):
    torch = torch_dev
    c, m = make_codec(1, N, M, gamma="dense", precision=2, max_h=H, max_w=W, max_in_flight=1)
    P = m.P
    x = synth.frame_sinusoid(H, W, t=2)
    xd = torch.from_numpy(x)[None].cuda()
    a = torch.empty((1,) + layer_out_shape("GA0", H, W, N, M), device="cuda", dtype=torch.uint8)
    c.run_layer("GA0", 1, H, W, xd, a)
    # the image layer runs on bf16 operands and stores e4m3 activations
    ref = oracle.gdn(oracle.conv2d(bf16(oracle.pad64(x)), bf16(P["ga0.w"]), P["ga0.b"], 2, 2),
                     P["ga0.beta"], P["ga0.gamma"])
    assert np.max(np.abs(ref)) * Q < 448
    assert rel_err(act(a), ref) < FP8_OUT_TOL
    prev = a
    for i, L in ((1, "GA1"), (2, "GA2")):
        o = torch.empty((1,) + layer_out_shape(L, H, W, N, M), device="cuda", dtype=torch.uint8)
        c.run_layer(L, 1, H, W, prev, o)
        ref = oracle.gdn(oracle.conv2d(act(prev), w_fp8(P[f"ga{i}.w"], "conv"), P[f"ga{i}.b"], 2, 2),
                         P[f"ga{i}.beta"], P[f"ga{i}.gamma"])
        assert rel_err(act(o), ref) < FP8_OUT_TOL, L
        prev = o
    y = torch.empty((1,) + layer_out_shape("GA3", H, W, N, M), device="cuda")
    sy = torch.empty_like(y, dtype=torch.int8)
    c.run_layer("GA3", 1, H, W, prev, y, sy)
    yref = oracle.conv2d(act(prev), w_fp8(P["ga3.w"], "conv"), P["ga3.b"], 2, 2)
    assert rel_err(chw(y), yref) < 1e-4              # exact products, FP32 sums
    assert np.array_equal(np.transpose(sy[0].cpu().numpy(), (2, 0, 1)).astype(np.int32),
                          oracle.quantize_f32(np.transpose(y[0].cpu().numpy(), (2, 0, 1)), np.float32(0)))
    c.close()


@pytest.mark.parametrize("N,M,H,W", CASES)
def test_fp8_synthesis_layers(torch_dev, N, M, H, W):
    torch = torch_dev
    c, m = make_codec(1, N, M, gamma="dense", precision=2, max_h=H, max_w=W, max_in_flight=1)
    P = m.P
    rng = np.random.default_rng(H + W)
    d = layer_out_shape("GA3", H, W, N, M)
    sym = np.clip(np.rint(rng.normal(0, 1.5, (M, d[0], d[1]))), -64, 64).astype(np.int8)
    prev = torch.from_numpy(np.ascontiguousarray(np.transpose(sym, (1, 2, 0)))[None]).cuda()
    src = sym.astype(np.float64)            # exact on the first layer's bf16 operands
    for i, L in ((0, "GS0"), (1, "GS1"), (2, "GS2")):
        # GS2 stores bf16 (the output layer's operands), the others e4m3
        o = torch.empty((1,) + layer_out_shape(L, H, W, N, M), device="cuda",
                        dtype=torch.bfloat16 if L == "GS2" else torch.uint8)
        c.run_layer(L, 1, H, W, prev, o)
        # (the first layer runs on bf16 operands and stores e4m3)
        w = bf16(P["gs0.w"]) if i == 0 else w_fp8(P[f"gs{i}.w"], "deconv")
        ref = oracle.gdn(oracle.deconv2d(src, w, P[f"gs{i}.b"], 2, 2, 1),
                         P[f"gs{i}.beta"], P[f"gs{i}.gamma"], inverse=True)
        if L == "GS2":
            assert rel_err(chw_any(o), ref) < BF16_OUT_TOL, L
            src = chw_any(o)
        else:
            assert np.max(np.abs(ref)) * Q < 448, L
            assert rel_err(act(o), ref) < FP8_OUT_TOL, L
            src = act(o)
        prev = o
    img = torch.empty((1, 3, H, W), device="cuda")
    pre = torch.empty((1, 3, 64 * -(-H // 64), 64 * -(-W // 64)), device="cuda")
    c.run_layer("GS3", 1, H, W, prev, img, pre)
    ref = oracle.deconv2d(src, bf16(P["gs3.w"]), P["gs3.b"], 2, 2, 1)
    assert rel_err(pre[0].cpu().numpy(), ref) < 1e-4
    assert np.max(np.abs(img[0].cpu().numpy() - np.clip(ref, 0, 1)[:, :H, :W])) <= 1e-3
    c.close()


def _gpu_latents_fp8(torch, c, xd, H, W):
    shp = lambda L: (1,) + layer_out_shape(L, H, W, 128, 192)
    a = torch.empty(shp("GA0"), device="cuda", dtype=torch.uint8)
    c.run_layer("GA0", 1, H, W, xd, a)
    b = torch.empty(shp("GA1"), device="cuda", dtype=torch.uint8)
    c.run_layer("GA1", 1, H, W, a, b)
    a2 = torch.empty(shp("GA2"), device="cuda", dtype=torch.uint8)
    c.run_layer("GA2", 1, H, W, b, a2)
    y = torch.empty(shp("GA3"), device="cuda")
    sy = torch.empty_like(y, dtype=torch.int8)
    c.run_layer("GA3", 1, H, W, a2, y, sy)
    h = torch.empty(shp("HA0"), device="cuda")
    c.run_layer("HA0", 1, H, W, y, h)
    h2 = torch.empty(shp("HA1"), device="cuda")
    c.run_layer("HA1", 1, H, W, h, h2)
    z = torch.empty(shp("HA2"), device="cuda")
    sz = torch.empty_like(z, dtype=torch.int8)
    c.run_layer("HA2", 1, H, W, h2, z, sz)
    g = torch.empty(shp("HS0"), device="cuda")
    c.run_layer("HS0", 1, H, W, sz, g)
    g2 = torch.empty(shp("HS1"), device="cuda")
    c.run_layer("HS1", 1, H, W, g, g2)
    idx = torch.empty(shp("HS2"), device="cuda", dtype=torch.uint8)
    c.run_layer("HS2", 1, H, W, g2, idx, None)
    return {"y": y, "sym_y": sy, "sym_z": sz, "idx": idx}


def test_fp8_codec_rate_distortion_vs_fp64(torch_dev):
    torch = torch_dev
    H, W = 256, 384
    c, m = make_codec(1, 128, 192, precision=2, max_h=H, max_w=W, y_slices=2, entropy_threads=4)
    x = synth.frame_sinusoid(H, W, t=9)
    xd = torch.from_numpy(x)[None].cuda()
    xh = torch.empty((1, 3, H, W), device="cuda")
    bits = c.encode_decode(xd, xh)[0]
    lat = _gpu_latents_fp8(torch, c, xd, H, W)
    assert bits == _expected_stream(m, 2, H, W, lat)            # entropy side exact
    bits64, _ = m.encode(x, S=2)
    x64, _ = m.decode(bits64)
    xf = xh[0].cpu().numpy()
    d_psnr = oracle.psnr(x, xf) - oracle.psnr(x, x64)
    d_bpp = oracle.bpp(len(bits), H, W) - oracle.bpp(len(bits64), H, W)
    print(f"FP8 vs FP64: dPSNR {d_psnr:+.4f} dB, PSNR(x64, xfp8) {oracle.psnr(x64, xf):.2f} dB, "
          f"dbpp {d_bpp:+.5f}")
    assert abs(d_psnr) <= 0.1
    assert abs(d_bpp) <= 0.05 * oracle.bpp(len(bits64), H, W)
    # fidelity to the FP64 codec's own reconstruction: ~24 dB measured at 720p
    assert oracle.psnr(x64, xf) >= 20.0
    c.close()
