"""BF16 precision form of the analysis / synthesis transforms.

Layer parity: with bf16 operands the GEMM products are exact in FP32, so
the oracle is run in FP64 on the same bf16-rounded weights and on the GPU's
own (bf16) layer inputs; what remains is FP32 accumulation (latents within
1e-4) and, for layers that store bf16 activations, one bf16 rounding of the
output (within 2^-8 of max|ref|).  Codec level: the bitstream is bit-exact
given the GPU's symbols and indices, and the reconstruction's PSNR and the
rate are reported against the FP64 oracle codec (gate: 0.1 dB).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import chw, layer_out_shape, make_codec, rel_err
from test_gpu_codec import _expected_stream

pytestmark = pytest.mark.gpu

BF16_OUT_TOL = 2.0 ** -8
# (N, M, H, W): both channel widths of the transforms, ragged sizes included
CASES = [(128, 192, 128, 192), (128, 192, 200, 328), (192, 320, 136, 200)]


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def chw_any(t):
    return np.transpose(t[0].float().cpu().numpy().astype(np.float64), (2, 0, 1))


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("N,M,H,W", CASES)
def test_bf16_analysis_layers(torch_dev, N, M, H, W):
    torch = torch_dev
    c, m = make_codec(1, N, M, gamma="dense", precision=1, max_h=H, max_w=W, max_in_flight=1)
    P = m.P
    x = synth.frame_sinusoid(H, W, t=2)
    xd = torch.from_numpy(x)[None].cuda()
    a = torch.empty((1,) + layer_out_shape("GA0", H, W, N, M), device="cuda", dtype=torch.bfloat16)
    c.run_layer("GA0", 1, H, W, xd, a)
    ref = oracle.gdn(oracle.conv2d(bf16(oracle.pad64(x)), bf16(P["ga0.w"]), P["ga0.b"], 2, 2),
                     P["ga0.beta"], P["ga0.gamma"])
    assert rel_err(chw_any(a), ref) < BF16_OUT_TOL
    prev = a
    for i, L in ((1, "GA1"), (2, "GA2")):
        o = torch.empty((1,) + layer_out_shape(L, H, W, N, M), device="cuda", dtype=torch.bfloat16)
        c.run_layer(L, 1, H, W, prev, o)
        ref = oracle.gdn(oracle.conv2d(chw_any(prev), bf16(P[f"ga{i}.w"]), P[f"ga{i}.b"], 2, 2),
                         P[f"ga{i}.beta"], P[f"ga{i}.gamma"])
        assert rel_err(chw_any(o), ref) < BF16_OUT_TOL, L
        prev = o
    y = torch.empty((1,) + layer_out_shape("GA3", H, W, N, M), device="cuda")
    sy = torch.empty_like(y, dtype=torch.int8)
    c.run_layer("GA3", 1, H, W, prev, y, sy)
    yref = oracle.conv2d(chw_any(prev), bf16(P["ga3.w"]), P["ga3.b"], 2, 2)
    assert rel_err(chw(y), yref) < 1e-4              # exact products, FP32 sums
    assert np.array_equal(np.transpose(sy[0].cpu().numpy(), (2, 0, 1)).astype(np.int32),
                          oracle.quantize_f32(np.transpose(y[0].cpu().numpy(), (2, 0, 1)), np.float32(0)))
    c.close()


@pytest.mark.parametrize("N,M,H,W", CASES)
def test_bf16_synthesis_layers(torch_dev, N, M, H, W):
    torch = torch_dev
    c, m = make_codec(1, N, M, gamma="dense", precision=1, max_h=H, max_w=W, max_in_flight=1)
    P = m.P
    rng = np.random.default_rng(H + W)
    d = layer_out_shape("GA3", H, W, N, M)
    sym = np.clip(np.rint(rng.normal(0, 1.5, (M, d[0], d[1]))), -64, 64).astype(np.int8)
    prev = torch.from_numpy(np.ascontiguousarray(np.transpose(sym, (1, 2, 0)))[None]).cuda()
    src = sym.astype(np.float64)
    for i, L in ((0, "GS0"), (1, "GS1"), (2, "GS2")):
        o = torch.empty((1,) + layer_out_shape(L, H, W, N, M), device="cuda", dtype=torch.bfloat16)
        c.run_layer(L, 1, H, W, prev, o)
        ref = oracle.gdn(oracle.deconv2d(src, bf16(P[f"gs{i}.w"]), P[f"gs{i}.b"], 2, 2, 1),
                         P[f"gs{i}.beta"], P[f"gs{i}.gamma"], inverse=True)
        assert rel_err(chw_any(o), ref) < BF16_OUT_TOL, L
        prev = o
        src = chw_any(o)
    img = torch.empty((1, 3, H, W), device="cuda")
    pre = torch.empty((1, 3, 64 * -(-H // 64), 64 * -(-W // 64)), device="cuda")
    c.run_layer("GS3", 1, H, W, prev, img, pre)
    ref = oracle.deconv2d(src, bf16(P["gs3.w"]), P["gs3.b"], 2, 2, 1)
    assert rel_err(pre[0].cpu().numpy(), ref) < 1e-4
    assert np.max(np.abs(img[0].cpu().numpy() - np.clip(ref, 0, 1)[:, :H, :W])) <= 1e-3
    c.close()


def _gpu_latents_bf16(torch, c, xd, H, W):
    shp = lambda L: (1,) + layer_out_shape(L, H, W, 128, 192)
    a = torch.empty(shp("GA0"), device="cuda", dtype=torch.bfloat16)
    c.run_layer("GA0", 1, H, W, xd, a)
    b = torch.empty(shp("GA1"), device="cuda", dtype=torch.bfloat16)
    c.run_layer("GA1", 1, H, W, a, b)
    a2 = torch.empty(shp("GA2"), device="cuda", dtype=torch.bfloat16)
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


def test_bf16_codec_rate_distortion_vs_fp64(torch_dev):
    torch = torch_dev
    H, W = 256, 384
    c, m = make_codec(1, 128, 192, precision=1, max_h=H, max_w=W, y_slices=2, entropy_threads=4)
    x = synth.frame_sinusoid(H, W, t=9)
    xd = torch.from_numpy(x)[None].cuda()
    xh = torch.empty((1, 3, H, W), device="cuda")
    bits = c.encode_decode(xd, xh)[0]
    lat = _gpu_latents_bf16(torch, c, xd, H, W)
    assert bits == _expected_stream(m, 2, H, W, lat)            # entropy side exact
    bits64, _ = m.encode(x, S=2)
    x64, _ = m.decode(bits64)
    xb = xh[0].cpu().numpy()
    d_psnr = oracle.psnr(x, xb) - oracle.psnr(x, x64)
    d_bpp = oracle.bpp(len(bits), H, W) - oracle.bpp(len(bits64), H, W)
    print(f"BF16 vs FP64: dPSNR {d_psnr:+.4f} dB, PSNR(x64, xbf16) {oracle.psnr(x64, xb):.2f} dB, "
          f"dbpp {d_bpp:+.5f}")
    assert abs(d_psnr) <= 0.1
    assert abs(d_bpp) <= 0.01 * oracle.bpp(len(bits64), H, W)
    # fidelity to the FP64 codec's own reconstruction (the random-weight
    # codec is ~7 dB from the source, so the gap above barely moves): ~36 dB
    # measured at 720p
    assert oracle.psnr(x64, xb) >= 30.0
    c.close()
