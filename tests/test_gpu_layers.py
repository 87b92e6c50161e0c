"""Layer-by-layer parity of the HIP kernels against the FP64 oracle.

Each layer runs through the C ABI (codec_run_layer) on the GPU's own output
of the previous layer, and the oracle recomputes that layer in FP64 from the
same input.  Sizes span several tiles and ragged tails (non-multiples of 64
padded to the next multiple; pixel counts that do not fill the last tile).
Tolerances: latents / activations within 1e-4 of max|ref| (relative), symbols
bit-exact against the quantiser applied to the GPU's own float32 values and
within the 1e-3 rounding band against FP64 values, scale indices bit-exact
against the float32 decision and within 1e-4 t_k of a boundary against FP64,
reconstructions within 1e-3 absolute.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import boundary_mismatches, chw, index_mismatches, layer_out_shape, make_codec, rel_err, to_nhwc

pytestmark = pytest.mark.gpu

SIZES = [(128, 128), (200, 328)]
# (N, M, H, W): the two channel widths of the transforms (N=128 M=192 and
# N=192 M=320, the larger of which uses 12-row-block weight tiles)
CASES = [(128, 192, 128, 128), (128, 192, 200, 328), (192, 320, 136, 200)]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _empty(torch, shape, dtype=None):
    return torch.empty((1,) + tuple(shape), dtype=dtype or torch.float32, device="cuda")


@pytest.mark.parametrize("gamma", ["diag", "dense"])
@pytest.mark.parametrize("N,M,H,W", CASES)
def test_analysis_layers(torch_dev, N, M, H, W, gamma):
    torch = torch_dev
    c, m = make_codec(1, N, M, gamma=gamma, max_h=H, max_w=W, max_in_flight=1)
    P = m.P
    x = synth.frame_sinusoid(H, W, t=3)
    xd = torch.from_numpy(x)[None].cuda()
    # GA0: NCHW image (padding and layout change fused in the loader)
    out = _empty(torch, layer_out_shape("GA0", H, W, N, M))
    c.run_layer("GA0", 1, H, W, xd, out)
    ref = oracle.gdn(oracle.conv2d(oracle.pad64(x), P["ga0.w"], P["ga0.b"], 2, 2), P["ga0.beta"], P["ga0.gamma"])
    assert rel_err(chw(out), ref) < 1e-4
    prev = out
    for i, L in ((1, "GA1"), (2, "GA2")):
        out = _empty(torch, layer_out_shape(L, H, W, N, M))
        c.run_layer(L, 1, H, W, prev, out)
        ref = oracle.gdn(oracle.conv2d(chw(prev), P[f"ga{i}.w"], P[f"ga{i}.b"], 2, 2),
                         P[f"ga{i}.beta"], P[f"ga{i}.gamma"])
        assert rel_err(chw(out), ref) < 1e-4, L
        prev = out
    y = _empty(torch, layer_out_shape("GA3", H, W, N, M))
    sym = _empty(torch, layer_out_shape("GA3", H, W, N, M), torch.int8)
    c.run_layer("GA3", 1, H, W, prev, y, sym)
    yref = oracle.conv2d(chw(prev), P["ga3.w"], P["ga3.b"], 2, 2)
    assert rel_err(chw(y), yref) < 1e-4
    sg = np.transpose(sym[0].cpu().numpy(), (2, 0, 1)).astype(np.int32)
    # same decision in float32 on the GPU's own y: bit-exact
    assert np.array_equal(sg, oracle.quantize_f32(np.transpose(y[0].cpu().numpy(), (2, 0, 1)), np.float32(0)))
    # against FP64 y: mismatches only inside the rounding band
    n, ok = boundary_mismatches(sg, yref, 0.0)
    assert ok, f"{n} symbol mismatches outside the 1e-3 band"
    c.close()


@pytest.mark.parametrize("hs_out", [1, 0])
@pytest.mark.parametrize("H,W", SIZES)
def test_hyper_layers(torch_dev, H, W, hs_out):
    torch = torch_dev
    c, m = make_codec(1, 128, 192, hs_out=hs_out, max_h=H, max_w=W, max_in_flight=1)
    P = m.P
    rng = np.random.default_rng(H * W)
    d = layer_out_shape("GA3", H, W, 128, 192)
    y = rng.normal(0.0, 1.3, (192, d[0], d[1]))
    yd = to_nhwc(y.astype(np.float32), "cuda")
    h = _empty(torch, layer_out_shape("HA0", H, W, 128, 192))
    c.run_layer("HA0", 1, H, W, yd, h)
    ref = oracle.relu(oracle.conv2d(np.abs(y.astype(np.float32).astype(np.float64)), P["ha0.w"], P["ha0.b"], 1, 1))
    assert rel_err(chw(h), ref) < 1e-4
    h2 = _empty(torch, layer_out_shape("HA1", H, W, 128, 192))
    c.run_layer("HA1", 1, H, W, h, h2)
    assert rel_err(chw(h2), oracle.relu(oracle.conv2d(chw(h), P["ha1.w"], P["ha1.b"], 2, 2))) < 1e-4
    z = _empty(torch, layer_out_shape("HA2", H, W, 128, 192))
    sz = _empty(torch, layer_out_shape("HA2", H, W, 128, 192), torch.int8)
    c.run_layer("HA2", 1, H, W, h2, z, sz)
    zref = oracle.conv2d(chw(h2), P["ha2.w"], P["ha2.b"], 2, 2)
    assert rel_err(chw(z), zref) < 1e-4
    szg = np.transpose(sz[0].cpu().numpy(), (2, 0, 1)).astype(np.int32)
    mu = m.medians[:, None, None]
    assert np.array_equal(szg, oracle.quantize_f32(np.transpose(z[0].cpu().numpy(), (2, 0, 1)), mu))
    n, ok = boundary_mismatches(szg, zref, mu.astype(np.float64))
    assert ok, f"{n} z-symbol mismatches outside the band"
    # h_s from the GPU's own symbols (dequantised with the medians in the loader)
    zhat = szg + mu.astype(np.float64)
    a = _empty(torch, layer_out_shape("HS0", H, W, 128, 192))
    c.run_layer("HS0", 1, H, W, sz, a)
    assert rel_err(chw(a), oracle.relu(oracle.deconv2d(zhat, P["hs0.w"], P["hs0.b"], 2, 2, 1))) < 1e-4
    b = _empty(torch, layer_out_shape("HS1", H, W, 128, 192))
    c.run_layer("HS1", 1, H, W, a, b)
    assert rel_err(chw(b), oracle.relu(oracle.deconv2d(chw(a), P["hs1.w"], P["hs1.b"], 2, 2, 1))) < 1e-4
    idx = _empty(torch, layer_out_shape("HS2", H, W, 128, 192), torch.uint8)
    v = _empty(torch, layer_out_shape("HS2", H, W, 128, 192))
    c.run_layer("HS2", 1, H, W, b, idx, v)
    vref = oracle.conv2d(chw(b), P["hs2.w"], P["hs2.b"], 1, 1)
    assert rel_err(chw(v), vref) < 1e-4
    ig = np.transpose(idx[0].cpu().numpy(), (2, 0, 1)).astype(np.int32)
    assert np.array_equal(ig, oracle.scale_index_f32(np.transpose(v[0].cpu().numpy(), (2, 0, 1)), hs_out))
    n, ok = index_mismatches(ig, oracle.scales_from_hs(vref, hs_out), m.t)
    assert ok, f"{n} index mismatches away from a table boundary"
    # without the optional v output the indices are the same
    idx2 = torch.zeros_like(idx)
    c.run_layer("HS2", 1, H, W, b, idx2, None)
    assert torch.equal(idx, idx2)
    c.close()


@pytest.mark.parametrize("kind", [1, 0])
@pytest.mark.parametrize("N,M,H,W", CASES)
def test_synthesis_layers(torch_dev, N, M, H, W, kind):
    torch = torch_dev
    c, m = make_codec(kind, N, M, gamma="dense", max_h=H, max_w=W, max_in_flight=1)
    P = m.P
    rng = np.random.default_rng(7 + H)
    d = layer_out_shape("GA3", H, W, N, M)
    sym = np.clip(np.rint(rng.normal(0, 1.5, (M, d[0], d[1]))), -64, 64).astype(np.int8)
    mu = (m.medians if kind == 0 else np.zeros(M, np.float32))[:, None, None].astype(np.float64)
    yhat = sym.astype(np.float64) + mu
    prev = to_nhwc(sym, "cuda")
    src = yhat
    for i, L in ((0, "GS0"), (1, "GS1"), (2, "GS2")):
        out = _empty(torch, layer_out_shape(L, H, W, N, M))
        c.run_layer(L, 1, H, W, prev, out)
        ref = oracle.gdn(oracle.deconv2d(src, P[f"gs{i}.w"], P[f"gs{i}.b"], 2, 2, 1),
                         P[f"gs{i}.beta"], P[f"gs{i}.gamma"], inverse=True)
        assert rel_err(chw(out), ref) < 1e-4, L
        prev = out
        src = chw(out)
    img = torch.empty((1, 3, H, W), device="cuda")
    pre = torch.empty((1, 3, 64 * -(-H // 64), 64 * -(-W // 64)), device="cuda")
    c.run_layer("GS3", 1, H, W, prev, img, pre)
    ref = oracle.deconv2d(src, P["gs3.w"], P["gs3.b"], 2, 2, 1)
    assert rel_err(pre[0].cpu().numpy(), ref) < 1e-4
    got = img[0].cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - np.clip(ref, 0, 1)[:, :H, :W])) <= 1e-3
    c.close()


def test_batched_layers_equal_single(torch_dev):
    """n images in one launch give the same bits as one launch per image."""
    torch = torch_dev
    H, W = 136, 200
    c, m = make_codec(1, 128, 192, max_h=H, max_w=W, max_in_flight=1)
    xs = np.stack([synth.frame_sinusoid(H, W, t=t) for t in range(3)])
    xd = torch.from_numpy(xs).cuda()
    outb = torch.empty((3,) + layer_out_shape("GA0", H, W, 128, 192), device="cuda")
    c.run_layer("GA0", 3, H, W, xd, outb)
    for i in range(3):
        o = _empty(torch, layer_out_shape("GA0", H, W, 128, 192))
        c.run_layer("GA0", 1, H, W, xd[i:i + 1].contiguous(), o)
        assert torch.equal(o[0], outb[i])
    # split-K layers too: the tile configuration depends on the image size only
    g = torch.Generator(device="cuda").manual_seed(3)
    for L, src in (("GA3", "GA2"), ("HA1", "HA0"), ("HS2", "HS1")):
        shp = layer_out_shape(src, H, W, 128, 192)
        inp = torch.randn((3,) + shp, device="cuda", generator=g)
        dt = torch.uint8 if L == "HS2" else torch.float32
        ob = torch.empty((3,) + layer_out_shape(L, H, W, 128, 192), device="cuda", dtype=dt)
        ab = torch.empty((3,) + layer_out_shape(L, H, W, 128, 192), device="cuda", dtype=torch.int8) if L == "GA3" else None
        c.run_layer(L, 3, H, W, inp, ob, ab)
        for i in range(3):
            o1 = torch.empty_like(ob[:1])
            a1 = torch.empty_like(ab[:1]) if ab is not None else None
            c.run_layer(L, 1, H, W, inp[i:i + 1].contiguous(), o1, a1)
            assert torch.equal(o1[0], ob[i]), L
            if ab is not None:
                assert torch.equal(a1[0], ab[i])
    c.close()


def test_layer_kernel_forms(torch_dev):
    """The kernel choice follows the precision and the frame size: whole
    frames run the GDN layers of the FP32 form on split-FP32 operands, small
    frames split K over the waves of a block (FP32 matrix cores)."""
    c, _ = make_codec(1, 128, 192, max_h=720, max_w=1280, max_in_flight=1)
    assert c.layer_kernel("GA1", 720, 1280) == ("f32x", 1)
    assert c.layer_kernel("GS2", 720, 1280) == ("f32x", 1)
    assert c.layer_kernel("GA2", 720, 1280) == ("f32x", 1)     # one pixel group per wave
    assert c.layer_kernel("GS0", 720, 1280) == ("f32x", 1)
    assert c.layer_kernel("GA0", 720, 1280) == ("f32x", 1)     # image loader
    assert c.layer_kernel("GS3", 720, 1280) == ("f32", 1)      # output layer: FP32 matrix cores
    assert c.layer_kernel("GA1", 128, 128) == ("f32", 4)
    assert c.layer_kernel("HS2", 720, 1280)[0] == "f32"
    c.close()
    c, _ = make_codec(1, 128, 192, precision=1, max_h=720, max_w=1280, max_in_flight=1)
    assert c.layer_kernel("GA1", 720, 1280) == ("bf16", 1)
    assert c.layer_kernel("HA1", 720, 1280)[0] == "f32"       # the hyper path stays FP32
    c.close()
    c, _ = make_codec(1, 128, 192, precision=2, max_h=720, max_w=1280, max_in_flight=1)
    assert c.layer_kernel("GA1", 720, 1280) == ("fp8", 1)
    assert c.layer_kernel("GS2", 720, 1280) == ("fp8", 1)
    assert c.layer_kernel("GA0", 720, 1280) == ("bf16", 1)    # image layer: bf16 operands
    assert c.layer_kernel("GS0", 720, 1280) == ("bf16", 1)    # g_s's first layer: bf16 operands
    assert c.layer_kernel("GS3", 720, 1280) == ("bf16", 1)    # output layer: bf16 halo tiles
    # GS2 stores bf16 for it; the other GDN layers e4m3 bytes
    n_px = 384 * 640 * 128
    assert c.layer_bytes("GS2", 1, 720, 1280)[1] == 2 * n_px
    assert c.layer_bytes("GS3", 1, 720, 1280)[0] == 2 * n_px
    assert c.layer_bytes("GA0", 1, 720, 1280)[1] == n_px
    c.close()
