"""Activation scales of the e4m3 form calibrated per layer (codec_calibrate).

With the synthesis weights scaled up so that g_s's activations exceed 56
(beyond what the fixed scale 8 can store in e4m3, whose largest value is
448), an uncalibrated codec clamps values and counts them; after
calibration on a seeded frame every e4m3-storing layer has q = 448 / (2
amax), no value is clamped, each layer matches the FP64 oracle on the same
dequantised operands within one e4m3 rounding (decoding the stored bytes
with the layer's own q), and the codec reconstruction is closer to the FP64
codec's than the uncalibrated one.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import chw, layer_out_shape, rel_err
from test_gpu_fp8 import FP8_OUT_TOL, e4m3_decode, w_fp8
from test_gpu_precision import BF16_OUT_TOL, bf16, chw_any

pytestmark = pytest.mark.gpu
N, M, H, W = 128, 192, 256, 384


def _big_model():
    P = synth.model_params(1, N, M, gamma="dense")
    P["gs0.w"] = (P["gs0.w"] * 4.0).astype(np.float32)
    blob = synth.weight_blob(P, 1, N, M)
    return P, blob


def _codec(blob):
    from paper_2208_01641_amd import Codec
    return Codec(blob, kind=1, N=N, M=M, precision=2, max_h=H, max_w=W, y_slices=2, entropy_threads=4,
                 max_in_flight=1)


def _act(t, q):
    return np.transpose(e4m3_decode(t[0].cpu().numpy()) / q, (2, 0, 1))


def _synthesis(c, sym_dev):
    import torch
    o = {}
    prev = sym_dev
    for L in ("GS0", "GS1", "GS2"):
        t = torch.empty((1,) + layer_out_shape(L, H, W, N, M), device="cuda",
                        dtype=torch.bfloat16 if L == "GS2" else torch.uint8)
        c.run_layer(L, 1, H, W, prev, t)
        o[L] = prev = t
    torch.cuda.synchronize()
    return o


def test_calibration_removes_clamping_and_keeps_parity():
    import torch
    P, blob = _big_model()
    x = torch.from_numpy(synth.frame_sinusoid(H, W, t=3))[None].cuda()
    # y_hat of the frame from the codec's own analysis transform
    c0 = _codec(blob)
    shp = lambda L: (1,) + layer_out_shape(L, H, W, N, M)
    a = torch.empty(shp("GA0"), device="cuda", dtype=torch.uint8)
    c0.run_layer("GA0", 1, H, W, x, a)
    b = torch.empty(shp("GA1"), device="cuda", dtype=torch.uint8)
    c0.run_layer("GA1", 1, H, W, a, b)
    a2 = torch.empty(shp("GA2"), device="cuda", dtype=torch.uint8)
    c0.run_layer("GA2", 1, H, W, b, a2)
    y = torch.empty(shp("GA3"), device="cuda")
    sym = torch.empty_like(y, dtype=torch.int8)
    c0.run_layer("GA3", 1, H, W, a2, y, sym)
    # uncalibrated: every q is 8 and g_s's activations overflow e4m3
    q0, sat0 = c0.fp8_scales()
    assert q0[10] == 8.0 and q0[11] == 8.0
    _synthesis(c0, sym)
    _, sat1 = c0.fp8_scales()
    print(f"uncalibrated: {sat1 - sat0} values clamped at +-448")
    assert sat1 > sat0
    x2 = synth.frame_sinusoid(H, W, t=4)
    x2d = torch.from_numpy(x2)[None].cuda()
    xh0 = torch.empty((1, 3, H, W), device="cuda")
    c0.encode_decode(x2d, xh0)
    c0.close()

    c = _codec(blob)
    c.calibrate(x)
    q, sat_before = c.fp8_scales()
    names = ["GA0", "GA1", "GA2", "GS0", "GS1"]
    ids = [0, 1, 2, 10, 11]
    print("calibrated q:", {n: float(q[i]) for n, i in zip(names, ids)})
    assert all(q[i] > 0 for i in ids) and q[12] == 0.0 and q[13] == 0.0
    assert q[10] < 8.0                      # the enlarged layer needs a smaller scale
    o = _synthesis(c, sym)
    src = np.transpose(sym[0].cpu().numpy(), (2, 0, 1)).astype(np.float64)
    for i, L in enumerate(("GS0", "GS1", "GS2")):
        w = bf16(P["gs0.w"]) if i == 0 else w_fp8(P[f"gs{i}.w"], "deconv")    # first layer: bf16 operands
        ref = oracle.gdn(oracle.deconv2d(src, w, P[f"gs{i}.b"], 2, 2, 1),
                         P[f"gs{i}.beta"], P[f"gs{i}.gamma"], inverse=True)
        got = chw_any(o[L]) if L == "GS2" else _act(o[L], q[10 + i])
        err = rel_err(got, ref)
        print(f"{L}: max |ref| {np.max(np.abs(ref)):.1f}, max error / max |ref| = {err:.2e}")
        if L != "GS2":
            assert np.max(np.abs(ref)) > 56.0, "the test needs activations beyond the fixed scale's range"
        assert err < (BF16_OUT_TOL if L == "GS2" else FP8_OUT_TOL), L
        src = got
    # codec level on another frame of the stream: nothing clamped, and
    # closer to the FP64 codec's own reconstruction than without calibration
    xh = torch.empty((1, 3, H, W), device="cuda")
    c.encode_decode(x2d, xh)
    _, sat_after = c.fp8_scales()
    assert sat_after == sat_before
    m = oracle.Model(P, 1, N, M, blob)
    x64, _ = m.decode(m.encode(x2, S=2)[0])
    p = oracle.psnr(x64, xh[0].cpu().numpy())
    p0 = oracle.psnr(x64, xh0[0].cpu().numpy())
    print(f"PSNR against the FP64 codec's reconstruction: calibrated {p:.2f} dB, fixed scale 8 {p0:.2f} dB")
    assert p > p0
    c.close()
