"""Full-size parity of the analysis / synthesis transforms in every operand
form (FP32, bf16, e4m3) and both channel widths, in the launch configuration
of whole frames (one frame per launch: no split-K, the block-shared weight
and gamma staging of the GDN layers).

Each layer runs on the GPU's own output of the previous layer; the oracle
recomputes all channels of sampled output pixels (corners and edges
included) in FP64 on the same operands the form feeds the matrix cores:
bf16-rounded weights, per-row-scaled e4m3 weights, the GPU's stored bf16 /
e4m3 activations.  Tolerances (relative to max |ref|): 1e-4 for FP32 values
(FP32 accumulation), plus one rounding of the stored activation for the bf16
(2^-8) and e4m3 (2^-4) forms.  The symbols of y are checked over the whole
tensor against the same decision taken in float32 on the GPU's y.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import chw, layer_out_shape, make_codec
from test_gpu_fp8 import FP8_OUT_TOL, act, w_fp8
from test_gpu_precision import BF16_OUT_TOL, bf16, chw_any

pytestmark = pytest.mark.gpu

NPTS = 32
# (precision, N, M, H, W); FP32 at N=128 M=192 720p is covered layer by layer
# (hyper path included) in test_gpu_fullsize
CASES = [(1, 128, 192, 720, 1280), (2, 128, 192, 720, 1280),
         (0, 192, 320, 1080, 1920), (1, 192, 320, 1080, 1920), (2, 192, 320, 1080, 1920)]


def _points(Hout, Wout, rng):
    edge = [(0, 0), (0, Wout - 1), (Hout - 1, 0), (Hout - 1, Wout - 1), (Hout // 2, 0), (0, Wout // 2)]
    return edge + [(int(rng.integers(Hout)), int(rng.integers(Wout))) for _ in range(NPTS - len(edge))]


def _rel(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


class Form:
    """How one operand form stores activations and rounds weights."""

    def __init__(self, prec):
        self.prec = prec

    def _bf16_out(self, L):         # the e4m3 form's GS2 stores bf16 (the output layer's operands)
        return self.prec == 1 or (self.prec == 2 and L == "GS2")

    def tolerance(self, L):
        return 1e-4 if self.prec == 0 else BF16_OUT_TOL if self._bf16_out(L) else FP8_OUT_TOL

    def dtype(self, torch, L=None):
        return torch.float32 if self.prec == 0 else torch.bfloat16 if self._bf16_out(L) else torch.uint8

    def values(self, t):            # stored activation [1, H, W, C] -> CHW float64
        import torch
        return chw(t) if t.dtype == torch.float32 else chw_any(t) if t.dtype == torch.bfloat16 else act(t)

    def w(self, w, kind):
        if self.prec == 0:
            return w
        if self.prec == 1 or kind == "rows":    # the output layer runs on bf16 operands in both forms
            return bf16(w)
        return w_fp8(w, kind)

    def image(self, x):             # the image layer of the e4m3 form runs on bf16 operands
        return x if self.prec == 0 else bf16(x)

    def w_first(self, w):           # the e4m3 form's first layers of g_a and g_s: bf16 operands
        return w if self.prec == 0 else bf16(w)

    def yhat(self, sym):            # symbols (|sym| <= 64) are exact in every form's first g_s layer
        return sym


@pytest.fixture(scope="module", params=CASES, ids=lambda c: "p%d-N%d-M%d-%dx%d" % c)
def chain(request):
    import torch
    assert torch.cuda.is_available()
    prec, N, M, H, W = request.param
    f = Form(prec)
    c, m = make_codec(1, N, M, gamma="dense", precision=prec, max_h=H, max_w=W, max_in_flight=1)
    x = synth.frame_sinusoid(H, W, t=5)
    shp = lambda L: (1,) + layer_out_shape(L, H, W, N, M)
    o = {"x": x}
    o["GA0"] = torch.empty(shp("GA0"), device="cuda", dtype=f.dtype(torch, "GA0"))
    c.run_layer("GA0", 1, H, W, torch.from_numpy(x)[None].cuda(), o["GA0"])
    for L, src in (("GA1", "GA0"), ("GA2", "GA1")):
        o[L] = torch.empty(shp(L), device="cuda", dtype=f.dtype(torch, L))
        c.run_layer(L, 1, H, W, o[src], o[L])
    o["GA3"] = torch.empty(shp("GA3"), device="cuda")
    o["sym"] = torch.empty(shp("GA3"), device="cuda", dtype=torch.int8)
    c.run_layer("GA3", 1, H, W, o["GA2"], o["GA3"], o["sym"])
    o["GS0"] = torch.empty(shp("GS0"), device="cuda", dtype=f.dtype(torch, "GS0"))
    c.run_layer("GS0", 1, H, W, o["sym"], o["GS0"])
    for L, src in (("GS1", "GS0"), ("GS2", "GS1")):
        o[L] = torch.empty(shp(L), device="cuda", dtype=f.dtype(torch, L))
        c.run_layer(L, 1, H, W, o[src], o[L])
    Hp, Wp = 64 * -(-H // 64), 64 * -(-W // 64)
    o["img"] = torch.empty((1, 3, H, W), device="cuda")
    o["pre"] = torch.empty((1, 3, Hp, Wp), device="cuda")
    c.run_layer("GS3", 1, H, W, o["GS2"], o["img"], o["pre"])
    torch.cuda.synchronize()
    yield f, m, o, (N, M, H, W)
    c.close()


def _sampled(out_chw, pts):
    return np.stack([out_chw[:, i, j] for i, j in pts])


def test_analysis_sampled(chain):
    f, m, o, (N, M, H, W) = chain
    P = m.P
    src = f.image(oracle.pad64(o["x"]))
    for i, L in enumerate(("GA0", "GA1", "GA2")):
        out = f.values(o[L])
        pts = _points(out.shape[1], out.shape[2], np.random.default_rng(11 + i))
        w = f.w_first(P["ga0.w"]) if i == 0 else f.w(P[f"ga{i}.w"], "conv")
        ref = oracle.conv2d_points(src, w, P[f"ga{i}.b"], 2, 2, pts)
        ref = oracle.gdn(ref.T, P[f"ga{i}.beta"], P[f"ga{i}.gamma"]).T
        err = _rel(_sampled(out, pts), ref)
        print(f"{L}: max error / max |ref| = {err:.2e}")
        assert err < f.tolerance(L), L
        src = out
    y = chw(o["GA3"])
    pts = _points(y.shape[1], y.shape[2], np.random.default_rng(14))
    ref = oracle.conv2d_points(src, f.w(P["ga3.w"], "conv"), P["ga3.b"], 2, 2, pts)
    assert _rel(_sampled(y, pts), ref) < 1e-4              # FP32 values
    sym = np.transpose(o["sym"][0].cpu().numpy(), (2, 0, 1)).astype(np.int32)
    assert np.array_equal(sym, oracle.quantize_f32(np.transpose(o["GA3"][0].cpu().numpy(), (2, 0, 1)), np.float32(0)))


def test_synthesis_sampled(chain):
    f, m, o, (N, M, H, W) = chain
    P = m.P
    src = f.yhat(np.transpose(o["sym"][0].cpu().numpy(), (2, 0, 1)).astype(np.float64))
    for i, L in enumerate(("GS0", "GS1", "GS2")):
        out = f.values(o[L])
        pts = _points(out.shape[1], out.shape[2], np.random.default_rng(21 + i))
        w = f.w_first(P["gs0.w"]) if i == 0 else f.w(P[f"gs{i}.w"], "deconv")
        ref = oracle.deconv2d_points(src, w, P[f"gs{i}.b"], 2, 2, pts)
        ref = oracle.gdn(ref.T, P[f"gs{i}.beta"], P[f"gs{i}.gamma"], inverse=True).T
        err = _rel(_sampled(out, pts), ref)
        print(f"{L}: max error / max |ref| = {err:.2e}")
        assert err < f.tolerance(L), L
        src = out
    pre = o["pre"][0].cpu().numpy().astype(np.float64)
    pts = _points(pre.shape[1], pre.shape[2], np.random.default_rng(24))
    ref = oracle.deconv2d_points(src, f.w(P["gs3.w"], "rows"), P["gs3.b"], 2, 2, pts)
    assert _rel(_sampled(pre, pts), ref) < 1e-4
    img = o["img"][0].cpu().numpy()
    for q, (i, j) in enumerate(pts):
        if i < H and j < W:
            assert np.max(np.abs(img[:, i, j] - np.clip(ref[q], 0, 1))) <= 1e-3
