"""1DN (the normalisation of the paper's implementation C, Section IV.C, read
as y_i = x_i / (beta_i + sum_j gamma_ij |x_j|) and its inverse x_i (...)) on
the GPU against the FP64 oracle.

The 1DN layers run the same kernels as GDN with the |x| contraction and the
division / multiplication epilogue.  Layers run on the GPU's own output of
the previous layer, with a dense gamma so the channel mix is exercised:
  * FP32 form, whole tensors: a small frame (split-K kernels) and a full
    720p frame (whole-frame split-FP32 kernels), within 1e-4 of max |ref|;
  * bf16 and e4m3 forms at 720p, sampled outputs (corners and edges
    included) against the oracle on the operands the form feeds the matrix
    cores, within one rounding of the stored activation;
  * the codec: the oracle (1DN) decodes the library's 1DN bitstream to the
    GPU's y_hat, the library's reconstruction matches the oracle's synthesis
    on it within 1e-3, and a GDN decoder refuses the stream.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import boundary_mismatches, chw, layer_out_shape, make_codec, rel_err
from test_gpu_fullsize_forms import Form, _points, _rel, _sampled

pytestmark = pytest.mark.gpu
N, M = 128, 192


def _chain(prec, H, W, t=7):
    import torch
    f = Form(prec)
    c, m = make_codec(1, N, M, gamma="dense", precision=prec, max_h=H, max_w=W, max_in_flight=1, norm=1)
    x = synth.frame_sinusoid(H, W, t=t)
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
    torch.cuda.synchronize()
    c.close()
    return f, m, o


@pytest.mark.parametrize("H,W", [(136, 200), (720, 1280)])
def test_fp32_1dn_layers_whole_tensor(H, W):
    print(f"1DN FP32 layers at {H}x{W}", flush=True)
    f, m, o = _chain(0, H, W)
    P = m.P
    src = oracle.pad64(o["x"])
    for i, L in enumerate(("GA0", "GA1", "GA2")):
        ref = oracle.gdn1(oracle.conv2d(src, P[f"ga{i}.w"], P[f"ga{i}.b"], 2, 2), P[f"ga{i}.beta"], P[f"ga{i}.gamma"])
        got = chw(o[L])
        err = rel_err(got, ref)
        print(f"{L} (1DN): {ref.size} elements, max error / max |ref| = {err:.2e}")
        assert err <= 1e-4, L
        src = got
    yref = oracle.conv2d(src, P["ga3.w"], P["ga3.b"], 2, 2)
    assert rel_err(chw(o["GA3"]), yref) <= 1e-4
    sy = np.transpose(o["sym"][0].cpu().numpy(), (2, 0, 1)).astype(np.int32)
    n, ok = boundary_mismatches(sy, yref, 0.0)
    assert ok, f"{n} symbols outside the band"
    src = sy.astype(np.float64)
    for i, L in enumerate(("GS0", "GS1", "GS2")):
        ref = oracle.gdn1(oracle.deconv2d(src, P[f"gs{i}.w"], P[f"gs{i}.b"], 2, 2, 1), P[f"gs{i}.beta"],
                          P[f"gs{i}.gamma"], inverse=True)
        got = chw(o[L])
        err = rel_err(got, ref)
        print(f"{L} (inverse 1DN): {ref.size} elements, max error / max |ref| = {err:.2e}")
        assert err <= 1e-4, L
        src = got


@pytest.mark.parametrize("prec", [1, 2])
def test_reduced_forms_1dn_sampled_720p(prec):
    H, W = 720, 1280
    print(f"1DN precision form {prec} at 720p", flush=True)
    f, m, o = _chain(prec, H, W, t=9)
    P = m.P
    src = f.image(oracle.pad64(o["x"]))
    for i, L in enumerate(("GA0", "GA1", "GA2")):
        out = f.values(o[L])
        pts = _points(out.shape[1], out.shape[2], np.random.default_rng(31 + i))
        w = f.w_first(P["ga0.w"]) if i == 0 else f.w(P[f"ga{i}.w"], "conv")
        ref = oracle.conv2d_points(src, w, P[f"ga{i}.b"], 2, 2, pts)
        ref = oracle.gdn1(ref.T, P[f"ga{i}.beta"], P[f"ga{i}.gamma"]).T
        if prec == 2 and L != "GS2":
            assert 8 * np.max(np.abs(ref)) < 448, "e4m3 activations would saturate"
        err = _rel(_sampled(out, pts), ref)
        print(f"{L}: max error / max |ref| = {err:.2e}")
        assert err < f.tolerance(L), L
        src = out
    src = f.yhat(np.transpose(o["sym"][0].cpu().numpy(), (2, 0, 1)).astype(np.float64))
    for i, L in enumerate(("GS0", "GS1", "GS2")):
        out = f.values(o[L])
        pts = _points(out.shape[1], out.shape[2], np.random.default_rng(41 + i))
        w = f.w_first(P["gs0.w"]) if i == 0 else f.w(P[f"gs{i}.w"], "deconv")
        ref = oracle.deconv2d_points(src, w, P[f"gs{i}.b"], 2, 2, pts)
        ref = oracle.gdn1(ref.T, P[f"gs{i}.beta"], P[f"gs{i}.gamma"], inverse=True).T
        if prec == 2 and L != "GS2":
            assert 8 * np.max(np.abs(ref)) < 448, "e4m3 activations would saturate"
        err = _rel(_sampled(out, pts), ref)
        print(f"{L}: max error / max |ref| = {err:.2e}")
        assert err < f.tolerance(L), L
        src = out


@pytest.mark.parametrize("lanes", [0, 8])
def test_1dn_codec_round_trip_with_oracle(lanes):
    """The library's 1DN bitstream equals the oracle's coder and container on
    the GPU's symbols and scale indices (both entropy coders); the GPU's
    latents match the FP64 1DN analysis; the GPU decoder's image matches the
    oracle's 1DN synthesis of the GPU's y_hat; a GDN decoder refuses it."""
    import torch
    from paper_2208_01641_amd import LicError
    from test_gpu_codec import _gpu_latents
    H, W, S = 256, 384, 3
    print(f"1DN codec 256x384, rANS lanes {lanes}", flush=True)
    c, m = make_codec(1, N, M, max_h=H, max_w=W, y_slices=S, entropy_threads=4, max_in_flight=2, norm=1,
                      rans_lanes=lanes)
    x = synth.frame_sinusoid(H, W, t=11)
    xd = torch.from_numpy(x)[None].cuda()
    bits = c.encode(xd)[0]
    lat = _gpu_latents(torch, c, xd, H, W, N, M, True)
    sy = lat["sym_y"][0].cpu().numpy().astype(np.int32)
    sz = lat["sym_z"][0].cpu().numpy().astype(np.int32)
    idx = lat["idx"][0].cpu().numpy().astype(np.int32)
    zb = m._enc(sz.ravel() + 64, np.broadcast_to(np.arange(N, dtype=np.int32), sz.shape).ravel(), m.freq_fact)
    ys = [m._enc(sy[a:b].ravel() + 64, idx[a:b].ravel(), m.freq_gauss) for a, b in m.slice_rows(sy.shape[0], S)]
    assert bits == oracle.pack_container(1, 1, S, H, W, N, M, m.model_id, zb, ys, norm=1, lanes=lanes)
    hdr = oracle.parse_container(bits)
    assert hdr["norm"] == 1 and hdr["lanes"] == lanes
    yref = m.g_a(oracle.pad64(x))
    assert rel_err(chw(lat["y"]), yref) <= 1e-4
    n, ok = boundary_mismatches(np.transpose(sy, (2, 0, 1)), yref, 0.0)
    assert ok, f"{n} symbols outside the band"
    xh = torch.empty((1, 3, H, W), device="cuda")
    assert c.decode([bits], xh) == (H, W)
    xo = np.clip(m.g_s(np.transpose(sy, (2, 0, 1)).astype(np.float64)), 0, 1)[:, :H, :W]
    err = float(np.max(np.abs(xh[0].cpu().numpy() - xo)))
    print(f"1DN codec: {len(bits)} bytes, max |x_hat - oracle| = {err:.2e}")
    assert err <= 1e-3
    c.close()
    # a GDN codec of the same weights refuses the 1DN stream
    g, _ = make_codec(1, N, M, max_h=H, max_w=W, y_slices=S, entropy_threads=2, max_in_flight=1, rans_lanes=lanes)
    with pytest.raises(LicError):
        g.decode([bits], xh)
    g.close()
