"""Context model (kind 2: mean-scale hyperprior with checkerboard context
prediction) on the GPU against the FP64 oracle, through the C ABI.

Layer by layer: psi (h_s's last layer), the hidden entropy-parameter layers,
the means / scale indices / symbols of both passes and the context
convolution, each on the GPU's own upstream values, within FP32 tolerances
(relative 1e-5 of the tensor's largest value) and with symbol / index
mismatches only inside the rounding bands.  Codec level: the oracle's coder
on the GPU's symbols and indices gives the library's bitstream byte for
byte; the library decoder reproduces the encoder's y_hat exactly (its x_hat
equals g_s run on the encoder's y_hat, bit for bit); the FP64 decoder reads
the library's stream.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import boundary_mismatches, chw, dims, index_mismatches, layer_out_shape, make_codec, rel_err

pytestmark = pytest.mark.gpu

N, M = 128, 192
E1, E2 = synth.context_widths(M)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch


def _cb(t, part):
    """Set `part` of a checkerboard-major GPU tensor [1][2][Hy][Wy/2][M] as Hy x Wy/2 x M."""
    return t[0, part].cpu().numpy()


def _take(chw_arr, part):
    return oracle.checkerboard_take(np.transpose(chw_arr, (1, 2, 0)), part)


def _encoder_chain(torch, c, xd, H, W):
    """Every GPU layer of the context model's encoder, run one by one."""
    d = dims(H, W)
    Hy, Wy = d["Hy"], d["Wy"]
    L = {}
    a = torch.empty((1,) + layer_out_shape("GA0", H, W, N, M), device="cuda")
    c.run_layer("GA0", 1, H, W, xd, a)
    b = torch.empty((1,) + layer_out_shape("GA1", H, W, N, M), device="cuda")
    c.run_layer("GA1", 1, H, W, a, b)
    a2 = torch.empty((1,) + layer_out_shape("GA2", H, W, N, M), device="cuda")
    c.run_layer("GA2", 1, H, W, b, a2)
    y = torch.empty((1, Hy, Wy, M), device="cuda")
    c.run_layer("GA3", 1, H, W, a2, y, torch.empty_like(y, dtype=torch.int8))
    h = torch.empty((1, Hy, Wy, N), device="cuda")
    c.run_layer("HA0", 1, H, W, y, h)
    h2 = torch.empty((1, Hy // 2, Wy // 2, N), device="cuda")
    c.run_layer("HA1", 1, H, W, h, h2)
    z = torch.empty((1, d["Hz"], d["Wz"], N), device="cuda")
    sz = torch.empty_like(z, dtype=torch.int8)
    c.run_layer("HA2", 1, H, W, h2, z, sz)
    g = torch.empty((1, Hy // 2, Wy // 2, N), device="cuda")
    c.run_layer("HS0", 1, H, W, sz, g)
    g2 = torch.empty((1, Hy, Wy, N), device="cuda")
    c.run_layer("HS1", 1, H, W, g, g2)
    Z = torch.zeros((1, Hy, Wy, 4 * M), device="cuda")
    c.run_layer("HS2", 1, H, W, g2, Z)
    L.update(y=y, z=z, sym_z=sz, hs1=g2, psi=Z[..., :2 * M].clone())
    e1 = torch.empty((1, Hy, Wy, E1), device="cuda")
    e2 = torch.empty((1, Hy, Wy, E2), device="cuda")
    idx = torch.zeros((1, 2, Hy, Wy // 2, M), device="cuda", dtype=torch.uint8)
    sym = torch.zeros((1, 2, Hy, Wy // 2, M), device="cuda", dtype=torch.int8)
    yq = torch.zeros((1, Hy, Wy, M), device="cuda")
    c.run_layer("EP0A", 1, H, W, Z, e1)
    c.run_layer("EP1A", 1, H, W, e1, e2)
    L.update(e1a=e1.clone(), e2a=e2.clone())
    c.run_layer("EP2A", 1, H, W, e2, idx, sym, in2=y, out2=yq)
    L["yq_a"] = yq.clone()
    c.run_layer("CX", 1, H, W, yq, Z)
    L["ctx"] = Z[..., 2 * M:].clone()
    c.run_layer("EP0N", 1, H, W, Z, e1)
    c.run_layer("EP1N", 1, H, W, e1, e2)
    L.update(e1n=e1.clone(), e2n=e2.clone())
    c.run_layer("EP2N", 1, H, W, e2, idx, sym, in2=y, out2=yq)
    L.update(idx=idx, sym=sym, yhat=yq)
    return L


def _expected_stream(m, S, H, W, L):
    """The bitstream the oracle's coder makes from the GPU's symbols / indices."""
    sz = L["sym_z"][0].cpu().numpy().astype(np.int32)
    ztab = np.broadcast_to(np.arange(N, dtype=np.int32), sz.shape)
    zb = oracle.rans_encode(sz.ravel() + 64, ztab.ravel(), m.freq_fact)
    ys = []
    for part in (0, 1):
        sy = _cb(L["sym"], part).astype(np.int32)
        ix = _cb(L["idx"], part).astype(np.int32)
        Hy = sy.shape[0]
        ys += [oracle.rans_encode(sy[a:b].ravel() + 64, ix[a:b].ravel(), m.freq_gauss) for a, b in m.slice_rows(Hy, S)]
    return oracle.pack_container(2, m.hs_out, S, H, W, N, M, m.model_id, zb, ys)


def _check_pass(m, L, part, psi, ctx, y):
    """Hidden layers, means, indices and symbols of one pass against FP64."""
    A = oracle.checkerboard(*psi.shape[1:])
    sel = A if part == 0 else ~A
    tag = "a" if part == 0 else "n"
    h1 = oracle.relu(oracle.conv1x1(np.concatenate([psi, ctx]), m.P["ep0.w"], m.P["ep0.b"]))
    assert rel_err(chw(L["e1" + tag])[:, sel], h1[:, sel]) < 1e-5
    h2 = oracle.relu(oracle.conv1x1(chw(L["e1" + tag]), m.P["ep1.w"], m.P["ep1.b"]))
    assert rel_err(chw(L["e2" + tag])[:, sel], h2[:, sel]) < 1e-5
    mu, sraw = oracle.entropy_parameters(m.P, psi, ctx)
    # indices (the scale decision) and symbols (the rounding of y - mean)
    ig = np.transpose(_cb(L["idx"], part), (2, 0, 1)).astype(np.int32)
    n_i, ok = index_mismatches(ig, np.transpose(_take(oracle.scales_from_hs(sraw, m.hs_out), part), (2, 0, 1)), m.t)
    assert ok, f"pass {part}: {n_i} index mismatches outside the band"
    sg = np.transpose(_cb(L["sym"], part), (2, 0, 1)).astype(np.int32)
    n_s, ok = boundary_mismatches(sg, np.transpose(_take(y, part), (2, 0, 1)),
                                  np.transpose(_take(mu, part), (2, 0, 1)))
    assert ok, f"pass {part}: {n_s} symbol mismatches outside the band"
    return mu, n_i, n_s


@pytest.mark.parametrize("H,W", [(128, 192), (200, 328)])
def test_context_layers_match_oracle(torch_dev, H, W):
    torch = torch_dev
    c, m = make_codec(2, N, M, max_h=H, max_w=W, y_slices=2, entropy_threads=4, max_in_flight=2)
    xd = torch.from_numpy(synth.frame_sinusoid(H, W, t=3))[None].cuda()
    L = _encoder_chain(torch, c, xd, H, W)
    y = chw(L["y"])
    Hy, Wy = y.shape[1:]
    A = oracle.checkerboard(Hy, Wy)
    # h_a sees y itself (not |y|)
    zref = m.h_a(y)
    assert rel_err(chw(L["z"]), zref) < 1e-4
    # psi: h_s's last layer into the first 2M channels of [psi; ctx]
    psi = chw(L["psi"])
    assert rel_err(psi, oracle.conv2d(chw(L["hs1"]), m.P["hs2.w"], m.P["hs2.b"], 1, 1)) < 1e-5
    # pass 1 (zero context), its y_hat at the anchors
    zero = np.zeros_like(psi)
    mu1, _, _ = _check_pass(m, L, 0, psi, zero, y)
    s1 = np.transpose(_cb(L["sym"], 0), (2, 0, 1)).astype(np.float64)
    yq1 = _take(chw(L["yq_a"]), 0)
    assert np.max(np.abs(yq1 - (np.transpose(s1, (1, 2, 0)) + _take(mu1, 0)))) < 1e-4
    # the context: zero at the anchors, the masked convolution of the GPU's
    # anchor y_hat at the others
    ctx_g = chw(L["ctx"])
    assert np.all(ctx_g[:, A] == 0.0)
    ctx_ref = oracle.context(chw(L["yq_a"]), m.P["cx.w"], m.P["cx.b"])
    assert rel_err(ctx_g[:, ~A], ctx_ref[:, ~A]) < 1e-5
    # pass 2 on the GPU's context
    mu2, _, _ = _check_pass(m, L, 1, psi, ctx_g, y)
    # encoder's y_hat = sym + mean on the full grid
    yh = chw(L["yhat"])
    for part, mu in ((0, mu1), (1, mu2)):
        sp = _cb(L["sym"], part).astype(np.float64)
        assert np.max(np.abs(_take(yh, part) - (sp + _take(mu, part)))) < 1e-4
    # decoder side of the last layer: the means, checkerboard-major
    mu_g = torch.zeros((1, 2, Hy, Wy // 2, M), device="cuda")
    idx2 = torch.zeros_like(L["idx"])
    c.run_layer("EP2A", 1, H, W, L["e2a"], idx2, None, out2=mu_g)
    c.run_layer("EP2N", 1, H, W, L["e2n"], idx2, None, out2=mu_g)
    assert torch.equal(idx2, L["idx"])
    for part, mu in ((0, mu1), (1, mu2)):
        assert rel_err(_cb(mu_g, part), _take(mu, part)) < 1e-5
    c.close()


def _gs_chain(torch, c, H, W, yhat):
    """x_hat from the synthesis layers run one by one on y_hat (float32; the
    bf16 and e4m3 forms take it as bf16), buffers sized by the library."""
    gin = yhat if c.precision == 0 else yhat.to(torch.bfloat16)
    cur = gin
    for L in ("GS0", "GS1", "GS2"):
        nb = c.layer_bytes(L, 1, H, W)[1]
        out = torch.empty(nb, device="cuda", dtype=torch.uint8)
        c.run_layer(L, 1, H, W, cur, out)
        cur = out
    xg = torch.empty((1, 3, H, W), device="cuda")
    c.run_layer("GS3", 1, H, W, cur, xg)
    return xg


@pytest.mark.parametrize("H,W,S,lanes,prec,hs_out", [(128, 192, 2, 0, 0, 1), (200, 328, 3, 8, 0, 1),
                                                     (200, 328, 2, 8, 1, 1), (136, 200, 2, 0, 0, 0),
                                                     (200, 328, 2, 8, 2, 1)])
def test_context_codec(torch_dev, H, W, S, lanes, prec, hs_out):
    torch = torch_dev
    c, m = make_codec(2, N, M, max_h=H, max_w=W, y_slices=S, entropy_threads=4, max_in_flight=3,
                      rans_lanes=lanes, precision=prec, hs_out=hs_out)
    x = synth.frame_sinusoid(H, W, t=7)
    xd = torch.from_numpy(x)[None].cuda()
    bits = c.encode(xd)[0]
    L = _encoder_chain(torch, c, xd, H, W)
    if lanes == 0:
        assert bits == _expected_stream(m, S, H, W, L)
    hdr = oracle.parse_container(bits)
    assert hdr["kind"] == 2 and len(hdr["y"]) == 2 * S and hdr["lanes"] == lanes
    # the library decoder rebuilds the encoder's y_hat exactly: its x_hat is
    # g_s of the encoder's y_hat (run layer by layer), bit for bit
    xh = torch.empty((1, 3, H, W), device="cuda")
    assert c.decode([bits], xh) == (H, W)
    xg = _gs_chain(torch, c, H, W, L["yhat"])
    assert torch.equal(xh, xg)
    # FP64 synthesis of the same y_hat: the FP32 form within 1e-3, the
    # reduced forms above the same fidelity floors as the scale hyperprior's
    xo = np.clip(m.g_s(chw(L["yhat"])), 0, 1)[:, :H, :W]
    if prec == 0:
        assert np.max(np.abs(xh[0].cpu().numpy() - xo)) <= 1e-3
    else:
        assert oracle.psnr(xo, xh[0].cpu().numpy().astype(np.float64)) >= (30.0 if prec == 1 else 20.0)
    # chained encoder + decoder: the same bytes and pixels
    xh2 = torch.empty_like(xh)
    assert c.encode_decode(xd, xh2)[0] == bits
    assert torch.equal(xh, xh2)
    # the FP64 decoder reads the library's stream when it takes the same
    # decisions (no scale index on a table boundary in either pass)
    zg = L["sym_z"][0].cpu().numpy()
    psi64 = m.h_s(np.transpose(zg, (2, 0, 1)).astype(np.float64) + m.medians[:, None, None].astype(np.float64))
    mu1, s1 = oracle.entropy_parameters(m.P, psi64, np.zeros_like(psi64))
    same = np.array_equal(_cb(L["idx"], 0), _take(oracle.scale_index(oracle.scales_from_hs(s1, m.hs_out), m.t), 0))
    if same:
        Hy, Wy = mu1.shape[1:]
        s_a = np.zeros((Hy, Wy, M))
        oracle.checkerboard_put(s_a, 0, _cb(L["sym"], 0).astype(np.float64))
        A = oracle.checkerboard(Hy, Wy)[None]
        ctx64 = oracle.context(np.where(A, np.transpose(s_a, (2, 0, 1)) + mu1, 0.0), m.P["cx.w"], m.P["cx.b"])
        _, s2 = oracle.entropy_parameters(m.P, psi64, ctx64)
        same = np.array_equal(_cb(L["idx"], 1), _take(oracle.scale_index(oracle.scales_from_hs(s2, m.hs_out), m.t), 1))
    if same:
        xr_o, dd = m.decode(bits)
        for part in (0, 1):
            assert np.array_equal(_cb(L["sym"], part), _take(dd["sym_y"], part))
    c.close()


@pytest.mark.parametrize("H,W", [(720, 1280), (1080, 1920)])
def test_context_codec_720p_sampled(torch_dev, H, W):
    """The full-size kernels (their own tile shapes: 720p and 1080p grids
    choose other split-K configurations) against FP64 on the GPU's y: every
    index and symbol of both passes within the bands, and the decoder
    reproduces the encoder's y_hat."""
    torch = torch_dev
    c, m = make_codec(2, N, M, max_h=H, max_w=W, y_slices=8, entropy_threads=8, max_in_flight=2)
    xd = torch.from_numpy(synth.frame_sinusoid(H, W, t=11))[None].cuda()
    L = _encoder_chain(torch, c, xd, H, W)
    y = chw(L["y"])
    psi = chw(L["psi"])
    assert rel_err(psi, oracle.conv2d(chw(L["hs1"]), m.P["hs2.w"], m.P["hs2.b"], 1, 1)) < 1e-5
    _check_pass(m, L, 0, psi, np.zeros_like(psi), y)
    ctx_g = chw(L["ctx"])
    A = oracle.checkerboard(*y.shape[1:])
    ctx_ref = oracle.context(chw(L["yq_a"]), m.P["cx.w"], m.P["cx.b"])
    assert rel_err(ctx_g[:, ~A], ctx_ref[:, ~A]) < 1e-5
    _check_pass(m, L, 1, psi, ctx_g, y)
    bits = c.encode(xd)[0]
    xh = torch.empty((1, 3, H, W), device="cuda")
    assert c.decode([bits], xh) == (H, W)
    # the decoder's y_hat: g_s of the encoder's y_hat gives the same pixels
    a = torch.empty((1,) + layer_out_shape("GS0", H, W, N, M), device="cuda")
    c.run_layer("GS0", 1, H, W, L["yhat"], a)
    b = torch.empty((1,) + layer_out_shape("GS1", H, W, N, M), device="cuda")
    c.run_layer("GS1", 1, H, W, a, b)
    a2 = torch.empty((1,) + layer_out_shape("GS2", H, W, N, M), device="cuda")
    c.run_layer("GS2", 1, H, W, b, a2)
    xg = torch.empty((1, 3, H, W), device="cuda")
    c.run_layer("GS3", 1, H, W, a2, xg)
    assert torch.equal(xh, xg)
    c.close()


def test_context_codec_batches_equal_single_frames(torch_dev):
    """Tasks of two frames (one launch per layer for both) give every frame
    the bits and pixels it gets alone: the per-frame copies of the two
    checkerboard sets and the batched kernels keep frames apart."""
    torch = torch_dev
    H, W = 200, 328
    xs = torch.from_numpy(np.stack([synth.frame_sinusoid(H, W, t=t) for t in (1, 2, 3)])).cuda()
    c1, _ = make_codec(2, N, M, max_h=H, max_w=W, y_slices=2, entropy_threads=4, max_in_flight=2, max_batch=1)
    c2, _ = make_codec(2, N, M, max_h=H, max_w=W, y_slices=2, entropy_threads=4, max_in_flight=2, max_batch=2)
    b1 = c1.encode(xs)
    b2 = c2.encode(xs)
    assert b1 == b2
    x1 = torch.empty_like(xs)
    x2 = torch.empty_like(xs)
    c1.decode(b1, x1)
    c2.decode(b2, x2)
    assert torch.equal(x1, x2)
    x3 = torch.empty_like(xs)
    assert c2.encode_decode(xs, x3) == b1
    assert torch.equal(x3, x1)
    c1.close()
    c2.close()


def test_context_codec_errors_leave_it_usable(torch_dev):
    """Truncated streams, streams of another model and damaged anchor
    payloads are refused (or, where the coder cannot tell, decoded to some
    image) without harm: the next decode gives the right pixels."""
    from paper_2208_01641_amd import LicError
    torch = torch_dev
    H, W = 128, 192
    c, _ = make_codec(2, N, M, max_h=H, max_w=W, y_slices=2, entropy_threads=2, max_in_flight=2)
    xd = torch.from_numpy(synth.frame_sinusoid(H, W, t=2))[None].cuda()
    bits = c.encode(xd)[0]
    good = torch.empty((1, 3, H, W), device="cuda")
    c.decode([bits], good)
    out = torch.empty_like(good)
    with pytest.raises(LicError) as e:
        c.decode([bits[:-3]], out)
    assert e.value.code == -4                        # LIC_E_CORRUPT
    c1, _ = make_codec(1, N, M, max_h=H, max_w=W, y_slices=2, entropy_threads=2)
    with pytest.raises(LicError) as e:
        c.decode([c1.encode(xd)[0]], out)
    assert e.value.code == -8                        # LIC_E_MODEL (another kind)
    c1.close()
    hdr = oracle.parse_container(bits)
    start = len(bits) - sum(len(y) for y in hdr["y"])     # first anchor slice
    bad = bytearray(bits)
    for i in range(start + 8, start + 40):
        bad[i] ^= 0x5A
    try:
        c.decode([bytes(bad)], out)
    except LicError as err:
        assert err.code == -4
    c.decode([bits], out)
    assert torch.equal(out, good)
    c.close()
