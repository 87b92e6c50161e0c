"""Whole-codec parity through the C ABI (pipelined encode / decode).

Stage-wise, as the mismatch-propagation reading requires: the GPU's own
symbols and scale indices feed the oracle's entropy coder, whose bytes must
equal the library's bitstream exactly; the GPU decoder's reconstruction must
match the oracle's synthesis transform on the identical y_hat within 1e-3;
the GPU latents must match the FP64 analysis transform within 1e-4 (relative)
with symbol mismatches only inside the 1e-3 rounding band.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import boundary_mismatches, chw, index_mismatches, layer_out_shape, make_codec, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch


def _gpu_latents(torch, c, xd, H, W, N, M, hyper):
    """Runs the analysis (and hyper) transforms layer by layer on the GPU."""
    a = torch.empty((1,) + layer_out_shape("GA0", H, W, N, M), device="cuda")
    c.run_layer("GA0", 1, H, W, xd, a)
    b = torch.empty((1,) + layer_out_shape("GA1", H, W, N, M), device="cuda")
    c.run_layer("GA1", 1, H, W, a, b)
    a2 = torch.empty((1,) + layer_out_shape("GA2", H, W, N, M), device="cuda")
    c.run_layer("GA2", 1, H, W, b, a2)
    y = torch.empty((1,) + layer_out_shape("GA3", H, W, N, M), device="cuda")
    sy = torch.empty_like(y, dtype=torch.int8)
    c.run_layer("GA3", 1, H, W, a2, y, sy)
    out = {"y": y, "sym_y": sy}
    if hyper:
        h = torch.empty((1,) + layer_out_shape("HA0", H, W, N, M), device="cuda")
        c.run_layer("HA0", 1, H, W, y, h)
        h2 = torch.empty((1,) + layer_out_shape("HA1", H, W, N, M), device="cuda")
        c.run_layer("HA1", 1, H, W, h, h2)
        z = torch.empty((1,) + layer_out_shape("HA2", H, W, N, M), device="cuda")
        sz = torch.empty_like(z, dtype=torch.int8)
        c.run_layer("HA2", 1, H, W, h2, z, sz)
        g = torch.empty((1,) + layer_out_shape("HS0", H, W, N, M), device="cuda")
        c.run_layer("HS0", 1, H, W, sz, g)
        g2 = torch.empty((1,) + layer_out_shape("HS1", H, W, N, M), device="cuda")
        c.run_layer("HS1", 1, H, W, g, g2)
        idx = torch.empty((1,) + layer_out_shape("HS2", H, W, N, M), device="cuda", dtype=torch.uint8)
        v = torch.empty((1,) + layer_out_shape("HS2", H, W, N, M), device="cuda")
        c.run_layer("HS2", 1, H, W, g2, idx, v)
        out.update({"z": z, "sym_z": sz, "idx": idx, "v": v})
    return out


def _expected_stream(m, S, H, W, lat):
    """The bitstream the oracle's coder makes from the GPU's symbols/indices."""
    sy = lat["sym_y"][0].cpu().numpy().astype(np.int32)       # Hy x Wy x M
    Hy, Wy, M = sy.shape
    rows = m.slice_rows(Hy, S)
    if m.kind == 0:
        tab = np.broadcast_to(np.arange(M, dtype=np.int32), sy.shape)
        ys = [oracle.rans_encode(sy[a:b].ravel() + 64, tab[a:b].ravel(), m.freq_fact) for a, b in rows]
        return oracle.pack_container(0, m.hs_out, S, H, W, m.N, m.M, m.model_id, None, ys)
    sz = lat["sym_z"][0].cpu().numpy().astype(np.int32)
    ztab = np.broadcast_to(np.arange(m.N, dtype=np.int32), sz.shape)
    zb = oracle.rans_encode(sz.ravel() + 64, ztab.ravel(), m.freq_fact)
    idx = lat["idx"][0].cpu().numpy().astype(np.int32)
    ys = [oracle.rans_encode(sy[a:b].ravel() + 64, idx[a:b].ravel(), m.freq_gauss) for a, b in rows]
    return oracle.pack_container(1, m.hs_out, S, H, W, m.N, m.M, m.model_id, zb, ys)


def test_factorized_codec_cfg1(torch_dev):
    torch = torch_dev
    H = W = 128
    c, m = make_codec(0, 128, 192, max_h=H, max_w=W, y_slices=3, entropy_threads=4)
    x = synth.image_1f(H, W)
    xd = torch.from_numpy(x)[None].cuda()
    bits = c.encode(xd)[0]
    lat = _gpu_latents(torch, c, xd, H, W, 128, 192, False)
    assert bits == _expected_stream(m, 3, H, W, lat)
    # FP64 analysis transform: latents and symbols
    yref = m.g_a(oracle.pad64(x))
    assert rel_err(chw(lat["y"]), yref) < 1e-4
    n, ok = boundary_mismatches(np.transpose(lat["sym_y"][0].cpu().numpy(), (2, 0, 1)).astype(np.int32),
                                yref, m.medians[:, None, None].astype(np.float64))
    assert ok, f"{n} mismatches outside the rounding band"
    # the oracle decodes the library's stream to the GPU's y_hat; g_s agrees
    xr_o, d = m.decode(bits)
    sy = np.transpose(lat["sym_y"][0].cpu().numpy(), (2, 0, 1)).astype(np.float64)
    assert np.array_equal(d["yhat"], sy + m.medians[:, None, None].astype(np.float64))
    xh = torch.empty((1, 3, H, W), device="cuda")
    assert c.decode([bits], xh) == (H, W)
    assert np.max(np.abs(xh[0].cpu().numpy() - xr_o)) <= 1e-3
    c.close()


@pytest.mark.parametrize("H,W,S", [(256, 256, 4), (200, 328, 3)])
def test_hyperprior_codec(torch_dev, H, W, S):
    torch = torch_dev
    c, m = make_codec(1, 128, 192, max_h=H, max_w=W, y_slices=S, entropy_threads=4, max_in_flight=3)
    x = synth.frame_sinusoid(H, W, t=5)
    xd = torch.from_numpy(x)[None].cuda()
    bits = c.encode(xd)[0]
    lat = _gpu_latents(torch, c, xd, H, W, 128, 192, True)
    assert bits == _expected_stream(m, S, H, W, lat)

    # FP64 transforms on the GPU's upstream values
    yref = m.g_a(oracle.pad64(x))
    assert rel_err(chw(lat["y"]), yref) < 1e-4
    zref = m.h_a(chw(lat["y"]))
    assert rel_err(chw(lat["z"]), zref) < 1e-4
    szg = np.transpose(lat["sym_z"][0].cpu().numpy(), (2, 0, 1)).astype(np.int32)
    n, ok = boundary_mismatches(szg, zref, m.medians[:, None, None].astype(np.float64))
    assert ok
    vref = m.h_s(szg + m.medians[:, None, None].astype(np.float64))
    assert rel_err(chw(lat["v"]), vref) < 1e-4
    ig = np.transpose(lat["idx"][0].cpu().numpy(), (2, 0, 1)).astype(np.int32)
    n_idx, ok = index_mismatches(ig, oracle.scales_from_hs(vref, 1), m.t)
    assert ok

    # decode on the GPU: equals the synthesis layers on the encoder's symbols
    xh = torch.empty((1, 3, H, W), device="cuda")
    assert c.decode([bits], xh) == (H, W)
    sy = np.transpose(lat["sym_y"][0].cpu().numpy(), (2, 0, 1)).astype(np.float64)
    xo = np.clip(m.g_s(sy), 0, 1)[:, :H, :W]
    assert np.max(np.abs(xh[0].cpu().numpy() - xo)) <= 1e-3
    if n_idx == 0:
        xr_o, d = m.decode(bits)      # FP64 decoder reads the library stream
        assert np.array_equal(d["yhat"], sy)
    # chained encoder + decoder gives the same bytes and pixels
    xh2 = torch.empty_like(xh)
    bits2 = c.encode_decode(xd, xh2)[0]
    assert bits2 == bits
    assert torch.equal(xh, xh2)
    c.close()


def test_pipeline_many_frames_in_order(torch_dev):
    """Frames pipelined through every stage come back in order and equal
    the frame-by-frame results."""
    torch = torch_dev
    H, W = 192, 256
    c, m = make_codec(1, 128, 192, max_h=H, max_w=W, y_slices=2, entropy_threads=6, max_in_flight=4)
    xs = torch.from_numpy(np.stack([synth.frame_sinusoid(H, W, t=t) for t in range(10)])).cuda()
    bits = c.encode(xs)
    assert len(bits) == 10
    for i in (0, 4, 9):
        assert c.encode(xs[i:i + 1].contiguous())[0] == bits[i]
    out = torch.empty((10, 3, H, W), device="cuda")
    c.decode(bits, out)
    out2 = torch.empty_like(out)
    bits2 = c.encode_decode(xs, out2)
    assert bits2 == bits and torch.equal(out, out2)
    lat = c.latencies_ms()                   # of the last call: 10 chained frames
    assert lat.shape == (10,) and np.all(lat > 0)
    st = c.stats()
    assert st["frames"] == 10 and st["fps"] > 0
    one = torch.empty((1, 3, H, W), device="cuda")
    c.decode([bits[7]], one)
    assert torch.equal(one[0], out[7])
    assert c.latencies_ms().shape == (1,)
    c.close()


def test_batched_tasks_equal_per_frame(torch_dev):
    """Frames coded in tasks of 3 (one launch per layer for 3 frames) give
    the same bytes and pixels as frame-by-frame tasks."""
    torch = torch_dev
    H, W = 136, 264
    c1, _ = make_codec(1, 128, 192, max_h=H, max_w=W, y_slices=3, entropy_threads=4, max_in_flight=3)
    c3, _ = make_codec(1, 128, 192, max_h=H, max_w=W, y_slices=3, entropy_threads=4, max_in_flight=2, max_batch=3)
    xs = torch.from_numpy(np.stack([synth.frame_sinusoid(H, W, t=t) for t in range(7)])).cuda()
    b1 = c1.encode(xs)
    b3 = c3.encode(xs)
    assert b1 == b3
    o1 = torch.empty((7, 3, H, W), device="cuda")
    o3 = torch.empty_like(o1)
    c1.decode(b1, o1)
    c3.decode(b3, o3)
    assert torch.equal(o1, o3)
    o4 = torch.empty_like(o1)
    assert c3.encode_decode(xs, o4) == b1 and torch.equal(o4, o1)
    c1.close()
    c3.close()


def test_host_buffers_and_errors(torch_dev):
    from paper_2208_01641_amd import LicError
    torch = torch_dev
    H, W = 64, 64
    c, m = make_codec(1, 128, 192, max_h=H, max_w=W, y_slices=1, entropy_threads=2)
    x = synth.frame_sinusoid(H, W)
    b_host = c.encode(x[None].copy())[0]
    b_dev = c.encode(torch.from_numpy(x)[None].cuda())[0]
    assert b_host == b_dev
    xh = np.zeros((1, 3, H, W), np.float32)
    c.decode([b_host], xh)
    xd = torch.empty((1, 3, H, W), device="cuda")
    c.decode([b_dev], xd)
    assert np.array_equal(xh, xd.cpu().numpy())
    with pytest.raises(LicError) as e:
        c.decode([b_host[:-5]], xh)
    assert e.value.code == -4                    # LIC_E_CORRUPT
    bad = bytearray(b_host)
    bad[16] ^= 1                                 # model id
    with pytest.raises(LicError) as e:
        c.decode([bytes(bad)], xh)
    assert e.value.code == -8                    # LIC_E_MODEL
    with pytest.raises(LicError) as e:
        c.encode(np.zeros((1, 3, 128, 64), np.float32))
    assert e.value.code == -6                    # larger than max_h x max_w
    c.close()
