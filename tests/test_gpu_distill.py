"""Distilled synthesis network on the GPU against the FP64 oracle.

Forward output, loss and every parameter gradient of the HIP path (FP32
GEMMs) match the oracle's definitions within 1e-4 relative to the largest
magnitude of each tensor; one AdamW step matches the oracle's update applied
to the gradients the step used; repeated calls are bit-identical; a short
training run lowers the loss.  The bf16 forward is compared with the oracle
run on bf16-rounded parameters.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import rel_err

pytestmark = pytest.mark.gpu
M, F = 192, 64


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch


def _sym(rng, n, hy, wy):
    """int8 latent symbols with a heavy-tailed spread like y_hat's."""
    return np.clip(np.rint(rng.laplace(0.0, 2.0, (n, hy, wy, M))), -64, 64).astype(np.int8)


def _params(seed=2209):
    return synth.distill_params(M, F, seed=seed)


def _oracle_in(sym):
    return np.transpose(sym.astype(np.float64), (0, 3, 1, 2))


@pytest.mark.parametrize("n,hy,wy", [(2, 4, 6), (3, 5, 3), (1, 1, 1)])
def test_forward_matches_oracle(torch_dev, n, hy, wy):
    torch = torch_dev
    from paper_2208_01641_amd import Distill
    rng = np.random.default_rng(100 + n * 10 + hy)
    P = _params()
    sym = _sym(rng, n, hy, wy)
    d = Distill(P, M, F, max_batch=4, max_hy=8, max_wy=8, train=False)
    pre = torch.empty((n, 3, 16 * hy, 16 * wy), device="cuda")
    H, W = 16 * hy - 5, 16 * wy - 3
    xh = torch.empty((n, 3, H, W), device="cuda")
    d.forward(torch.from_numpy(sym).cuda(), pre=pre, x_hat=xh)
    ref, _ = oracle.distill_forward(P, _oracle_in(sym))
    got = pre.cpu().numpy()
    assert rel_err(got, ref) <= 1e-4
    # the decoded image is the clamped, cropped output of the same pass
    assert np.array_equal(xh.cpu().numpy(), np.clip(got[:, :, :H, :W], 0.0, 1.0))
    d.close()


def test_bf16_forward_matches_oracle_on_rounded_operands(torch_dev):
    torch = torch_dev
    from paper_2208_01641_amd import Distill
    rng = np.random.default_rng(7)
    n, hy, wy = 2, 4, 5
    P = _params()
    sym = _sym(rng, n, hy, wy)
    d = Distill(P, M, F, precision=1, max_batch=2, max_hy=4, max_wy=5, train=False)
    pre = torch.empty((n, 3, 16 * hy, 16 * wy), device="cuda")
    d.forward(torch.from_numpy(sym).cuda(), pre=pre)
    # bf16 weights, bf16 hidden activations, FP32 accumulation: the error
    # against the FP64 result on bf16-rounded weights stays near 2^-8
    Pb = {k: (torch.from_numpy(v).bfloat16().float().numpy() if k.endswith(".w") else v) for k, v in P.items()}
    ref, _ = oracle.distill_forward(Pb, _oracle_in(sym))
    assert rel_err(pre.cpu().numpy(), ref) <= 2.0 ** -6
    d.close()


@pytest.mark.parametrize("n,hy,wy", [(2, 4, 4), (3, 3, 5)])
def test_gradients_match_oracle(torch_dev, n, hy, wy):
    torch = torch_dev
    from paper_2208_01641_amd import Distill
    from paper_2208_01641_amd.distill import unflatten
    rng = np.random.default_rng(200 + n + hy)
    P = _params()
    sym = _sym(rng, n, hy, wy)
    tgt = rng.uniform(0.0, 1.0, (n, 3, 16 * hy, 16 * wy)).astype(np.float32)
    d = Distill(P, M, F, max_batch=4, max_hy=8, max_wy=8)
    loss, g = d.grads(torch.from_numpy(sym).cuda(), torch.from_numpy(tgt).cuda())
    rloss, rg = oracle.distill_loss_and_grads(P, _oracle_in(sym), tgt)
    assert loss == pytest.approx(rloss, rel=1e-5)
    G = unflatten(g, M, F)
    for k in rg:
        e = rel_err(G[k], rg[k])
        assert e <= 1e-4, (k, e)
    # the same call again gives the same bits (fixed-order reductions)
    loss2, g2 = d.grads(torch.from_numpy(sym).cuda(), torch.from_numpy(tgt).cuda())
    assert loss2 == loss and np.array_equal(g2, g)
    d.close()


def test_adamw_step_matches_oracle_update(torch_dev):
    torch = torch_dev
    from paper_2208_01641_amd import Distill
    rng = np.random.default_rng(31)
    n, hy, wy = 4, 3, 3
    P = _params()
    sym = torch.from_numpy(_sym(rng, 6, hy, wy)).cuda()
    tgt = torch.from_numpy(rng.uniform(0.0, 1.0, (6, 3, 16 * hy, 16 * wy)).astype(np.float32)).cuda()
    d = Distill(P, M, F, max_batch=4, max_hy=3, max_wy=3, lr=1e-3, weight_decay=0.01)
    idx = np.array([5, 0, 3, 1], np.int32)
    # the step's gradients equal a plain gradient call on the gathered batch
    _, g_ref = d.grads(sym[torch.from_numpy(idx).long().cuda()].contiguous(),
                       tgt[torch.from_numpy(idx).long().cuda()].contiguous())
    eps32 = float(np.finfo(np.float32).eps)
    for t in (1, 2):
        # the state the step starts from, as the GPU holds it
        w = d.get(0).astype(np.float64)
        m = d.get(1).astype(np.float64)
        v = d.get(2).astype(np.float64)
        m_prev, v_prev = m.copy(), v.copy()
        loss = torch.zeros(1, device="cuda")
        d.step(sym, tgt, idx, loss_out=loss)
        d.sync()
        g = d.get(3)
        if t == 1:
            assert np.array_equal(g, g_ref)
        oracle.adamw_step(w, m, v, g.astype(np.float64), t, lr=1e-3, wd=0.01)
        assert d.step_count == t
        # FP32 update against the FP64 update of the same state, element by
        # element: each moment is a sum of two FP32 products, so its error is
        # a few ulp of the larger of the two terms (where the terms cancel,
        # only the operands bound the error, not the result)
        g64 = g.astype(np.float64)
        bound_m = 4 * eps32 * np.maximum(np.abs(0.9 * m_prev), np.abs(0.1 * g64))
        bound_v = 4 * eps32 * np.maximum(np.abs(0.999 * v_prev), np.abs(0.001 * g64 * g64))
        dm = np.abs(d.get(1) - m)
        dv = np.abs(d.get(2) - v)
        assert np.all(dm <= bound_m), float(np.max(dm / np.maximum(bound_m, 1e-300)))
        assert np.all(dv <= bound_v), float(np.max(dv / np.maximum(bound_v, 1e-300)))
        np.testing.assert_allclose(d.get(0), w, rtol=0, atol=2e-6)
        assert float(loss.item()) > 0
    d.close()


def test_training_lowers_the_loss(torch_dev):
    """Fit a student to a teacher net of the same shape on 64 latents."""
    torch = torch_dev
    from paper_2208_01641_amd import Distill
    rng = np.random.default_rng(5)
    hy = wy = 2
    sym_np = _sym(rng, 64, hy, wy)
    sym = torch.from_numpy(sym_np).cuda()
    teacher = Distill(_params(seed=1), M, F, max_batch=64, max_hy=hy, max_wy=wy, train=False)
    tgt = torch.empty((64, 3, 16 * hy, 16 * wy), device="cuda")
    teacher.forward(sym, pre=tgt)
    student = Distill(_params(seed=2), M, F, max_batch=16, max_hy=hy, max_wy=wy, lr=1e-3)
    losses = torch.zeros(200, device="cuda")
    order = np.random.default_rng(9)
    for s in range(200):
        student.step(sym, tgt, order.choice(64, 16, replace=False), loss_out=losses[s:s + 1])
    student.sync()
    L = losses.cpu().numpy()
    assert np.all(np.isfinite(L))
    assert L[-20:].mean() < 0.5 * L[:5].mean(), (L[:5], L[-20:])
    teacher.close()
    student.close()


def _frames(torch, H, W, n, stream=3):
    return torch.from_numpy(np.stack([synth.frame_sinusoid(H, W, t=t, stream=stream) for t in range(n)])).cuda()


def _symbols(torch, codec, x):
    """Quantised latents of x through the codec's own encoder layers."""
    n, _, H, W = x.shape
    N, M_ = codec.N, codec.M
    a = torch.empty((n, H // 2, W // 2, N), device="cuda")
    b = torch.empty((n, H // 4, W // 4, N), device="cuda")
    c = torch.empty((n, H // 8, W // 8, N), device="cuda")
    y = torch.empty((n, H // 16, W // 16, M_), device="cuda")
    s = torch.empty((n, H // 16, W // 16, M_), dtype=torch.int8, device="cuda")
    codec.run_layer("GA0", n, H, W, x, a)
    codec.run_layer("GA1", n, H, W, a, b)
    codec.run_layer("GA2", n, H, W, b, c)
    codec.run_layer("GA3", n, H, W, c, y, s)
    return s


@pytest.mark.parametrize("precision", [0, 1])
def test_codec_decodes_with_the_distilled_gs(torch_dev, precision):
    """gs_mode 1: every decoded frame is the distilled net's output for the
    frame's symbols (same kernels, same bits)."""
    torch = torch_dev
    from gpu_util import make_codec
    from paper_2208_01641_amd import Distill
    H, W = 128, 192
    Pd = _params()
    c, _ = make_codec(1, 128, M, max_h=H, max_w=W, y_slices=2, entropy_threads=4, max_in_flight=2,
                      gs_mode=1, precision=precision)
    c.load_distilled(Pd)
    x = _frames(torch, H, W, 3)
    out = torch.empty_like(x)
    c.encode_decode(x, out)
    torch.cuda.synchronize()
    ref = torch.empty_like(x)
    d = Distill(Pd, M, F, precision=precision, max_batch=3, max_hy=H // 16, max_wy=W // 16, train=False)
    d.forward(_symbols(torch, c, x), x_hat=ref)
    assert torch.equal(out, ref)
    d.close()
    c.close()


def test_sampled_judge_keeps_or_falls_back(torch_dev):
    """gs_mode 2: with a threshold no frame can miss, the judge runs and the
    distilled output stays; with one no frame can meet, the codec falls back
    and the judged frames equal the full g_s decode."""
    torch = torch_dev
    from gpu_util import make_codec
    H, W = 128, 128
    x = _frames(torch, H, W, 4, stream=5)
    full, _ = make_codec(1, 128, M, max_h=H, max_w=W, y_slices=1, entropy_threads=2, max_in_flight=2)
    ref_full = torch.empty_like(x)
    full.encode_decode(x, ref_full)
    kept, _ = make_codec(1, 128, M, max_h=H, max_w=W, y_slices=1, entropy_threads=2, max_in_flight=2, gs_mode=2)
    kept.load_distilled(_params(), judge_psnr_db=-1e9, judge_every=2)
    o1 = torch.empty_like(x)
    kept.encode_decode(x, o1)
    st = kept.stats()
    assert st["gs_judged"] == 2 and st["gs_fallback"] == 0
    assert not torch.equal(o1, ref_full)
    fb, _ = make_codec(1, 128, M, max_h=H, max_w=W, y_slices=1, entropy_threads=2, max_in_flight=2, gs_mode=2)
    fb.load_distilled(_params(), judge_psnr_db=1e9, judge_every=2)
    o2 = torch.empty_like(x)
    fb.encode_decode(x, o2)
    st = fb.stats()
    assert st["gs_fallback"] == 1 and st["gs_judged"] == 1
    assert torch.equal(o2, ref_full)
    for c in (full, kept, fb):
        c.close()


def test_serving_decodes_with_the_distilled_gs_in_graphs(torch_dev):
    """Serving path (captured graphs, batches of up to 2): each decoded frame
    equals the distilled net's output for its symbols; judged tasks (every
    2nd frame here) run eagerly and keep the distilled output."""
    torch = torch_dev
    from gpu_util import make_codec
    from paper_2208_01641_amd import Distill
    H, W = 128, 192
    Pd = _params()
    c, _ = make_codec(1, 128, M, max_h=H, max_w=W, y_slices=2, entropy_threads=4, max_in_flight=3, max_batch=2,
                      use_graphs=1, gs_mode=2)
    c.load_distilled(Pd, judge_psnr_db=-1e9, judge_every=2)
    x = _frames(torch, H, W, 6, stream=8)
    bits = c.encode(x)
    sid = c.open_stream(H, W)
    for rep in range(2):                         # second round replays the graphs
        outs, tick, keep = {}, {}, []
        for i, b in enumerate(bits):
            outs[i] = torch.empty((3, H, W), device="cuda")
            keep.append(np.frombuffer(b, np.uint8).copy())      # alive until polled
            tick[c.submit_decode(sid, keep[-1], outs[i])] = i
        got = []
        import time
        t0 = time.time()
        while len(got) < len(tick):
            got += c.poll(64, 20000)
            assert time.time() - t0 < 60
        assert all(r["status"] == 0 for r in got)
        torch.cuda.synchronize()
        ref = torch.empty_like(x)
        d = Distill(Pd, M, F, max_batch=6, max_hy=H // 16, max_wy=W // 16, train=False)
        d.forward(_symbols(torch, c, x), x_hat=ref)
        d.close()
        for i in range(len(bits)):
            assert torch.equal(outs[i], ref[i]), (rep, i)
    st = c.stats()
    assert st["gs_judged"] >= 2 and st["gs_fallback"] == 0
    c.close_stream(sid)
    c.close()


def _serve_decode(torch, c, sid, bits, H, W):
    """All bitstreams through submit_decode / poll; returns the images in order."""
    import time
    outs, tick, keep = {}, {}, []
    for i, b in enumerate(bits):
        outs[i] = torch.empty((3, H, W), device="cuda")
        keep.append(np.frombuffer(b, np.uint8).copy())      # alive until polled
        tick[c.submit_decode(sid, keep[-1], outs[i])] = i
    got = []
    t0 = time.time()
    while len(got) < len(tick):
        got += c.poll(64, 20000)
        assert time.time() - t0 < 60
    assert all(r["status"] == 0 for r in got)
    torch.cuda.synchronize()
    return [outs[i] for i in range(len(bits))]


def test_serving_fallback_stops_replaying_distilled_graphs(torch_dev):
    """gs_mode 2 with a threshold no frame can meet, graphs on: once the judge
    has switched to the full g_s, later rounds (which would replay graphs
    captured with the distilled net if the graph cache ignored the switch)
    decode exactly like a codec with the full g_s."""
    torch = torch_dev
    from gpu_util import make_codec
    H, W = 128, 192
    x = _frames(torch, H, W, 6, stream=9)
    full, _ = make_codec(1, 128, M, max_h=H, max_w=W, y_slices=2, entropy_threads=4, max_in_flight=2)
    bits = full.encode(x)
    ref = torch.empty_like(x)
    full.decode(bits, ref)
    c, _ = make_codec(1, 128, M, max_h=H, max_w=W, y_slices=2, entropy_threads=4, max_in_flight=3, max_batch=2,
                      use_graphs=1, gs_mode=2)
    c.load_distilled(_params(), judge_psnr_db=1e9, judge_every=4)
    sid = c.open_stream(H, W)
    rounds = [_serve_decode(torch, c, sid, bits, H, W) for _ in range(3)]
    st = c.stats()
    assert st["gs_fallback"] == 1
    for rep in (1, 2):
        for i in range(len(bits)):
            assert torch.equal(rounds[rep][i], ref[i]), (rep, i)
    c.close_stream(sid)
    c.close()
    full.close()


def test_serving_reload_of_the_distilled_net_drops_its_graphs(torch_dev):
    """Loading a second distilled net into a serving codec with graphs: the
    next rounds decode with the new net (no graph of the first net, whose
    device buffers were freed, is replayed)."""
    torch = torch_dev
    from gpu_util import make_codec
    from paper_2208_01641_amd import Distill
    H, W = 128, 192
    x = _frames(torch, H, W, 4, stream=10)
    c, _ = make_codec(1, 128, M, max_h=H, max_w=W, y_slices=2, entropy_threads=4, max_in_flight=3, max_batch=2,
                      use_graphs=1, gs_mode=1)
    bits = c.encode(x)
    sid = c.open_stream(H, W)
    sym = _symbols(torch, c, x)
    for seed in (2209, 77):
        P = _params(seed)
        c.load_distilled(P)
        ref = torch.empty_like(x)
        d = Distill(P, M, F, max_batch=4, max_hy=H // 16, max_wy=W // 16, train=False)
        d.forward(sym, x_hat=ref)
        d.close()
        for rep in range(2):
            got = _serve_decode(torch, c, sid, bits, H, W)
            for i in range(len(bits)):
                assert torch.equal(got[i], ref[i]), (seed, rep, i)
    c.close_stream(sid)
    c.close()


def test_trained_net_gains_decode_speed_at_a_bounded_fidelity_cost(torch_dev):
    """What the distilled net gains over the method without it: the same
    bitstreams decode faster (g_s is the decoder's largest GPU stage and the
    net has about a twelfth of its FLOPs), and training on the full decoder's
    own (y_hat, x_hat) pairs is what makes its output usable — fidelity to
    the full g_s far above the untrained net's, and within 1 dB of the full
    g_s's PSNR against the source."""
    torch = torch_dev
    import time

    from gpu_util import make_codec
    from paper_2208_01641_amd import Distill
    from paper_2208_01641_amd import distill_train as dtr
    H = W = 128
    count, hold = 640, 64
    teacher, _ = make_codec(1, 128, M, max_h=H, max_w=W, y_slices=1, entropy_threads=2, max_in_flight=1)
    imgs = torch.from_numpy(np.stack([synth.frame_sinusoid(H, W, t=0, stream=10 ** 6 + i)
                                      for i in range(count)])).cuda()
    sym, rec = dtr.build_pairs(teacher, imgs)
    teacher.close()
    net = Distill(_params(seed=3), M, F, max_batch=32, max_hy=H // 16, max_wy=W // 16)
    fid0, _ = dtr.evaluate(net, sym[-hold:], rec[-hold:], imgs[-hold:])
    losses = dtr.train(net, sym[:-hold], rec[:-hold], steps=800, batch=32, seed=4)
    fid1, gap1 = dtr.evaluate(net, sym[-hold:], rec[-hold:], imgs[-hold:])
    print(f"held-out fidelity to the full g_s: untrained {fid0.mean():.2f} dB, trained {fid1.mean():.2f} dB; "
          f"gap against the source {gap1.mean():+.3f} dB; loss {losses[:10].mean():.4f} -> {losses[-50:].mean():.4f}")
    assert losses[-50:].mean() < 0.5 * losses[:10].mean()
    assert fid1.mean() > fid0.mean() + 5.0
    assert abs(gap1.mean()) < 1.0
    params = net.get(0)
    net.close()
    # 720p decode of the same bitstreams with the full and the distilled g_s:
    # the busy time of the decoder's g_s stage and the wall time
    Hd, Wd, n = 720, 1280, 96
    frames = synth.frames_sinusoid_torch(Hd, Wd, range(n), device="cuda")
    times, busy, outs = {}, {}, {}
    bits = None
    for mode in (0, 1):
        c, _ = make_codec(1, 128, M, max_h=Hd, max_w=Wd, y_slices=8, entropy_threads=16, max_in_flight=6,
                          gs_mode=mode)
        if mode:
            c.load_distilled(params, judge_psnr_db=0.0, judge_every=1000)
        bits = bits or c.encode(frames)
        xr = torch.empty_like(frames)
        c.decode(bits[:6], xr[:6])                      # warm-up
        torch.cuda.synchronize()
        b0 = c.stats()["gpu_busy_s"][2]
        t0 = time.perf_counter()
        c.decode(bits, xr)
        torch.cuda.synchronize()
        times[mode] = time.perf_counter() - t0
        busy[mode] = c.stats()["gpu_busy_s"][2] - b0
        outs[mode] = xr
        c.close()
    fid = 10 * np.log10(1.0 / float(torch.mean((outs[0] - outs[1]) ** 2)))
    print(f"720p decode of {n} frames: full g_s {1e3 * times[0]:.1f} ms (g_s stage busy {1e3 * busy[0]:.1f} ms), "
          f"distilled {1e3 * times[1]:.1f} ms ({1e3 * busy[1]:.1f} ms); PSNR(full, distilled) {fid:.2f} dB")
    # the g_s stage's GPU work shrinks severalfold; the wall time less, since
    # the other stages (entropy decoding on the host, h_s) remain
    assert busy[1] < 0.5 * busy[0]
    assert times[1] < 0.9 * times[0]
    assert fid > fid0.mean() + 5.0
