"""Serving: continuous batching of mixed-size streams (C ABI submit / poll).

Each request's bitstream and reconstruction must be bit-identical to the
same frame coded alone through the synchronous path (eager launches, batch
1), whatever it was batched with and however many times the captured graphs
were replayed.  Admission by the device-memory budget refuses a stream that
does not fit, and serving allocates no device memory after warm-up.
"""
import time

import numpy as np
import pytest

import synth
from gpu_util import make_codec

pytestmark = pytest.mark.gpu

SIZES = [(128, 192), (192, 256), (128, 192)]     # stream 0 and 2 share a bucket


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch


def _drain(c, n, timeout_s=60.0):
    res = []
    t0 = time.time()
    while len(res) < n:
        res += c.poll(256, 20000)
        assert time.time() - t0 < timeout_s, "serving results did not arrive"
    return res


@pytest.mark.parametrize("use_graphs", [1, 0])
def test_mixed_streams_equal_alone(torch_dev, use_graphs):
    torch = torch_dev
    alone, _ = make_codec(1, 128, 192, max_h=192, max_w=256, y_slices=2, entropy_threads=4, max_in_flight=2)
    srv, _ = make_codec(1, 128, 192, max_h=192, max_w=256, y_slices=2, entropy_threads=6, max_in_flight=3,
                        max_batch=3, use_graphs=use_graphs)
    frames = {s: [torch.from_numpy(synth.frame_sinusoid(H, W, t=t, stream=s)).cuda() for t in range(5)]
              for s, (H, W) in enumerate(SIZES)}
    # references: each frame alone, synchronous path
    ref_bits, ref_img = {}, {}
    for s, (H, W) in enumerate(SIZES):
        for t, x in enumerate(frames[s]):
            b = alone.encode(x[None])[0]
            o = torch.empty((1, 3, H, W), device="cuda")
            alone.decode([b], o)
            ref_bits[(s, t)], ref_img[(s, t)] = b, o[0]
    sids = [srv.open_stream(H, W) for H, W in SIZES]
    allocs = None
    for rep in range(3):                       # graphs are replayed on later rounds
        outs, tick = {}, {}
        for t in range(5):                     # interleave the streams
            for s, sid in enumerate(sids):
                buf = np.zeros(srv.max_stream_bytes(*SIZES[s]), np.uint8)
                outs[(s, t)] = buf
                tick[srv.submit_encode(sid, frames[s][t], buf)] = (s, t)
        res = _drain(srv, len(tick))
        bits = {}
        for r in res:
            assert r["status"] == 0 and r["direction"] == 0
            key = tick[r["ticket"]]
            bits[key] = outs[key][:r["bytes"]].tobytes()
            assert bits[key] == ref_bits[key], f"encode {key} differs from the frame coded alone"
        # decode them back, mixed
        imgs, dtick, keep = {}, {}, []
        for key, b in bits.items():
            s, t = key
            H, W = SIZES[s]
            arr = np.frombuffer(b, np.uint8).copy()
            keep.append(arr)
            imgs[key] = torch.empty((3, H, W), device="cuda")
            dtick[srv.submit_decode(sids[s], arr, imgs[key])] = key
        for r in _drain(srv, len(dtick)):
            assert r["status"] == 0 and r["direction"] == 1
            key = dtick[r["ticket"]]
            assert torch.equal(imgs[key], ref_img[key]), f"decode {key} differs from the frame decoded alone"
        torch.cuda.synchronize()
        st = srv.stats()
        if allocs is None:
            allocs = st["alloc_events"]
        assert st["alloc_events"] == allocs, "device memory allocated on the serving path"
    for sid in sids:
        srv.close_stream(sid)
    srv.close()
    alone.close()


def test_admission_by_budget(torch_dev):
    from paper_2208_01641_amd import LicError
    c, _ = make_codec(1, 128, 192, max_h=256, max_w=256, y_slices=1, entropy_threads=2, max_in_flight=1)
    base = c.stats()["device_bytes"]
    c.close()
    one = 4 * (6 * 256 * 256 + 128 * 128 * 128 + 128 * 64 * 64)     # one 256x256 stream's reservation
    c, _ = make_codec(1, 128, 192, max_h=256, max_w=256, y_slices=1, entropy_threads=2, max_in_flight=1,
                      hbm_budget_bytes=base + 2 * one + one // 2)
    a = c.open_stream(256, 256)
    b = c.open_stream(256, 256)
    with pytest.raises(LicError) as e:
        c.open_stream(256, 256)
    assert e.value.code == -6                     # LIC_E_BUDGET
    c.close_stream(a)
    c.open_stream(256, 256)                       # fits again once a stream closed
    with pytest.raises(LicError):
        c.open_stream(512, 256)                   # larger than max_h x max_w
    c.close()


@pytest.mark.timeout(180)
def test_slot_reuse_with_varying_batches_drains_and_closes(torch_dev):
    """Many requests over three frame sizes through two pool slots, batches
    of 1..4: every result arrives once, the pending count returns to zero and
    close() returns (a finished task's slot is reused by the batcher only
    after the task's bookkeeping is done)."""
    torch = torch_dev
    sizes = [(128, 128), (128, 192), (192, 256)]
    c, _ = make_codec(1, 128, 192, max_h=192, max_w=256, y_slices=1, entropy_threads=4, max_in_flight=2,
                      max_batch=4, use_graphs=1)
    sids = [c.open_stream(H, W) for H, W in sizes]
    frames = {s: torch.from_numpy(synth.frame_sinusoid(H, W, t=0, stream=20 + s)).cuda() for s, (H, W) in
              enumerate(sizes)}
    rng = np.random.default_rng(3)
    order = rng.integers(0, 3, 120)
    outs, tick = {}, {}
    for i, s in enumerate(order):
        outs[i] = np.zeros(c.max_stream_bytes(*sizes[s]), np.uint8)
        tick[c.submit_encode(sids[s], frames[int(s)], outs[i])] = i
    res = _drain(c, len(tick), timeout_s=120.0)
    assert sorted(tick[r["ticket"]] for r in res) == list(range(len(order)))
    assert all(r["status"] == 0 for r in res)
    bits = {tick[r["ticket"]]: outs[tick[r["ticket"]]][:r["bytes"]].copy() for r in res}
    imgs, dtick = {}, {}
    for i, s in enumerate(order):
        H, W = sizes[s]
        imgs[i] = torch.empty((3, H, W), device="cuda")
        dtick[c.submit_decode(sids[s], bits[i], imgs[i])] = i
    res = _drain(c, len(dtick), timeout_s=120.0)
    assert sorted(dtick[r["ticket"]] for r in res) == list(range(len(order)))
    assert all(r["status"] == 0 for r in res)
    c.close()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("precision", [1, 0])
def test_mixed_resolutions_at_serving_sizes_equal_alone(torch_dev, precision):
    """The serving mix at its real frame sizes (360p, 720p and 1080p streams
    in the ratio 2:1:1; whole-frame kernels, batches of up to 4, captured
    graphs): every bitstream and reconstruction equals the frame coded alone
    (eager, batch 1), on the first round and on a round that replays the
    graphs."""
    torch = torch_dev
    sizes = [(360, 640), (360, 640), (720, 1280), (1080, 1920)]
    alone, _ = make_codec(1, 128, 192, precision=precision, max_h=1080, max_w=1920, y_slices=4, entropy_threads=8,
                          max_in_flight=2)
    srv, _ = make_codec(1, 128, 192, precision=precision, max_h=1080, max_w=1920, y_slices=4, entropy_threads=8,
                        max_in_flight=4, max_batch=4, use_graphs=1)
    nf = 3
    frames = {s: [torch.from_numpy(synth.frame_sinusoid(H, W, t=t, stream=30 + s)).cuda() for t in range(nf)]
              for s, (H, W) in enumerate(sizes)}
    ref_bits, ref_img = {}, {}
    for s, (H, W) in enumerate(sizes):
        for t, x in enumerate(frames[s]):
            b = alone.encode(x[None])[0]
            o = torch.empty((1, 3, H, W), device="cuda")
            alone.decode([b], o)
            ref_bits[(s, t)], ref_img[(s, t)] = b, o[0]
    sids = [srv.open_stream(H, W) for H, W in sizes]
    for rep in range(2):
        outs, tick = {}, {}
        for t in range(nf):
            for s, sid in enumerate(sids):
                buf = np.zeros(srv.max_stream_bytes(*sizes[s]), np.uint8)
                outs[(s, t)] = buf
                tick[srv.submit_encode(sid, frames[s][t], buf)] = (s, t)
        bits = {}
        for r in _drain(srv, len(tick), timeout_s=120.0):
            assert r["status"] == 0 and r["direction"] == 0
            key = tick[r["ticket"]]
            bits[key] = outs[key][:r["bytes"]].tobytes()
            assert bits[key] == ref_bits[key], f"encode {key} differs from the frame coded alone (round {rep})"
        imgs, dtick, keep = {}, {}, []
        for key, b in bits.items():
            s, t = key
            H, W = sizes[s]
            keep.append(np.frombuffer(b, np.uint8).copy())
            imgs[key] = torch.empty((3, H, W), device="cuda")
            dtick[srv.submit_decode(sids[s], keep[-1], imgs[key])] = key
        for r in _drain(srv, len(dtick), timeout_s=120.0):
            assert r["status"] == 0 and r["direction"] == 1
            key = dtick[r["ticket"]]
            assert torch.equal(imgs[key], ref_img[key]), f"decode {key} differs from the frame alone (round {rep})"
    for sid in sids:
        srv.close_stream(sid)
    srv.close()
    alone.close()
