#!/usr/bin/env python3
"""720p scale-hyperprior encode+decode throughput and latency on one MI355X.

One step = one 3x720x1280 frame through the whole hot path: the GPU analysis
transform with GDN, quantisation of y, h_a, quantisation of z, h_s and the
scale-table index (encoder GPU stage), CPU rANS encoding into the bitstream,
then the 4-stage decoder (CPU rANS of z, GPU h_s + index, CPU rANS of y,
GPU synthesis transform with IGDN) back to a reconstructed frame.  Frames
are pipelined through the library's runtime (encoder chained into decoder
per frame); the input frames are resident in device memory before timing.

The headline line is the FP32 form at N=128, M=192.  Unless --no-variants
is given, the same JSON line also carries the comparison runs ("variants"):
the unpipelined per-frame form (one frame in flight), the BF16 and e4m3 forms at
720p, and the FP32 / BF16 / e4m3 forms of the 1080p N=192 M=320 batch-4 workload,
each with frames/s, p50/p99 latency, PSNR and bits per pixel, and the
serving loop (16 mixed-resolution streams, Poisson arrivals, BF16).

Prints one JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "720p hyperprior enc+dec frames/s + p99 ms; BF16/FP8 vs FP32 at fixed PSNR"
# MI355X dense matrix peaks per operand form of a kernel's GEMM; the
# split-FP32 form issues six bf16 products per FP32 product, so its ceiling
# in FP32 FLOP/s is the bf16 peak / 6
PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0, "fp8": 5000.0, "f32x": 2500.0 / 6}
PEAK_BASIS = {"f32": "FP32 matrix cores", "bf16": "bf16 matrix cores", "fp8": "fp8 matrix cores",
              "f32x": "bf16 matrix cores / 6 (six bf16 products per FP32 product)"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2208_01641_amd", "csrc", "conv_kernels.hip")
LAYERS = ("GA0", "GA1", "GA2", "GA3", "HA0", "HA1", "HA2", "HS0", "HS1", "HS2", "GS0", "GS1", "GS2", "GS3")
# the context model's layers beyond those (context convolution, entropy
# parameters of the anchor pass and of the second pass)
CTX_LAYERS = ("CX", "EP0A", "EP1A", "EP2A", "EP0N", "EP1N", "EP2N")
CODEC_NAME = {0: "factorized-prior", 1: "scale-hyperprior", 2: "context-model (checkerboard) mean-scale hyperprior"}


def layer_flops(layer, H, W, N, M, kind=1):
    """Algorithmic FLOPs (2 x MAC) of one layer on one frame, on the
    64-multiple padded frame the method codes (GDN contraction included).
    Context model (kind 2): h_s's last layer has 2M outputs; the context
    convolution has 12 taps at half the latent positions; the entropy-
    parameter layers run at half the positions each, the first on 4M inputs."""
    Hp, Wp = 64 * math.ceil(H / 64), 64 * math.ceil(W / 64)
    Hy, Wy = Hp // 16, Wp // 16
    E1, E2 = 32 * round(10 * M / 96), 32 * round(8 * M / 96)
    half = Hy * Wy // 2
    ctx = {"CX": (half, M, 2 * M, 12), "EP0A": (half, 4 * M, E1, 1), "EP0N": (half, 4 * M, E1, 1),
           "EP1A": (half, E1, E2, 1), "EP1N": (half, E1, E2, 1), "EP2A": (half, E2, 2 * M, 1),
           "EP2N": (half, E2, 2 * M, 1), "HS2": (Hy * Wy, N, 2 * M, 9)}
    if kind == 2 and layer in ctx:
        c = ctx[layer]
        return 2.0 * c[0] * c[1] * c[2] * c[3]
    conv = {  # (output pixels, or input pixels for transposed convs, C_in, C_out, k*k)
        "GA0": (Hp // 2 * Wp // 2, 3, N, 25), "GA1": (Hp // 4 * Wp // 4, N, N, 25),
        "GA2": (Hp // 8 * Wp // 8, N, N, 25), "GA3": (Hy * Wy, N, M, 25),
        "HA0": (Hy * Wy, M, N, 9), "HA1": (Hy // 2 * Wy // 2, N, N, 25), "HA2": (Hy // 4 * Wy // 4, N, N, 25),
        "HS0": (Hy // 4 * Wy // 4, N, N, 25), "HS1": (Hy // 2 * Wy // 2, N, N, 25), "HS2": (Hy * Wy, N, M, 9),
        "GS0": (Hy * Wy, M, N, 25), "GS1": (Hp // 8 * Wp // 8, N, N, 25), "GS2": (Hp // 4 * Wp // 4, N, N, 25),
        "GS3": (Hp // 2 * Wp // 2, N, 3, 25),
    }[layer]
    mac = conv[0] * conv[1] * conv[2] * conv[3]
    gdn_px = {"GA0": Hp // 2 * Wp // 2, "GA1": Hp // 4 * Wp // 4, "GA2": Hp // 8 * Wp // 8,
              "GS0": Hp // 8 * Wp // 8, "GS1": Hp // 4 * Wp // 4, "GS2": Hp // 2 * Wp // 2}.get(layer, 0)
    return 2.0 * (mac + gdn_px * N * N)


def kernel_src_hash():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_for(layer, precision):
    """HBM bytes per launch (one 720p frame) of a layer of the codec in a
    precision form (fp32, bf16, fp8) from the committed rocprofv3 counter
    summary, or None if there is none or the kernel source changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_src_sha256_16") != kernel_src_hash():
        return None
    ent = t.get("forms", {}).get(precision, {}).get(layer)
    return None if ent is None else ent.get("bytes_per_launch")


def rans_rate(blob, n=737280, seed=5):
    """Host rANS speed on one core: one 720p frame's worth of y symbols (N=128
    M=192: 48 x 80 x 192) with the codec's Gaussian tables and scale indices
    spread over the table, through the C ABI's encoder and decoder."""
    import numpy as np

    from paper_2208_01641_amd import rans_decode, rans_encode, rans_ileave_decode, rans_ileave_encode
    from paper_2208_01641_amd._lib import lib

    freq = np.zeros(64 * 129, np.uint32)
    buf = np.frombuffer(blob, np.uint8).copy()
    k = lib.lic_blob_tables(buf.ctypes.data, len(blob), 1, freq.ctypes.data, freq.size, None, 0)
    assert k == freq.size, k
    freq = freq.reshape(64, 129)
    rng = np.random.default_rng(seed)
    tab = rng.integers(0, 40, n).astype(np.uint8)
    cum = np.cumsum(freq, axis=1)
    slot = rng.integers(0, 1 << 16, n)
    sym = np.array([np.searchsorted(cum[t], s, side="right") for t, s in zip(tab[:4096], slot[:4096])], np.uint8)
    sym = np.resize(sym, n)
    tab = np.resize(tab[:4096], n)
    def rate(enc, dec):
        best = [1e9, 1e9]
        for _ in range(3):                  # best of three (one core, no other load)
            t0 = time.perf_counter()
            data = enc()
            t1 = time.perf_counter()
            back = dec(data)
            t2 = time.perf_counter()
            assert np.array_equal(back, sym)
            best = [min(best[0], t1 - t0), min(best[1], t2 - t1)]
        return {"encode_msym_per_s_per_core": round(n / best[0] / 1e6, 1),
                "decode_msym_per_s_per_core": round(n / best[1] / 1e6, 1),
                "bits_per_symbol": round(8 * len(data) / n, 4)}

    out = {"symbols": n}
    out.update(rate(lambda: rans_encode(sym, tab, freq), lambda d: rans_decode(d, tab, freq, n)))
    out["interleaved_8_states"] = rate(lambda: rans_ileave_encode(sym, tab, freq, 8),
                                       lambda d: rans_ileave_decode(d, tab, freq, n, 8))
    return out


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo, as lscpu reports it)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(x_np, P, blob, N, M):
    """The FP64 oracle on the host cores: one whole 720p frame encoded and
    decoded with every core the process may use (per-stage seconds), and a
    3x192x320 crop (1/16 of the padded frame) on one core, scaled to the frame.
    Also returns the oracle's reconstruction and stream length of the frame,
    the FP64 reference of the precision forms."""
    import oracle
    m = oracle.Model(P, 1, N, M, blob)
    cores = host_cores()
    oracle.set_threads(cores)
    used = oracle.set_threads(0)
    times = {}
    t0 = time.perf_counter()
    bits, _ = m.encode(x_np, S=8, times=times)
    xr, _ = m.decode(bits, times=times)
    dt_all = time.perf_counter() - t0
    progress(f"cpu baseline: FP64 oracle, one 720p frame on {used} threads in {dt_all:.1f} s")
    oracle.set_threads(1)
    crop = x_np[:, :192, :320].copy()
    t0 = time.perf_counter()
    b1, _ = m.encode(crop, S=1)
    m.decode(b1)
    dt_one = time.perf_counter() - t0
    oracle.set_threads(cores)
    scale = (768 * 1280) / (192 * 320)
    progress(f"cpu baseline: FP64 oracle, 192x320 crop on 1 thread in {dt_one:.1f} s")
    base = {"value": round(1.0 / dt_all, 5), "unit": "frames/s", "cores": used, "kind": "oracle",
            "sample": f"FP64 oracle encode+decode of one whole 3x720x1280 frame on {used} OpenMP threads "
                      f"({dt_all:.1f} s wall), and of a 3x192x320 crop (1/16 of the padded frame) on 1 thread "
                      f"({dt_one:.1f} s wall, scaled x{scale:.0f})",
            "cpu_model": cpu_model(),
            "stage_s": {k: round(v, 3) for k, v in times.items()},
            "one_thread": {"value": round(1.0 / (dt_one * scale), 6), "unit": "frames/s", "cores": 1}}
    return base, xr, len(bits)


def psnr(a, b) -> float:
    import numpy as np
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10 * math.log10(1.0 / mse)


RANS_LANES = 8      # entropy coder of every run unless a variant says otherwise (--rans-lanes)


def run_workload(*, H, W, N, M, precision, batch, steps, warmup, threads, inflight, slices, zero_copy,
                 timed_layers, copy_probe_mib=0, host_frames=False, kind=1, mode="encdec", norm=0, rans_lanes=None):
    """Creates a codec, pipelines warmup + steps frames through the encoder
    chained into the decoder (mode "encdec"), the encoder alone ("enc") or
    the decoder alone ("dec", on bitstreams encoded before the timed
    region), and returns the measurements, frame 0 (input), the weights."""
    import numpy as np
    import torch

    import synth
    from paper_2208_01641_amd import Codec

    P = synth.model_params(kind, N, M)
    blob = synth.weight_blob(P, kind, N, M)
    rans_lanes = RANS_LANES if rans_lanes is None else rans_lanes
    codec = Codec(blob, kind=kind, N=N, M=M, hs_out=1, precision=precision, y_slices=slices,
                  entropy_threads=threads, zero_copy=zero_copy, max_in_flight=inflight, max_h=H, max_w=W,
                  max_batch=batch, norm=norm, rans_lanes=rans_lanes)
    frames = synth.frames_sinusoid_torch(H, W, range(steps + warmup), device="cuda")
    out = torch.empty_like(frames)
    if precision == 2:                    # e4m3 activation scales from a calibration frame of the stream
        codec.calibrate(synth.frames_sinusoid_torch(H, W, [10_000], device="cuda"))
    if kind == 0 and (H, W) == (128, 128):   # the factorized-prior case: 1/f-spectrum noise images
        frames = torch.from_numpy(np.stack([synth.image_1f(H, W, seed=1641 + i)
                                            for i in range(steps + warmup)])).cuda()
    if host_frames:                        # frames and reconstructions in pinned host memory (PCIe both ways)
        frames = frames.cpu().pin_memory()
        out = out.cpu().pin_memory()
    if copy_probe_mib:
        src = torch.ones(copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    pre_bits = codec.encode(frames[:steps]) if mode == "dec" else None
    if warmup:
        if mode == "enc":
            codec.encode(frames[steps:])
        elif mode == "dec":
            codec.decode(codec.encode(frames[steps:]), out[steps:])
        else:
            codec.encode_decode(frames[steps:], out[steps:])
    codec.time_layers(timed_layers)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if mode == "enc":
        bits = codec.encode(frames[:steps])
    elif mode == "dec":
        codec.decode(pre_bits, out[:steps])
        bits = pre_bits
    else:
        bits = codec.encode_decode(frames[:steps], out[:steps])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lat = codec.latencies_ms()
    st = codec.stats()
    progress(f"{H}x{W} N={N} M={M} precision={precision} batch={batch} in_flight={inflight} mode={mode} kind={kind} "
             f"norm={norm} rans_lanes={rans_lanes}: {steps / dt:.1f} frames/s")
    layers = {}
    for L in timed_layers:
        ms, n = codec.layer_time(L)
        if n:
            per_launch = ms / n
            flops = layer_flops(L, H, W, N, M, kind) * batch      # a launch covers one task of `batch` frames
            layers[L] = {"avg_us": 1e3 * per_launch, "launches": n, "tflops": flops / (per_launch * 1e-3) / 1e12,
                         "flops_per_launch": flops, "form": codec.layer_kernel(L, H, W)[0]}
    if mode == "enc":                     # reconstructions of the encoded frames, untimed
        codec.decode(bits, out[:steps])
        torch.cuda.synchronize()
    mse = torch.mean((out[:steps] - frames[:steps]) ** 2, dim=(1, 2, 3))
    # GPU work per frame: the summed kernel time of every timed layer
    kernel_ms = sum(codec.layer_time(L)[0] for L in timed_layers) / (steps * batch)
    res = {
        "fps": steps / dt,
        "ms_per_step": 1e3 * dt / steps,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "psnr_db": float(torch.mean(10 * torch.log10(1.0 / mse)).item()),
        "bpp": float(np.mean([8.0 * len(b) / (H * W) for b in bits])),
        "gpu_busy_s": st["gpu_busy_s"],
        "cpu_busy_s": st["cpu_busy_s"],
        "layers": layers,
        "kernel_ms_per_frame": kernel_ms,
        "xhat0": out[0].cpu().numpy(),
        "bits0": len(bits[0]),
    }
    codec.close()
    x0 = frames[0].cpu().numpy()
    del frames, out
    torch.cuda.empty_cache()
    return res, x0, P, blob


def run_serving(*, precision, threads, duration_s=4.0, warmup_s=1.0, seed=7, use_graphs=1, rate=30.0):
    """16 concurrent streams (8 x 360p, 4 x 720p, 4 x 1080p), Poisson frame
    arrivals at `rate` frames/s per stream (30 by default), served through
    submit/poll with continuous batching (per-size buckets, batches of up to
    4, captured HIP graphs); every encoded frame is resubmitted for decoding.
    A stream holds at most 48 frames in flight (its buffer ring): arrivals
    beyond that are dropped and counted.  Returns the completed frames/s and
    the latency percentiles after the warm-up."""
    import numpy as np
    import torch

    import synth
    from paper_2208_01641_amd import Codec

    N, M = 128, 192
    progress(f"serving: 16 streams at {rate:g} frames/s each, precision={precision}, graphs={use_graphs}")
    sizes = [(360, 640)] * 8 + [(720, 1280)] * 4 + [(1080, 1920)] * 4
    P = synth.model_params(1, N, M)
    blob = synth.weight_blob(P, 1, N, M)
    codec = Codec(blob, kind=1, N=N, M=M, hs_out=1, precision=precision, y_slices=4, entropy_threads=threads,
                  zero_copy=1, max_in_flight=8, max_h=1080, max_w=1920, max_batch=4, use_graphs=use_graphs,
                  rans_lanes=RANS_LANES)
    sids = [codec.open_stream(H, W) for H, W in sizes]
    frames = [synth.frames_sinusoid_torch(H, W, range(4), stream=s, device="cuda") for s, (H, W) in enumerate(sizes)]
    ring = 48
    bits_buf = [[np.zeros(codec.max_stream_bytes(H, W), np.uint8) for _ in range(ring)] for H, W in sizes]
    img_buf = [[torch.empty((3, H, W), device="cuda") for _ in range(ring)] for H, W in sizes]
    rng = np.random.default_rng(seed)
    total = warmup_s + duration_s
    arrivals = []
    for s in range(len(sizes)):
        t = rng.exponential(1 / rate)
        while t < total:
            arrivals.append((t, s))
            t += rng.exponential(1 / rate)
    arrivals.sort()
    torch.cuda.synchronize()
    enc_of, dec_of, meta = {}, {}, {}
    lat_enc, lat_dec, lat_e2e = [], [], []
    done_frames = 0
    nxt = 0
    k = [0] * len(sizes)
    free = [list(range(ring)) for _ in sizes]     # buffer slots of each stream not in flight
    dropped = 0
    t0 = time.perf_counter()
    t_meas = None
    outstanding = 0
    while nxt < len(arrivals) or outstanding:
        now = time.perf_counter() - t0
        while nxt < len(arrivals) and arrivals[nxt][0] <= now:
            ta, s = arrivals[nxt]
            nxt += 1
            if not free[s]:
                dropped += ta >= warmup_s
                continue
            j = free[s].pop()
            tk = codec.submit_encode(sids[s], frames[s][k[s] % 4], bits_buf[s][j])
            enc_of[tk] = (s, j, ta)
            k[s] += 1
            outstanding += 1
        for r in codec.poll(256, 200):
            if r["direction"] == 0:
                s, j, ta = enc_of.pop(r["ticket"])
                assert r["status"] == 0, r
                arr = bits_buf[s][j][:r["bytes"]]
                tk = codec.submit_decode(sids[s], arr, img_buf[s][j])
                dec_of[tk] = (s, j, ta)
                if ta >= warmup_s:
                    lat_enc.append(r["latency_ms"])
            else:
                s, j, ta = dec_of.pop(r["ticket"])
                assert r["status"] == 0, r
                outstanding -= 1
                free[s].append(j)
                if ta >= warmup_s:
                    lat_dec.append(r["latency_ms"])
                    lat_e2e.append(1e3 * (time.perf_counter() - t0 - ta))
                    done_frames += 1
                    if t_meas is None:
                        t_meas = time.perf_counter()
        if nxt < len(arrivals) and not outstanding:
            time.sleep(max(0.0, arrivals[nxt][0] - (time.perf_counter() - t0)))
    t_end = time.perf_counter()
    codec.close()
    del frames, img_buf
    torch.cuda.empty_cache()
    pct = lambda a, q: float(np.percentile(a, q)) if a else None
    offered = sum(1 for ta, _ in arrivals if ta >= warmup_s) / duration_s
    return {"streams": len(sizes), "rate_per_stream": rate, "offered_fps": offered, "frames": done_frames,
            "dropped": dropped, "measured_s": duration_s, "warmup_s": warmup_s,
            "fps": done_frames / (t_end - t_meas) if t_meas else 0.0,
            "enc_p50_ms": pct(lat_enc, 50), "enc_p99_ms": pct(lat_enc, 99),
            "dec_p50_ms": pct(lat_dec, 50), "dec_p99_ms": pct(lat_dec, 99),
            "e2e_p50_ms": pct(lat_e2e, 50), "e2e_p99_ms": pct(lat_e2e, 99)}


def run_distilled(*, pairs, steps, threads, batch=32, holdout=256, deploy_frames=120, seed=0):
    """Distilled g_s: pairs (y_hat, x_hat) of 256x256 crops from the FP32
    N=128 M=192 decoder, GPU training (AdamW, batch 32), judge calibration
    on held-out crops, then 720p decoding with the full and the distilled
    g_s (frames/s, p99, PSNR gap)."""
    import numpy as np
    import torch

    import synth
    from paper_2208_01641_amd import Codec, Distill
    from paper_2208_01641_amd import distill_train as dtr

    N, M, F = 128, 192, 64
    P = synth.model_params(1, N, M)
    blob = synth.weight_blob(P, 1, N, M)
    teacher = Codec(blob, kind=1, N=N, M=M, hs_out=1, precision=0, y_slices=1, entropy_threads=2, max_in_flight=1,
                    max_h=256, max_w=256)
    total = pairs + holdout
    imgs = torch.empty((total, 3, 256, 256), device="cuda")
    for i in range(total):                 # one generator stream per crop
        imgs[i] = synth.frames_sinusoid_torch(256, 256, [0], stream=10 ** 6 + i, device="cuda")[0]
    torch.cuda.synchronize()
    progress(f"distilled g_s: {total} crops generated")
    t0 = time.perf_counter()
    sym, rec = dtr.build_pairs(teacher, imgs)
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    progress(f"distilled g_s: {total} (y_hat, x_hat) pairs in {t_pairs:.1f} s")
    teacher.close()
    net = Distill(synth.distill_params(M, F), M, F, max_batch=batch, max_hy=16, max_wy=16)
    dtr.train(net, sym[:pairs], rec[:pairs], 5, batch, seed=seed + 1)          # warm-up (discarded state below)
    net.set(0, synth_flat(synth.distill_params(M, F)))
    net.set(1, np.zeros(net.n_params, np.float32))
    net.set(2, np.zeros(net.n_params, np.float32))
    net.step_count = 0
    t0 = time.perf_counter()
    losses = []
    for s0 in range(0, steps, 1000):            # chunks of 1000 steps, with a progress line each
        n = min(1000, steps - s0)
        losses.append(dtr.train(net, sym[:pairs], rec[:pairs], n, batch, seed=seed + s0))
        progress(f"distilled g_s: {s0 + n}/{steps} steps, loss {float(losses[-1][-50:].mean()):.5f}")
    losses = np.concatenate(losses)
    t_train = time.perf_counter() - t0
    fid, gap = dtr.evaluate(net, sym[pairs:], rec[pairs:], imgs[pairs:])
    T = dtr.judge_threshold(fid, gap)
    params = net.get(0)
    net.close()
    del sym, rec, imgs
    torch.cuda.empty_cache()

    # deployment: decode 720p frames with the full and the distilled g_s
    H, W = 720, 1280
    frames = synth.frames_sinusoid_torch(H, W, range(deploy_frames), device="cuda")
    out = {}
    for name, mode, prec in (("full_fp32", 0, 0), ("distilled_fp32", 1, 0), ("distilled_bf16", 1, 1),
                             ("distilled_judged_fp32", 2, 0)):
        c = Codec(blob, kind=1, N=N, M=M, hs_out=1, precision=0 if mode == 0 else prec, y_slices=8,
                  entropy_threads=threads, max_in_flight=6, max_h=H, max_w=W, gs_mode=mode, rans_lanes=RANS_LANES)
        if mode:
            c.load_distilled(params, judge_psnr_db=T if math.isfinite(T) else 1e9, judge_every=30)
        bits = c.encode(frames) if mode == 0 or "enc" not in out else out["enc"]
        out.setdefault("enc", bits)
        xr = torch.empty_like(frames)
        c.decode(bits[:8], xr[:8])                     # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.decode(bits, xr)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        lat = c.latencies_ms()
        mse = torch.mean((xr - frames) ** 2, dim=(1, 2, 3))
        r = {"decode_fps": deploy_frames / dt, "p50_ms": float(np.percentile(lat, 50)),
             "p99_ms": float(np.percentile(lat, 99)), "psnr_db": float(torch.mean(10 * torch.log10(1.0 / mse)))}
        if mode:
            st = c.stats()
            r.update(gs_judged=st["gs_judged"], gs_fallback=st["gs_fallback"])
            r["psnr_vs_full_db"] = float(torch.mean(10 * torch.log10(1.0 / torch.mean((xr - out["full_xr"]) ** 2,
                                                                                     dim=(1, 2, 3)))))
        else:
            out["full_xr"] = xr
        out[name] = _round(r)
        progress(f"distilled g_s: 720p decode {name}: {r['decode_fps']:.1f} frames/s")
        c.close()
    full = out.pop("full_xr")
    del full, frames
    out.pop("enc")
    for k in ("distilled_fp32", "distilled_bf16", "distilled_judged_fp32"):
        out[k]["gap_db_vs_full"] = round(out["full_fp32"]["psnr_db"] - out[k]["psnr_db"], 4)
    flops_per_sample = 3 * 2 * 0.2338e9           # forward + input and weight gradients
    return {
        "pairs": pairs, "steps": steps, "batch": batch, "pairs_s": round(t_pairs, 3), "train_s": round(t_train, 3),
        "train_samples_per_s": round(steps * batch / t_train, 1),
        "train_tflops": round(steps * batch * flops_per_sample / t_train / 1e12, 2),
        "loss_first": float(losses[:10].mean()), "loss_last": float(losses[-100:].mean()),
        "holdout_fidelity_db": round(float(np.mean(fid)), 3), "holdout_gap_db": round(float(np.mean(gap)), 4),
        "judge_threshold_db": T if math.isfinite(T) else None,
        "deploy_720p": out,
    }


def synth_flat(P):
    from paper_2208_01641_amd.distill import flatten
    return flatten(P)


def progress(msg):
    """One line per finished piece of work, on stderr (the JSON line is the
    only stdout output)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _round(d, nd=3):
    return {k: (round(v, nd) if isinstance(v, float) else v) for k, v in d.items()}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300, help="timed frames")
    ap.add_argument("--warmup", type=int, default=30, help="untimed frames first")
    ap.add_argument("--height", type=int, default=720)
    ap.add_argument("--width", type=int, default=1280)
    ap.add_argument("--precision", choices=["fp32", "bf16", "fp8"], default="fp32")
    ap.add_argument("--threads", type=int, default=0, help="entropy worker threads (0: min(16, cores))")
    ap.add_argument("--inflight", type=int, default=6, help="tasks in flight (pooled slots)")
    ap.add_argument("--slices", type=int, default=8, help="rANS row slices of y")
    ap.add_argument("--zero-copy", type=int, default=1)
    ap.add_argument("--rans-lanes", type=int, default=8,
                    help="entropy coder: interleaved rANS states (0: byte-wise single-state rANS)")
    ap.add_argument("--serial", action="store_true", help="one frame in flight (unpipelined)")
    ap.add_argument("--channels", choices=["128x192", "192x320"], default="128x192",
                    help="N x M of the main workload's codec")
    ap.add_argument("--batch", type=int, default=1, help="frames per codec task of the main workload")
    ap.add_argument("--kind", type=int, choices=[0, 1, 2], default=1,
                    help="codec of the main workload: 1 scale hyperprior (the metric's), 0 factorized prior, "
                         "2 context model (for profiles of those codecs)")
    ap.add_argument("--all-layers", action="store_true", help="time every layer (per-layer breakdown)")
    ap.add_argument("--no-variants", action="store_true", help="headline workload only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--distill-pairs", type=int, default=20000,
                    help="distilled g_s variant: training pairs (0 skips the variant)")
    ap.add_argument("--distill-steps", type=int, default=12500,
                    help="distilled g_s variant: AdamW steps (12500 = 20 epochs of 20k pairs at batch 32)")
    ap.add_argument("--distill-only", action="store_true", help="run only the distilled g_s variant")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (calibrates HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported by this build "
              "(frames are independent keyframes: each GPU would run its own codec)", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    threads = args.threads or min(16, os.cpu_count() or 1)
    global RANS_LANES
    RANS_LANES = args.rans_lanes
    if args.distill_only:
        print(json.dumps({"distilled_gs": run_distilled(pairs=args.distill_pairs, steps=args.distill_steps,
                                                        threads=threads)}), flush=True)
        return
    prec = {"fp32": 0, "bf16": 1, "fp8": 2}[args.precision]
    dtype = {0: "f32", 1: "bf16", 2: "fp8"}[prec]
    H, W, K, Wm = args.height, args.width, args.steps, args.warmup
    N, M = (int(v) for v in args.channels.split("x"))
    # (the headline run times two layers only: events between every launch
    # perturb the pipelined run; the one-frame-in-flight variant times all)
    timed = ["GA1", "GS2"]
    if args.all_layers:
        timed = [L for L in LAYERS if args.kind or not L.startswith("H")] + (list(CTX_LAYERS) if args.kind == 2 else [])
    main_res, x0, P, blob = run_workload(
        H=H, W=W, N=N, M=M, precision=prec, batch=args.batch, steps=K, warmup=Wm, threads=threads,
        inflight=1 if args.serial else args.inflight, slices=args.slices, zero_copy=args.zero_copy,
        timed_layers=timed, copy_probe_mib=args.copy_probe_mib, kind=args.kind)

    per_layer = main_res["layers"]
    dom = max(per_layer, key=lambda L: per_layer[L]["avg_us"] * per_layer[L]["launches"])
    form = per_layer[dom]["form"]
    peak = round(PEAK_TFLOPS[form], 2)
    ach = per_layer[dom]["tflops"]
    roofline = {"bound": "mfma", "achieved": round(ach, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(ach / peak, 4),
                "traffic": (traffic_for(dom, args.precision)
                            if (H, W, N, M, args.kind, args.batch) == (720, 1280, 128, 192, 1, 1) else None),
                "kernel": dom, "form": form, "peak_basis": PEAK_BASIS[form],
                "avg_us": round(per_layer[dom]["avg_us"], 2),
                "flops_per_launch": per_layer[dom]["flops_per_launch"]}

    res = {
        "metric": METRIC,
        "value": round(main_res["fps"], 3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": round(main_res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"{CODEC_NAME[args.kind]} N={N} M={M} {args.precision.upper()} encode chained into decode, "
                               f"3x{H}x{W} frames (32 moving sinusoids + noise)"
                               + (f", batches of {args.batch}" if args.batch > 1 else "") + ", pipelined",
                   "frames": K, "entropy_threads": threads, "max_in_flight": 1 if args.serial else args.inflight,
                   "y_slices": args.slices, "zero_copy": args.zero_copy, "rans_lanes": args.rans_lanes},
        "p50_ms": round(main_res["p50_ms"], 3),
        "p99_ms": round(main_res["p99_ms"], 3),
        "psnr_db": round(main_res["psnr_db"], 3),
        "bpp": round(main_res["bpp"], 4),
        "gpu_busy_s": main_res["gpu_busy_s"],
        "cpu_busy_s": main_res["cpu_busy_s"],
        "layers": {L: {"avg_us": round(v["avg_us"], 2), "tflops": round(v["tflops"], 2), "form": v["form"]}
                   for L, v in per_layer.items()},
        "roofline": roofline,
        "variants": None,
        "cpu_baseline": None,
    }

    if not args.no_variants:
        var = {}
        keys = ("fps", "p50_ms", "p99_ms", "psnr_db", "bpp")
        common = dict(threads=threads, slices=args.slices, zero_copy=args.zero_copy, timed_layers=["GA1", "GS2"])
        hd = dict(H=720, W=1280, N=128, M=192, batch=1)
        # steady state over 300 pipelined frames (the latency percentiles of
        # the FP32 form, whatever --steps the headline ran with)
        r, _, _, _ = run_workload(precision=0, steps=300, warmup=30, inflight=args.inflight, **hd, **common)
        var["fp32_720p_300_frames"] = _round({k: r[k] for k in keys})
        fp32_ref = r
        r, _, _, _ = run_workload(precision=0, steps=60, warmup=5, inflight=1, **hd,
                                  **dict(common, timed_layers=list(LAYERS)))
        var["fp32_720p_one_frame_in_flight"] = _round({k: r[k] for k in keys})
        # GPU-only bound: frames/s if the GPU ran one frame's kernels back to
        # back with nothing else (no entropy coding, no overlap)
        var["fp32_720p_one_frame_in_flight"]["gpu_kernel_ms_per_frame"] = round(r["kernel_ms_per_frame"], 4)
        var["fp32_720p_one_frame_in_flight"]["gpu_only_fps"] = round(1e3 / r["kernel_ms_per_frame"], 1)
        var["fp32_720p_one_frame_in_flight"]["layers_us"] = {L: round(v["avg_us"], 1) for L, v in r["layers"].items()}
        # encoder and decoder apart (the paper reports them separately), for
        # the scale hyperprior and the factorized prior, pipelined and with
        # one frame in flight (the paper's implementation A)
        for kind, kname in ((1, "hyper"), (0, "factor")):
            for mode in ("enc", "dec"):
                for infl, tag in ((args.inflight, "pipelined"), (1, "one_frame_in_flight")):
                    r, _, _, _ = run_workload(precision=0, steps=150 if infl > 1 else 60, warmup=10, inflight=infl,
                                              kind=kind, mode=mode, **hd, **common)
                    var[f"fp32_720p_{kname}_{mode}_{tag}"] = _round({k: r[k] for k in ("fps", "p50_ms", "p99_ms")})
        # the factorized-prior case at 3x128x128: per-frame latency of encode
        # + decode with one frame in flight, and pipelined frames/s
        for infl, tag in ((1, "one_frame_in_flight"), (args.inflight, "pipelined")):
            r, _, _, _ = run_workload(H=128, W=128, N=128, M=192, batch=1, precision=0, steps=200, warmup=20,
                                      inflight=infl, kind=0, **dict(common, slices=1))
            var[f"factor_128x128_{tag}"] = _round({k: r[k] for k in keys})
            var[f"factor_128x128_{tag}"]["us_per_frame"] = round(1e3 / r["fps"], 1)
        var["rans_one_core"] = rans_rate(blob)
        # ladder rungs: symbols and indices through device buffers and async
        # copies instead of zero-copy stores; frames in pinned host memory
        zc = dict(common, zero_copy=0)
        r, _, _, _ = run_workload(precision=0, steps=150, warmup=10, inflight=args.inflight, **hd, **zc)
        var["fp32_720p_async_copies"] = _round({k: r[k] for k in ("fps", "p50_ms", "p99_ms")})
        r, _, _, _ = run_workload(precision=0, steps=150, warmup=10, inflight=args.inflight, host_frames=True,
                                  **hd, **common)
        var["fp32_720p_host_frames"] = _round({k: r[k] for k in ("fps", "p50_ms", "p99_ms")})
        forms = {}
        for name, p in (("bf16", 1), ("fp8", 2)):
            r, _, _, _ = run_workload(precision=p, steps=300, warmup=30, inflight=args.inflight, **hd, **common)
            forms[name] = r
            v = _round({k: r[k] for k in keys})
            v["d_psnr_db_vs_fp32"] = round(r["psnr_db"] - fp32_ref["psnr_db"], 4)
            v["d_bpp_vs_fp32"] = round(r["bpp"] - fp32_ref["bpp"], 5)
            var[f"{name}_720p"] = v
        # the byte-wise single-state rANS coder instead of the interleaved one
        for name, p in (("fp32", 0), ("bf16", 1), ("fp8", 2)):
            r, _, _, _ = run_workload(precision=p, steps=300, warmup=30, inflight=args.inflight, rans_lanes=0,
                                      **hd, **common)
            var[f"{name}_720p_bytewise_rans"] = _round({k: r[k] for k in keys})
        # 1DN instead of GDN (the paper's implementation C) in every form
        for name, p in (("fp32", 0), ("bf16", 1), ("fp8", 2)):
            r, _, _, _ = run_workload(precision=p, steps=150, warmup=15, inflight=args.inflight, norm=1,
                                      **hd, **dict(common, timed_layers=["GA1", "GS2"]))
            var[f"{name}_720p_1dn"] = _round({k: r[k] for k in keys})
            var[f"{name}_720p_1dn"]["layers_us"] = {L: round(v["avg_us"], 1) for L, v in r["layers"].items()}
        # per-layer kernel times of 1DN with one frame in flight (compare
        # fp32_720p_one_frame_in_flight for GDN)
        r, _, _, _ = run_workload(precision=0, steps=30, warmup=5, inflight=1, norm=1, **hd,
                                  **dict(common, timed_layers=list(LAYERS)))
        var["fp32_720p_1dn_one_frame_in_flight"] = _round({k: r[k] for k in ("fps", "p50_ms", "p99_ms")})
        var["fp32_720p_1dn_one_frame_in_flight"]["layers_us"] = {L: round(v["avg_us"], 1) for L, v in r["layers"].items()}
        # the context model (checkerboard-parallel context prediction) at
        # 720p: encode chained into decode, pipelined, in every form;
        # and one frame in flight with the kernel time of every layer
        for name, p in (("fp32", 0), ("bf16", 1), ("fp8", 2)):
            r, _, _, _ = run_workload(precision=p, steps=150, warmup=15, inflight=args.inflight, kind=2, **hd,
                                      **common)
            var[f"{name}_720p_context"] = _round({k: r[k] for k in keys})
        r, _, _, _ = run_workload(precision=0, steps=30, warmup=5, inflight=1, kind=2, **hd,
                                  **dict(common, timed_layers=list(LAYERS) + list(CTX_LAYERS)))
        v = _round({k: r[k] for k in keys})
        v["gpu_kernel_ms_per_frame"] = round(r["kernel_ms_per_frame"], 4)
        v["layers_us"] = {L: round(x["avg_us"], 1) for L, x in r["layers"].items()}
        v["layers_tflops"] = {L: round(x["tflops"], 1) for L in CTX_LAYERS for x in [r["layers"].get(L)] if x}
        var["fp32_720p_context_one_frame_in_flight"] = v
        big = {}
        for name, p in (("fp32", 0), ("bf16", 1), ("fp8", 2)):
            r, _, _, _ = run_workload(H=1080, W=1920, N=192, M=320, precision=p, batch=4, steps=40, warmup=8,
                                      inflight=3, **common)
            big[name] = r
            var[f"{name}_1080p_n192_m320_batch4"] = _round({k: r[k] for k in keys})
        for name in ("bf16", "fp8"):
            var[f"{name}_1080p_n192_m320_batch4"]["d_psnr_db_vs_fp32"] = round(big[name]["psnr_db"] - big["fp32"]["psnr_db"], 4)
            var[f"{name}_1080p_n192_m320_batch4"]["d_bpp_vs_fp32"] = round(big[name]["bpp"] - big["fp32"]["bpp"], 5)
        var["serving_16_streams_bf16"] = _round(run_serving(precision=1, threads=threads, duration_s=10.0,
                                                            warmup_s=2.0))
        var["serving_16_streams_bf16_no_graphs"] = _round(run_serving(precision=1, threads=threads, use_graphs=0))
        # offered-load sweep: 16 streams at 60 to 180 frames/s each
        var["serving_load_sweep_bf16"] = [_round(run_serving(precision=1, threads=threads, rate=rate,
                                                             duration_s=4.0, warmup_s=1.0))
                                          for rate in (60.0, 120.0, 180.0)]
        # the streaming sample application: sender and receiver processes over
        # TCP on this host, factorized prior at 720p, paced at 30 frames/s and
        # unpaced (8 frames per codec call)
        from paper_2208_01641_amd import stream
        for name, fps, n, chunk in (("stream_720p30_factorized_tcp", 30.0, 120, 1),
                                    ("stream_720p_factorized_tcp_unpaced", 0.0, 320, 8)):
            r = stream.run_loopback(frames=n, fps=fps, kind=0, chunk=chunk, lanes=RANS_LANES, timeout_s=240)
            rv = r["received"]
            assert rv["frames"] == n and rv["bitstream_sha16"] == r["sent"]["bitstream_sha16"]
            var[name] = _round({"frames": n, "fps": rv["fps"], "latency_p50_ms": rv["latency_p50_ms"],
                                "latency_p99_ms": rv["latency_p99_ms"], "bytes_per_frame": r["sent"]["bytes"] / n})
            progress(f"{name}: {rv['fps']:.1f} frames/s")
        if args.distill_pairs > 0:
            var["distilled_gs"] = run_distilled(pairs=args.distill_pairs, steps=args.distill_steps, threads=threads)
        res["variants"] = var
        forms["fp32"] = fp32_ref

    if not args.no_cpu_baseline:
        base, x64, bytes64 = cpu_baseline(x0, P, blob, N, M)
        res["cpu_baseline"] = base
        # fidelity of each form against the FP64 oracle on frame 0 (the
        # random-weight codec's PSNR to the source is about 7 dB, so this is
        # the informative figure), and its rate against the oracle's
        fid = {"fp32_headline": {"psnr_vs_fp64_db": round(psnr(main_res["xhat0"], x64), 3),
                                 "d_bpp_vs_fp64": round(8.0 * (main_res["bits0"] - bytes64) / (H * W), 5)}}
        if not args.no_variants:
            for name in ("fp32", "bf16", "fp8"):
                r = forms[name]
                fid[name] = {"psnr_vs_fp64_db": round(psnr(r["xhat0"], x64), 3),
                             "d_bpp_vs_fp64": round(8.0 * (r["bits0"] - bytes64) / (H * W), 5),
                             "d_psnr_db_vs_fp64": round(psnr(r["xhat0"], x0) - psnr(x64, x0), 4)}
        res["vs_fp64_frame0"] = fid
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
