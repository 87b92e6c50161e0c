"""Streaming sample application: a sender that encodes frames and a receiver
that decodes them, connected by TCP (the paper's streaming demonstration,
Section VI: an encoder streams a 1280x720 factorized-prior codec at 30
frames/s to a decoder on another machine).  Here both ends run on one GPU,
each in its own process; the frames are seeded synthetic frames standing in
for a camera.

Wire format, one message per frame: the header "<4sIQI" = b"LICF", frame
index, capture time (CLOCK_MONOTONIC, ns, the same clock in both processes
of one host) and payload length, then the codec's bitstream.  A header with
index 0xFFFFFFFF and length 0 ends the stream.

Every step of the codec runs in liblic.so; this module only paces frames,
moves bytes over the socket and records timings.

    python -m paper_2208_01641_amd.stream --frames 120 --fps 30
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import socket
import struct
import subprocess
import sys
import time

HEADER = struct.Struct("<4sIQI")
MAGIC = b"LICF"
END = 0xFFFFFFFF


def pack_message(index: int, capture_ns: int, payload: bytes) -> bytes:
    return HEADER.pack(MAGIC, index, capture_ns, len(payload)) + payload


def _recv_exact(sock, n: int) -> bytes:
    buf = bytearray()
    while len(buf) < n:
        chunk = sock.recv(n - len(buf))
        if not chunk:
            raise ConnectionError("stream closed inside a message")
        buf += chunk
    return bytes(buf)


def read_message(sock):
    """(index, capture_ns, payload), or None at the end of the stream."""
    magic, index, capture_ns, length = HEADER.unpack(_recv_exact(sock, HEADER.size))
    if magic != MAGIC:
        raise ValueError("not a LICF message")
    if index == END:
        return None
    return index, capture_ns, _recv_exact(sock, length)


def image_digest(t) -> str:
    """Checksum of a decoded frame (device tensor), computed on the GPU: the
    sum of its 32-bit words and their position-weighted sum, mod 2^64."""
    import torch
    v = t.contiguous().view(torch.int32).reshape(-1).to(torch.int64)
    w = torch.arange(1, v.numel() + 1, device=v.device, dtype=torch.int64)
    return "%016x%016x" % (int(v.sum().item()) & (2 ** 64 - 1), int((v * w).sum().item()) & (2 ** 64 - 1))


def _codec(kind: int, H: int, W: int, precision: int, lanes: int, max_batch: int):
    import synth
    from .codec import Codec
    N, M = 128, 192
    P = synth.model_params(kind, N, M)
    blob = synth.weight_blob(P, kind, N, M)
    return Codec(blob, kind=kind, N=N, M=M, precision=precision, y_slices=8, entropy_threads=8,
                 max_in_flight=4, max_h=H, max_w=W, max_batch=max_batch, rans_lanes=lanes)


def run_sender(host: str, port: int, frames: int, fps: float, H: int = 720, W: int = 1280, kind: int = 0,
               precision: int = 0, lanes: int = 8, chunk: int = 1) -> dict:
    """Encodes `frames` frames and sends them as they are ready.  With fps > 0
    frame i is captured at t0 + i / fps (paced, chunk frames per codec call);
    with fps = 0 frames are sent as fast as the encoder produces them."""
    import torch

    import synth
    torch.cuda.init()                        # torch's device context before the library's
    src = synth.frames_sinusoid_torch(H, W, range(frames), device="cuda")      # the camera's frames
    codec = _codec(kind, H, W, precision, lanes, chunk)
    codec.encode(src[:1])                                                        # warm-up
    sock = socket.create_connection((host, port))
    sock.setsockopt(socket.IPPROTO_TCP, socket.TCP_NODELAY, 1)
    digests = []
    sent_bytes = 0
    t0 = time.monotonic_ns() + 50_000_000
    for f0 in range(0, frames, chunk):
        n = min(chunk, frames - f0)
        cap = [t0 + int((f0 + i) * 1e9 / fps) if fps > 0 else time.monotonic_ns() for i in range(n)]
        if fps > 0:
            wait = (cap[-1] - time.monotonic_ns()) / 1e9              # the chunk's last frame is captured
            if wait > 0:
                time.sleep(wait)
        bits = codec.encode(src[f0:f0 + n])
        for i, b in enumerate(bits):
            sock.sendall(pack_message(f0 + i, cap[i], b))
            digests.append(hashlib.sha256(b).hexdigest()[:16])
            sent_bytes += len(b)
    sock.sendall(HEADER.pack(MAGIC, END, 0, 0))
    sock.close()
    codec.close()
    del src
    torch.cuda.empty_cache()
    return {"frames": frames, "bytes": sent_bytes, "bitstream_sha16": digests}


def run_receiver(port: int, H: int = 720, W: int = 1280, kind: int = 0, precision: int = 0, lanes: int = 8,
                 chunk: int = 1, ready=None, listen_host: str = "127.0.0.1") -> dict:
    """Accepts one sender, decodes its frames (chunk at a time) and returns the
    per-frame latency (capture to decoded), throughput and digests of the
    received bitstreams and decoded frames."""
    import numpy as np
    import torch

    torch.cuda.init()                        # torch's device context before the library's
    out = torch.empty((chunk, 3, H, W), device="cuda")
    codec = _codec(kind, H, W, precision, lanes, chunk)
    codec.encode(torch.zeros((1, 3, H, W), device="cuda"))                       # warm-up
    srv = socket.socket(socket.AF_INET, socket.SOCK_STREAM)
    srv.setsockopt(socket.SOL_SOCKET, socket.SO_REUSEADDR, 1)
    srv.bind((listen_host, port))
    srv.listen(1)
    if ready is not None:
        ready(srv.getsockname()[1])
    conn, _ = srv.accept()
    lat, bit_d, img_d = [], [], []
    first = last = None
    pend = []

    def flush():
        nonlocal last
        n = len(pend)
        codec.decode([p[2] for p in pend], out[:n])
        torch.cuda.synchronize()
        now = time.monotonic_ns()
        last = now
        for k, (idx, cap, b) in enumerate(pend):
            lat.append((now - cap) / 1e6)
            bit_d.append(hashlib.sha256(b).hexdigest()[:16])
            img_d.append(image_digest(out[k]))
        pend.clear()

    while True:
        msg = read_message(conn)
        if msg is None:
            break
        if first is None:
            first = time.monotonic_ns()
        pend.append(msg)
        if len(pend) == chunk:
            flush()
    if pend:
        flush()
    conn.close()
    srv.close()
    codec.close()
    frames = len(lat)
    span = (last - first) / 1e9 if frames > 1 else 0.0
    return {"frames": frames, "fps": (frames - 1) / span if span > 0 else 0.0,
            "latency_p50_ms": float(np.percentile(lat, 50)) if lat else None,
            "latency_p99_ms": float(np.percentile(lat, 99)) if lat else None,
            "bitstream_sha16": bit_d, "image_sha16": img_d}


def run_loopback(frames: int = 120, fps: float = 30.0, H: int = 720, W: int = 1280, kind: int = 0,
                 precision: int = 0, lanes: int = 8, chunk: int = 1, timeout_s: float = 300.0) -> dict:
    """Receiver in a child process, sender in this one, over 127.0.0.1."""
    import tempfile
    with tempfile.TemporaryDirectory() as td:
        port_file = os.path.join(td, "port")
        res_file = os.path.join(td, "recv.json")
        cmd = [sys.executable, "-m", "paper_2208_01641_amd.stream", "--role", "recv", "--port", "0",
               "--port-file", port_file, "--out", res_file, "--height", str(H), "--width", str(W),
               "--kind", str(kind), "--precision", str(precision), "--rans-lanes", str(lanes), "--chunk", str(chunk)]
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        env = dict(os.environ, PYTHONPATH=root + os.pathsep + os.environ.get("PYTHONPATH", ""))
        child = subprocess.Popen(cmd, cwd=root, env=env)
        try:
            t_end = time.monotonic() + timeout_s
            while not os.path.exists(port_file):
                if child.poll() is not None:
                    raise RuntimeError(f"receiver exited with {child.returncode}")
                if time.monotonic() > t_end:
                    raise TimeoutError("receiver did not start")
                time.sleep(0.05)
            time.sleep(0.05)
            with open(port_file) as fh:
                port = int(fh.read())
            sent = run_sender("127.0.0.1", port, frames, fps, H, W, kind, precision, lanes, chunk)
            rc = child.wait(timeout=max(1.0, t_end - time.monotonic()))
            if rc != 0:
                raise RuntimeError(f"receiver exited with {rc}")
            with open(res_file) as fh:
                recv = json.load(fh)
        finally:
            if child.poll() is None:
                child.kill()
                child.wait()
    return {"sent": sent, "received": recv}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--role", choices=["loopback", "send", "recv"], default="loopback")
    ap.add_argument("--host", default="127.0.0.1")
    ap.add_argument("--port", type=int, default=0)
    ap.add_argument("--port-file", default=None, help="recv: write the bound port here once listening")
    ap.add_argument("--out", default=None, help="recv: write the result JSON here")
    ap.add_argument("--frames", type=int, default=120)
    ap.add_argument("--fps", type=float, default=30.0, help="capture rate (0: as fast as the encoder runs)")
    ap.add_argument("--height", type=int, default=720)
    ap.add_argument("--width", type=int, default=1280)
    ap.add_argument("--kind", type=int, default=0, help="0 factorized prior (the paper's demo), 1 hyperprior")
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--rans-lanes", type=int, default=8)
    ap.add_argument("--chunk", type=int, default=1, help="frames per codec call")
    a = ap.parse_args()
    if a.role == "recv":
        def ready(port):
            if a.port_file:
                tmp = a.port_file + ".tmp"
                with open(tmp, "w") as fh:
                    fh.write(str(port))
                os.replace(tmp, a.port_file)
        res = run_receiver(a.port, a.height, a.width, a.kind, a.precision, a.rans_lanes, a.chunk, ready)
    elif a.role == "send":
        res = run_sender(a.host, a.port, a.frames, a.fps, a.height, a.width, a.kind, a.precision, a.rans_lanes,
                         a.chunk)
    else:
        res = run_loopback(a.frames, a.fps, a.height, a.width, a.kind, a.precision, a.rans_lanes, a.chunk)
    text = json.dumps(res)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text)
    else:
        print(text)


if __name__ == "__main__":
    main()
