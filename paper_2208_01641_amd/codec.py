"""Python handle over the C ABI (marshalling only; torch supplies device memory)."""
from __future__ import annotations

import ctypes
import json

import numpy as np

from . import _lib
from ._lib import lib


class LicError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_lib.STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _ptr(a) -> int:
    """Address of a torch tensor (host or device) or numpy array."""
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def _is_device(a) -> int:
    return int(hasattr(a, "is_cuda") and a.is_cuda)


def _sync(*tensors):
    if any(_is_device(t) for t in tensors if t is not None):
        import torch
        torch.cuda.synchronize()


class Codec:
    """A codec instance: packed weights, tables, pools and pipeline threads."""

    def __init__(self, blob: bytes, kind: int = 1, N: int = 128, M: int = 192, hs_out: int = 1, precision: int = 0,
                 y_slices: int = 8, entropy_threads: int = 8, zero_copy: int = 1, max_in_flight: int = 6,
                 max_h: int = 1088, max_w: int = 1920, max_batch: int = 1, hbm_budget_bytes: int = 0,
                 device: int = 0, use_graphs: int = 1, gs_mode: int = 0, norm: int = 0, rans_lanes: int = 0):
        cfg = _lib.CodecConfig()
        lib.codec_default_config(ctypes.byref(cfg))
        cfg.kind, cfg.N, cfg.M, cfg.hs_out, cfg.precision = kind, N, M, hs_out, precision
        cfg.y_slices, cfg.entropy_threads, cfg.zero_copy = y_slices, entropy_threads, zero_copy
        cfg.max_in_flight, cfg.max_h, cfg.max_w, cfg.max_batch = max_in_flight, max_h, max_w, max_batch
        cfg.hbm_budget_bytes, cfg.hip_device, cfg.use_graphs = hbm_budget_bytes, device, use_graphs
        cfg.gs_mode, cfg.norm, cfg.rans_lanes = gs_mode, norm, rans_lanes
        self.cfg = cfg
        self.kind, self.N, self.M, self.S, self.precision = kind, N, M, y_slices, precision
        self._blob = ctypes.create_string_buffer(bytes(blob), len(blob))
        h = ctypes.c_void_p()
        rc = lib.codec_create(ctypes.byref(cfg), self._blob, len(blob), ctypes.byref(h))
        if rc != 0:
            raise LicError(rc, lib.codec_last_error(None).decode())
        self._h = h

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib.codec_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc):
        if rc < 0:
            raise LicError(rc, lib.codec_last_error(self._h).decode())
        return rc

    def max_stream_bytes(self, H: int, W: int) -> int:
        Hp, Wp = 64 * -(-H // 64), 64 * -(-W // 64)
        ny = (Hp // 16) * (Wp // 16) * self.M
        nz = (Hp // 64) * (Wp // 64) * self.N if self.kind >= 1 else 0
        ns = 2 * self.S if self.kind == 2 else self.S          # y streams
        return 20 + 4 * (ns + 1) + 2 * (ny + nz) + 160 * (ns + 1)

    # ------------------------------------------------------------------
    def encode(self, x) -> list:
        """x: [n, 3, H, W] float32 (torch tensor on the GPU or host, or numpy)."""
        n, _, H, W = x.shape
        cap = n * self.max_stream_bytes(H, W)
        out = np.empty(cap, np.uint8)
        lens = np.zeros(n, np.uint64)
        _sync(x)
        self._check(lib.codec_encode(self._h, _ptr(x), n, H, W, _is_device(x), out.ctypes.data, cap,
                                     lens.ctypes.data))
        res, off = [], 0
        for ln in lens.tolist():
            res.append(out[off:off + ln].tobytes())
            off += ln
        return res

    def decode(self, streams, out):
        """Decodes a list of bitstreams into out ([n, 3, H, W] float32, device or host)."""
        n = len(streams)
        buf = np.frombuffer(b"".join(streams), np.uint8).copy()
        lens = np.array([len(s) for s in streams], np.uint64)
        H, W = ctypes.c_int(), ctypes.c_int()
        _sync(out)
        self._check(lib.codec_decode(self._h, buf.ctypes.data, lens.ctypes.data, n, _ptr(out), out.numel()
                                     if hasattr(out, "numel") else out.size, _is_device(out),
                                     ctypes.byref(H), ctypes.byref(W)))
        return H.value, W.value

    def encode_decode(self, x, out) -> list:
        """Encoder chained into the decoder, frame by frame; returns the bitstreams."""
        n, _, H, W = x.shape
        cap = n * self.max_stream_bytes(H, W)
        bits = np.empty(cap, np.uint8)
        lens = np.zeros(n, np.uint64)
        _sync(x, out)
        self._check(lib.codec_encode_decode(self._h, _ptr(x), n, H, W, _is_device(x), bits.ctypes.data, cap,
                                            lens.ctypes.data, _ptr(out)))
        res, off = [], 0
        for ln in lens.tolist():
            res.append(bits[off:off + ln].tobytes())
            off += ln
        return res

    def load_distilled(self, params, judge_psnr_db: float = 0.0, judge_every: int = 30):
        """Distilled g_s for gs_mode 1 / 2: params is the flat float32 vector
        (or the dict) of paper_2208_01641_amd.distill."""
        from .distill import flatten
        if isinstance(params, dict):
            params = flatten(params, self.M, 64)
        v = np.ascontiguousarray(params, np.float32)
        self._check(lib.codec_load_distilled(self._h, v.ctypes.data, v.size, judge_psnr_db, judge_every))

    def calibrate(self, x):
        """FP8 form: per-layer e4m3 activation scales from frames x [n, 3, H, W]."""
        n, _, H, W = x.shape
        _sync(x)
        self._check(lib.codec_calibrate(self._h, _ptr(x), n, H, W, _is_device(x)))

    def fp8_scales(self):
        """(q per layer, as a list of LIC_NUM_LAYERS floats (0: no e4m3 output),
        values clamped to +-448 by e4m3 stores since create)."""
        q = np.zeros(len(_lib.LAYERS), np.float32)
        sat = ctypes.c_ulonglong()
        self._check(lib.codec_fp8_scales(self._h, q.ctypes.data, q.size, ctypes.byref(sat)))
        return q.tolist(), int(sat.value)

    def layer_bytes(self, layer, n: int, H: int, W: int):
        """(in, out, aux) bytes of codec_run_layer's buffers for this layer."""
        lid = _lib.LAYER_ID[layer] if isinstance(layer, str) else int(layer)
        b = (ctypes.c_size_t * 3)()
        self._check(lib.codec_layer_bytes(self._h, lid, n, H, W, ctypes.byref(b, 0), ctypes.byref(b, 8),
                                          ctypes.byref(b, 16)))
        return tuple(int(v) for v in b)

    def run_layer(self, layer, n: int, H: int, W: int, inp, out, aux=None, in2=None, out2=None):
        """One layer on device buffers.  in2 / out2: the last entropy-parameter
        layer of the context model (y, and y_hat or the means)."""
        lid = _lib.LAYER_ID[layer] if isinstance(layer, str) else int(layer)
        # refuse buffers smaller than what the layer reads or writes
        need = self.layer_bytes(lid, n, H, W)
        pl = n * (64 * -(-H // 64) // 16) * (64 * -(-W // 64) // 16) * self.M * 4   # float latent tensor
        ep2 = _lib.LAYERS[lid] in ("EP2A", "EP2N")
        for name, t, nb in (("input", inp, need[0]), ("output", out, need[1]), ("aux", aux, need[2]),
                            ("in2", in2, pl if ep2 else 0), ("out2", out2, pl if ep2 else 0)):
            if t is None or nb == 0:
                continue
            have = t.numel() * t.element_size() if hasattr(t, "element_size") else t.nbytes
            if have < nb:
                raise LicError(_lib.LIC_E_SMALLBUF, f"{_lib.LAYERS[lid]} {name} buffer holds {have} bytes, needs {nb}")
        _sync(inp, out, aux, in2, out2)
        opt = lambda t: 0 if t is None else _ptr(t)    # noqa: E731
        self._check(lib.codec_run_layer_ex(self._h, lid, n, H, W, _ptr(inp), opt(out), opt(aux), opt(in2),
                                           opt(out2)))

    def latencies_ms(self) -> np.ndarray:
        buf = np.zeros(1 << 16, np.float64)
        n = self._check(lib.codec_last_latencies(self._h, buf.ctypes.data, buf.size))
        return buf[:n].copy()

    def stats(self) -> dict:
        buf = ctypes.create_string_buffer(4096)
        self._check(lib.codec_get_stats(self._h, buf, 4096))
        return json.loads(buf.value.decode())

    # ------------------------------------------------------------ serving
    def open_stream(self, H: int, W: int) -> int:
        sid = ctypes.c_int()
        self._check(lib.codec_open_stream(self._h, H, W, ctypes.byref(sid)))
        return sid.value

    def close_stream(self, sid: int):
        self._check(lib.codec_close_stream(self._h, sid))

    def submit_encode(self, sid: int, x, out) -> int:
        """Queues one frame (3 x H x W float32); the bitstream goes to the
        uint8 buffer `out`.  Both must stay alive until the result is polled."""
        t = ctypes.c_uint64()
        self._check(lib.codec_submit_encode(self._h, sid, _ptr(x), _is_device(x), _ptr(out),
                                            out.nbytes if hasattr(out, "nbytes") else out.numel(), ctypes.byref(t)))
        return t.value

    def submit_decode(self, sid: int, bits, x_hat) -> int:
        """Queues one bitstream (a uint8 numpy array kept alive by the
        caller) for decoding into x_hat (3 x H x W float32)."""
        t = ctypes.c_uint64()
        self._check(lib.codec_submit_decode(self._h, sid, _ptr(bits), bits.size, _ptr(x_hat),
                                            x_hat.numel() if hasattr(x_hat, "numel") else x_hat.size,
                                            _is_device(x_hat), ctypes.byref(t)))
        return t.value

    def poll(self, max_results: int = 256, timeout_us: int = 0) -> list:
        buf = (_lib.LicResult * max_results)()
        n = self._check(lib.codec_poll(self._h, buf, max_results, timeout_us))
        return [{"ticket": r.ticket, "status": r.status, "stream_id": r.stream_id, "direction": r.direction,
                 "H": r.H, "W": r.W, "bytes": r.bytes, "latency_ms": r.latency_ms} for r in buf[:n]]

    def time_layers(self, layers):
        """Bracket every pipeline launch of these layers with HIP events."""
        mask = 0
        for L in layers or ():
            mask |= 1 << (_lib.LAYER_ID[L] if isinstance(L, str) else int(L))
        self._check(lib.codec_time_layers(self._h, mask))

    FORMS = {0: "f32", 1: "bf16", 2: "fp8", 3: "f32x"}

    def layer_kernel(self, layer, H, W):
        """(operand form name, K-split waves) of the kernel a layer launches
        for one H x W frame."""
        lid = _lib.LAYER_ID[layer] if isinstance(layer, str) else int(layer)
        form, ks = ctypes.c_int(), ctypes.c_int()
        self._check(lib.codec_layer_kernel(self._h, lid, H, W, ctypes.byref(form), ctypes.byref(ks)))
        return self.FORMS[form.value], ks.value

    def layer_time(self, layer):
        """(summed kernel milliseconds, launches) of a timed layer."""
        lid = _lib.LAYER_ID[layer] if isinstance(layer, str) else int(layer)
        ms, n = ctypes.c_double(), ctypes.c_long()
        self._check(lib.codec_layer_time(self._h, lid, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def tables(self, which: int) -> np.ndarray:
        buf = np.zeros(512 * 129, np.uint32)
        n = self._check(lib.codec_tables(self._h, which, buf.ctypes.data, buf.size))
        return buf[:n].reshape(-1, 129).copy()

    def medians(self) -> np.ndarray:
        buf = np.zeros(512, np.float32)
        n = self._check(lib.codec_medians(self._h, buf.ctypes.data, buf.size))
        return buf[:n].copy()


# ---------------------------------------------------------------- host coder
def rans_encode(sym, tab, freq) -> bytes:
    sym = np.ascontiguousarray(sym, np.uint8).ravel()
    tab = np.ascontiguousarray(tab, np.uint8).ravel()
    freq = np.ascontiguousarray(freq, np.uint32)
    cap = 2 * sym.size + 64
    out = np.empty(cap, np.uint8)
    n = lib.lic_rans_encode(sym.ctypes.data, tab.ctypes.data, sym.size, freq.ctypes.data, freq.shape[0],
                            out.ctypes.data, cap)
    if n < 0:
        raise LicError(n, "lic_rans_encode")
    return out[:n].tobytes()


def rans_decode(data: bytes, tab, freq, n: int) -> np.ndarray:
    tab = np.ascontiguousarray(tab, np.uint8).ravel()
    freq = np.ascontiguousarray(freq, np.uint32)
    buf = np.frombuffer(data, np.uint8).copy() if data else np.zeros(1, np.uint8)
    sym = np.empty(n, np.uint8)
    rc = lib.lic_rans_decode(buf.ctypes.data, len(data), tab.ctypes.data, n, freq.ctypes.data, freq.shape[0],
                             sym.ctypes.data)
    if rc != 0:
        raise LicError(rc, "lic_rans_decode")
    return sym


def rans_ileave_encode(sym, tab, freq, lanes: int = 8) -> bytes:
    sym = np.ascontiguousarray(sym, np.uint8).ravel()
    tab = np.ascontiguousarray(tab, np.uint8).ravel()
    freq = np.ascontiguousarray(freq, np.uint32)
    cap = 2 * sym.size + 4 * lanes + 64
    out = np.empty(cap, np.uint8)
    n = lib.lic_rans_ileave_encode(lanes, sym.ctypes.data, tab.ctypes.data, sym.size, freq.ctypes.data,
                                   freq.shape[0], out.ctypes.data, cap)
    if n < 0:
        raise LicError(n, "lic_rans_ileave_encode")
    return out[:n].tobytes()


def rans_ileave_decode(data: bytes, tab, freq, n: int, lanes: int = 8) -> np.ndarray:
    tab = np.ascontiguousarray(tab, np.uint8).ravel()
    freq = np.ascontiguousarray(freq, np.uint32)
    buf = np.frombuffer(data, np.uint8).copy() if data else np.zeros(1, np.uint8)
    sym = np.empty(max(n, 1), np.uint8)
    rc = lib.lic_rans_ileave_decode(lanes, buf.ctypes.data, len(data), tab.ctypes.data, n, freq.ctypes.data,
                                    freq.shape[0], sym.ctypes.data)
    if rc != 0:
        raise LicError(rc, "lic_rans_ileave_decode")
    return sym[:n]


def fnv1a(data: bytes) -> int:
    buf = np.frombuffer(data, np.uint8).copy() if data else np.zeros(1, np.uint8)
    return int(lib.lic_fnv1a(buf.ctypes.data, len(data)))
