"""FP64 CPU oracle of the learned-codec hot path.

TEST INFRASTRUCTURE ONLY: this package may be imported by ``tests/``, by
``__graft_entry__.smoke()`` and by the CPU-baseline leg of ``bench.py``, and
by nothing else.  It shares no code with ``paper_2208_01641_amd`` (the HIP
library): neither imports the other.  The only module both use is ``synth``
(seeded inputs, none of the method's arithmetic).

The numerical primitives live in ``lic_oracle.c`` (plain double-precision
loops); this module strings them together into the codecs of the paper:

  * factorized prior (Section III.A, Fig. 1): x -> g_a -> y -> quantise with
    a per-channel offset -> entropy code with per-channel tables;
  * scale hyperprior (Section III.B, Fig. 1): additionally z = h_a(|y|) is
    quantised and coded, and h_s(z_hat) gives the scales whose table index
    selects the Gaussian table each element of y is coded with;
  * context model with parallel context prediction (the class of codecs that
    Sections II and VII name as the next step): a mean-scale hyperprior whose
    entropy parameters also see a context of already decoded latents, in the
    two-pass checkerboard order, so that each pass is one parallel step.

The architecture details the paper leaves to its cited models (layer shapes,
GDN, quantiser, tables, rANS, bitstream) follow the readings listed in the
design notes; each function below states the one it implements.

Parity status: pinned by ``tests/test_oracle_*.py`` (brute force, closed
forms, identities, round trips).  No function here is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import math
import os
import struct
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lic_oracle.c")
_SO = os.path.join(_HERE, "liblic_oracle.so")

NSYM = 129          # symbols -64..64
SYM_MIN = -64
SYM_MAX = 64
PREC = 16           # frequency precision, totals 2^16
RANS_L = 1 << 23


def build(force: bool = False) -> str:
    """Compile lic_oracle.c with gcc (plain -O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        d, i, l = ctypes.c_double, ctypes.c_int, ctypes.c_long
        P = ctypes.c_void_p
        L.or_conv2d_at.restype = d
        L.or_conv2d_at.argtypes = [P, i, i, i, P, P, i, i, i, i, i, i]
        L.or_conv2d.restype = None
        L.or_conv2d.argtypes = [P, i, i, i, P, P, i, i, i, i, P, i, i]
        L.or_deconv2d_at.restype = d
        L.or_deconv2d_at.argtypes = [P, i, i, i, P, P, i, i, i, i, i, i, i]
        L.or_deconv2d.restype = None
        L.or_deconv2d.argtypes = [P, i, i, i, P, P, i, i, i, i, P, i, i]
        L.or_conv2d_points.restype = None
        L.or_conv2d_points.argtypes = [P, i, i, i, P, P, i, i, i, i, i, P, P]
        L.or_deconv2d_points.restype = None
        L.or_deconv2d_points.argtypes = [P, i, i, i, P, P, i, i, i, i, i, P, P]
        L.or_deconv2d_wgrad.restype = None
        L.or_deconv2d_wgrad.argtypes = [P, i, i, i, P, i, i, i, i, i, i, P, P]
        L.or_adamw.restype = None
        L.or_adamw.argtypes = [P, P, P, P, l, l, d, d, d, d, d]
        L.or_gdn.restype = None
        L.or_gdn.argtypes = [P, i, l, P, P, i, P]
        L.or_gdn1.restype = None
        L.or_gdn1.argtypes = [P, i, l, P, P, i, P]
        L.or_density_logit.restype = d
        L.or_density_logit.argtypes = [P, d]
        L.or_density_cdf.restype = d
        L.or_density_cdf.argtypes = [P, d]
        L.or_density_median.restype = d
        L.or_density_median.argtypes = [P]
        L.or_pmf_factorized.restype = None
        L.or_pmf_factorized.argtypes = [P, d, P]
        L.or_pmf_gaussian.restype = None
        L.or_pmf_gaussian.argtypes = [d, P]
        L.or_quantize_pmf.restype = None
        L.or_quantize_pmf.argtypes = [P, P]
        L.or_scale_table.restype = None
        L.or_scale_table.argtypes = [P]
        L.or_scale_index.restype = i
        L.or_scale_index.argtypes = [P, d]
        L.or_rans_encode.restype = l
        L.or_rans_encode.argtypes = [P, P, l, P, P, l]
        L.or_rans_decode.restype = i
        L.or_rans_decode.argtypes = [P, l, P, l, P, P]
        L.or_rans_ileave_encode.restype = l
        L.or_rans_ileave_encode.argtypes = [P, P, l, i, P, P, l]
        L.or_rans_ileave_decode.restype = i
        L.or_rans_ileave_decode.argtypes = [P, l, P, l, i, P, P]
        L.or_set_threads.restype = i
        L.or_set_threads.argtypes = [i]
        _lib = L
    return _lib


def set_threads(n: int = 0) -> int:
    """Sets the OpenMP threads of the oracle's loops (0: leave); returns the count."""
    return int(lib().or_set_threads(int(n)))


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------------------
# neural-transform primitives (single image, C x H x W, float64)
# ----------------------------------------------------------------------------
def conv2d(x, w, b, s: int, p: int) -> np.ndarray:
    """Strided convolution with zero padding p; w is [C_out, C_in, k, k]."""
    x, w = _f64(x), _f64(w)
    b = None if b is None else _f64(b)
    C, H, W = x.shape
    Co, Ci, k, _ = w.shape
    assert Ci == C
    Ho = (H + 2 * p - k) // s + 1
    Wo = (W + 2 * p - k) // s + 1
    out = np.empty((Co, Ho, Wo), np.float64)
    lib().or_conv2d(_p(x), C, H, W, _p(w), None if b is None else _p(b), Co, k, s, p, _p(out), Ho, Wo)
    return out


def conv2d_at(x, w, b, s: int, p: int, o: int, i: int, j: int) -> float:
    x, w = _f64(x), _f64(w)
    b = None if b is None else _f64(b)
    C, H, W = x.shape
    return lib().or_conv2d_at(_p(x), C, H, W, _p(w), None if b is None else _p(b), w.shape[2], s, p, o, i, j)


def deconv2d(x, w, b, s: int, p: int, op: int) -> np.ndarray:
    """Transposed convolution; w is [C_in, C_out, k, k]; H_out = (H-1)s - 2p + k + op."""
    x, w = _f64(x), _f64(w)
    b = None if b is None else _f64(b)
    C, H, W = x.shape
    Ci, Co, k, _ = w.shape
    assert Ci == C
    Ho = (H - 1) * s - 2 * p + k + op
    Wo = (W - 1) * s - 2 * p + k + op
    out = np.empty((Co, Ho, Wo), np.float64)
    lib().or_deconv2d(_p(x), C, H, W, _p(w), None if b is None else _p(b), Co, k, s, p, _p(out), Ho, Wo)
    return out


def deconv2d_at(x, w, b, s: int, p: int, o: int, i: int, j: int) -> float:
    x, w = _f64(x), _f64(w)
    b = None if b is None else _f64(b)
    C, H, W = x.shape
    return lib().or_deconv2d_at(_p(x), C, H, W, _p(w), None if b is None else _p(b), w.shape[1], w.shape[2],
                                s, p, o, i, j)


def conv2d_points(x, w, b, s: int, p: int, pts) -> np.ndarray:
    """Every output channel of a convolution at output positions pts [(i, j)]:
    returns [len(pts), C_out].  Each value is the single-output definition."""
    x, w = _f64(x), _f64(w)
    b = None if b is None else _f64(b)
    C, H, W = x.shape
    Co, _, k, _ = w.shape
    ij = np.ascontiguousarray(pts, np.int32).reshape(-1, 2)
    out = np.empty((ij.shape[0], Co), np.float64)
    lib().or_conv2d_points(_p(x), C, H, W, _p(w), None if b is None else _p(b), Co, k, s, p, ij.shape[0],
                           _p(ij), _p(out))
    return out


def deconv2d_points(x, w, b, s: int, p: int, pts) -> np.ndarray:
    """Every output channel of a transposed convolution at output positions pts."""
    x, w = _f64(x), _f64(w)
    b = None if b is None else _f64(b)
    C, H, W = x.shape
    _, Co, k, _ = w.shape
    ij = np.ascontiguousarray(pts, np.int32).reshape(-1, 2)
    out = np.empty((ij.shape[0], Co), np.float64)
    lib().or_deconv2d_points(_p(x), C, H, W, _p(w), None if b is None else _p(b), Co, k, s, p, ij.shape[0],
                             _p(ij), _p(out))
    return out


def gdn(x, beta, gamma, inverse: bool = False) -> np.ndarray:
    """GDN y_i = x_i / sqrt(beta_i + sum_j gamma_ij x_j^2); IGDN multiplies instead."""
    x = _f64(x)
    C = x.shape[0]
    HW = int(np.prod(x.shape[1:]))
    out = np.empty_like(x)
    lib().or_gdn(_p(x), C, HW, _p(_f64(beta)), _p(_f64(gamma)), int(inverse), _p(out))
    return out


def gdn1(x, beta, gamma, inverse: bool = False) -> np.ndarray:
    """1DN (implementation C of Section IV.C; the paper gives no formula):
    y_i = x_i / (beta_i + sum_j gamma_ij |x_j|); the inverse multiplies."""
    x = _f64(x)
    C = x.shape[0]
    HW = int(np.prod(x.shape[1:]))
    out = np.empty_like(x)
    lib().or_gdn1(_p(x), C, HW, _p(_f64(beta)), _p(_f64(gamma)), int(inverse), _p(out))
    return out


def norm(x, beta, gamma, inverse: bool, kind: int) -> np.ndarray:
    """The transforms' normalisation: GDN / IGDN (kind 0) or 1DN (kind 1)."""
    return gdn1(x, beta, gamma, inverse) if kind == 1 else gdn(x, beta, gamma, inverse)


def relu(x):
    return np.maximum(x, 0.0)


# ----------------------------------------------------------------------------
# quantiser and entropy parameters
# ----------------------------------------------------------------------------
def rne(v):
    """Round half to even (numpy's rint under the default rounding mode)."""
    return np.rint(v)


def quantize(v, mu):
    """sym = clamp(rne(v - mu), -64, 64); v_hat = sym + mu.  mu broadcasts per channel."""
    d = np.asarray(v, np.float64) - np.asarray(mu, np.float64)
    sym = np.clip(rne(d), SYM_MIN, SYM_MAX)
    return sym.astype(np.int32), sym + np.asarray(mu, np.float64)


def quantize_f32(v32, mu32):
    """The same decision taken in single precision: rne(float32(v - mu))."""
    d = np.asarray(v32, np.float32) - np.asarray(mu32, np.float32)
    return np.clip(np.rint(d), SYM_MIN, SYM_MAX).astype(np.int32)


def scale_table() -> np.ndarray:
    t = np.empty(64, np.float64)
    lib().or_scale_table(_p(t))
    return t


def scale_index(s, t=None) -> np.ndarray:
    """idx = #{k in [0,62] : t_k < max(s, t_0)} elementwise."""
    t = scale_table() if t is None else t
    s = np.asarray(s, np.float64)
    s = np.maximum(s, t[0])
    return np.sum(t[None, :63] < s.reshape(-1, 1), axis=1).reshape(s.shape).astype(np.int32)


def scales_from_hs(v, hs_out: int) -> np.ndarray:
    """Output activation of h_s: exp (hs_out=1) or ReLU (hs_out=0)."""
    v = np.asarray(v, np.float64)
    return np.exp(v) if hs_out == 1 else np.maximum(v, 0.0)


def scale_index_f32(v32, hs_out: int) -> np.ndarray:
    """The scale-index decision taken in single precision.

    exp output: exp(v) > t_k  <=>  v > ln t_k, so the comparison is made on
    v against float32(ln t_k).  ReLU output: float32(max(v, 0)) against the
    float32 table after the clamp to t_0.
    """
    t = scale_table()
    v = np.asarray(v32, np.float32).reshape(-1, 1)
    if hs_out == 1:
        lt = np.array([math.log(tk) for tk in t[:63]], np.float64).astype(np.float32)
        cnt = np.sum(lt[None, :] < v, axis=1)
    else:
        t32 = t.astype(np.float32)
        s = np.maximum(np.maximum(v, np.float32(0.0)), t32[0])
        cnt = np.sum(t32[None, :63] < s, axis=1)
    return cnt.reshape(np.shape(v32)).astype(np.int32)


def density_logit(prm, x: float) -> float:
    return lib().or_density_logit(_p(_f64(prm)), float(x))


def density_cdf(prm, x: float) -> float:
    return lib().or_density_cdf(_p(_f64(prm)), float(x))


def density_median(prm) -> float:
    return lib().or_density_median(_p(_f64(prm)))


def pmf_factorized(prm, mu: float) -> np.ndarray:
    p = np.empty(NSYM, np.float64)
    lib().or_pmf_factorized(_p(_f64(prm)), float(mu), _p(p))
    return p


def pmf_gaussian(t: float) -> np.ndarray:
    p = np.empty(NSYM, np.float64)
    lib().or_pmf_gaussian(float(t), _p(p))
    return p


def quantize_pmf(p) -> np.ndarray:
    p = _f64(p)
    f = np.empty(NSYM, np.uint32)
    lib().or_quantize_pmf(_p(p), _p(f))
    return f


# ----------------------------------------------------------------------------
# rANS
# ----------------------------------------------------------------------------
def rans_encode(sym, tab, freq) -> bytes:
    """Alphabet indices sym (0..128), table id per symbol, freq [ntab, 129]."""
    sym = np.ascontiguousarray(sym, np.int32).ravel()
    tab = np.ascontiguousarray(tab, np.int32).ravel()
    freq = np.ascontiguousarray(freq, np.uint32)
    n = sym.size
    cap = 4 * n + 64
    out = np.empty(cap, np.uint8)
    ln = lib().or_rans_encode(_p(sym), _p(tab), n, _p(freq), _p(out), cap)
    if ln < 0:
        raise RuntimeError("rANS output overflow")
    return out[:ln].tobytes()


def rans_decode(data: bytes, tab, freq, n: int) -> np.ndarray:
    tab = np.ascontiguousarray(tab, np.int32).ravel()
    freq = np.ascontiguousarray(freq, np.uint32)
    buf = np.frombuffer(data, np.uint8).copy() if len(data) else np.zeros(1, np.uint8)
    sym = np.empty(n, np.int32)
    rc = lib().or_rans_decode(_p(buf), len(data), _p(tab), n, _p(freq), _p(sym))
    if rc != 0:
        raise ValueError("corrupt rANS stream (code %d)" % rc)
    return sym


RANS_LANES = 8       # states of the interleaved coder


def rans_ileave_encode(sym, tab, freq, K: int = RANS_LANES) -> bytes:
    """Interleaved word-wise rANS with K states (symbol i on state i mod K)."""
    sym = np.ascontiguousarray(sym, np.int32).ravel()
    tab = np.ascontiguousarray(tab, np.int32).ravel()
    freq = np.ascontiguousarray(freq, np.uint32)
    n = sym.size
    cap = 4 * n + 4 * K + 64
    out = np.empty(cap, np.uint8)
    ln = lib().or_rans_ileave_encode(_p(sym), _p(tab), n, K, _p(freq), _p(out), cap)
    if ln < 0:
        raise RuntimeError("rANS output overflow")
    return out[:ln].tobytes()


def rans_ileave_decode(data: bytes, tab, freq, n: int, K: int = RANS_LANES) -> np.ndarray:
    tab = np.ascontiguousarray(tab, np.int32).ravel()
    freq = np.ascontiguousarray(freq, np.uint32)
    buf = np.frombuffer(data, np.uint8).copy() if len(data) else np.zeros(1, np.uint8)
    sym = np.empty(n, np.int32)
    rc = lib().or_rans_ileave_decode(_p(buf), len(data), _p(tab), n, K, _p(freq), _p(sym))
    if rc != 0:
        raise ValueError("corrupt rANS stream (code %d)" % rc)
    return sym


def fnv1a32(data: bytes) -> int:
    h = 2166136261
    for byte in data:
        h ^= byte
        h = (h * 16777619) & 0xFFFFFFFF
    return h


# ----------------------------------------------------------------------------
# the codec
# ----------------------------------------------------------------------------
# ----------------------------------------------------------------------------
# context model with checkerboard-parallel prediction (kind 2)
# ----------------------------------------------------------------------------
def checkerboard(Hy: int, Wy: int) -> np.ndarray:
    """Anchor positions of the two-pass order: (r + c) even.  Anchors get
    their entropy parameters from the hyperprior alone; the other half also
    from a context of the anchors."""
    r = np.arange(Hy)[:, None]
    c = np.arange(Wy)[None, :]
    return (r + c) % 2 == 0


def context_mask(k: int = 5) -> np.ndarray:
    """Taps of the k x k context kernel: offsets (dy, dx) with dy + dx odd.
    Seen from a non-anchor these are exactly the anchors of the window."""
    d = np.arange(k) - k // 2
    return (d[:, None] + d[None, :]) % 2 != 0


def context(yhat, w, b) -> np.ndarray:
    """Context of the non-anchors: a k x k convolution (stride 1, zero
    padding k // 2) with the masked kernel over y_hat with every non-anchor
    set to zero, plus bias; zero at the anchors (their context is empty)."""
    yhat = np.asarray(yhat, np.float64)
    C, Hy, Wy = yhat.shape
    A = checkerboard(Hy, Wy)[None]
    k = w.shape[-1]
    wm = np.asarray(w, np.float64) * context_mask(k)[None, None]
    out = conv2d(np.where(A, yhat, 0.0), wm, b, 1, k // 2)
    return np.where(A, 0.0, out)


def conv1x1(x, w, b) -> np.ndarray:
    """1 x 1 convolution: one matrix product over all positions."""
    x = np.asarray(x, np.float64)
    C, H, W = x.shape
    w2 = np.asarray(w, np.float64).reshape(w.shape[0], C)
    return (w2 @ x.reshape(C, H * W)).reshape(-1, H, W) + np.asarray(b, np.float64)[:, None, None]


def entropy_parameters(P, psi, ctx):
    """Mean and pre-activation scale of every latent element from the
    concatenation [psi; ctx]: 1 x 1 layers with ReLU between them.  The
    first M output channels are the means, the last M the scales."""
    h = relu(conv1x1(np.concatenate([psi, ctx]), P["ep0.w"], P["ep0.b"]))
    h = relu(conv1x1(h, P["ep1.w"], P["ep1.b"]))
    out = conv1x1(h, P["ep2.w"], P["ep2.b"])
    M = out.shape[0] // 2
    return out[:M], out[M:]


def checkerboard_take(hwc, part: int) -> np.ndarray:
    """Hy x Wy/2 x C: row by row, the positions of the anchors (part 0) or of
    the other half (part 1) in increasing column order."""
    Hy, Wy = hwc.shape[:2]
    A = checkerboard(Hy, Wy)
    sel = A if part == 0 else ~A
    return np.stack([hwc[r][sel[r]] for r in range(Hy)])


def checkerboard_put(hwc, part: int, vals) -> None:
    """Inverse of checkerboard_take: writes vals into the positions of the set."""
    Hy, Wy = hwc.shape[:2]
    A = checkerboard(Hy, Wy)
    sel = A if part == 0 else ~A
    for r in range(Hy):
        hwc[r][sel[r]] = vals[r]


def pad64(x):
    """Zero-pad a C x H x W image at the bottom and right to multiples of 64."""
    C, H, W = x.shape
    Hp, Wp = 64 * math.ceil(H / 64), 64 * math.ceil(W / 64)
    out = np.zeros((C, Hp, Wp), np.float64)
    out[:, :H, :W] = x
    return out


class Model:
    """Parameters of one codec plus the entropy tables derived from them.

    kind 0 = factorized prior, 1 = scale hyperprior, 2 = mean-scale
    hyperprior with a checkerboard context model.  hs_out selects the
    output activation of h_s (1 = exp, 0 = ReLU); norm the normalisation of
    g_a / g_s (0 = GDN / IGDN, 1 = 1DN and its inverse); lanes the entropy
    coder (0 = byte-wise rANS, K = interleaved word-wise rANS with K states).
    """

    def __init__(self, params, kind: int, N: int, M: int, blob: bytes = b"", hs_out: int = 1, norm: int = 0,
                 lanes: int = 0):
        self.P = {k: np.asarray(v) for k, v in params.items()}
        self.kind, self.N, self.M, self.hs_out, self.norm = kind, N, M, hs_out, norm
        self.lanes = lanes
        self.model_id = fnv1a32(blob) if blob else 0
        dens = self.P["eb.density"]
        # channel offsets: FP64 bisection, rounded to float32
        self.medians = np.array([np.float32(density_median(dens[c])) for c in range(dens.shape[0])],
                                np.float32)
        self.freq_fact = np.stack([quantize_pmf(pmf_factorized(dens[c], float(self.medians[c])))
                                   for c in range(dens.shape[0])])
        self.t = scale_table()
        self.freq_gauss = np.stack([quantize_pmf(pmf_gaussian(self.t[k])) for k in range(64)])

    # ---- transforms (one image, C x H x W) ----
    def g_a(self, x, keep=None):
        P = self.P
        h = x
        for i in range(4):
            h = conv2d(h, P[f"ga{i}.w"], P[f"ga{i}.b"], 2, 2)
            if i < 3:
                h = norm(h, P[f"ga{i}.beta"], P[f"ga{i}.gamma"], False, self.norm)
            if keep is not None:
                keep.append(h)
        return h

    def g_s(self, y, keep=None):
        P = self.P
        h = y
        for i in range(4):
            h = deconv2d(h, P[f"gs{i}.w"], P[f"gs{i}.b"], 2, 2, 1)
            if i < 3:
                h = norm(h, P[f"gs{i}.beta"], P[f"gs{i}.gamma"], True, self.norm)
            if keep is not None:
                keep.append(h)
        return h

    def h_a(self, y, keep=None):
        P = self.P
        # the scale hyperprior sees |y|; the mean-scale model needs the signs
        h = relu(conv2d(np.abs(y) if self.kind == 1 else y, P["ha0.w"], P["ha0.b"], 1, 1))
        if keep is not None: keep.append(h)
        h = relu(conv2d(h, P["ha1.w"], P["ha1.b"], 2, 2))
        if keep is not None: keep.append(h)
        h = conv2d(h, P["ha2.w"], P["ha2.b"], 2, 2)
        if keep is not None: keep.append(h)
        return h

    def h_s(self, zhat, keep=None):
        """Pre-activation output v of h_s; scales = exp(v) or ReLU(v).  For
        the context model (kind 2) the 2M channels psi that feed the
        entropy-parameter layers."""
        P = self.P
        h = relu(deconv2d(zhat, P["hs0.w"], P["hs0.b"], 2, 2, 1))
        if keep is not None: keep.append(h)
        h = relu(deconv2d(h, P["hs1.w"], P["hs1.b"], 2, 2, 1))
        if keep is not None: keep.append(h)
        h = conv2d(h, P["hs2.w"], P["hs2.b"], 1, 1)
        if keep is not None: keep.append(h)
        return h

    # ---- context model (kind 2): the two checkerboard passes ----
    def checkerboard_passes(self, psi, y=None, decode_set=None, keep=None):
        """Entropy parameters, symbols and y_hat of the context model.

        Pass 1 (anchors, (r + c) even): mean and scale from psi alone (zero
        context).  The anchors are then quantised (encoder, from y) or decoded
        (decoder, decode_set(0, idx)), giving y_hat at the anchors.  Pass 2
        (the other half): the context of the anchors' y_hat joins psi.  A
        decoder thus repeats the encoder's computation exactly: pass 1 needs
        only z_hat, pass 2 only z_hat and the anchors.  Returns a dict of
        M x Hy x Wy arrays mu, sraw (pre-activation scale), idx, sym, yhat."""
        P = self.P
        M2, Hy, Wy = psi.shape
        M = M2 // 2
        A = checkerboard(Hy, Wy)[None]
        mu1, s1 = entropy_parameters(P, psi, np.zeros_like(psi))
        idx1 = scale_index(scales_from_hs(s1, self.hs_out), self.t)
        if y is not None:
            sym1, _ = quantize(y, mu1)
        else:
            sym1 = decode_set(0, idx1)
        yhat1 = np.where(A, sym1 + mu1, 0.0)
        ctx = context(yhat1, P["cx.w"], P["cx.b"])
        mu2, s2 = entropy_parameters(P, psi, ctx)
        idx2 = scale_index(scales_from_hs(s2, self.hs_out), self.t)
        if y is not None:
            sym2, _ = quantize(y, mu2)
        else:
            sym2 = decode_set(1, idx2)
        r = {"mu": np.where(A, mu1, mu2), "sraw": np.where(A, s1, s2), "idx": np.where(A, idx1, idx2),
             "sym": np.where(A, sym1, sym2).astype(np.int32), "ctx": ctx}
        r["yhat"] = r["sym"] + r["mu"]
        return r

    def _code_sets(self, sym, idx, S):
        """rANS streams of the anchors, then of the other half: S row slices
        each, positions of the set in raster order, channels fastest."""
        M, Hy, Wy = sym.shape
        out = []
        for part in (0, 1):
            ys = checkerboard_take(np.transpose(sym, (1, 2, 0)), part).reshape(Hy, -1) - SYM_MIN
            yt = checkerboard_take(np.transpose(idx, (1, 2, 0)), part).reshape(Hy, -1)
            out += [self._enc(ys[a:b], yt[a:b], self.freq_gauss) for a, b in self.slice_rows(Hy, S)]
        return out

    # ---- entropy coding helpers (HWC raster, channel fastest) ----
    @staticmethod
    def slice_rows(Hy: int, S: int):
        return [(s * Hy // S, (s + 1) * Hy // S) for s in range(S)]

    def _code_factorized(self, sym_chw):
        C = sym_chw.shape[0]
        hwc = np.transpose(sym_chw, (1, 2, 0))
        tab = np.broadcast_to(np.arange(C, dtype=np.int32), hwc.shape)
        return hwc.ravel() - SYM_MIN, np.ascontiguousarray(tab).ravel()

    def _enc(self, sym, tab, freq):
        if self.lanes:
            return rans_ileave_encode(sym, tab, freq, K=self.lanes)
        return rans_encode(sym, tab, freq)

    def _dec(self, data, tab, freq, n):
        if self.lanes:
            return rans_ileave_decode(data, tab, freq, n, K=self.lanes)
        return rans_decode(data, tab, freq, n)

    # ---- codec ----
    def encode(self, x, S: int = 1, times=None):
        """x: 3 x H x W in [0,1].  Returns (bitstream bytes, intermediates).
        times: optional dict that receives the wall seconds of each stage."""
        T = _Stages(times)
        _, H, W = x.shape
        xp = pad64(np.asarray(x, np.float64))
        inter = {"ga": []}
        with T("g_a"):
            y = self.g_a(xp, inter["ga"])
        inter["y"] = y
        M, Hy, Wy = y.shape
        payloads = []
        if self.kind == 0:
            sym_y, yhat = quantize(y, self.medians[:, None, None])
            inter["sym_y"] = sym_y
            with T("rans_y"):
                syms, tabs = self._code_factorized(sym_y)
                syms = syms.reshape(Hy, Wy * M)
                tabs = tabs.reshape(Hy, Wy * M)
                ys = [self._enc(syms[a:b], tabs[a:b], self.freq_fact) for a, b in self.slice_rows(Hy, S)]
        else:
            inter["ha"] = []
            with T("h_a"):
                z = self.h_a(y, inter["ha"])
            inter["z"] = z
            sym_z, zhat = quantize(z, self.medians[:, None, None])
            inter["sym_z"] = sym_z
            with T("h_s"):
                v = self.h_s(zhat, inter.setdefault("hs", []))
            inter["v"] = v
            if self.kind == 1:
                idx = scale_index(scales_from_hs(v, self.hs_out), self.t)
                sym_y, yhat = quantize(y, 0.0)
            else:
                with T("context"):
                    cp = self.checkerboard_passes(v, y=y)
                inter.update(mu=cp["mu"], sraw=cp["sraw"], ctx=cp["ctx"])
                idx, sym_y, yhat = cp["idx"], cp["sym"], cp["yhat"]
            inter["idx"] = idx
            inter["sym_y"] = sym_y
            with T("rans_z"):
                zs, zt = self._code_factorized(sym_z)
                payloads.append(self._enc(zs, zt, self.freq_fact))
            with T("rans_y"):
                if self.kind == 1:
                    ysym = (np.transpose(sym_y, (1, 2, 0)) - SYM_MIN).reshape(Hy, Wy * M)
                    ytab = np.transpose(idx, (1, 2, 0)).reshape(Hy, Wy * M)
                    ys = [self._enc(ysym[a:b], ytab[a:b], self.freq_gauss) for a, b in self.slice_rows(Hy, S)]
                else:
                    ys = self._code_sets(sym_y, idx, S)
        inter["yhat"] = yhat
        bits = pack_container(self.kind, self.hs_out, S, H, W, self.N, self.M, self.model_id,
                              payloads[0] if self.kind else None, ys, norm=self.norm, lanes=self.lanes)
        return bits, inter

    def decode(self, bits: bytes, keep=None, times=None):
        T = _Stages(times)
        hdr = parse_container(bits)
        if (hdr["model_id"] != self.model_id or hdr["kind"] != self.kind or hdr["norm"] != self.norm
                or hdr["lanes"] != self.lanes):
            raise ValueError("bitstream was made by another model")
        H, W, S = hdr["H"], hdr["W"], hdr["S"]
        Hy, Wy = 4 * math.ceil(H / 64), 4 * math.ceil(W / 64)
        M, N = self.M, self.N
        inter = {} if keep is None else keep
        if self.kind == 0:
            yhat_hwc = np.empty((Hy, Wy, M), np.float64)
            with T("rans_y"):
                for (a, b), data in zip(self.slice_rows(Hy, S), hdr["y"]):
                    tab = np.broadcast_to(np.arange(M, dtype=np.int32), (b - a, Wy, M))
                    sym = self._dec(data, tab, self.freq_fact, (b - a) * Wy * M).reshape(b - a, Wy, M)
                    yhat_hwc[a:b] = sym + SYM_MIN + self.medians[None, None, :].astype(np.float64)
            yhat = np.transpose(yhat_hwc, (2, 0, 1))
        else:
            Hz, Wz = Hy // 4, Wy // 4
            with T("rans_z"):
                tab = np.broadcast_to(np.arange(N, dtype=np.int32), (Hz, Wz, N))
                sz = self._dec(hdr["z"], tab, self.freq_fact, Hz * Wz * N).reshape(Hz, Wz, N) + SYM_MIN
            zhat = np.transpose(sz, (2, 0, 1)) + self.medians[:, None, None].astype(np.float64)
            inter["sym_z"] = np.transpose(sz, (2, 0, 1))
            with T("h_s"):
                v = self.h_s(zhat)
            if self.kind == 1:
                idx = scale_index(scales_from_hs(v, self.hs_out), self.t)
                idx_hwc = np.transpose(idx, (1, 2, 0))
                yhat_hwc = np.empty((Hy, Wy, M), np.float64)
                with T("rans_y"):
                    for (a, b), data in zip(self.slice_rows(Hy, S), hdr["y"]):
                        sym = self._dec(data, idx_hwc[a:b], self.freq_gauss, (b - a) * Wy * M)
                        yhat_hwc[a:b] = sym.reshape(b - a, Wy, M) + SYM_MIN
                yhat = np.transpose(yhat_hwc, (2, 0, 1))
            else:
                def decode_set(part, idx_chw):
                    tab = checkerboard_take(np.transpose(idx_chw, (1, 2, 0)), part)       # Hy x Wy/2 x M
                    got = np.empty(tab.shape, np.int32)
                    for (a, b), data in zip(self.slice_rows(Hy, S), hdr["y"][part * S:(part + 1) * S]):
                        got[a:b] = self._dec(data, tab[a:b], self.freq_gauss, tab[a:b].size).reshape(
                            tab[a:b].shape) + SYM_MIN
                    out = np.zeros((Hy, Wy, M), np.int32)
                    checkerboard_put(out, part, got)
                    return np.transpose(out, (2, 0, 1))

                with T("context"):
                    cp = self.checkerboard_passes(v, decode_set=decode_set)
                idx, yhat = cp["idx"], cp["yhat"]
                inter.update(mu=cp["mu"], sym_y=cp["sym"])
            inter["idx"] = idx
        inter["yhat"] = yhat
        with T("g_s"):
            xr = self.g_s(yhat)
        inter["x_pre"] = xr
        return np.clip(xr, 0.0, 1.0)[:, :H, :W], inter


class _Stages:
    """Accumulates the wall time of named stages into a dict (or does nothing)."""

    def __init__(self, times):
        self.times = times

    def __call__(self, name):
        self.name = name
        return self

    def __enter__(self):
        self.t0 = time.perf_counter()

    def __exit__(self, *exc):
        if self.times is not None:
            self.times[self.name] = self.times.get(self.name, 0.0) + time.perf_counter() - self.t0


# ----------------------------------------------------------------------------
# bitstream container: "LICS", u8 version, u8 kind, u8 flags (bit 0 = exp
# output of h_s, bit 1 = 1DN, bits 2..4 = log2 of the interleaved rANS
# states, 0 for the byte-wise coder), u8 S, u16 H, u16 W, u16 N, u16 M, u32 model id,
# [u32 len_z], S x u32 len_y, payloads z, y_0 .. y_{S-1}; little-endian.
# The context model (kind 2) has 2S y payloads: the S row slices of the
# anchors, then the S row slices of the other half.
# ----------------------------------------------------------------------------
def pack_container(kind, hs_out, S, H, W, N, M, model_id, z, ys, norm: int = 0, lanes: int = 0) -> bytes:
    """flags: bit 0 = exp output of h_s, bit 1 = 1DN instead of GDN, bits 2..4
    = log2(lanes) of the interleaved coder (0 = byte-wise rANS)."""
    lg = 0 if lanes == 0 else int(lanes).bit_length() - 1
    assert lanes == 0 or (lanes == 1 << lg and 1 <= lg <= 5)
    out = bytearray(b"LICS")
    out += struct.pack("<BBBBHHHHI", 1, kind, (hs_out & 1) | ((norm & 1) << 1) | (lg << 2), S, H, W, N, M,
                       model_id)
    assert len(ys) == (2 * S if kind == 2 else S)
    if kind:
        out += struct.pack("<I", len(z))
    out += struct.pack(f"<{len(ys)}I", *[len(y) for y in ys])
    if kind:
        out += z
    for y in ys:
        out += y
    return bytes(out)


def parse_container(bits: bytes) -> dict:
    if len(bits) < 20 or bits[:4] != b"LICS":
        raise ValueError("not a LICS bitstream")
    ver, kind, flags, S, H, W, N, M, mid = struct.unpack_from("<BBBBHHHHI", bits, 4)
    if ver != 1 or kind not in (0, 1, 2) or S < 1 or H == 0 or W == 0 or flags >> 5 or ((flags >> 2) & 7) > 5:
        raise ValueError("bad header")
    pos = 20
    nlen = (2 * S if kind == 2 else S) + (1 if kind else 0)
    if len(bits) < pos + 4 * nlen:
        raise ValueError("truncated header")
    lens = struct.unpack_from(f"<{nlen}I", bits, pos)
    pos += 4 * nlen
    if pos + sum(lens) != len(bits):
        raise ValueError("length mismatch")
    lg = (flags >> 2) & 7
    hdr = {"kind": kind, "hs_out": flags & 1, "norm": (flags >> 1) & 1, "lanes": (1 << lg) if lg else 0, "S": S,
           "H": H, "W": W, "N": N, "M": M, "model_id": mid}
    if kind:
        hdr["z"] = bits[pos:pos + lens[0]]
        pos += lens[0]
        lens = lens[1:]
    ys = []
    for ln in lens:
        ys.append(bits[pos:pos + ln])
        pos += ln
    hdr["y"] = ys
    return hdr


# ----------------------------------------------------------------------------
# distilled synthesis network (a learned stand-in for g_s)
#   T1: transposed conv 5x5 s2 p2 op1, M -> F, ReLU
#   T2: transposed conv 5x5 s2 p2 op1, F -> F, ReLU
#   T3: transposed conv 8x8 s4 p2,     F -> 3
# so a latent of Hy x Wy maps to 16 Hy x 16 Wy pixels, like g_s.
# ----------------------------------------------------------------------------
DISTILL_LAYERS = (("t1", 5, 2, 2, 1), ("t2", 5, 2, 2, 1), ("t3", 8, 4, 2, 0))   # name, k, s, p, output padding


def deconv2d_wgrad(x, dy, k: int, s: int, p: int):
    """Gradients of a transposed convolution's weights [C_in, C_out, k, k]
    and bias for one image x [C_in, H, W] and output gradient dy."""
    x, dy = _f64(x), _f64(dy)
    C, H, W = x.shape
    Co, Ho, Wo = dy.shape
    dw = np.zeros((C, Co, k, k))
    db = np.zeros(Co)
    lib().or_deconv2d_wgrad(_p(x), C, H, W, _p(dy), Co, Ho, Wo, k, s, p, _p(dw), _p(db))
    return dw, db


def deconv2d_dgrad(dy, w, s: int, p: int, H: int, W: int):
    """Gradient of a transposed convolution's input: the strided convolution
    of dy with the same weights read as [C_out = C_in, C_in = C_out, k, k],
    cropped to the input size."""
    g = conv2d(dy, w, None, s, p)
    return g[:, :H, :W]


def distill_forward(P, yhat):
    """yhat [B, M, Hy, Wy] -> (out [B, 3, 16Hy, 16Wy], activations)."""
    outs, acts = [], []
    for n in range(yhat.shape[0]):
        h = _f64(yhat[n])
        a = [h]
        for name, k, s, p, op in DISTILL_LAYERS:
            h = deconv2d(h, P[name + ".w"], P[name + ".b"], s, p, op)
            if name != "t3":
                h = relu(h)
            a.append(h)
        outs.append(h)
        acts.append(a)
    return np.stack(outs), acts


def distill_loss_and_grads(P, yhat, target):
    """MSE over every output element and its gradients (FP64)."""
    out, acts = distill_forward(P, yhat)
    n = out.size
    loss = float(np.mean((out - target) ** 2))
    grads = {k: np.zeros_like(np.asarray(v, np.float64)) for k, v in P.items()}
    for b in range(out.shape[0]):
        g = 2.0 * (out[b] - target[b]) / n
        for li in (2, 1, 0):
            name, k, s, p, op = DISTILL_LAYERS[li]
            x_in = acts[b][li]
            dw, db = deconv2d_wgrad(x_in, g, k, s, p)
            grads[name + ".w"] += dw
            grads[name + ".b"] += db
            if li > 0:
                g = deconv2d_dgrad(g, P[name + ".w"], s, p, x_in.shape[1], x_in.shape[2])
                g = g * (x_in > 0)              # ReLU of the previous layer
    return loss, grads


def adamw_step(w, m, v, g, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, wd=0.01):
    """In place, on float64 arrays; t counts from 1."""
    for a in (w, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(g)
    lib().or_adamw(_p(w), _p(m), _p(v), _p(g), w.size, t, lr, b1, b2, eps, wd)


def psnr(x, xr) -> float:
    mse = float(np.mean((np.asarray(x, np.float64) - np.asarray(xr, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10.0 * math.log10(1.0 / mse)


def bpp(nbytes: int, H: int, W: int) -> float:
    return 8.0 * nbytes / (H * W)
