"""Seeded synthetic inputs shared by the FP64 oracle and the HIP codec.

This module only draws random numbers and packs them into arrays and bytes.
It holds none of the codec's arithmetic (no convolution, normalisation,
quantisation, probability model or entropy coding), so that the oracle and
the GPU library can both consume it without sharing any of the method.

Contents
  * image generators with the statistics of the workloads:
      - ``image_1f``      : 1/f-spectrum noise image (factorized-prior case)
      - ``frame_sinusoid``: smooth moving frame, sum of 32 random 2-D
                            sinusoids plus Gaussian noise (hyperprior cases)
      - ``frames_sinusoid_torch``: the same sinusoid field evaluated on a
                            torch device for long frame sequences
  * ``model_params``      : seeded random-init weights of the factorized-prior
                            and scale-hyperprior models (He-normal convs,
                            uniform biases, GDN beta/gamma, raw parameters of
                            the per-channel factorized density)
  * ``weight_blob``       : the "LICW" little-endian container that the C-ABI
                            library reads at create time.
"""
from __future__ import annotations

import math
import struct
from collections import OrderedDict

import numpy as np

IMAGE_SEED = 1641
WEIGHT_SEED = 2208

# Raw parameter count of one channel's factorized density: a 1-3-3-3-1
# network, i.e. matrices 3x1, 3x3, 3x3, 1x3, biases 3,3,3,1, and the three
# non-linearity factors of the hidden layers (3 each).
DENSITY_DIMS = (1, 3, 3, 3, 1)
DENSITY_PARAMS_PER_CHANNEL = 43


# ----------------------------------------------------------------------------
# images
# ----------------------------------------------------------------------------
def image_1f(H: int, W: int, seed: int = IMAGE_SEED) -> np.ndarray:
    """3xHxW float32 image of 1/f-spectrum noise in [0, 1].

    Per channel: white N(0,1) -> FFT -> amplitude x 1/max(f, 1/128) with f the
    radial frequency in cycles per pixel and the DC term set to 0 -> real part
    of the inverse FFT -> standardise -> clamp(0.5 + 0.2 n, 0, 1).
    """
    rng = np.random.default_rng(seed)
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.fftfreq(W)[None, :]
    f = np.sqrt(fx * fx + fy * fy)
    amp = 1.0 / np.maximum(f, 1.0 / 128.0)
    amp[0, 0] = 0.0
    out = np.empty((3, H, W), np.float64)
    for c in range(3):
        white = rng.standard_normal((H, W))
        n = np.real(np.fft.ifft2(np.fft.fft2(white) * amp))
        n = (n - n.mean()) / n.std()
        out[c] = np.clip(0.5 + 0.2 * n, 0.0, 1.0)
    return out.astype(np.float32)


def sinusoid_params(stream: int = 0, seed: int = IMAGE_SEED, n_sin: int = 32) -> dict:
    """Amplitudes, spatial frequencies, phases and motion of one stream."""
    rng = np.random.default_rng([seed, stream])
    return {
        "a": rng.uniform(0.0, 0.05, n_sin),
        "u": rng.uniform(-8.0, 8.0, n_sin),          # cycles across the width
        "v": rng.uniform(-8.0, 8.0, n_sin),          # cycles across the height
        "phi": rng.uniform(0.0, 2.0 * math.pi, (n_sin, 3)),
        "omega": rng.uniform(-0.2, 0.2, n_sin),      # radians per frame
    }


def _sinusoid_factors(H, W, t, p, xp):
    """Row and column factors whose product is the sinusoid field.

    sin(A_j + B_i) = sin A_j cos B_i + cos A_j sin B_i, so each channel is one
    [H x 2K] @ [2K x W] product (an exact rewrite of the sum, not a model).
    """
    i = xp.arange(H, dtype=xp.float64)[:, None]
    j = xp.arange(W, dtype=xp.float64)[:, None]
    B = 2.0 * math.pi * i * xp.asarray(p["v"])[None, :] / H            # H x K
    rows = xp.concatenate([xp.cos(B), xp.sin(B)], axis=1)               # H x 2K
    cols = []
    for c in range(3):
        A = (2.0 * math.pi * j * xp.asarray(p["u"])[None, :] / W
             + xp.asarray(p["phi"][:, c])[None, :] + xp.asarray(p["omega"])[None, :] * t)
        a = xp.asarray(p["a"])[None, :]
        cols.append(xp.concatenate([a * xp.sin(A), a * xp.cos(A)], axis=1).T)  # 2K x W
    return rows, cols


def frame_sinusoid(H: int, W: int, t: int = 0, stream: int = 0,
                   seed: int = IMAGE_SEED, sigma: float = 0.02) -> np.ndarray:
    """3xHxW float32 frame t of a stream: 0.5 + sum of 32 sinusoids + N(0, sigma^2), clamped."""
    p = sinusoid_params(stream, seed)
    rows, cols = _sinusoid_factors(H, W, t, p, np)
    noise_rng = np.random.default_rng([seed, stream, t + 1])
    out = np.empty((3, H, W), np.float64)
    for c in range(3):
        out[c] = 0.5 + rows @ cols[c] + sigma * noise_rng.standard_normal((H, W))
    return np.clip(out, 0.0, 1.0).astype(np.float32)


def frames_sinusoid_torch(H: int, W: int, ts, stream: int = 0, device="cuda",
                          seed: int = IMAGE_SEED, sigma: float = 0.02):
    """len(ts) x 3 x H x W float32 frames evaluated on a torch device.

    The sinusoid field is the one ``frame_sinusoid`` draws; the Gaussian noise
    comes from torch's generator on that device (seeded per stream), so these
    frames are a different noise realisation of the same recipe.
    """
    import torch

    p = sinusoid_params(stream, seed)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed * 1_000_003 + stream)
    out = torch.empty((len(ts), 3, H, W), dtype=torch.float32, device=device)
    for n, t in enumerate(ts):
        rows, cols = _sinusoid_factors(H, W, float(t), p, np)
        r = torch.from_numpy(rows).to(device)
        for c in range(3):
            field = r @ torch.from_numpy(cols[c]).to(device)
            noise = torch.randn((H, W), generator=gen, device=device, dtype=torch.float32)
            out[n, c] = (0.5 + field).float() + sigma * noise
    return out.clamp_(0.0, 1.0)


# ----------------------------------------------------------------------------
# model parameters
# ----------------------------------------------------------------------------
def layer_specs(kind: int, N: int, M: int):
    """(name, op, C_in, C_out, k, post) for every layer, in forward order.

    op is "conv" (weights [C_out, C_in, k, k]) or "deconv" (transposed
    convolution, weights [C_in, C_out, k, k]).  post names what follows the
    layer: "gdn", "igdn", "relu" or "".
    """
    ga = [("ga0", "conv", 3, N, 5, "gdn"), ("ga1", "conv", N, N, 5, "gdn"),
          ("ga2", "conv", N, N, 5, "gdn"), ("ga3", "conv", N, M, 5, "")]
    gs = [("gs0", "deconv", M, N, 5, "igdn"), ("gs1", "deconv", N, N, 5, "igdn"),
          ("gs2", "deconv", N, N, 5, "igdn"), ("gs3", "deconv", N, 3, 5, "")]
    if kind == 0:
        return ga + gs
    ha = [("ha0", "conv", M, N, 3, "relu"), ("ha1", "conv", N, N, 5, "relu"),
          ("ha2", "conv", N, N, 5, "")]
    hs = [("hs0", "deconv", N, N, 5, "relu"), ("hs1", "deconv", N, N, 5, "relu"),
          ("hs2", "conv", N, M if kind == 1 else 2 * M, 3, "")]
    if kind == 1:
        return ga + gs + ha + hs
    # kind 2: context model with checkerboard-parallel prediction; cx is the
    # 5x5 context convolution (its checkerboard mask is applied by the user
    # of the weights, not stored), ep0..ep2 the 1x1 entropy-parameter layers
    E1, E2 = context_widths(M)
    ctx = [("cx", "conv", M, 2 * M, 5, ""), ("ep0", "conv", 4 * M, E1, 1, "relu"),
           ("ep1", "conv", E1, E2, 1, "relu"), ("ep2", "conv", E2, 2 * M, 1, "")]
    return ga + gs + ha + hs + ctx


def context_widths(M: int):
    """Hidden widths of the entropy-parameter layers of the context model:
    about 10 M / 3 and 8 M / 3, in multiples of 32 (640 and 512 for M = 192)."""
    return 32 * round(10 * M / 96), 32 * round(8 * M / 96)


def model_params(kind: int, N: int, M: int, seed: int = WEIGHT_SEED,
                 gamma: str = "diag") -> "OrderedDict[str, np.ndarray]":
    """Seeded random-init parameters.

    * conv / transposed-conv weights: He normal, N(0, 2 / (C_in k^2)) with C_in
      the layer's input channels; biases U(-0.05, 0.05)   (float32)
    * GDN / IGDN: beta = 1; gamma = 0.1 I ("diag") or
      0.1 I + (0.1 / C) U(0,1) ("dense")                   (float32)
    * entropy bottleneck: raw parameters of one 1-3-3-3-1 density per channel
      (C = N for the hyperprior's z, C = M for the factorized prior's y):
      matrices log(expm1(1 / (s d_k))) + 0.1 N(0,1) with s = 2^(1/4) and d_k the
      layer's output width, biases U(-0.5, 0.5), factors 0.5 N(0,1)  (float64)
    """
    rng = np.random.default_rng(seed)
    P: "OrderedDict[str, np.ndarray]" = OrderedDict()
    for name, op, cin, cout, k, post in layer_specs(kind, N, M):
        shape = (cout, cin, k, k) if op == "conv" else (cin, cout, k, k)
        # fan-in of the context convolution: the 12 taps its mask keeps
        std = math.sqrt(2.0 / (cin * (12 if name == "cx" else k * k)))
        P[name + ".w"] = (rng.standard_normal(shape) * std).astype(np.float32)
        P[name + ".b"] = rng.uniform(-0.05, 0.05, cout).astype(np.float32)
        if post in ("gdn", "igdn"):
            P[name + ".beta"] = np.ones(cout, np.float32)
            g = 0.1 * np.eye(cout)
            if gamma == "dense":
                g = g + (0.1 / cout) * rng.uniform(0.0, 1.0, (cout, cout))
            P[name + ".gamma"] = g.astype(np.float32)
    C = M if kind == 0 else N
    P["eb.density"] = density_params(C, rng)
    return P


def density_params(C: int, rng) -> np.ndarray:
    """C x 43 float64 raw density parameters, in the order
    H1(3x1) b1(3) a1(3) H2(3x3) b2(3) a2(3) H3(3x3) b3(3) a3(3) H4(1x3) b4(1)."""
    s = 2.0 ** 0.25
    out = np.empty((C, DENSITY_PARAMS_PER_CHANNEL), np.float64)
    for c in range(C):
        parts = []
        for k in range(4):
            din, dout = DENSITY_DIMS[k], DENSITY_DIMS[k + 1]
            init = math.log(math.expm1(1.0 / (s * dout)))
            parts.append(init + 0.1 * rng.standard_normal(dout * din))
            parts.append(rng.uniform(-0.5, 0.5, dout))
            if k < 3:
                parts.append(0.5 * rng.standard_normal(dout))
        out[c] = np.concatenate(parts)
    return out


def distill_params(M: int = 192, F: int = 64, seed: int = WEIGHT_SEED + 1) -> "OrderedDict[str, np.ndarray]":
    """Initial parameters of the distilled synthesis network (three
    transposed convolutions M -> F -> F -> 3 with kernels 5, 5, 8):
    He-normal weights [C_in, C_out, k, k] and U(-0.05, 0.05) biases."""
    rng = np.random.default_rng(seed)
    P: "OrderedDict[str, np.ndarray]" = OrderedDict()
    for name, cin, cout, k in (("t1", M, F, 5), ("t2", F, F, 5), ("t3", F, 3, 8)):
        std = math.sqrt(2.0 / (cin * k * k))
        P[name + ".w"] = (rng.standard_normal((cin, cout, k, k)) * std).astype(np.float32)
        P[name + ".b"] = rng.uniform(-0.05, 0.05, cout).astype(np.float32)
    return P


def weight_blob(params: "OrderedDict[str, np.ndarray]", kind: int, N: int, M: int) -> bytes:
    """Serialise parameters as the little-endian "LICW" container.

    header: "LICW", u32 version=1, u32 kind, u32 N, u32 M, u32 entry count
    entry : u16 name length, name (ASCII), u8 dtype (0 f32, 1 f64), u8 ndim,
            ndim x u32 dims, then the C-order data.
    """
    out = bytearray(b"LICW")
    out += struct.pack("<5I", 1, kind, N, M, len(params))
    for name, arr in params.items():
        nb = name.encode("ascii")
        if arr.dtype == np.float32:
            code = 0
        elif arr.dtype == np.float64:
            code = 1
        else:
            raise TypeError(f"{name}: unsupported dtype {arr.dtype}")
        out += struct.pack("<H", len(nb)) + nb + struct.pack("<BB", code, arr.ndim)
        out += struct.pack(f"<{arr.ndim}I", *arr.shape)
        out += np.ascontiguousarray(arr).astype(arr.dtype.newbyteorder("<")).tobytes()
    return bytes(out)


def read_blob(blob: bytes):
    """Inverse of ``weight_blob``: (kind, N, M, OrderedDict of arrays)."""
    if blob[:4] != b"LICW":
        raise ValueError("not a LICW blob")
    version, kind, N, M, count = struct.unpack_from("<5I", blob, 4)
    if version != 1:
        raise ValueError("unsupported LICW version")
    pos = 24
    P: "OrderedDict[str, np.ndarray]" = OrderedDict()
    for _ in range(count):
        (ln,) = struct.unpack_from("<H", blob, pos); pos += 2
        name = blob[pos:pos + ln].decode("ascii"); pos += ln
        code, ndim = struct.unpack_from("<BB", blob, pos); pos += 2
        dims = struct.unpack_from(f"<{ndim}I", blob, pos); pos += 4 * ndim
        dt = np.dtype("<f4") if code == 0 else np.dtype("<f8")
        n = int(np.prod(dims)) if ndim else 1
        P[name] = np.frombuffer(blob, dt, n, pos).reshape(dims).copy()
        pos += n * dt.itemsize
    return kind, N, M, P
