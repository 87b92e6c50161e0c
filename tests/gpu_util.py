"""Shared helpers of the GPU parity tests (device plumbing and comparisons)."""
import math

import numpy as np

import oracle
import synth


def rel_err(got, ref) -> float:
    """max |got - ref| / max |ref| over a tensor."""
    ref = np.asarray(ref, np.float64)
    d = np.max(np.abs(np.asarray(got, np.float64) - ref))
    m = np.max(np.abs(ref))
    return float(d / m) if m > 0 else float(d)


def chw(nhwc, i=0):
    """One image of an NHWC torch tensor as a float64 C x H x W array."""
    return np.transpose(nhwc[i].detach().cpu().numpy().astype(np.float64), (2, 0, 1))


def to_nhwc(chw_arr, device, dtype=None):
    import torch
    a = np.ascontiguousarray(np.transpose(chw_arr, (1, 2, 0)))[None]
    t = torch.from_numpy(a)
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device)


def dims(H, W):
    Hp, Wp = 64 * math.ceil(H / 64), 64 * math.ceil(W / 64)
    return {"Hp": Hp, "Wp": Wp, "Hy": Hp // 16, "Wy": Wp // 16, "Hz": Hp // 64, "Wz": Wp // 64}


def layer_out_shape(layer, H, W, N, M):
    d = dims(H, W)
    Hp, Wp, Hy, Wy, Hz, Wz = d["Hp"], d["Wp"], d["Hy"], d["Wy"], d["Hz"], d["Wz"]
    return {
        "GA0": (Hp // 2, Wp // 2, N), "GA1": (Hp // 4, Wp // 4, N), "GA2": (Hp // 8, Wp // 8, N),
        "GA3": (Hy, Wy, M), "HA0": (Hy, Wy, N), "HA1": (Hy // 2, Wy // 2, N), "HA2": (Hz, Wz, N),
        "HS0": (2 * Hz, 2 * Wz, N), "HS1": (Hy, Wy, N), "HS2": (Hy, Wy, M),
        "GS0": (2 * Hy, 2 * Wy, N), "GS1": (Hp // 4, Wp // 4, N), "GS2": (Hp // 2, Wp // 2, N),
    }[layer]


def make_codec(kind=1, N=128, M=192, gamma="diag", hs_out=1, seed=synth.WEIGHT_SEED, **kw):
    from paper_2208_01641_amd import Codec
    P = synth.model_params(kind, N, M, seed=seed, gamma=gamma)
    blob = synth.weight_blob(P, kind, N, M)
    c = Codec(blob, kind=kind, N=N, M=M, hs_out=hs_out, **kw)
    m = oracle.Model(P, kind, N, M, blob, hs_out=hs_out, norm=kw.get("norm", 0), lanes=kw.get("rans_lanes", 0))
    return c, m


def boundary_mismatches(sym_gpu, v_ref, mu, band=1e-3):
    """Symbols that differ from the FP64 quantiser; each must lie within
    `band` of a rounding boundary of v_ref - mu.  Returns (count, ok)."""
    ref_sym, _ = oracle.quantize(v_ref, mu)
    diff = sym_gpu != ref_sym
    d = np.asarray(v_ref, np.float64) - np.asarray(mu, np.float64)
    near = np.abs(np.abs(d - np.floor(d)) - 0.5) <= band
    return int(diff.sum()), bool(np.all(near[diff]))


def index_mismatches(idx_gpu, s_ref, t, band=1e-4):
    """Scale indices that differ from FP64; each must have s_ref within
    band * t_k of a table boundary t_k."""
    ref = oracle.scale_index(s_ref, t)
    diff = idx_gpu != ref
    s = np.asarray(s_ref, np.float64)[diff]
    k = np.minimum(ref[diff], idx_gpu[diff])       # boundary between the two indices
    near = np.abs(s - t[np.clip(k, 0, 63)]) <= band * t[np.clip(k, 0, 63)]
    return int(diff.sum()), bool(np.all(near))
