"""Python handle over the distilled-synthesis entry points of the C ABI
(marshalling only; the forward, backward and optimizer run in liblic.so)."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import lib
from .codec import LicError, _ptr

PARAM_NAMES = ("t1.w", "t1.b", "t2.w", "t2.b", "t3.w", "t3.b")


def param_shapes(M: int = 192, F: int = 64):
    """Shapes of the parameter arrays, in the order of the flat vector."""
    return {"t1.w": (M, F, 5, 5), "t1.b": (F,), "t2.w": (F, F, 5, 5), "t2.b": (F,), "t3.w": (F, 3, 8, 8),
            "t3.b": (3,)}


def flatten(P: dict, M: int = 192, F: int = 64) -> np.ndarray:
    shapes = param_shapes(M, F)
    parts = []
    for n in PARAM_NAMES:
        a = np.asarray(P[n], np.float32)
        assert a.shape == shapes[n], (n, a.shape)
        parts.append(a.reshape(-1))
    return np.ascontiguousarray(np.concatenate(parts))


def unflatten(v: np.ndarray, M: int = 192, F: int = 64) -> dict:
    out, o = {}, 0
    for n, s in param_shapes(M, F).items():
        k = int(np.prod(s))
        out[n] = np.asarray(v[o:o + k]).reshape(s)
        o += k
    assert o == v.size
    return out


class Distill:
    """The distilled synthesis network: FP32 master parameters, AdamW state
    and device buffers for batches of up to max_batch latents."""

    def __init__(self, params, M: int = 192, F: int = 64, precision: int = 0, max_batch: int = 32, max_hy: int = 16,
                 max_wy: int = 16, train: bool = True, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8, weight_decay: float = 0.01, device: int = 0):
        if isinstance(params, dict):
            params = flatten(params, M, F)
        params = np.ascontiguousarray(params, np.float32)
        cfg = _lib.DistillConfig()
        lib.lic_distill_default_config(ctypes.byref(cfg))
        cfg.M, cfg.F, cfg.precision, cfg.max_batch, cfg.max_hy, cfg.max_wy = M, F, precision, max_batch, max_hy, max_wy
        cfg.train, cfg.lr, cfg.beta1, cfg.beta2, cfg.eps = int(train), lr, beta1, beta2, eps
        cfg.weight_decay, cfg.hip_device = weight_decay, device
        self.cfg, self.M, self.F = cfg, M, F
        self.n_params = int(lib.lic_distill_param_count(M, F))
        h = ctypes.c_void_p()
        rc = lib.lic_distill_create(ctypes.byref(cfg), params.ctypes.data, params.size, ctypes.byref(h))
        self._h = h
        if rc != 0:
            msg = lib.lic_distill_last_error(h).decode()
            self.close()
            raise LicError(rc, msg)

    def close(self):
        if getattr(self, "_h", None):
            lib.lic_distill_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, rc):
        if rc < 0:
            raise LicError(rc, lib.lic_distill_last_error(self._h).decode())
        return rc

    @staticmethod
    def _mu(mu):
        return None if mu is None else _ptr(mu)

    def forward(self, sym, mu=None, pre=None, x_hat=None, H: int = 0, W: int = 0):
        """sym: int8 device tensor [n, hy, wy, M]; pre [n, 3, 16hy, 16wy] and/or
        x_hat [n, 3, H, W] (float32 device tensors) receive the outputs."""
        n, hy, wy, _ = sym.shape
        if x_hat is not None and not H:
            H, W = x_hat.shape[2], x_hat.shape[3]
        self._check(lib.lic_distill_forward(self._h, _ptr(sym), self._mu(mu), n, hy, wy,
                                            None if pre is None else _ptr(pre),
                                            None if x_hat is None else _ptr(x_hat), H, W))

    def forward_noalloc(self, sym, mu=None, pre=None, x_hat=None, H: int = 0, W: int = 0):
        """forward() with the hidden activations in the library's fixed
        per-device workspace (the call allocates no device memory)."""
        n, hy, wy, _ = sym.shape
        if x_hat is not None and not H:
            H, W = x_hat.shape[2], x_hat.shape[3]
        self._check(lib.lic_distill_forward_noalloc(self._h, _ptr(sym), self._mu(mu), n, hy, wy,
                                                    None if pre is None else _ptr(pre),
                                                    None if x_hat is None else _ptr(x_hat), H, W))

    def grads(self, sym, target, mu=None):
        """Loss and parameter gradients (flat float32 vector) without an update."""
        n, hy, wy, _ = sym.shape
        g = np.zeros(self.n_params, np.float32)
        loss = ctypes.c_float()
        self._check(lib.lic_distill_grads(self._h, _ptr(sym), self._mu(mu), _ptr(target), n, hy, wy, g.ctypes.data,
                                          ctypes.byref(loss)))
        return float(loss.value), g

    def step(self, sym_all, target_all, idx, mu=None, loss_out=None):
        """One AdamW step on samples idx of the device-resident data set;
        loss_out: optional float32 device tensor element for the step's loss."""
        idx = np.ascontiguousarray(idx, np.int32)
        _, hy, wy, _ = sym_all.shape
        self._check(lib.lic_distill_step(self._h, _ptr(sym_all), self._mu(mu), _ptr(target_all), sym_all.shape[0],
                                         idx.ctypes.data, idx.size, hy, wy,
                                         None if loss_out is None else _ptr(loss_out)))

    def sync(self):
        self._check(lib.lic_distill_sync(self._h))

    def get(self, what: int = 0) -> np.ndarray:
        """0 parameters, 1 first moments, 2 second moments, 3 last gradients."""
        out = np.zeros(self.n_params, np.float32)
        self._check(lib.lic_distill_get(self._h, what, out.ctypes.data, out.size))
        return out

    def set(self, what: int, values):
        v = np.ascontiguousarray(values, np.float32)
        self._check(lib.lic_distill_set(self._h, what, v.ctypes.data, v.size))

    @property
    def step_count(self) -> int:
        t = ctypes.c_int64()
        self._check(lib.lic_distill_get_step(self._h, ctypes.byref(t)))
        return int(t.value)

    @step_count.setter
    def step_count(self, t: int):
        self._check(lib.lic_distill_set_step(self._h, t))

    def params(self) -> dict:
        return unflatten(self.get(0), self.M, self.F)
