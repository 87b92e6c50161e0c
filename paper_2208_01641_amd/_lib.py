"""ctypes binding of liblic.so (argument marshalling only).

The library must have been built (``python -m paper_2208_01641_amd.build`` or
``__graft_entry__.build()``).  There is no fallback: if the shared library is
missing or fails to load, importing this module raises.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblic.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("liblic.so is not built: run `python paper_2208_01641_amd/build.py` (HIP library for gfx950)")

# One HIP runtime per process: PyTorch's wheel carries its own HIP runtime,
# which the library's libamdhip64.so.7 dependency resolves to once torch is
# loaded.  Loaded the other way round, the process would hold two runtimes and
# the second to start would find no device.
try:
    import torch  # noqa: F401
except ImportError:
    pass

lib = ctypes.CDLL(LIB_PATH)

c_int, c_long, c_size_t, c_void_p, c_uint32, c_double = (ctypes.c_int, ctypes.c_long, ctypes.c_size_t,
                                                          ctypes.c_void_p, ctypes.c_uint32, ctypes.c_double)


class CodecConfig(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("kind", ctypes.c_int32),
        ("N", ctypes.c_int32),
        ("M", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("hs_out", ctypes.c_int32),
        ("gs_mode", ctypes.c_int32),
        ("y_slices", ctypes.c_int32),
        ("entropy_threads", ctypes.c_int32),
        ("zero_copy", ctypes.c_int32),
        ("max_in_flight", ctypes.c_int32),
        ("max_h", ctypes.c_int32),
        ("max_w", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("hip_device", ctypes.c_int32),
        ("use_graphs", ctypes.c_int32),
        ("norm", ctypes.c_int32),
        ("rans_lanes", ctypes.c_int32),
    ]


class DistillConfig(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("M", ctypes.c_int32),
        ("F", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("max_hy", ctypes.c_int32),
        ("max_wy", ctypes.c_int32),
        ("train", ctypes.c_int32),
        ("lr", ctypes.c_double),
        ("beta1", ctypes.c_double),
        ("beta2", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("weight_decay", ctypes.c_double),
        ("hip_device", ctypes.c_int32),
    ]


class LicResult(ctypes.Structure):
    _fields_ = [
        ("ticket", ctypes.c_uint64),
        ("status", ctypes.c_int32),
        ("stream_id", ctypes.c_int32),
        ("direction", ctypes.c_int32),
        ("H", ctypes.c_int32),
        ("W", ctypes.c_int32),
        ("bytes", ctypes.c_uint64),
        ("latency_ms", ctypes.c_double),
    ]


P = c_void_p
SIGNATURES = {
    "codec_default_config": (None, [P]),
    "codec_create": (c_int, [P, P, c_size_t, P]),
    "codec_encode": (c_int, [P, P, c_int, c_int, c_int, c_int, P, c_size_t, P]),
    "codec_decode": (c_int, [P, P, P, c_int, P, c_size_t, c_int, P, P]),
    "codec_encode_decode": (c_int, [P, P, c_int, c_int, c_int, c_int, P, c_size_t, P, P]),
    "codec_last_latencies": (c_int, [P, P, c_int]),
    "codec_get_stats": (c_int, [P, P, c_size_t]),
    "codec_destroy": (None, [P]),
    "codec_last_error": (ctypes.c_char_p, [P]),
    "codec_run_layer": (c_int, [P, c_int, c_int, c_int, c_int, P, P, P]),
    "codec_run_layer_ex": (c_int, [P, c_int, c_int, c_int, c_int, P, P, P, P, P]),
    "codec_tables": (c_long, [P, c_int, P, c_size_t]),
    "codec_time_layers": (c_int, [P, c_uint32]),
    "codec_layer_kernel": (c_int, [P, c_int, c_int, c_int, P, P]),
    "codec_layer_bytes": (c_int, [P, c_int, c_int, c_int, c_int, P, P, P]),
    "codec_layer_time": (c_int, [P, c_int, P, P]),
    "codec_medians": (c_long, [P, P, c_size_t]),
    "lic_rans_encode": (c_long, [P, P, c_long, P, c_int, P, c_size_t]),
    "lic_rans_decode": (c_int, [P, c_size_t, P, c_long, P, c_int, P]),
    "lic_rans_ileave_encode": (c_long, [c_int, P, P, c_long, P, c_int, P, c_size_t]),
    "lic_rans_ileave_decode": (c_int, [c_int, P, c_size_t, P, c_long, P, c_int, P]),
    "lic_fnv1a": (c_uint32, [P, c_size_t]),
    "lic_blob_tables": (c_long, [P, c_size_t, c_int, P, c_size_t, P, c_size_t]),
    "codec_open_stream": (c_int, [P, c_int, c_int, P]),
    "codec_close_stream": (c_int, [P, c_int]),
    "codec_submit_encode": (c_int, [P, c_int, P, c_int, P, c_size_t, P]),
    "codec_submit_decode": (c_int, [P, c_int, P, c_size_t, P, c_size_t, c_int, P]),
    "codec_poll": (c_int, [P, P, c_int, c_int]),
    "codec_load_distilled": (c_int, [P, P, c_size_t, ctypes.c_float, c_int]),
    "codec_calibrate": (c_int, [P, P, c_int, c_int, c_int, c_int]),
    "codec_fp8_scales": (c_int, [P, P, c_int, P]),
    "lic_distill_default_config": (None, [P]),
    "lic_distill_param_count": (c_size_t, [c_int, c_int]),
    "lic_distill_create": (c_int, [P, P, c_size_t, P]),
    "lic_distill_destroy": (None, [P]),
    "lic_distill_last_error": (ctypes.c_char_p, [P]),
    "lic_distill_forward": (c_int, [P, P, P, c_int, c_int, c_int, P, P, c_int, c_int]),
    "lic_distill_forward_noalloc": (c_int, [P, P, P, c_int, c_int, c_int, P, P, c_int, c_int]),
    "lic_distill_grads": (c_int, [P, P, P, P, c_int, c_int, c_int, P, P]),
    "lic_distill_step": (c_int, [P, P, P, P, c_long, P, c_int, c_int, c_int, P]),
    "lic_distill_sync": (c_int, [P]),
    "lic_distill_get": (c_int, [P, c_int, P, c_size_t]),
    "lic_distill_set": (c_int, [P, c_int, P, c_size_t]),
    "lic_distill_get_step": (c_int, [P, P]),
    "lic_distill_set_step": (c_int, [P, ctypes.c_int64]),
}
for _name, (_res, _args) in SIGNATURES.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args

# status codes (include/lic.h)
LIC_OK, LIC_E_ARG, LIC_E_NOMEM, LIC_E_HIP, LIC_E_CORRUPT, LIC_E_SMALLBUF, LIC_E_BUDGET, LIC_E_STATE, LIC_E_MODEL = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
STATUS_NAMES = {0: "LIC_OK", -1: "LIC_E_ARG", -2: "LIC_E_NOMEM", -3: "LIC_E_HIP", -4: "LIC_E_CORRUPT",
                -5: "LIC_E_SMALLBUF", -6: "LIC_E_BUDGET", -7: "LIC_E_STATE", -8: "LIC_E_MODEL"}
LAYERS = ["GA0", "GA1", "GA2", "GA3", "HA0", "HA1", "HA2", "HS0", "HS1", "HS2", "GS0", "GS1", "GS2", "GS3",
          "CX", "EP0A", "EP1A", "EP2A", "EP0N", "EP1N", "EP2N"]
LAYER_ID = {n: i for i, n in enumerate(LAYERS)}
