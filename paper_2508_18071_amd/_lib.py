"""ctypes declarations of libevs.so (mirrors include/evs.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation anywhere in this package.
"""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# EVS_LIB_PATH selects another build of the same library (the host-sanitized
# one of the CPU tests); the default is the in-tree libevs.so
LIB_PATH = os.environ.get("EVS_LIB_PATH") or os.path.join(_HERE, "libevs.so")

EVS_OK, EVS_EINVAL, EVS_EUNSUPPORTED, EVS_EWORKSPACE, EVS_EHIP, EVS_EOVERFLOW = range(6)
EVS_FP32, EVS_BF16 = 0, 1
EVS_SURR_SIGMOID, EVS_SURR_ATAN = 0, 1
EVS_INPUT_DIRECT, EVS_INPUT_RGB_LOGDIFF = 0, 1
EVS_OP_FORWARD, EVS_OP_BACKWARD, EVS_OP_EMD, EVS_OP_COMPACT = range(4)
# device status word: EVS_STATUS_WORDS int32 values
EVS_STATUS_WORDS, EVS_STATUS_NAN_X, EVS_STATUS_NAN_GRAD, EVS_STATUS_FLAGS = 4, 0, 1, 2
EVS_FLAG_EVENT_OVERFLOW = 1
EVS_FLAG_X_RANGE = 2
EVS_MAX_LAYERS = 8


class EvsNet(ctypes.Structure):
    _fields_ = [
        ("n_layers", ctypes.c_int32),
        ("ch", ctypes.c_int32 * (EVS_MAX_LAYERS + 1)),
        ("theta", ctypes.c_float),
        ("leak", ctypes.c_float),
        ("surr_alpha", ctypes.c_float),
        ("precision", ctypes.c_int32),
        ("relaxed", ctypes.c_int32),
        ("detach_reset", ctypes.c_int32),
        ("surrogate", ctypes.c_int32),
        ("input", ctypes.c_int32),
        ("lum_scale", ctypes.c_float),
        ("knee", ctypes.c_float),
    ]


class EvsTnet(ctypes.Structure):
    _fields_ = [
        ("hidden", ctypes.c_int32),
        ("theta", ctypes.c_float),
        ("leak", ctypes.c_float),
    ]


class EvsClip(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int32), ("T", ctypes.c_int32), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
        ("x", ctypes.c_void_p),
        ("s_out", ctypes.c_void_p),
        ("s_fp32", ctypes.c_int32),
        ("v_state", ctypes.c_void_p),
        ("h_trace", ctypes.c_void_p),
        ("trace_box", ctypes.c_int32 * 4),
    ]


# (name, restype, argtypes) of every exported entry point
_P = ctypes.c_void_p
_SIGS = [
    ("evs_workspace_bytes", ctypes.c_size_t,
     [ctypes.POINTER(EvsNet), ctypes.POINTER(EvsClip), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    ("evs_packed_weights_bytes", ctypes.c_size_t, [ctypes.POINTER(EvsNet)]),
    ("evs_pack_weights", ctypes.c_int, [ctypes.POINTER(EvsNet), ctypes.POINTER(_P), _P, _P]),
    ("evs_forward", ctypes.c_int,
     [ctypes.POINTER(EvsNet), _P, ctypes.POINTER(EvsClip), ctypes.c_int32, _P, ctypes.c_int32,
      _P, ctypes.c_size_t, _P, _P]),
    ("evs_backward", ctypes.c_int,
     [ctypes.POINTER(EvsNet), _P, ctypes.POINTER(EvsClip), _P, ctypes.c_int32, _P,
      ctypes.POINTER(_P), _P, _P, _P, ctypes.c_size_t, _P, _P]),
    ("evs_emd_loss", ctypes.c_int,
     [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
      ctypes.c_float, _P, _P, _P, ctypes.c_size_t, _P]),
    ("evs_emd_loss_noalloc", ctypes.c_int,
     [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
      ctypes.c_float, _P, _P, _P]),
    ("evs_compact_events", ctypes.c_int,
     [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int64, _P,
      _P, ctypes.c_size_t, _P, _P]),
    ("evs_tnet_weight_floats", ctypes.c_size_t, [_P]),
    ("evs_tnet_forward", ctypes.c_int,
     [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P, _P]),
    ("evs_logdiff", ctypes.c_int,
     [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_float, _P, _P]),
    ("evs_contrast_events", ctypes.c_int,
     [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
      ctypes.c_float, _P, _P]),
    ("evs_autotune", ctypes.c_int,
     [ctypes.POINTER(EvsNet), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
      ctypes.POINTER(ctypes.c_int32), _P]),
    ("evs_tile_count", ctypes.c_int32, [ctypes.POINTER(EvsNet)]),
    ("evs_tile_name", ctypes.c_char_p, [ctypes.POINTER(EvsNet), ctypes.c_int32]),
    ("evs_set_tile", ctypes.c_int, [ctypes.POINTER(EvsNet), ctypes.c_int32]),
    ("evs_graph_begin", ctypes.c_int, [_P]),
    ("evs_graph_end", ctypes.c_int, [_P, ctypes.POINTER(_P)]),
    ("evs_graph_launch", ctypes.c_int, [_P, _P]),
    ("evs_graph_destroy", ctypes.c_int, [_P]),
    ("evs_status_str", ctypes.c_char_p, [ctypes.c_int]),
    ("evs_last_error", ctypes.c_char_p, []),
    ("evs_version", ctypes.c_char_p, []),
]

EXPORTED = [n for n, _, _ in _SIGS]

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class EvsError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        msg = L.evs_last_error().decode(errors="replace")
        super().__init__(f"{where}: {L.evs_status_str(status).decode()} ({status}): {msg}")
        self.status = status


def check(status: int, where: str):
    if status != EVS_OK:
        raise EvsError(status, where)
