"""ctypes declarations of the C ABI in include/lsp.h (argument marshalling only).

The library is the in-tree liblsp.so built by paper_2102_08518_amd/build.py.
There is no fallback: if it is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblsp.so")

LSP_F32, LSP_F64, LSP_BF16, LSP_F16 = 0, 1, 2, 3

STATUS = {0: "LSP_OK", 1: "LSP_E_INVALID_ARG", 2: "LSP_E_UNSUPPORTED", 3: "LSP_E_DTYPE",
          4: "LSP_E_SHAPE", 5: "LSP_E_WORKSPACE", 6: "LSP_E_HIP", 7: "LSP_E_OOM"}

# Every symbol include/lsp.h declares.
EXPORTS = ("lsp_status_string", "lsp_last_error", "lsp_version", "lsp_set_option", "lsp_spline_create",
           "lsp_spline_load_plugin",
           "lsp_spline_destroy", "lsp_spline_get_info", "lsp_volume_create", "lsp_volume_destroy",
           "lsp_volume_info", "lsp_volume_set_coeffs", "lsp_eval", "lsp_eval_grad",
           "lsp_eval_hessian", "lsp_eval_binned_workspace_size", "lsp_eval_binned",
           "lsp_backward_workspace_size", "lsp_backward", "lsp_backward_dx_from_grad",
           "lsp_batch_plan_create",
           "lsp_batch_plan_info", "lsp_batch_run", "lsp_batch_plan_destroy",
           "lsp_debug_tap_offsets", "lsp_debug_geometry")

LSP_BATCH_AUTOTUNE = 1
LSP_OPT_MFMA = 1
LSP_OPT_PREDICATED = 2
LSP_OPT_SPLIT_MAXN = 3


class LspError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class SplineInfo(ctypes.Structure):
    _fields_ = [("s", ctypes.c_int), ("kind", ctypes.c_int), ("n_cosets", ctypes.c_int),
                ("D", ctypes.c_int * 3), ("shift", (ctypes.c_int * 3) * 4), ("taps", ctypes.c_int),
                ("union_taps", ctypes.c_int), ("n_reference", ctypes.c_int),
                ("degree", ctypes.c_int), ("radius", ctypes.c_int), ("fma_eval", ctypes.c_int),
                ("pad", ctypes.c_int), ("continuity", ctypes.c_int)]


_lock = threading.Lock()
_lib = None

vp = ctypes.c_void_p
i64 = ctypes.c_int64
i32p = ctypes.POINTER(ctypes.c_int32)


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError("liblsp.so not built: run __graft_entry__.build() "
                              "(python -m paper_2102_08518_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "lsp_status_string": (ctypes.c_char_p, [ctypes.c_int]),
            "lsp_last_error": (ctypes.c_char_p, []),
            "lsp_version": (ctypes.c_char_p, []),
            "lsp_set_option": (ctypes.c_int, [ctypes.c_int, ctypes.c_int]),
            "lsp_spline_load_plugin": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(vp)]),
            "lsp_spline_create": (ctypes.c_int, [ctypes.c_int, i32p, i32p, ctypes.c_int,
                                                 ctypes.POINTER(vp)]),
            "lsp_spline_destroy": (None, [vp]),
            "lsp_spline_get_info": (ctypes.c_int, [vp, ctypes.POINTER(SplineInfo)]),
            "lsp_volume_create": (ctypes.c_int, [vp, ctypes.POINTER(i64), ctypes.c_int,
                                                 ctypes.POINTER(vp)]),
            "lsp_volume_destroy": (None, [vp]),
            "lsp_volume_info": (ctypes.c_int, [vp, ctypes.POINTER(SplineInfo), ctypes.POINTER(i64),
                                               ctypes.POINTER(ctypes.c_int)]),
            "lsp_volume_set_coeffs": (ctypes.c_int, [vp, ctypes.POINTER(vp), ctypes.c_int, vp]),
            "lsp_eval": (ctypes.c_int, [vp, vp, ctypes.c_int, i64, vp, vp]),
            "lsp_eval_grad": (ctypes.c_int, [vp, vp, ctypes.c_int, i64, vp, vp, vp]),
            "lsp_eval_hessian": (ctypes.c_int, [vp, vp, ctypes.c_int, i64, vp, vp, vp, vp]),
            "lsp_eval_binned_workspace_size": (ctypes.c_int, [vp, ctypes.c_int, i64,
                                                              ctypes.POINTER(ctypes.c_size_t)]),
            "lsp_eval_binned": (ctypes.c_int, [vp, vp, ctypes.c_int, i64, vp, vp, vp, ctypes.c_size_t,
                                               vp]),
            "lsp_backward_workspace_size": (ctypes.c_int, [vp, i64, ctypes.POINTER(ctypes.c_size_t)]),
            "lsp_backward": (ctypes.c_int, [vp, vp, ctypes.c_int, i64, vp, vp, vp, vp,
                                            ctypes.c_size_t, vp]),
            "lsp_backward_dx_from_grad": (ctypes.c_int, [ctypes.c_int64, vp, vp, vp, vp]),
            "lsp_batch_plan_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                                     ctypes.POINTER(i64), ctypes.POINTER(vp),
                                                     ctypes.POINTER(vp), ctypes.c_int, vp,
                                                     ctypes.POINTER(vp)]),
            "lsp_batch_plan_info": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int),
                                                   ctypes.POINTER(ctypes.c_int),
                                                   ctypes.POINTER(ctypes.c_int)]),
            "lsp_batch_run": (ctypes.c_int, [vp, vp]),
            "lsp_batch_plan_destroy": (None, [vp]),
            "lsp_debug_tap_offsets": (ctypes.c_int, [vp, ctypes.POINTER(i64), ctypes.c_int,
                                                     ctypes.POINTER(ctypes.c_double), i64, i32p,
                                                     i32p]),
            "lsp_debug_geometry": (ctypes.c_int, [vp, ctypes.POINTER(i64), ctypes.c_int, i32p,
                                                  ctypes.POINTER(ctypes.c_size_t)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        return L


def check(status: int) -> None:
    if status != 0:
        raise LspError(status, lib().lsp_last_error().decode(errors="replace"))
