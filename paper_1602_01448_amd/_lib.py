"""ctypes binding of libsharp.so (argument marshalling only).

torch is imported first so that the library binds to the HIP runtime torch
already loaded; every device computation runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, Structure, c_char_p, c_float, c_int, c_int32, c_longlong, c_size_t, c_void_p

import torch  # noqa: F401  (must precede loading the library: shared HIP runtime)

HERE = os.path.dirname(os.path.abspath(__file__))
# SHARP_LIBRARY selects another build of the same sources (for instance the
# host-sanitizer build the CPU tests make); default: the in-tree library
LIB_PATH = os.environ.get("SHARP_LIBRARY") or os.path.join(HERE, "libsharp.so")

SHARP_OK = 0
STATUS = {
    0: "SHARP_OK", -1: "SHARP_ERR_INVALID_ARG", -2: "SHARP_ERR_UNSUPPORTED_SIZE",
    -3: "SHARP_ERR_POSITION_OUT_OF_RANGE", -4: "SHARP_ERR_NOT_READY",
    -5: "SHARP_ERR_WORKSPACE_TOO_SMALL", -6: "SHARP_ERR_NONFINITE", -7: "SHARP_ERR_HIP",
    -8: "SHARP_ERR_HOST_ALLOC", -9: "SHARP_ERR_SCRATCH_LIMIT",
}
OPS = {"F": 0, "FINV": 1, "Q": 2, "QSTAR": 3, "PA": 4, "PQ": 5, "OBJECT": 6}


class SharpError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        name = STATUS.get(status, str(status))
        msg = lib.sharp_status_string(status).decode() if _lib is not None else name
        super().__init__(f"{where}: {name} ({msg})")


class SharpOptions(Structure):
    _fields_ = [("periodic", c_int), ("probe_every", c_int), ("probe_start", c_int), ("eps_D", c_float),
                ("tile", c_int), ("merge_split", c_int), ("grad_groups", c_int), ("frame_launch", c_int),
                ("fft_block", c_int), ("strip_rows", c_int), ("probe_center", c_int),
                ("reserved", c_int * 1)]


class SharpPlanInfo(Structure):
    _fields_ = [("nx", c_int), ("ny", c_int), ("m", c_int), ("K", c_int), ("periodic", c_int),
                ("tile", c_int), ("tiles_x", c_int), ("tiles_y", c_int), ("merge_split", c_int),
                ("grad_groups", c_int), ("frame_launch", c_int), ("fft_block", c_int), ("strip_rows", c_int),
                ("streaming", c_int), ("csr_nnz", c_longlong),
                ("iteration", c_longlong)]


# (name, restype, argtypes) for every symbol declared in include/sharp.h
SIGNATURES = [
    ("sharp_status_string", c_char_p, [c_int]),
    ("sharp_plan_create", c_int, [POINTER(c_void_p), c_int, c_int, c_int, c_int, POINTER(c_int32),
                                  POINTER(SharpOptions)]),
    ("sharp_plan_destroy", None, [c_void_p]),
    ("sharp_workspace_bytes", c_size_t, [c_void_p]),
    ("sharp_set_workspace", c_int, [c_void_p, c_void_p, c_size_t]),
    ("sharp_set_stream", c_int, [c_void_p, c_void_p]),
    ("sharp_set_data", c_int, [c_void_p, c_void_p]),
    ("sharp_set_probe", c_int, [c_void_p, c_void_p]),
    ("sharp_init_probe", c_int, [c_void_p]),
    ("sharp_set_probe_constraint", c_int, [c_void_p, c_int, c_void_p]),
    ("sharp_set_object", c_int, [c_void_p, c_void_p]),
    ("sharp_raar_iterate", c_int, [c_void_p, c_int, c_float]),
    ("sharp_get_object", c_int, [c_void_p, c_void_p]),
    ("sharp_get_probe", c_int, [c_void_p, c_void_p]),
    ("sharp_get_metrics", c_int, [c_void_p, POINTER(c_float), c_int, POINTER(c_int)]),
    ("sharp_sync", c_int, [c_void_p]),
    ("sharp_grad", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("sharp_simulate", c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    ("sharp_apply", c_int, [c_void_p, c_int, c_void_p, c_void_p]),
    ("sharp_apply_noalloc", c_int, [c_void_p, c_int, c_void_p, c_void_p]),
    ("sharp_state_bytes", c_size_t, [c_void_p]),
    ("sharp_get_state", c_int, [c_void_p, c_void_p]),
    ("sharp_set_state", c_int, [c_void_p, c_void_p]),
    ("sharp_get_plan_info", c_int, [c_void_p, POINTER(SharpPlanInfo)]),
    ("sharp_get_plan_csr", c_int, [c_void_p, POINTER(c_int32), POINTER(c_int32)]),
    ("sharp_timing_enable", c_int, [c_void_p, c_int]),
    ("sharp_timing_read", c_int, [c_void_p, POINTER(ctypes.c_double), POINTER(c_longlong)]),
    ("sharp_batch_create", c_int, [POINTER(c_void_p), c_int, POINTER(c_void_p)]),
    ("sharp_batch_destroy", None, [c_void_p]),
    ("sharp_batch_workspace_bytes", c_size_t, [c_void_p]),
    ("sharp_batch_set_workspace", c_int, [c_void_p, c_void_p, c_size_t]),
    ("sharp_batch_set_stream", c_int, [c_void_p, c_void_p]),
    ("sharp_batch_raar_iterate", c_int, [c_void_p, c_int, c_float]),
    ("sharp_read_reference", c_int, [c_void_p, c_size_t, c_void_p, c_void_p]),
]

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libsharp.so.  Fails loudly when it has not been built: there is
    no fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1602_01448_amd.build` "
                          "(or __graft_entry__.build()); the library has no CPU fallback")
    L = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


class _LazyLib:
    def __getattr__(self, name):
        return getattr(load(), name)


lib = _LazyLib()


def check(status: int, where: str = "") -> None:
    if status != SHARP_OK:
        raise SharpError(status, where)
