"""ctypes binding of libsht.so (the C ABI in include/sht.h).

Argument marshalling only: every step of the transform runs in the library's
HIP kernels.  Loading fails loudly if the library has not been built.
"""

from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsht.so")

SHT_OK = 0
SHT_ERR_INVALID_ARG = -1
SHT_ERR_UNSUPPORTED = -2
SHT_ERR_WORKSPACE = -3
SHT_ERR_ALIGNMENT = -4
SHT_ERR_OOM = -5
SHT_ERR_HIP = -6
SHT_ERR_BUSY = -7
SHT_ERR_NOT_READY = -8

SHT_SAMPLING_MW = 0
SHT_FP64, SHT_FP32, SHT_BF16X3 = 0, 1, 2
SHT_TRI_L_MAX = 512
SHT_MULTI_SEG_MAX = 8
SHT_BATCH_MAX = 64
SHT_L_MAX = 4096
SHT_NOALLOC_SCRATCH_BYTES = 64 << 20

#: every symbol include/sht.h declares
EXPORTS = ("sht_inverse", "sht_inverse_noalloc", "sht_forward", "sht_inverse_multi", "sht_forward_multi", "sht_inverse_real", "sht_forward_real", "sht_forward_triangular",
           "sht_forward_lstsq",
           "sht_spin_pair", "sht_workspace_bytes", "sht_plan_warmup",
           "sht_plan_tables", "sht_graph_create", "sht_graph_launch", "sht_graph_destroy",
           "sht_tile_set", "sht_tune", "sht_error_workspace_bytes", "sht_error_metrics",
           "sht_release_all", "sht_status_string", "sht_version", "sht_last_hip_error",
           "sht_trace_enable", "sht_trace_read")

#: stage ids of sht_trace_read (enum sht_stage)
STAGES = ("layout_in", "contract_inv", "theta_inv", "phi_inv", "phi_fwd", "theta_fwd",
          "contract_fwd", "layout_out")

_lib = None


class ShtError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        lib = load()
        msg = lib.sht_status_string(code).decode()
        if code == SHT_ERR_HIP:
            msg += ": " + lib.sht_last_hip_error().decode()
        super().__init__(f"{where} failed ({code}): {msg}")


def load() -> ctypes.CDLL:
    """Load libsht.so from the package directory (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_0807_4494_amd.build.build() "
                          "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    for name in ("sht_inverse", "sht_forward", "sht_forward_triangular", "sht_forward_lstsq"):
        f = getattr(lib, name)
        f.argtypes = [i, i, i, i, i, vp, vp, vp, sz, vp]
        f.restype = i
    for name in ("sht_inverse_real", "sht_forward_real"):
        f = getattr(lib, name)
        f.argtypes = [i, i, i, i, vp, vp, vp, sz, vp]
        f.restype = i
    for name in ("sht_inverse_multi", "sht_forward_multi"):
        f = getattr(lib, name)
        f.argtypes = [i, i, ctypes.POINTER(i), ctypes.POINTER(i), i, i, vp, vp, vp, sz, vp]
        f.restype = i
    lib.sht_inverse_noalloc.argtypes = [i, i, i, i, i, vp, vp, vp]
    lib.sht_inverse_noalloc.restype = i
    lib.sht_spin_pair.argtypes = [i, i, i, i, vp, vp, vp]
    lib.sht_spin_pair.restype = i
    lib.sht_workspace_bytes.argtypes = [i, i, i, i, i]
    lib.sht_workspace_bytes.restype = sz
    lib.sht_plan_warmup.argtypes = [i, i, i, i, vp]
    lib.sht_plan_warmup.restype = i
    lib.sht_plan_tables.argtypes = [i, i, i, i, vp]
    lib.sht_plan_tables.restype = i
    lib.sht_graph_create.argtypes = [i, i, i, i, i, vp, vp, vp, vp, sz, vp, ctypes.POINTER(vp)]
    lib.sht_graph_create.restype = i
    lib.sht_graph_launch.argtypes = [vp, vp]
    lib.sht_graph_launch.restype = i
    lib.sht_graph_destroy.argtypes = [vp]
    lib.sht_graph_destroy.restype = i
    lib.sht_tile_set.argtypes = [i, i, i, i]
    lib.sht_tile_set.restype = i
    lib.sht_tune.argtypes = [i, i, i, i, vp, sz, vp, ctypes.POINTER(i)]
    lib.sht_tune.restype = i
    lib.sht_error_workspace_bytes.argtypes = []
    lib.sht_error_workspace_bytes.restype = sz
    lib.sht_error_metrics.argtypes = [i, sz, vp, vp, vp, vp, sz, vp]
    lib.sht_error_metrics.restype = i
    lib.sht_release_all.argtypes = []
    lib.sht_release_all.restype = i
    lib.sht_status_string.argtypes = [i]
    lib.sht_status_string.restype = ctypes.c_char_p
    lib.sht_version.argtypes = []
    lib.sht_version.restype = i
    lib.sht_last_hip_error.argtypes = []
    lib.sht_last_hip_error.restype = ctypes.c_char_p
    lib.sht_trace_enable.argtypes = [i]
    lib.sht_trace_enable.restype = i
    lib.sht_trace_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int), i]
    lib.sht_trace_read.restype = i
    _lib = lib
    return lib


def check(code: int, where: str) -> None:
    if code != SHT_OK:
        raise ShtError(code, where)
