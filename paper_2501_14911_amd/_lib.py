"""ctypes binding of libp2o.so (include/p2o.h).  Argument marshalling only.

Importing this module loads the in-tree shared library and raises
``ImportError`` if it is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_size_t, c_void_p

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libp2o.so")

P2O_FP64, P2O_FP32, P2O_BF16, P2O_FP16 = 0, 1, 2, 3
P2O_SRC_F64, P2O_SRC_F32 = 0, 1
PRECISIONS = {"fp64": P2O_FP64, "fp32": P2O_FP32, "bf16": P2O_BF16, "fp16": P2O_FP16}

STAGES = {"r2c": 0, "gemv_fwd": 1, "gemv_adj": 2, "c2r": 3, "project": 4, "reduce": 5, "load": 6,
          "gemm_fwd": 7, "gemm_adj": 8}
BATCHED = {"auto": 0, "gemv": 1, "mfma": 2}

STATUS = {
    0: "P2O_OK", -1: "P2O_ERR_ARG", -2: "P2O_ERR_STATE", -3: "P2O_ERR_DTYPE",
    -4: "P2O_ERR_STORAGE", -5: "P2O_ERR_NONFINITE", -6: "P2O_ERR_HIP", -7: "P2O_ERR_NO_DEVICE",
}


class P2OError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


def _load():
    # PyTorch ships its own HIP runtime.  Load it first so that libp2o binds to
    # the same runtime (same SONAME) as the device memory and streams torch
    # hands us; loading libp2o first would put a second runtime in the process.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} not found: build the HIP library first "
            "(python paper_2501_14911_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    pv = c_void_p
    sigs = {
        "p2o_create": [POINTER(c_void_p), c_int64, c_int64, c_int64, c_int32, c_int64],
        "p2o_destroy": [pv],
        "p2o_get_layout": [pv, POINTER(c_int64), POINTER(c_int64), POINTER(c_int64), POINTER(c_int64)],
        "p2o_required_bytes": [pv, POINTER(c_size_t), POINTER(c_size_t)],
        "p2o_bind_storage": [pv, pv, c_size_t, pv, c_size_t],
        "p2o_set_stream": [pv, pv],
        "p2o_load_blocks": [pv, pv, c_int64, c_int64, c_int32],
        "p2o_load_finalize": [pv],
        "p2o_apply_F": [pv, pv, pv, c_int64, pv],
        "p2o_apply_F_noalloc": [pv, pv, pv, c_int64, pv],
        "p2o_apply_Ft": [pv, pv, pv, c_int64, pv],
        "p2o_apply_FFt": [pv, pv, pv, c_int64, pv],
        "p2o_misfit_grad": [pv, pv, pv, pv, c_int64, pv, pv, c_int64, pv],
        "p2o_assemble_K": [pv, c_double, pv, c_int64, pv, c_int64, c_int64, c_int64],
        "p2o_gram_accumulate": [pv, c_int64, c_int64, c_int64, c_int64, pv, c_int64, pv],
        "p2o_gram_to_K": [pv, c_int64, c_int64, c_int64, c_double, pv, c_int64, pv],
        "p2o_cholesky": [pv, c_int64, c_int64, pv, pv],
        "p2o_cholesky_solve": [pv, c_int64, c_int64, pv, c_int64, c_int64, pv],
        "p2o_map_point": [pv, c_double, pv, c_int64, pv, c_int64, pv, pv, c_int64],
        "p2o_posterior_cov_apply": [pv, c_double, pv, c_int64, pv, pv, c_int64],
        "p2o_apply_FGt": [pv, pv, pv, pv, c_int64],
        "p2o_d2q_rows": [pv, pv, c_double, pv, c_int64, pv, c_int64, c_int64, c_int64, pv, c_int64],
        "p2o_qoi_posterior_cov": [pv, pv, c_double, pv, c_int64, c_int64, c_int64, pv, c_int64],
        "p2o_d2q_apply": [pv, c_int64, c_int64, c_int64, pv, pv, c_int64, pv],
        "p2o_profile_enable": [pv, c_int32],
        "p2o_set_option": [pv, c_int32, c_int64],
        "p2o_profile_read_nrhs": [pv, c_int32, c_int64, POINTER(c_double), POINTER(c_int64)],
        "p2o_bandwidth_probe": [c_int32, pv, pv, c_size_t, c_int32, pv],
        "p2o_profile_read": [pv, c_int32, POINTER(c_double), POINTER(c_int64)],
        "p2o_gemm_tile_info": [c_int32, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32), POINTER(c_int32)],
        "p2o_autotune": [pv, c_int64, c_int32, POINTER(c_int32), POINTER(c_int32), POINTER(c_double),
                         POINTER(c_double)],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = c_int32
    lib.p2o_status_string.argtypes = [c_int32]
    lib.p2o_status_string.restype = c_char_p
    lib.p2o_last_error.argtypes = []
    lib.p2o_last_error.restype = c_char_p
    return lib


lib = _load()


def check(status: int) -> None:
    if status != 0:
        raise P2OError(status, lib.p2o_last_error().decode(errors="replace"))


def status_name(status: int) -> str:
    return lib.p2o_status_string(status).decode()


def last_error() -> str:
    return lib.p2o_last_error().decode(errors="replace")


__all__ = ["BATCHED", "STAGES", "lib", "check", "P2OError", "PRECISIONS", "P2O_FP64", "P2O_FP32", "P2O_BF16", "P2O_FP16",
           "P2O_SRC_F64", "P2O_SRC_F32", "status_name", "last_error", "LIB_PATH",
           "c_double", "c_int64", "c_size_t", "c_void_p"]
