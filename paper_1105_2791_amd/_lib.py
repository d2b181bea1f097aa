"""ctypes loader for libmodal.so (the HIP library).  Argument marshalling only.

Importing this module fails loudly when the library has not been built: there
is no CPU fallback anywhere in the package.
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmodal.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "modal.h")

OK, EINVAL, ESHAPE, EDEVICE, ENOTPD, ENOTREADY, EUNSUPPORTED, ENOSPACE = range(8)
NOALLOC_SCRATCH_BYTES = 64 << 20   # MODAL_NOALLOC_SCRATCH_BYTES
CTX_LAMBDA_TABLE = 1              # MODAL_CTX_LAMBDA_TABLE
F64, F32, BF16X3, F16X3 = range(4)
OP_FILTER_MAPS, OP_BETA, OP_LINEAR_ACCUMULATE, OP_LINEAR_APPLY, OP_BETA_VJP, \
    OP_COVARIANCE_SAMPLE, OP_COVARIANCE_FISHER, OP_FNL, OP_LINEAR_FINALIZE, OP_NOISE_VECTORS, OP_FNL_LOWRANK, \
    OP_ALPHA_SEPARABLE, OP_IDEAL_COVARIANCE, OP_POWER_BETA, OP_POWER_ALPHA, OP_POWER_COVARIANCE, \
    OP_POWER_FNL, OP_TRISPECTRUM, OP_FRAME, OP_FNL_FRAME, OP_COVARIANCE_CENTERED, OP_BETA_LOO = range(22)
LIN_RESET, LIN_ACCUMULATE, LIN_FINALIZE, LIN_APPLY = range(4)
COV_SAMPLE, COV_FISHER, COV_SAMPLE_CENTERED = range(3)

STATUS_NAMES = {OK: "OK", EINVAL: "EINVAL", ESHAPE: "ESHAPE", EDEVICE: "EDEVICE", ENOTPD: "ENOTPD",
                ENOTREADY: "ENOTREADY", EUNSUPPORTED: "EUNSUPPORTED", ENOSPACE: "ENOSPACE"}
PREC_NAMES = {"f64": F64, "f32": F32, "bf16x3": BF16X3, "f16x3": F16X3}


class ModalError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None

vp = C.c_void_p
ip = C.c_int
sz = C.c_size_t
dp = C.POINTER(C.c_double)

_SIGS = {
    "modal_ctx_bytes": (sz, [ip, ip, ip, ip, ip, C.c_uint]),
    "modal_create": (ip, [C.POINTER(vp), ip, ip, ip, ip, ip, C.c_uint, vp, vp, vp, vp, sz]),
    "modal_destroy": (None, [vp]),
    "modal_last_error": (C.c_char_p, [vp]),
    "modal_version": (C.c_char_p, []),
    "modal_nalm": (ip, [vp]),
    "modal_nmax": (ip, [vp]),
    "modal_npairs": (ip, [vp]),
    "modal_grid": (ip, [vp, vp, vp]),
    "modal_workspace_size": (ip, [vp, ip, ip, C.POINTER(sz)]),
    "modal_linear_state_size": (sz, [vp]),
    "modal_filter_maps": (ip, [vp, vp, ip, vp, vp, sz, vp]),
    "modal_linear_term": (ip, [vp, ip, vp, ip, vp, vp, vp, sz, vp]),
    "modal_beta": (ip, [vp, vp, ip, vp, vp, vp, sz, vp]),
    "modal_beta_loo": (ip, [vp, vp, ip, vp, vp, vp, sz, vp]),
    "modal_beta_noalloc": (ip, [vp, vp, ip, vp, vp, vp]),
    "modal_beta_vjp": (ip, [vp, vp, ip, vp, vp, vp, vp, sz, vp]),
    "modal_covariance": (ip, [vp, ip, vp, vp, vp, vp, ip, vp, vp, sz, vp]),
    "modal_fnl": (ip, [vp, vp, vp, vp, ip, vp, vp, vp, vp, sz, vp]),
    "modal_profile_enable": (ip, [vp, ip]),
    "modal_cubic_path": (ip, [vp]),
    "modal_cubic_issued_macs": (C.c_double, [vp]),
    "modal_cubic_plan": (ip, [ip, ip, vp, vp, vp, vp]),
    "modal_beta_graph_create": (ip, [ip, vp, vp, vp, vp, vp, vp, vp, vp]),
    "modal_graph_launch": (ip, [vp, vp]),
    "modal_graph_destroy": (None, [vp]),
    "modal_autotune": (ip, [vp, vp, ip, vp, vp, vp, sz, vp, vp, vp]),
    "modal_profile_read": (ip, [vp, vp, vp, ip]),
    "modal_noise_vectors": (ip, [vp, vp, ip, ip, ip, vp, vp, vp, sz, vp]),
    "modal_fnl_lowrank": (ip, [vp, vp, ip, vp, vp, ip, vp, vp, vp, sz, vp]),
    "modal_bivector_rotate": (ip, [vp, vp, vp, ip, vp, vp]),
    "modal_whiten": (ip, [vp, vp, vp, ip, vp, vp]),
    "modal_alpha_separable": (ip, [vp, vp, ip, vp, vp, sz, vp]),
    "modal_ideal_covariance": (ip, [vp, vp, vp, vp, sz, vp]),
    "modal_power_beta": (ip, [vp, vp, ip, vp, vp, vp, sz, vp]),
    "modal_power_alpha": (ip, [vp, vp, vp, vp, sz, vp]),
    "modal_power_ideal_covariance": (ip, [vp, vp, vp, vp, sz, vp]),
    "modal_power_fnl": (ip, [vp, vp, vp, vp, ip, vp, vp, vp, sz, vp]),
    "modal_trispectrum": (ip, [vp, vp, ip, vp, vp, vp, sz, vp]),
    "modal_nquad": (ip, [vp]),
    "modal_frame": (ip, [vp, vp, C.c_double, vp, vp, vp, vp, sz, vp]),
    "modal_frame_rotate": (ip, [vp, ip, vp, vp, vp, ip, vp, vp]),
    "modal_fnl_frame": (ip, [vp, vp, ip, vp, vp, vp, ip, vp, vp, vp, sz, vp]),
}

STAGES = ["legendre", "fft", "cubic", "reduce", "linacc", "adj_pair", "adj_fft", "adj_legendre",
          "covariance", "cholesky", "linear"]


def lib():
    """The loaded library (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libmodal.so not built at {LIB_PATH}; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def header_functions(path: str = HEADER):
    """Names of every function the public header declares."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(modal_[a-z0-9_]+)\s*\(", txt)))
