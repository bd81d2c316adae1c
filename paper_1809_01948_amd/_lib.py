"""ctypes declarations of the C ABI in include/pbicgstab.h (marshalling only)."""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpbicgstab.so")

FP64, MIXED = 0, 1
PC_NONE, PC_JACOBI, PC_BLOCK_JACOBI_BASE = 0, 1, 256
ST_2D5, ST_3D7, ST_DIA5, CSR = 0, 1, 2, 3

STATUS_NAMES = {
    0: "CONVERGED", 1: "MAXIT", 2: "BREAKDOWN_RHO", 3: "BREAKDOWN_OMEGA", 4: "NONFINITE",
    5: "TRUE_RES_NOT_MET", -1: "ERR_INVALID_ARG", -2: "ERR_HIP", -3: "ERR_ZERO_DIAG",
    -4: "ERR_WORKSPACE_TOO_SMALL", -5: "ERR_UNSUPPORTED",
}

# every exported entry point: name -> (restype, argtypes)
_c = ctypes
_P = _c.c_void_p
SIGNATURES = {
    "pbicgstab_default_opts": (None, [_P]),
    "pbicgstab_workspace_bytes": (_c.c_size_t, [_c.c_int, _c.c_int64, _c.c_int64, _c.c_int32,
                                                _c.c_int, _c.c_int, _c.c_int]),
    "pbicgstab_create_csr": (_c.c_int, [_c.POINTER(_P), _c.c_int64, _c.c_int64, _P, _P, _P,
                                        _c.c_int, _c.c_int, _P, _c.c_size_t, _P]),
    "pbicgstab_create_stencil": (_c.c_int, [_c.POINTER(_P), _c.c_int, _P, _P, _c.c_int, _c.c_int,
                                            _P, _c.c_size_t, _P]),
    "pbicgstab_solve": (_c.c_int, [_P, _P, _P, _P, _P]),
    "pbicgstab_solve_noalloc": (_c.c_int, [_P, _P, _P, _P, _P]),
    "classic_bicgstab_solve": (_c.c_int, [_P, _P, _P, _P, _P]),
    "pbicgstab_apply": (_c.c_int, [_P, _P, _P, _c.c_int, _P]),
    "pbicgstab_grad_values": (_c.c_int, [_P, _P, _P, _P, _P]),
    "pbicgstab_update_values": (_c.c_int, [_P, _P, _c.c_int, _P]),
    "pbicgstab_dia5_assemble_kappa": (_c.c_int, [_P, _P, _c.c_double, _c.c_double, _c.c_double,
                                                 _P]),
    "pbicgstab_dia5_kappa_grad": (_c.c_int, [_P, _P, _P, _P, _P]),
    "pbicgstab_get_vector": (_c.c_int, [_P, _c.c_int, _P, _P]),
    "pbicgstab_time_kernel": (_c.c_int, [_P, _c.c_int, _c.c_int, _c.POINTER(_c.c_double), _P]),
    "pbicgstab_info": (_c.c_int, [_P, _P, _P, _P]),
    "pbicgstab_destroy": (None, [_P]),
    "pbicgstab_last_error": (_c.c_char_p, []),
}


class Opts(ctypes.Structure):
    _fields_ = [
        ("tol", _c.c_double),
        ("maxit", _c.c_int32),
        ("rr_period", _c.c_int32),
        ("rr_tau", _c.c_double),
        ("check_every", _c.c_int32),
        ("transpose", _c.c_int32),
        ("history", _P),
        ("history_len", _c.c_int32),
        ("gap_every", _c.c_int32),
        ("gap_history", _P),
        ("gap_len", _c.c_int32),
        ("use_graph", _c.c_int32),
        ("stream", _P),
        ("rr_auto", _c.c_int32),
        ("rr_eps", _c.c_double),
        ("bound_history", _P),
        ("bound_len", _c.c_int32),
        ("restarts", _c.c_int32),
        ("rhat", _P),
        ("bound_state", _P),
        ("bound_state_len", _c.c_int64),
        ("single_kernel", _c.c_int32),
        ("rr_nv", _c.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("status", _c.c_int32),
        ("iterations", _c.c_int32),
        ("replacements", _c.c_int32),
        ("spmvs", _c.c_int32),
        ("rel_res_recursive", _c.c_double),
        ("rel_res_true", _c.c_double),
        ("elapsed_ms", _c.c_double),
        ("rnorm0", _c.c_double),
        ("bnorm", _c.c_double),
        ("restarts", _c.c_int32),
        ("single_kernel", _c.c_int32),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if not k.startswith("pad")}
        d["status_name"] = STATUS_NAMES.get(self.status, str(self.status))
        return d


_lib = None


def load(path: str = LIB_PATH):
    """Load libpbicgstab.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build the HIP library first "
            "(python -m paper_1809_01948_amd.build); there is no fallback path")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class PbcgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code: int) -> int:
    """Raise on a negative return code (errors); solver outcomes pass through."""
    if code < 0:
        msg = load().pbicgstab_last_error()
        raise PbcgError(code, msg.decode() if msg else "")
    return code
