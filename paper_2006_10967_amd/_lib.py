"""ctypes declarations of the C ABI in include/pcpf.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PCPF_LIBRARY") or os.path.join(HERE, "libpcpf.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pcpf.h")

(PCPF_OK, PCPF_EINVAL, PCPF_EDEVICE, PCPF_EUNSUPPORTED, PCPF_ESTATE, PCPF_ENONFINITE,
 PCPF_ENOMEM) = range(7)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "EDEVICE", 3: "EUNSUPPORTED", 4: "ESTATE",
                5: "ENONFINITE", 6: "ENOMEM"}
PCPF_FP64, PCPF_FP32, PCPF_BF16 = 0, 1, 2
PCPF_MODE_PHYS, PCPF_MODE_PRECOND = 0, 1
PCPF_NORMAL_PSI, PCPF_NORMAL_PHI = 0, 1
PCPF_REDUCE_MASS, PCPF_REDUCE_L1, PCPF_REDUCE_RMS = 0, 1, 2
PCPF_SGN_PSI0, PCPF_SGN_CURRENT = 0, 1
PCPF_STOP_FIXED, PCPF_STOP_RMS = 0, 1
PCPF_SHAPE_TENSOR, PCPF_SHAPE_TRIANGLE = 0, 1
MAX_ORDER = 6
ABI_VERSION = 2
ADJOINT_STATIC_BYTES = 64 << 20

_dp = ctypes.POINTER(ctypes.c_double)


class PcpfMesh(ctypes.Structure):
    _fields_ = [("ndims", ctypes.c_int32), ("order", ctypes.c_int32), ("nelem", ctypes.c_int64),
                ("nodes", _dp), ("weights", _dp), ("deriv", _dp), ("lminus", _dp),
                ("lplus", _dp), ("cminus", _dp), ("cplus", _dp), ("vinv", _dp),
                ("x0", _dp), ("jac", _dp), ("nbr", ctypes.POINTER(ctypes.c_int32)),
                ("period", ctypes.c_double * 3)]


_u8p = ctypes.POINTER(ctypes.c_uint8)


class PcpfDenseMesh(ctypes.Structure):
    _fields_ = [("ndims", ctypes.c_int32), ("order", ctypes.c_int32), ("shape", ctypes.c_int32),
                ("nupts", ctypes.c_int32), ("nfpts", ctypes.c_int32), ("nelem", ctypes.c_int64),
                ("M0", _dp), ("D", _dp), ("LiftN", _dp), ("Lift", _dp), ("Vinv", _dp),
                ("topmask", _u8p), ("W", _dp), ("ref_fnorm", _dp), ("jinv", _dp),
                ("detj", _dp), ("fnorm", _dp), ("fscale", _dp), ("xorig", _dp), ("jac", _dp),
                ("nbr_slot", ctypes.POINTER(ctypes.c_int32)), ("owner", _u8p),
                ("period", ctypes.c_double * 3)]


class PcpfParams(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("eps", ctypes.c_double), ("eps_w", ctypes.c_double),
                ("tau", ctypes.c_double), ("nu_max", ctypes.c_double), ("s0", ctypes.c_double),
                ("kappa", ctypes.c_double), ("dtau", ctypes.c_double),
                ("delta_n", ctypes.c_double), ("delta_g", ctypes.c_double),
                ("delta_phi", ctypes.c_double), ("vel_amp", ctypes.c_double),
                ("vel_period", ctypes.c_double), ("vel_u0", ctypes.c_double * 3),
                ("vel_kind", ctypes.c_int32), ("reset_mode", ctypes.c_int32),
                ("reset_every", ctypes.c_int32), ("precond_iters", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("normal_mode", ctypes.c_int32),
                ("sgn_mode", ctypes.c_int32), ("stop_mode", ctypes.c_int32)]


class PcpfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"pcpf {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_LIB = None


def header_functions():
    """Names of the functions include/pcpf.h declares."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(pcpf_[a-z_0-9]+)\s*\(", txt)))


def load() -> ctypes.CDLL:
    """Load the in-tree HIP library; raises if it has not been built (there is no
    fallback implementation)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2006_10967_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    sig = {
        "pcpf_abi_version": (ctypes.c_int, []),
        "pcpf_last_error": (ctypes.c_char_p, [vp]),
        "pcpf_line_operators": (st, [i32] + [_dp] * 8),
        "pcpf_solution_coords": (st, [ctypes.POINTER(PcpfMesh), _dp]),
        "pcpf_triangle_operators": (st, [i32] + [_dp] * 7 + [_u8p, _dp, _dp]),
        "pcpf_workspace_bytes": (st, [ctypes.POINTER(PcpfMesh), ctypes.POINTER(PcpfParams),
                                      ctypes.POINTER(ctypes.c_size_t)]),
        "pcpf_create": (st, [ctypes.POINTER(PcpfMesh), ctypes.POINTER(PcpfParams), vp,
                             ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
        "pcpf_workspace_bytes_dense": (st, [ctypes.POINTER(PcpfDenseMesh),
                                            ctypes.POINTER(PcpfParams),
                                            ctypes.POINTER(ctypes.c_size_t)]),
        "pcpf_create_dense": (st, [ctypes.POINTER(PcpfDenseMesh), ctypes.POINTER(PcpfParams), vp,
                                   ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
        "pcpf_destroy": (None, [vp]),
        "pcpf_sizes": (st, [vp, ctypes.POINTER(i64), ctypes.POINTER(i32)]),
        "pcpf_set_state": (st, [vp, vp, vp, dbl, i64]),
        "pcpf_get_state": (st, [vp, vp, vp, ctypes.POINTER(dbl), ctypes.POINTER(i64)]),
        "pcpf_step": (st, [vp, dbl, i64]),
        "pcpf_precondition": (st, [vp, i32]),
        "pcpf_precond_info": (st, [vp, ctypes.POINTER(i32), ctypes.POINTER(dbl)]),
        "pcpf_residual": (st, [vp, vp, vp, dbl, i32, vp, vp]),
        "pcpf_get_sign": (st, [vp, vp]),
        "pcpf_sensor": (st, [vp, vp, vp]),
        "pcpf_reduce": (st, [vp, i32, vp, vp, ctypes.POINTER(dbl)]),
        "pcpf_set_timing": (st, [vp, i32]),
        "pcpf_kernel_times": (st, [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64), i32]),
        "pcpf_set_velocity_amplitude": (st, [vp, dbl]),
        "pcpf_ckpt_bytes": (st, [vp, i64, i64, ctypes.POINTER(ctypes.c_size_t)]),
        "pcpf_forward_ckpt": (st, [vp, dbl, i64, i64, vp, ctypes.c_size_t]),
        "pcpf_adjoint_bytes": (st, [vp, i64, ctypes.POINTER(ctypes.c_size_t)]),
        "pcpf_adjoint": (st, [vp, vp, vp, ctypes.c_size_t, vp, vp, vp, vp, ctypes.POINTER(dbl)]),
        "pcpf_adjoint_static": (st, [vp, vp, vp, vp, vp, vp, ctypes.POINTER(dbl)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.pcpf_abi_version() != ABI_VERSION:
        raise ImportError("libpcpf ABI version mismatch")
    _LIB = lib
    return lib


def check(status: int, ctx=None):
    if status != PCPF_OK:
        lib = load()
        msg = lib.pcpf_last_error(ctx).decode()
        raise PcpfError(status, msg)
