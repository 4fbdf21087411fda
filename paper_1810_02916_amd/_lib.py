"""ctypes view of libnf.so (the C ABI in include/nf.h).

There is no fallback: if the library is missing the import of the compute
entry points fails loudly.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnf.so")

NF_OK = 0
NF_EINVAL = 1
NF_EWORKSPACE = 2
NF_EHIP = 3
NF_EUNSUPPORTED = 4

NF_COMPENSATED = 1 << 0
NF_SIMPLE = 1 << 1
NF_PLUMMER = 1 << 2
NF_SPLINE_EVERYWHERE = 1 << 3
NF_SERIAL = 1 << 4
NF_PAIR_SYMMETRIC = 1 << 5

NF_MAX_BOXES = 4096
NF_MAX_ORDER = 8
NF_NOALLOC_SCRATCH_BYTES = 32 << 20

EXPORTED = (
    "nf_version",
    "nf_strerror",
    "nf_last_error",
    "nf_workspace_bytes",
    "nf_bin_particles",
    "nf_accel",
    "nf_accel_noalloc",
    "nf_accel_vjp",
    "nf_plan_items",
    "nf_multipoles",
    "nf_step_stats",
    "nf_step_choose",
    "nf_kick_drift",
)


class NfBox(ctypes.Structure):
    """Mirror of ``struct nf_box``."""
    _fields_ = [
        ("n", ctypes.c_int64),
        ("K", ctypes.c_int32),
        ("dense_min", ctypes.c_int32),
        ("L", ctypes.c_double),
        ("eps_s", ctypes.c_double),
        ("pos", ctypes.c_void_p),
        ("off", ctypes.c_void_p),
        ("cell_start", ctypes.c_void_p),
        ("order", ctypes.c_void_p),
        ("nbad", ctypes.c_void_p),
        ("narrow_max", ctypes.c_int32),
        ("light_window", ctypes.c_int32),
        ("narrow_window", ctypes.c_int32),
        ("flush", ctypes.c_int32),
    ]


class NfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nf error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libnf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -c 'from paper_1810_02916_amd import build; build.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    P = ctypes.POINTER(NfBox)
    lib.nf_version.restype = ctypes.c_int
    lib.nf_strerror.restype = ctypes.c_char_p
    lib.nf_strerror.argtypes = [ctypes.c_int]
    lib.nf_last_error.restype = ctypes.c_char_p
    lib.nf_workspace_bytes.restype = ctypes.c_size_t
    lib.nf_workspace_bytes.argtypes = [ctypes.c_int, P, ctypes.c_uint32]
    lib.nf_bin_particles.restype = ctypes.c_int
    lib.nf_bin_particles.argtypes = [ctypes.c_int, P, vp, ctypes.c_size_t, vp]
    lib.nf_accel.restype = ctypes.c_int
    lib.nf_accel.argtypes = [ctypes.c_int, P, ctypes.c_double, ctypes.c_uint32,
                             ctypes.POINTER(vp), vp, ctypes.c_size_t, vp]
    lib.nf_accel_noalloc.restype = ctypes.c_int
    lib.nf_accel_noalloc.argtypes = [ctypes.c_int, P, ctypes.c_double, ctypes.c_uint32,
                                     ctypes.POINTER(vp), vp]
    lib.nf_accel_vjp.restype = ctypes.c_int
    lib.nf_accel_vjp.argtypes = [ctypes.c_int, P, ctypes.c_double, ctypes.c_uint32,
                                 ctypes.POINTER(vp), ctypes.POINTER(vp), vp, ctypes.c_size_t, vp]
    lib.nf_plan_items.restype = ctypes.c_int
    lib.nf_plan_items.argtypes = [ctypes.c_int, P, vp, ctypes.c_int64, vp, vp, ctypes.c_size_t,
                                  vp]
    PP = ctypes.POINTER(vp)
    lib.nf_step_stats.restype = ctypes.c_int
    lib.nf_step_stats.argtypes = [ctypes.c_int, P, PP, PP, PP, PP, vp, vp, ctypes.c_size_t, vp]
    lib.nf_step_choose.restype = ctypes.c_int
    lib.nf_step_choose.argtypes = [ctypes.c_int, P, PP, PP, vp, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, vp, vp, ctypes.c_size_t, vp]
    lib.nf_kick_drift.restype = ctypes.c_int
    lib.nf_kick_drift.argtypes = [ctypes.c_int, P, PP, PP, PP, ctypes.c_double, ctypes.c_double,
                                  vp, ctypes.c_size_t, vp]
    lib.nf_multipoles.restype = ctypes.c_int
    lib.nf_multipoles.argtypes = [ctypes.c_int, P, ctypes.c_int, ctypes.POINTER(vp), vp,
                                  ctypes.c_size_t, vp]
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != NF_OK:
        lib = load()
        msg = (lib.nf_last_error() or b"").decode() or lib.nf_strerror(rc).decode()
        if rc == NF_EINVAL:
            raise ValueError(f"nf error {rc}: {msg}")
        raise NfError(rc, msg)


def last_error() -> str:
    return (load().nf_last_error() or b"").decode()
