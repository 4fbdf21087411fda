"""ctypes front end of the C oracle (``nf_oracle.c``).

TEST INFRASTRUCTURE ONLY: the oracle defines what the near-field force is
(Sec. 2.1 cell decomposition with R = 2, Sec. 4.3 Eq. 2 spline softening or
the Plummer law of the same section, Sec. 4.5 FP64 comparison) and is never called by the product path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


class OracleError(RuntimeError):
    pass


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _get():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64, i32, dbl, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
        lib.oracle_cells.argtypes = [i64, vp, i32, dbl, vp, vp]
        lib.oracle_bin.argtypes = [i64, vp, i32, dbl, vp, vp, vp]
        ci = ctypes.c_int
        lib.oracle_accel.argtypes = [i64, vp, i32, dbl, dbl, dbl, ci, ci, i64, vp, vp, vp]
        lib.oracle_jvp.argtypes = [i64, vp, i32, dbl, dbl, dbl, ci, ci, vp, i64, vp, vp]
        lib.oracle_vjp.argtypes = [i64, vp, i32, dbl, dbl, dbl, ci, ci, vp, vp]
        lib.oracle_interactions.argtypes = [i64, vp, i32, dbl, vp]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        for f in ("oracle_cells", "oracle_bin", "oracle_accel", "oracle_jvp",
                  "oracle_vjp", "oracle_interactions"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _pos(pos) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(pos, dtype=np.float64))
    if a.ndim != 2 or a.shape[1] != 3:
        raise ValueError("positions must be an (n, 3) array")
    return a


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


def num_threads() -> int:
    return int(_get().oracle_num_threads())


def set_num_threads(t: int) -> None:
    _get().oracle_set_num_threads(int(t))


def cells(pos, K: int, L: float):
    """(cell[n,3] int64, offset[n,3] float64) in input order."""
    p = _pos(pos)
    n = p.shape[0]
    c = np.empty((n, 3), dtype=np.int64)
    o = np.empty((n, 3), dtype=np.float64)
    _check(_get().oracle_cells(n, _p(p), int(K), float(L), _p(c), _p(o)), "oracle_cells")
    return c, o


def bin_particles(pos, K: int, L: float):
    """(cell_start[K^3+1] int32, order[n] int32, off[n,4] float32)."""
    p = _pos(pos)
    n = p.shape[0]
    cs = np.empty(int(K) ** 3 + 1, dtype=np.int32)
    order = np.empty(n, dtype=np.int32)
    off = np.empty((n, 4), dtype=np.float32)
    _check(_get().oracle_bin(n, _p(p), int(K), float(L), _p(cs), _p(order), _p(off)),
           "oracle_bin")
    return cs, order, off


LAWS = {"spline": 0, "plummer": 1}


def _law(law: str) -> int:
    if law not in LAWS:
        raise ValueError(f"law must be one of {sorted(LAWS)}")
    return LAWS[law]


def accel(pos, K: int, L: float, eps_s: float, gm: float = 1.0, *,
          round_offsets: bool = False, sinks=None, return_count: bool = False,
          law: str = "spline"):
    """FP64 accelerations [n,3] (or [len(sinks),3]) in input order.  ``law``:
    "spline" (Eq. 2, eps_s is the spline radius) or "plummer" (eps_s is the
    Plummer length)."""
    p = _pos(pos)
    n = p.shape[0]
    s = None if sinks is None else np.ascontiguousarray(np.asarray(sinks, dtype=np.int64))
    m = n if s is None else s.shape[0]
    out = np.empty((m, 3), dtype=np.float64)
    cnt = np.zeros(1, dtype=np.int64)
    _check(_get().oracle_accel(n, _p(p), int(K), float(L), float(eps_s), float(gm), _law(law),
                               1 if round_offsets else 0, m, _p(s), _p(out), _p(cnt)),
           "oracle_accel")
    return (out, int(cnt[0])) if return_count else out


def jvp(pos, K: int, L: float, eps_s: float, tvec, gm: float = 1.0, *, sinks=None,
        law: str = "spline", round_offsets: bool = False):
    """Jacobian-vector product (gather form), FP64, binning frozen.
    ``round_offsets``: evaluate on the float-rounded cell offsets (the GPU's
    input representation) instead of the exact double offsets."""
    p = _pos(pos)
    n = p.shape[0]
    t = _pos(tvec)
    s = None if sinks is None else np.ascontiguousarray(np.asarray(sinks, dtype=np.int64))
    m = n if s is None else s.shape[0]
    out = np.empty((m, 3), dtype=np.float64)
    _check(_get().oracle_jvp(n, _p(p), int(K), float(L), float(eps_s), float(gm), _law(law),
                             1 if round_offsets else 0, _p(t), m, _p(s), _p(out)), "oracle_jvp")
    return out


def vjp(pos, K: int, L: float, eps_s: float, v, gm: float = 1.0, *, law: str = "spline",
        round_offsets: bool = False):
    """Vector-Jacobian product (scatter form, written from the chain rule)."""
    p = _pos(pos)
    n = p.shape[0]
    vv = _pos(v)
    out = np.empty((n, 3), dtype=np.float64)
    _check(_get().oracle_vjp(n, _p(p), int(K), float(L), float(eps_s), float(gm), _law(law),
                             1 if round_offsets else 0, _p(vv), _p(out)), "oracle_vjp")
    return out


def interactions(pos, K: int, L: float) -> int:
    p = _pos(pos)
    out = np.zeros(1, dtype=np.int64)
    _check(_get().oracle_interactions(p.shape[0], _p(p), int(K), float(L), _p(out)),
           "oracle_interactions")
    return int(out[0])
