"""Build and load the oracle's plain-C operator library (test infrastructure)."""
from __future__ import annotations

import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "projectors.c")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None


def build_oracle(force: bool = True) -> str:
    """Compile projectors.c with gcc (IEEE FP64: no fast-math, no contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


def load_oracle():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build_oracle(force=True)
    lib = ctypes.CDLL(LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    i, d = ctypes.c_int, ctypes.c_double
    lib.oracle_joseph2d.argtypes = [dp, dp, i, i, i, i, i, d, dp, dp, ip]
    lib.oracle_joseph2d_t.argtypes = [dp, dp, i, i, i, i, i, d, dp, dp, ip]
    lib.oracle_pixbp2d.argtypes = [dp, dp, i, i, i, i, i, d, dp, dp]
    lib.oracle_cone_fwd.argtypes = [dp, dp, i, i, i, i, i, i, d, d, dp, dp, dp, dp]
    lib.oracle_cone_bp.argtypes = [dp, dp, i, i, i, i, i, i, d, d, dp, dp, dp, dp]
    lib.oracle_cone_bp_points.argtypes = [dp, ctypes.POINTER(ctypes.c_longlong), dp, i, i, i, i, i, i, i, d, d,
                                          dp, dp, dp, dp]
    lib.oracle_fan_fwd.argtypes = [dp, dp, i, i, i, i, d, dp, dp, dp]
    lib.oracle_fan_bp.argtypes = [dp, dp, i, i, i, i, d, dp, dp, dp]
    for f in (lib.oracle_joseph2d, lib.oracle_joseph2d_t, lib.oracle_pixbp2d,
              lib.oracle_cone_fwd, lib.oracle_cone_bp, lib.oracle_cone_bp_points,
              lib.oracle_fan_fwd, lib.oracle_fan_bp):
        f.restype = None
    _lib = lib
    return lib
