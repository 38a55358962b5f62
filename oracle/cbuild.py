"""Build and load the oracle's C interpolation loops (oracle/nufft_c.c) with gcc and OpenMP.

Test infrastructure only, like the rest of ``oracle/``.  The library is built in
place as ``oracle/libnufft_oracle.so``; :func:`load` builds it on first use if it
is missing or older than its source.
"""
from __future__ import annotations

import ctypes as C
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nufft_c.c")
LIB = os.path.join(HERE, "libnufft_oracle.so")

_lib = None


def build() -> str:
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        raise RuntimeError("no C compiler (gcc) for the oracle's interpolation loops")
    tmp = LIB + ".tmp"
    cmd = [cc, "-O2", "-std=gnu99", "-fopenmp", "-fPIC", "-shared", SRC, "-o", tmp, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"building the oracle C library failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    lib = C.CDLL(LIB)
    vp, i64, i32, f64 = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    lib.oracle_bessel_i0.restype = f64
    lib.oracle_bessel_i0.argtypes = [f64]
    lib.oracle_kb.restype = f64
    lib.oracle_kb.argtypes = [f64, i32, f64]
    lib.oracle_taps.restype = None
    lib.oracle_taps.argtypes = [i64, vp, i32, i32, f64, vp, vp, i32]
    lib.oracle_interp_fwd.restype = None
    lib.oracle_interp_fwd.argtypes = [i64, i32, i32, vp, vp, vp, vp, vp, i32]
    lib.oracle_interp_adj.restype = i32
    lib.oracle_interp_adj.argtypes = [i64, i32, i32, vp, vp, vp, vp, vp, i32]
    _lib = lib
    return lib
