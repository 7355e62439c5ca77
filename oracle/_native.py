"""Build and load the oracle's one C helper (``nnpass.c``) -- test
infrastructure only.

The helper is compiled with gcc into ``oracle/libnnpass.so`` next to its
source (``build()``; ``load()`` builds it when the library is missing or older
than the source).  It shares nothing with the HIP library.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nnpass.c")
LIB = os.path.join(HERE, "libnnpass.so")

_lib = None


def build() -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"gcc failed for {SRC}:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    lib = ctypes.CDLL(LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int64)
    i64 = ctypes.c_int64
    lib.nn_block.argtypes = [dp, i64, i64, dp, dp, i64, i64, dp, ip, dp, ip]
    lib.nn_block.restype = ctypes.c_int
    _lib = lib
    return lib
