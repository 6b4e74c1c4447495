"""ctypes binding of the scalar C oracle (cbase.c; test infrastructure only).

``build()`` compiles cbase.c with gcc -O2 (no fast-math) into
liboracle_c.so beside it; ``lib()`` builds it when it is missing or older
than its source and loads it.  The functions take (n, 3) uint8 pixel arrays
and return (n, 3) float64 arrays; ``threads`` > 1 splits the pixels into equal
ranges on a thread pool (ctypes releases the interpreter lock during a call),
so the C code runs on that many cores.
"""
import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cbase.c")
OUT = os.path.join(HERE, "liboracle_c.so")
CFLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-Wall"]

_lib = None


def build():
    tmp = OUT + ".tmp"
    subprocess.check_call(["gcc"] + CFLAGS + ["-o", tmp, SRC, "-lm"])
    os.replace(tmp, OUT)
    return OUT


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(OUT) or os.path.getmtime(OUT) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(OUT)
        u8, f64, i64, i32 = (ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_double), ctypes.c_int64,
                             ctypes.c_int32)
        L.oc_lab_exact_u8.argtypes = [u8, i64, i64, f64]
        L.oc_lab_mact_u8.argtypes = [u8, i64, i64, f64, i32, f64, i32, f64]
        L.oc_lut_build_lab.argtypes = [i32, f64]
        L.oc_lut_tetra_u8.argtypes = [f64, i32, u8, i64, i64, f64]
        for f in (L.oc_lab_exact_u8, L.oc_lab_mact_u8, L.oc_lut_build_lab, L.oc_lut_tetra_u8):
            f.restype = None
        _lib = L
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _ranges(n, threads):
    step = -(-n // max(1, threads))
    return [(s, min(n, s + step)) for s in range(0, n, step)] if n else []


def _run(fn, n, threads):
    parts = _ranges(n, threads)
    if threads <= 1 or len(parts) <= 1:
        for a, b in parts:
            fn(a, b)
        return
    with ThreadPoolExecutor(len(parts)) as ex:
        list(ex.map(lambda ab: fn(*ab), parts))


def _pixels(v8):
    v = np.ascontiguousarray(np.asarray(v8, dtype=np.uint8).reshape(-1, 3))
    return v, np.empty(v.shape, dtype=np.float64)


def lab_exact_u8(v8, threads=1):
    """Exact FP64 RGB -> CIELAB (BT.709, D65) of 8-bit pixels."""
    L = lib()
    v, out = _pixels(v8)
    _run(lambda a, b: L.oc_lab_exact_u8(_ptr(v, ctypes.c_uint8), a, b, _ptr(out, ctypes.c_double)), len(v), threads)
    return out


def lab_mact_u8(v8, p, q, threads=1):
    """RGB -> CIELAB with the cube root replaced by p/q (coefficients in
    increasing degree) above 0.008856, FP64."""
    L = lib()
    v, out = _pixels(v8)
    pc = np.ascontiguousarray(p, dtype=np.float64)
    qc = np.ascontiguousarray(q, dtype=np.float64)
    _run(lambda a, b: L.oc_lab_mact_u8(_ptr(v, ctypes.c_uint8), a, b, _ptr(pc, ctypes.c_double), len(pc) - 1,
                                       _ptr(qc, ctypes.c_double), len(qc) - 1, _ptr(out, ctypes.c_double)),
         len(v), threads)
    return out


def lut_build_lab(N):
    """The packed (N, N, N, 3) FP64 CIELAB LUT."""
    out = np.empty((N, N, N, 3), dtype=np.float64)
    lib().oc_lut_build_lab(int(N), _ptr(out, ctypes.c_double))
    return out


def lut_tetra_u8(lut, v8, threads=1):
    """Tetrahedral interpolation of 8-bit pixels in a packed LUT."""
    L = lib()
    lut = np.ascontiguousarray(lut, dtype=np.float64)
    N = lut.shape[0]
    v, out = _pixels(v8)
    _run(lambda a, b: L.oc_lut_tetra_u8(_ptr(lut, ctypes.c_double), N, _ptr(v, ctypes.c_uint8), a, b,
                                        _ptr(out, ctypes.c_double)), len(v), threads)
    return out
