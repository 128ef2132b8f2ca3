"""Oracle: ctypes wrapper of the compiled fast algorithm in ``fast_cpu.c``.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  The C file restates the same
passages as ``operators.fast_apply_H`` (Sec. 1.2 set, Sec. 3.1 direct operation, Sec. 3.2
eq. Horner / Fig. 3 formal insertion, axis N applied first, each term restarted from the
input) for sets too large for NumPy, with OpenMP loops over rows.  It is pinned against
``operators.fast_apply_H`` by ``tests/test_oracle_fast_cpu.py``.

``build()`` compiles ``libfastcpu.so`` next to the source with gcc; ``load()`` builds it
when it is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fast_cpu.c")
LIB = os.path.join(HERE, "libfastcpu.so")
BASIS = {"mono": 0, "cheb": 1, "herm": 2}
_lib = None


def build() -> str:
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", SRC, "-o", tmp, "-lm"],
                   check=True)
    os.replace(tmp, LIB)
    return LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = C.CDLL(LIB)
        lib.fc_set_create.restype = C.c_void_p
        lib.fc_set_create.argtypes = [C.c_int, C.c_int64]
        lib.fc_set_size.restype = C.c_int64
        lib.fc_set_size.argtypes = [C.c_void_p]
        lib.fc_set_multi_indices.argtypes = [C.c_void_p, C.c_void_p]
        lib.fc_set_destroy.argtypes = [C.c_void_p]
        lib.fc_apply_h.restype = C.c_int
        lib.fc_apply_h.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_int, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_int]
        lib.fc_max_threads.restype = C.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return load().fc_max_threads()


class FastSet:
    """K_N(B) in lexicographic order with its neighbour tables (compiled)."""

    def __init__(self, N: int, B: int):
        self.lib = load()
        self.h = self.lib.fc_set_create(int(N), int(B))
        if not self.h:
            raise ValueError("fc_set_create: N or B out of range")
        self.N, self.B = N, B
        self.size = int(self.lib.fc_set_size(self.h))

    def multi_indices(self) -> np.ndarray:
        out = np.empty((self.size, self.N), dtype=np.uint16)
        self.lib.fc_set_multi_indices(self.h, out.ctypes.data)
        return out

    def apply_H(self, pot, v: np.ndarray, threads: int = 0) -> np.ndarray:
        """(D + W^pol(X_K)) v for an ``operators.Potential`` (v in lexicographic order)."""
        v = np.ascontiguousarray(v, dtype=np.complex128)
        assert v.shape == (self.size,)
        deg = np.ascontiguousarray(np.array([a for _, a in pot.terms], dtype=np.uint16).reshape(-1, self.N))
        coef = np.ascontiguousarray(np.array([c for c, _ in pot.terms], dtype=np.float64))
        y = np.empty_like(v)
        st = self.lib.fc_apply_h(self.h, BASIS[pot.basis], float(pot.scale), len(pot.terms), deg.ctypes.data,
                                 coef.ctypes.data, v.ctypes.data, y.ctypes.data, int(threads))
        if st != 0:
            raise ValueError("fc_apply_h: bad arguments")
        return y

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.lib.fc_set_destroy(self.h)
                self.h = None
        except Exception:
            pass
