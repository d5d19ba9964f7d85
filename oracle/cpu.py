"""C/OpenMP build of the FP64 oracle's A-DEF2 loop (``cpu_adef2.c``).

TEST INFRASTRUCTURE ONLY: the CPU baseline of the benchmark and a second CPU
check of the Python oracle.  The restricted system and the orthonormal
restricted basis come from the Python oracle (``restricted_operator``,
``restricted_basis``); the C code runs the coarse setup and the iteration
(Sec. "Online deflated solve (A-DEF2)", App. "CG stopping criterion").
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpu_adef2.c")
LIB = os.path.join(HERE, "libcpu_adef2.so")
# portable x86-64 level (AVX2 + FMA): the library is built on one machine
# and may run on another
CFLAGS = ["-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared"]

_lib = None


def build(force: bool = False) -> str:
    """Compile the shared library with gcc (skipped when up to date)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    res = subprocess.run(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"], capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"gcc failed building {LIB}:\n{res.stdout}{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        lib.cpu_adef2.restype = ctypes.c_int
        lib.cpu_adef2.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int32, P, P, ctypes.c_double,
                                  ctypes.c_int32, ctypes.c_int32, P, P, P, P, P]
        lib.cpu_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().cpu_max_threads())


@dataclass
class CpuResult:
    x: np.ndarray
    iters: int
    converged: bool
    setup_s: float
    solve_s: float
    fallback: bool


def adef2(S_II, b: np.ndarray, Zo: np.ndarray, tol: float, maxit: int = 100000,
          threads: int = 0) -> CpuResult:
    """A-DEF2 on the restricted system S_II (sparse, or an oracle FactoredOp)
    with the orthonormal restricted basis Zo (n_I x k), x0 = 0."""
    lib = _load()
    if not sp.issparse(S_II):
        S_II = S_II.assembled()
    A = sp.csr_matrix(S_II)
    A.sort_indices()
    n = A.shape[0]
    rp = np.ascontiguousarray(A.indptr, dtype=np.int64)
    ci = np.ascontiguousarray(A.indices, dtype=np.int32)
    v = np.ascontiguousarray(A.data, dtype=np.float64)
    k = int(Zo.shape[1])
    Z = np.asfortranarray(Zo, dtype=np.float64)
    bb = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(n)
    it = np.zeros(1, np.int32)
    conv = np.zeros(1, np.int32)
    t = np.zeros(2)
    rc = lib.cpu_adef2(n, rp.ctypes.data, ci.ctypes.data, v.ctypes.data, k,
                       Z.ctypes.data if k else None, bb.ctypes.data, float(tol), int(maxit),
                       int(threads), x.ctypes.data, it.ctypes.data, conv.ctypes.data,
                       t[0:].ctypes.data, t[1:].ctypes.data)
    if rc == -2:
        raise MemoryError("cpu_adef2: allocation failed")
    return CpuResult(x, int(it[0]), bool(conv[0]), float(t[0]), float(t[1]), rc == -1)
