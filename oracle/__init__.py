"""FP64 CPU oracle for hybrid CSR+BCSR SpMM -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP library never links, loads
or calls anything here, and nothing here imports the HIP library.

Contents
  oracle.c      plain FP64 SpMM, A^T*G by row scatter, SDDMM (C, OpenMP)
  loops_ref.py  CPU restatement of the hybrid format conversion (Alg. 1),
                the row boundary (Eq. 1), the quadratic model fit (Eq. 2)
                and its argmax (Eq. 3), and the per-row-block FP16/BF16
                quantisation with power-of-two scales.

Parity status: every function here is pinned by ``tests/test_oracle.py``
against closed forms, dense products, scipy, invariants, brute force and the
numbers the paper prints (see each test's docstring).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "oracle.c"
_LIB = _HERE / "liboracle.so"
_lib = None


def build(force: bool = False) -> Path:
    """Compile oracle.c with gcc -O2 -fopenmp into oracle/liboracle.so."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp%d" % os.getpid())
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                        str(_SRC), "-o", str(tmp)], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(str(_LIB))
        i64, i32p, f64p, i64p = ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p
        L.oracle_spmm_f64.argtypes = [i64, i64, i64p, i32p, f64p, i64, f64p, i64, f64p, i64, ctypes.c_int]
        L.oracle_spmm_t_f64.argtypes = [i64, i64, i64p, i32p, f64p, i64, f64p, i64, f64p, i64, ctypes.c_int]
        L.oracle_sddmm_f64.argtypes = [i64, i64, i64p, i32p, i64, f64p, i64, f64p, i64, f64p, ctypes.c_int]
        for f in (L.oracle_spmm_f64, L.oracle_spmm_t_f64, L.oracle_sddmm_f64):
            f.restype = ctypes.c_int
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr_arrays(row_ptr, col_idx, vals=None):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.float64)
    return rp, ci, v


def spmm(m, k, row_ptr, col_idx, vals, B, nthreads: int = 0) -> np.ndarray:
    """C = A*B in FP64 (A given as CSR; duplicates and any column order are
    summed as stored)."""
    rp, ci, v = _csr_arrays(row_ptr, col_idx, vals)
    B = np.ascontiguousarray(B, dtype=np.float64)
    n = B.shape[1]
    C = np.empty((m, n), dtype=np.float64)
    rc = lib().oracle_spmm_f64(m, k, _ptr(rp), _ptr(ci), _ptr(v), n, _ptr(B), n, _ptr(C), n, nthreads)
    if rc:
        raise ValueError("oracle_spmm_f64: invalid arguments")
    return C


def spmm_t(m, k, row_ptr, col_idx, vals, G, nthreads: int = 0) -> np.ndarray:
    """dB = A^T * G in FP64 by row scatter."""
    rp, ci, v = _csr_arrays(row_ptr, col_idx, vals)
    G = np.ascontiguousarray(G, dtype=np.float64)
    n = G.shape[1]
    dB = np.empty((k, n), dtype=np.float64)
    rc = lib().oracle_spmm_t_f64(m, k, _ptr(rp), _ptr(ci), _ptr(v), n, _ptr(G), n, _ptr(dB), n, nthreads)
    if rc:
        raise ValueError("oracle_spmm_t_f64: invalid arguments")
    return dB


def sddmm(m, k, row_ptr, col_idx, G, B, nthreads: int = 0) -> np.ndarray:
    """dA[e] = <G[row(e),:], B[col(e),:]> in FP64 for every stored entry."""
    rp, ci, _ = _csr_arrays(row_ptr, col_idx)
    G = np.ascontiguousarray(G, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    n = G.shape[1]
    assert B.shape[1] == n
    dA = np.empty(ci.shape[0], dtype=np.float64)
    rc = lib().oracle_sddmm_f64(m, k, _ptr(rp), _ptr(ci), n, _ptr(G), n, _ptr(B), n, _ptr(dA), nthreads)
    if rc:
        raise ValueError("oracle_sddmm_f64: invalid arguments")
    return dA


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def rel_err(x: np.ndarray, ref: np.ndarray) -> float:
    """Relative Frobenius error ||x - ref|| / ||ref|| (absolute if ref = 0)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    num = float(np.linalg.norm((x - ref).ravel()))
    den = float(np.linalg.norm(ref.ravel()))
    return num / den if den > 0 else num
