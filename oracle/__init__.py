"""Python handle on the CPU oracle (``oracle.c``) -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never does: it shares no code with the
oracle.  See ``oracle.h`` for what is computed and which passages of the
paper each function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

PLUS_TIMES_I64, MIN_PLUS_F32, PLUS_TIMES_F64, OR_AND_U32 = 0, 1, 2, 3
DTYPE = {PLUS_TIMES_I64: np.int64, MIN_PLUS_F32: np.float32, PLUS_TIMES_F64: np.float64,
         OR_AND_U32: np.uint32}


def build(out_path: str = LIB_PATH, src_dir: str = HERE) -> str:
    """Compile the oracle with gcc: one IEEE rounding per operation, no FMA."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-std=c11", "-Wall", "-Wextra", "-o", out_path, os.path.join(src_dir, "oracle.c"), "-lm"]
    subprocess.run(cmd, check=True)
    return out_path


_lib = None


def lib(path: str = LIB_PATH):
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        build(path)
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    L.orc_apply.restype = ctypes.c_int64
    L.orc_apply.argtypes = [ctypes.c_int, ctypes.c_int32, ctypes.c_int32, P, P, P, P, P, P, P,
                            ctypes.c_int64, P, P, P, P]
    L.orc_spgemm.restype = ctypes.c_int
    L.orc_spgemm.argtypes = [ctypes.c_int, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                             P, P, P, P, P, P, P, ctypes.c_int32, P, P, P, ctypes.c_int]
    L.orc_transpose.restype = ctypes.c_int64
    L.orc_transpose.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int, P, P, P, P, P, P]
    L.orc_axpby.restype = ctypes.c_int64
    L.orc_axpby.argtypes = [ctypes.c_int, ctypes.c_int32, P, P, P, P, P, P, P, P, P, P, P]
    if path == LIB_PATH:
        _lib = L
    return L


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Csr:
    """Sorted CSR (rows sorted by column, unique keys)."""

    def __init__(self, nrows, ncols, row_ptr, col, val):
        self.nrows, self.ncols = int(nrows), int(ncols)
        self.row_ptr = np.ascontiguousarray(row_ptr, np.int64)
        self.col = np.ascontiguousarray(col, np.int32)
        self.val = np.ascontiguousarray(val)

    @property
    def nnz(self):
        return int(self.row_ptr[-1])

    @classmethod
    def of(cls, m):
        return cls(m.nrows, m.ncols, m.row_ptr, m.col, m.val)


def apply(semiring: int, A, rows, cols, vals, ops, L=None):
    """Sequential application of a batch; returns (Csr, changed uint8[nrows])."""
    L = L or lib()
    dt = DTYPE[semiring]
    rows = np.ascontiguousarray(rows, np.int32)
    cols = np.ascontiguousarray(cols, np.int32)
    vals = np.ascontiguousarray(vals, dt)
    ops = np.ascontiguousarray(ops, np.uint8)
    b = rows.size
    cap = A.nnz + b
    orp = np.zeros(A.nrows + 1, np.int64)
    oci = np.zeros(max(cap, 1), np.int32)
    ov = np.zeros(max(cap, 1), dt)
    changed = np.zeros(A.nrows, np.uint8)
    Av = np.ascontiguousarray(A.val, dt)
    nnz = L.orc_apply(semiring, A.nrows, A.ncols, _p(A.row_ptr), _p(A.col), _p(Av), _p(rows),
                      _p(cols), _p(vals), _p(ops), b, _p(orp), _p(oci), _p(ov), _p(changed))
    if nnz < 0:
        raise ValueError("oracle apply: index out of range or unknown op")
    return Csr(A.nrows, A.ncols, orp, oci[:nnz].copy(), ov[:nnz].copy()), changed


def spgemm(semiring: int, A, B, rows=None, nthreads: int = 1, L=None):
    """C = A (x) B (all rows, or the listed rows in list order)."""
    L = L or lib()
    dt = DTYPE[semiring]
    if A.ncols != B.nrows:
        raise ValueError("shape mismatch")
    Av = np.ascontiguousarray(A.val, dt)
    Bv = np.ascontiguousarray(B.val, dt)
    r = None if rows is None else np.ascontiguousarray(rows, np.int32)
    nq = A.nrows if r is None else r.size
    crp = np.zeros(nq + 1, np.int64)
    args = (semiring, A.nrows, A.ncols, B.ncols, _p(A.row_ptr), _p(A.col), _p(Av),
            _p(B.row_ptr), _p(B.col), _p(Bv), _p(r), nq if r is not None else 0)
    if L.orc_spgemm(*args, _p(crp), None, None, nthreads) != 0:
        raise ValueError("oracle spgemm: bad arguments")
    nnz = int(crp[-1])
    cci = np.zeros(max(nnz, 1), np.int32)
    cv = np.zeros(max(nnz, 1), dt)
    if L.orc_spgemm(*args, _p(crp), _p(cci), _p(cv), nthreads) != 0:
        raise ValueError("oracle spgemm: bad arguments")
    return Csr(nq, B.ncols, crp, cci[:nnz], cv[:nnz])


def transpose(A, L=None):
    """A^T (t_ji = a_ij), sorted CSR; values keep their dtype."""
    L = L or lib()
    val = np.ascontiguousarray(A.val)
    vs = val.dtype.itemsize
    trp = np.zeros(A.ncols + 1, np.int64)
    tci = np.zeros(max(A.nnz, 1), np.int32)
    tv = np.zeros(max(A.nnz, 1), val.dtype)
    nnz = L.orc_transpose(A.nrows, A.ncols, vs, _p(A.row_ptr), _p(A.col), _p(val), _p(trp), _p(tci), _p(tv))
    if nnz < 0:
        raise ValueError("oracle transpose: bad arguments")
    return Csr(A.ncols, A.nrows, trp, tci[:nnz].copy(), tv[:nnz].copy())


def axpby(semiring: int, alpha, C, beta, X, L=None):
    """(alpha (x) C) (+) (beta (x) X) entry by entry; X None means empty."""
    L = L or lib()
    dt = DTYPE[semiring]
    if X is None:
        X = Csr(C.nrows, C.ncols, np.zeros(C.nrows + 1, np.int64), np.zeros(0, np.int32), np.zeros(0, dt))
    if (C.nrows, C.ncols) != (X.nrows, X.ncols):
        raise ValueError("shape mismatch")
    a = np.array([alpha], dt)
    b = np.array([beta], dt)
    Cv = np.ascontiguousarray(C.val, dt)
    Xv = np.ascontiguousarray(X.val, dt)
    cap = max(C.nnz + X.nnz, 1)
    drp = np.zeros(C.nrows + 1, np.int64)
    dci = np.zeros(cap, np.int32)
    dv = np.zeros(cap, dt)
    nnz = L.orc_axpby(semiring, C.nrows, _p(a), _p(C.row_ptr), _p(C.col), _p(Cv), _p(b), _p(X.row_ptr),
                      _p(X.col), _p(Xv), _p(drp), _p(dci), _p(dv))
    if nnz < 0:
        raise ValueError("oracle axpby: bad arguments")
    return Csr(C.nrows, C.ncols, drp, dci[:nnz].copy(), dv[:nnz].copy())
