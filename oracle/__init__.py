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
    I32, I64 = ctypes.c_int32, ctypes.c_int64
    L.orc_changed_entries.restype = ctypes.c_int
    L.orc_changed_entries.argtypes = [I32, ctypes.c_int, P, P, P, P, P, P, P, P]
    L.orc_bloom.restype = ctypes.c_int
    L.orc_bloom.argtypes = [I32, I32, P, P, P, P, P, P, P]
    L.orc_pattern.restype = ctypes.c_int
    L.orc_pattern.argtypes = [I32, I32] + [P] * 13
    L.orc_row_filter.restype = ctypes.c_int
    L.orc_row_filter.argtypes = [I32] + [P] * 7
    L.orc_masked_product.restype = ctypes.c_int
    L.orc_masked_product.argtypes = [ctypes.c_int, I32, I32] + [P] * 12
    L.orc_masked_merge.restype = ctypes.c_int
    L.orc_masked_merge.argtypes = [I32, ctypes.c_int] + [P] * 10
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


# ---- general updates filtered by a Bloom matrix (Section 5.2, Algorithm 2) ----

BLOOM_L = 64


def _two_phase(fn, nrows, args_before, dt=None, extra=None):
    """Run a two-phase oracle function: row pointers, then columns (and values)."""
    rp = np.zeros(nrows + 1, np.int64)
    if fn(*args_before, _p(rp), None, *([None] * (extra or 0))) != 0:
        raise ValueError("oracle: bad arguments")
    nnz = int(rp[-1])
    ci = np.zeros(max(nnz, 1), np.int32)
    outs = [np.zeros(max(nnz, 1), d) for d in (dt or [])]
    if fn(*args_before, _p(rp), _p(ci), *[_p(o) for o in outs]) != 0:
        raise ValueError("oracle: bad arguments")
    return rp, ci[:nnz], [o[:nnz] for o in outs]


def changed_entries(A, A2, L=None):
    """Structure of A*: entries present in exactly one of A, A', or in both with
    different value bits (Section 5: deletions count as changed entries)."""
    L = L or lib()
    v, v2 = np.ascontiguousarray(A.val), np.ascontiguousarray(A2.val)
    vs = v.dtype.itemsize
    rp, ci, _ = _two_phase(L.orc_changed_entries, A.nrows,
                           (A.nrows, vs, _p(A.row_ptr), _p(A.col), _p(v), _p(A2.row_ptr), _p(A2.col), _p(v2)))
    return Csr(A.nrows, A.ncols, rp, ci, np.zeros(ci.size, np.uint8))


def bloom(A, B, L=None):
    """F for C = A B: C's structure; bit (k mod 64) of f_ij set iff a_ik and b_kj
    are present (Section 5.2)."""
    L = L or lib()
    if A.ncols != B.nrows:
        raise ValueError("shape mismatch")
    rp, ci, (fv,) = _two_phase(L.orc_bloom, A.nrows,
                               (A.nrows, B.ncols, _p(A.row_ptr), _p(A.col), _p(B.row_ptr), _p(B.col)),
                               dt=[np.uint64], extra=1)
    return Csr(A.nrows, B.ncols, rp, ci, fv)


def general_update(semiring: int, A, A2, B, B2, C, F, L=None):
    """One dynamic multiply with general updates, Algorithm 2 on one process.
    A, B: operands before the batch; A2, B2 after; C = A B and F its Bloom
    matrix.  Returns a dict with C2 (C'), F2 (F'), Cstar (C* with f*_ij as
    values), R (r_i per row), Astar, Bstar (structures)."""
    L = L or lib()
    dt = DTYPE[semiring]
    n, m = A.nrows, B.ncols
    As = changed_entries(A, A2, L)
    Bs = changed_entries(B, B2, L)
    # computePattern
    rp, ci, (fs,) = _two_phase(L.orc_pattern, n,
                               (n, m, _p(A.row_ptr), _p(A.col), _p(As.row_ptr), _p(As.col), _p(A2.row_ptr),
                                _p(A2.col), _p(Bs.row_ptr), _p(Bs.col), _p(B2.row_ptr), _p(B2.col)),
                               dt=[np.uint64], extra=1)
    Cs = Csr(n, m, rp, ci, fs)
    # E, R
    r = np.zeros(max(n, 1), np.uint64)
    fv = np.ascontiguousarray(F.val, np.uint64)
    if L.orc_row_filter(n, _p(Cs.row_ptr), _p(Cs.col), _p(Cs.val), _p(F.row_ptr), _p(F.col), _p(fv), _p(r)) != 0:
        raise ValueError("oracle: bad arguments")
    r = r[:n]
    # Z, H = A^R B' masked at C*
    nz = max(Cs.nnz, 1)
    zv, zp, hv = np.zeros(nz, dt), np.zeros(nz, np.uint8), np.zeros(nz, np.uint64)
    a2v, b2v = np.ascontiguousarray(A2.val, dt), np.ascontiguousarray(B2.val, dt)
    if L.orc_masked_product(semiring, n, m, _p(A2.row_ptr), _p(A2.col), _p(a2v), _p(r), _p(B2.row_ptr),
                            _p(B2.col), _p(b2v), _p(Cs.row_ptr), _p(Cs.col), _p(zv), _p(zp), _p(hv)) != 0:
        raise ValueError("oracle: bad arguments")

    def merge(X, vals, dtype):
        xv = np.ascontiguousarray(X.val, dtype)
        rp2, ci2, (ov,) = _two_phase(L.orc_masked_merge, n,
                                     (n, np.dtype(dtype).itemsize, _p(X.row_ptr), _p(X.col), _p(xv),
                                      _p(Cs.row_ptr), _p(Cs.col), _p(vals), _p(zp)),
                                     dt=[dtype], extra=1)
        return Csr(n, m, rp2, ci2, ov)
    return {"C2": merge(C, zv, dt), "F2": merge(F, hv, np.uint64), "Cstar": Cs, "R": r,
            "Astar": As, "Bstar": Bs, "Z": zv[:Cs.nnz], "Zp": zp[:Cs.nnz], "H": hv[:Cs.nnz]}
