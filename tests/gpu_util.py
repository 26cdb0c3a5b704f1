"""Helpers for the GPU parity tests: compare library results with the oracle."""
from __future__ import annotations

import os

import numpy as np

import oracle
from paper_2202_08808_amd import inputs as I

U = 2.0 ** -53
THREADS = max(1, min(16, os.cpu_count() or 1))

# fp64 comparisons of the session: how many were bit for bit, how many needed
# the tolerance, and how many entries passed only through the cancellation
# clause (beyond 1e-12 relative, within the recursive-summation bound)
FP64_TALLY = {"comparisons": 0, "bitwise": 0, "entries": 0, "entries_differing": 0, "cancellation_clause": 0}


def assert_same_csr(sr, got, want, what="", A=None, B=None):
    """Structure bit-exact.  Values bit-exact for int64 and min-plus; for fp64
    either bit-exact or |got - want| <= max(1e-12 |want|, 2 n_ij u sum_k
    |a_ik b_kj|) when the operands are given (the second clause is the
    recursive-summation error bound, for sums that cancel)."""
    assert got.nrows == want.nrows, what
    assert np.array_equal(np.asarray(got.row_ptr), np.asarray(want.row_ptr)), f"{what}: row pointers differ"
    assert np.array_equal(np.asarray(got.col), np.asarray(want.col)), f"{what}: columns differ"
    gv = np.ascontiguousarray(got.val)
    wv = np.ascontiguousarray(want.val)
    if sr == I.PLUS_TIMES_F64:
        FP64_TALLY["comparisons"] += 1
        FP64_TALLY["entries"] += int(wv.size)
    if gv.tobytes() == wv.tobytes():
        if sr == I.PLUS_TIMES_F64:
            FP64_TALLY["bitwise"] += 1
        return
    if sr != I.PLUS_TIMES_F64:
        idx = np.nonzero(gv.view(np.int32 if gv.itemsize == 4 else np.int64) !=
                         wv.view(np.int32 if wv.itemsize == 4 else np.int64))[0][:5]
        raise AssertionError(f"{what}: values differ at {idx}: got {gv[idx]} want {wv[idx]}")
    tol = rel = 1e-12 * np.abs(wv)
    if A is not None and B is not None:
        absA = oracle.Csr(A.nrows, A.ncols, A.row_ptr, A.col, np.abs(A.val))
        absB = oracle.Csr(B.nrows, B.ncols, B.row_ptr, B.col, np.abs(B.val))
        mag = oracle.spgemm(I.PLUS_TIMES_F64, absA, absB, nthreads=THREADS)

        def ones(M):
            return oracle.Csr(M.nrows, M.ncols, M.row_ptr, M.col, np.ones(M.col.size))
        cnt = oracle.spgemm(I.PLUS_TIMES_F64, ones(A), ones(B), nthreads=THREADS)
        tol = np.maximum(tol, 2.0 * cnt.val * U * mag.val)
    err = np.abs(gv - wv)
    FP64_TALLY["entries_differing"] += int(np.count_nonzero(gv.view(np.int64) != wv.view(np.int64)))
    FP64_TALLY["cancellation_clause"] += int(np.count_nonzero((err > rel) & (err <= tol)))
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, f"{what}: {bad.size} fp64 values outside tolerance, e.g. {bad[:5]} {gv[bad[:5]]} {wv[bad[:5]]}"


def rows_of(C, rows):
    """Sub-CSR of the listed rows (in list order)."""
    rows = np.asarray(rows, np.int64)
    lens = C.row_ptr[rows + 1] - C.row_ptr[rows]
    rp = np.zeros(rows.size + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    if rows.size:
        idx = np.concatenate([np.arange(C.row_ptr[r], C.row_ptr[r + 1]) for r in rows])
    else:
        idx = np.zeros(0, np.int64)
    return oracle.Csr(rows.size, C.ncols, rp, C.col[idx], C.val[idx])


def changed_rows(before, after):
    """Rows whose (column, value-bit) content differs between two sorted CSRs."""
    n = before.nrows
    lb = np.diff(before.row_ptr)
    la = np.diff(after.row_ptr)
    diff = lb != la
    rid_b = np.repeat(np.arange(n), lb)
    rid_a = np.repeat(np.arange(n), la)
    pb = np.nonzero(~diff[rid_b])[0]
    pa = np.nonzero(~diff[rid_a])[0]
    assert pb.size == pa.size
    isz = np.asarray(before.val).dtype.itemsize
    vb = np.ascontiguousarray(before.val).view(np.uint8).reshape(before.val.size, isz)
    va = np.ascontiguousarray(after.val).view(np.uint8).reshape(after.val.size, isz)
    ne = (before.col[pb] != after.col[pa]) | (vb[pb] != va[pa]).any(axis=1)
    diff[rid_b[pb[ne]]] = True
    return np.nonzero(diff)[0].astype(np.int32)
