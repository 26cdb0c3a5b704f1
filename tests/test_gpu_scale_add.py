"""GPU: D = (alpha (x) C) (+) (beta (x) X) from a maintained product (the
general SpGEMM result alpha op(A) op(B) + beta X of Section 3) against the
oracle's entrywise definition, bit for bit (each operation is one rounding
on both sides, in the same order)."""
import sys

import numpy as np
import pytest

import oracle
from gpu_util import THREADS
from paper_2202_08808_amd import dsg
from paper_2202_08808_amd import inputs as I

pytestmark = pytest.mark.gpu

SRS = [I.PLUS_TIMES_I64, I.MIN_PLUS_F32, I.PLUS_TIMES_F64, I.OR_AND_U32]
SR_ID = {I.PLUS_TIMES_I64: "i64", I.MIN_PLUS_F32: "minplus", I.PLUS_TIMES_F64: "f64", I.OR_AND_U32: "orand"}
SCALARS = {I.PLUS_TIMES_I64: (3, -2), I.MIN_PLUS_F32: (2.5, -1.0), I.PLUS_TIMES_F64: (0.7, -1.3),
           I.OR_AND_U32: (0x0F0F0F0F, 0xFFFF0000)}


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return dsg.Context(0)


def values(sr, n, rng):
    if sr == I.OR_AND_U32:
        return I.draw_values(sr, n, rng, 0, (1 << 32) - 1)
    if sr == I.PLUS_TIMES_F64:
        return rng.standard_normal(n)
    return I.draw_values(sr, n, rng, 1, 9)


def rand_csr(rng, nr, nc, density, sr, extra_keys=None):
    keys = np.flatnonzero(rng.random(nr * nc) < density).astype(np.int64)
    if extra_keys is not None:
        keys = np.unique(np.concatenate([keys, extra_keys]))
    return I.csr_from_keys(nr, nc, keys, values(sr, keys.size, rng))


def same(sr, got, want, what):
    assert np.array_equal(np.asarray(got.row_ptr), np.asarray(want.row_ptr)), f"{what}: row pointers"
    assert np.array_equal(np.asarray(got.col), np.asarray(want.col)), f"{what}: columns"
    gv = np.ascontiguousarray(got.val, oracle.DTYPE[sr])
    wv = np.ascontiguousarray(want.val, oracle.DTYPE[sr])
    assert gv.tobytes() == wv.tobytes(), f"{what}: values"


def keys_of(C):
    rows = np.repeat(np.arange(C.nrows, dtype=np.int64), np.diff(C.row_ptr))
    return rows * C.ncols + C.col.astype(np.int64)


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
@pytest.mark.parametrize("trans", [False, True], ids=["AB", "AtB"])
def test_scale_add_matches_oracle(ctx, sr, trans):
    say(f"scale_add {SR_ID[sr]} {'AtB' if trans else 'AB'}")
    rng = np.random.default_rng(800 + sr + 10 * trans)
    m, k, n = 300, 200, 260
    A = rand_csr(rng, k if trans else m, m if trans else k, 0.02, sr)
    B = rand_csr(rng, k, n, 0.02, sr)
    Am, Bm = dsg.Matrix.from_csr(ctx, A, sr), dsg.Matrix.from_csr(ctx, B, sr)
    P = dsg.Product(ctx, Am, Bm, trans_a=trans)
    a, b = oracle.Csr.of(A), oracle.Csr.of(B)
    ba = I.random_batch(a.nrows, a.ncols, sr, 400, rng)
    Am.apply_batch(ba)
    a, _ = oracle.apply(sr, a, ba.rows, ba.cols, ba.vals, ba.ops)
    P.update()
    C = oracle.spgemm(sr, oracle.transpose(a) if trans else a, b, nthreads=THREADS)
    # X: its own entries plus a third of C's, so all three cases of the union occur
    ck = keys_of(C)
    X = rand_csr(rng, m, n, 0.01, sr, extra_keys=ck[rng.random(ck.size) < 0.33])
    Xm = dsg.Matrix.from_csr(ctx, X, sr)
    alpha, beta = SCALARS[sr]
    D = P.scale_add(alpha, Xm, beta)
    want = oracle.axpby(sr, alpha, C, beta, oracle.Csr.of(X))
    same(sr, D.export(), want, "alpha C + beta X")
    # X absent: alpha (x) C
    D2 = P.scale_add(alpha)
    same(sr, D2.export(), oracle.axpby(sr, alpha, C, beta, None), "alpha C")
    # D is a matrix like any other: it takes updates
    bd = I.random_batch(m, n, sr, 300, rng)
    D.apply_batch(bd)
    want2, _ = oracle.apply(sr, want, bd.rows, bd.cols, bd.vals, bd.ops)
    same(sr, D.export(), want2, "D after an apply")
    for o in (D, D2, P, Am, Bm, Xm):
        o.destroy()


def test_scale_add_edge_cases(ctx):
    say("scale_add edge cases")
    rng = np.random.default_rng(900)
    sr = I.PLUS_TIMES_I64
    # empty C: D = beta (x) X
    A = I.csr_from_keys(50, 40, np.zeros(0, np.int64), np.zeros(0, np.int64))
    B = rand_csr(rng, 40, 30, 0.1, sr)
    Am, Bm = dsg.Matrix.from_csr(ctx, A, sr), dsg.Matrix.from_csr(ctx, B, sr)
    P = dsg.Product(ctx, Am, Bm)
    X = rand_csr(rng, 50, 30, 0.1, sr)
    Xm = dsg.Matrix.from_csr(ctx, X, sr)
    D = P.scale_add(5, Xm, 7)
    C = oracle.spgemm(sr, oracle.Csr.of(A), oracle.Csr.of(B))
    assert C.nnz == 0
    same(sr, D.export(), oracle.axpby(sr, 5, C, 7, oracle.Csr.of(X)), "empty C")
    # errors: shape and semiring of X
    Xbad = dsg.Matrix.from_csr(ctx, rand_csr(rng, 49, 30, 0.1, sr), sr)
    with pytest.raises(dsg.DsgError) as e:
        P.scale_add(1, Xbad, 1)
    assert e.value.status == dsg.E_STATE
    Xf = dsg.Matrix.from_csr(ctx, rand_csr(rng, 50, 30, 0.1, I.MIN_PLUS_F32), I.MIN_PLUS_F32)
    h = dsg.P()
    one = np.array([1], np.int64)
    st = ctx.L.dsg_prod_scale_add(P.h, one.ctypes.data_as(dsg.P), Xf.h, one.ctypes.data_as(dsg.P),
                                  dsg.ctypes.byref(h))
    assert st == dsg.E_STATE
    st = ctx.L.dsg_prod_scale_add(P.h, None, None, None, dsg.ctypes.byref(h))
    assert st == dsg.E_ARG
    for o in (D, P, Am, Bm, Xm, Xbad, Xf):
        o.destroy()
