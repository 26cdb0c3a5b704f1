"""GPU: products with transposed operands, C = op(A) op(B), against the oracle
(its transpose, then its product).  Structure bit-exact, values bit-exact
(fp64 within the tolerance of ``assert_same_csr``), and the reported rows are
exactly the rows whose content changed.  Transposition follows Section 3 (either
SpGEMM operand may be transposed) and Section 5, "Handling Transposition"."""
import sys

import numpy as np
import pytest

import oracle
from gpu_util import THREADS, assert_same_csr, changed_rows
from paper_2202_08808_amd import dsg
from paper_2202_08808_amd import inputs as I

pytestmark = pytest.mark.gpu

SRS = [I.PLUS_TIMES_I64, I.MIN_PLUS_F32, I.PLUS_TIMES_F64, I.OR_AND_U32]
SR_ID = {I.PLUS_TIMES_I64: "i64", I.MIN_PLUS_F32: "minplus", I.PLUS_TIMES_F64: "f64", I.OR_AND_U32: "orand"}
OPS = {"AtB": (True, False), "ABt": (False, True), "AtBt": (True, True)}


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return dsg.Context(0)


def values(sr, n, rng):
    if sr == I.OR_AND_U32:
        return I.draw_values(sr, n, rng, 0, (1 << 32) - 1)
    if sr == I.MIN_PLUS_F32:
        return rng.integers(-5, 100, n).astype(np.float32)
    return I.draw_values(sr, n, rng, 1, 9)


def rand_csr(rng, nr, nc, density, sr, hubs=0):
    """Uniform entries; `hubs` rows and as many columns are nearly full, so
    rows of op(A) op(B) reach the large accumulator bins."""
    mask = rng.random((nr, nc)) < density
    for h in range(hubs):
        mask[rng.integers(nr), :] |= rng.random(nc) < 0.8
        mask[:, rng.integers(nc)] |= rng.random(nr) < 0.8
    ii, jj = np.nonzero(mask)
    return I.csr_from_keys(nr, nc, ii.astype(np.int64) * nc + jj, values(sr, ii.size, rng))


def op(M, t):
    return oracle.transpose(M) if t else M


def want_product(sr, a, b, ta, tb):
    return oracle.spgemm(sr, op(a, ta), op(b, tb), nthreads=THREADS)


def batch_values(sr, n, rng):
    return values(sr, n, rng)


def random_batch(sr, nr, nc, size, rng):
    b = I.random_batch(nr, nc, sr, size, rng)
    return I.Batch(b.rows, b.cols, batch_values(sr, size, rng), b.ops)


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
@pytest.mark.parametrize("form", list(OPS))
def test_transposed_static(ctx, sr, form):
    ta, tb = OPS[form]
    say(f"transposed static {SR_ID[sr]} {form}")
    rng = np.random.default_rng(100 + sr + 7 * len(form))
    m, k, n = 230, 170, 310
    A = rand_csr(rng, k if ta else m, m if ta else k, 0.03, sr)
    B = rand_csr(rng, n if tb else k, k if tb else n, 0.03, sr)
    Am, Bm = dsg.Matrix.from_csr(ctx, A, sr), dsg.Matrix.from_csr(ctx, B, sr)
    P = dsg.Product(ctx, Am, Bm, trans_a=ta, trans_b=tb)
    assert (P.nrows, P.ncols) == (m, n)
    a, b = oracle.Csr.of(A), oracle.Csr.of(B)
    assert_same_csr(sr, P.export(), want_product(sr, a, b, ta, tb), "static", A=op(a, ta), B=op(b, tb))
    P.destroy()
    Am.destroy()
    Bm.destroy()


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
@pytest.mark.parametrize("form", list(OPS))
def test_transposed_dynamic(ctx, sr, form):
    """Batches applied to both operands; each update equals the static
    product of the updated operands and reports exactly the changed rows.
    Hub rows and columns of the operands give rows of C from a few entries
    to nearly full."""
    ta, tb = OPS[form]
    say(f"transposed dynamic {SR_ID[sr]} {form}")
    rng = np.random.default_rng(200 + sr + 7 * len(form))
    m, k, n = 600, 500, 700
    A = rand_csr(rng, k if ta else m, m if ta else k, 0.01, sr, hubs=3)
    B = rand_csr(rng, n if tb else k, k if tb else n, 0.01, sr, hubs=3)
    Am, Bm = dsg.Matrix.from_csr(ctx, A, sr), dsg.Matrix.from_csr(ctx, B, sr)
    P = dsg.Product(ctx, Am, Bm, trans_a=ta, trans_b=tb)
    a, b = oracle.Csr.of(A), oracle.Csr.of(B)
    C = want_product(sr, a, b, ta, tb)
    assert_same_csr(sr, P.export(), C, "initial", A=op(a, ta), B=op(b, tb))
    for t, size in enumerate([1, 20, 300, 3000]):
        ba = random_batch(sr, a.nrows, a.ncols, size, rng)
        bb = random_batch(sr, b.nrows, b.ncols, size // 2 + 1, rng)
        Am.apply_batch(ba)
        Bm.apply_batch(bb)
        a, _ = oracle.apply(sr, a, ba.rows, ba.cols, ba.vals, ba.ops)
        b, _ = oracle.apply(sr, b, bb.rows, bb.cols, bb.vals, bb.ops)
        rs = P.update()
        want = want_product(sr, a, b, ta, tb)
        assert_same_csr(sr, P.export(), want, f"batch {t}", A=op(a, ta), B=op(b, tb))
        truth = changed_rows(C, want)
        if sr != I.PLUS_TIMES_F64:
            assert np.array_equal(rs.row_ids(), truth), f"batch {t}: reported rows"
        else:
            assert set(truth.tolist()) <= set(rs.row_ids().tolist())
        C = want
    st = P.stats()
    assert st["path"] == 0
    P.destroy()
    Am.destroy()
    Bm.destroy()


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
@pytest.mark.parametrize("force", [8, 9], ids=["dense", "global"])
def test_transposed_forced_bins(ctx, sr, force):
    """A^T B^T with every row in the dense bin (column passes and, for
    (min,+), the LDS hash) or in the global hash bin, C 6000 columns wide."""
    say(f"transposed forced bin {force} {SR_ID[sr]}")
    t = ctx.get_tuning()
    t.force_bin = force
    ctx.set_tuning(t)
    try:
        rng = np.random.default_rng(700 + force + 10 * sr)
        A = rand_csr(rng, 1200, 150, 0.01, sr, hubs=2)     # A^T: 150 x 1200
        B = rand_csr(rng, 6000, 1200, 0.004, sr, hubs=2)   # B^T: 1200 x 6000
        Am, Bm = dsg.Matrix.from_csr(ctx, A, sr), dsg.Matrix.from_csr(ctx, B, sr)
        P = dsg.Product(ctx, Am, Bm, trans_a=True, trans_b=True)
        a, b = oracle.Csr.of(A), oracle.Csr.of(B)
        assert_same_csr(sr, P.export(), want_product(sr, a, b, True, True), "initial",
                        A=op(a, True), B=op(b, True))
        for k, size in enumerate([40, 900]):
            ba = random_batch(sr, a.nrows, a.ncols, size, rng)
            bb = random_batch(sr, b.nrows, b.ncols, size, rng)
            Am.apply_batch(ba)
            Bm.apply_batch(bb)
            a, _ = oracle.apply(sr, a, ba.rows, ba.cols, ba.vals, ba.ops)
            b, _ = oracle.apply(sr, b, bb.rows, bb.cols, bb.vals, bb.ops)
            P.update()
            assert_same_csr(sr, P.export(), want_product(sr, a, b, True, True), f"batch {k}",
                            A=op(a, True), B=op(b, True))
        assert P.stats()["bin_rows"][force] > 0
        P.destroy()
        Am.destroy()
        Bm.destroy()
    finally:
        ctx.set_tuning(None)


@pytest.mark.parametrize("sr", [I.PLUS_TIMES_I64, I.MIN_PLUS_F32, I.OR_AND_U32], ids=lambda s: SR_ID[s])
@pytest.mark.parametrize("form", ["AtA", "AAt", "AtAt"])
def test_one_matrix_both_sides(ctx, sr, form):
    """Gram-type products of one matrix (A^T A, A A^T, A^T A^T) under updates
    of that matrix."""
    ta, tb = {"AtA": (True, False), "AAt": (False, True), "AtAt": (True, True)}[form]
    say(f"one matrix {SR_ID[sr]} {form}")
    rng = np.random.default_rng(300 + sr + 7 * len(form))
    nn = 450
    A = rand_csr(rng, nn, nn, 0.012, sr, hubs=2)
    Am = dsg.Matrix.from_csr(ctx, A, sr)
    P = dsg.Product(ctx, Am, Am, trans_a=ta, trans_b=tb)
    a = oracle.Csr.of(A)
    C = want_product(sr, a, a, ta, tb)
    assert_same_csr(sr, P.export(), C, "initial")
    for t, size in enumerate([5, 200, 2500]):
        ba = random_batch(sr, nn, nn, size, rng)
        Am.apply_batch(ba)
        a, _ = oracle.apply(sr, a, ba.rows, ba.cols, ba.vals, ba.ops)
        rs = P.update()
        want = want_product(sr, a, a, ta, tb)
        assert_same_csr(sr, P.export(), want, f"batch {t}")
        assert np.array_equal(rs.row_ids(), changed_rows(C, want)), f"batch {t}: reported rows"
        C = want
    P.destroy()
    Am.destroy()


@pytest.mark.parametrize("sr", [I.PLUS_TIMES_I64, I.MIN_PLUS_F32], ids=lambda s: SR_ID[s])
def test_plain_and_transposed_products_share_a_matrix(ctx, sr):
    """A B and A^T D kept current together from the same applies of A (the
    entry-granular path stays available to the plain product A A)."""
    say(f"shared operand {SR_ID[sr]}")
    rng = np.random.default_rng(400 + sr)
    nn = 400
    A = rand_csr(rng, nn, nn, 0.01, sr, hubs=2)
    D = rand_csr(rng, nn, 300, 0.01, sr)
    Am, Dm = dsg.Matrix.from_csr(ctx, A, sr), dsg.Matrix.from_csr(ctx, D, sr)
    P1 = dsg.Product(ctx, Am, Am)
    P2 = dsg.Product(ctx, Am, Dm, trans_a=True)
    a, d = oracle.Csr.of(A), oracle.Csr.of(D)
    for t, size in enumerate([3, 100, 1500]):
        ba = random_batch(sr, nn, nn, size, rng)
        Am.apply_batch(ba)
        a, _ = oracle.apply(sr, a, ba.rows, ba.cols, ba.vals, ba.ops)
        P1.update()
        P2.update()
        assert_same_csr(sr, P1.export(), oracle.spgemm(sr, a, a, nthreads=THREADS), f"A A, batch {t}")
        assert_same_csr(sr, P2.export(), want_product(sr, a, d, True, False), f"A^T D, batch {t}")
    P1.destroy()
    P2.destroy()
    Am.destroy()
    Dm.destroy()


def to_dev(b):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (b.rows, b.cols, b.vals, b.ops)]


def test_transposed_in_batched_form(ctx):
    """Batched runs (graph and plain path) of transposed products give the
    same C as per-product updates."""
    say("transposed batched")
    rng = np.random.default_rng(500)
    sr = I.MIN_PLUS_F32
    specs = [(True, False), (False, True), (True, True), (False, False)]
    mats, prods, host = [], [], []
    for ta, tb in specs:
        A = rand_csr(rng, 300, 300, 0.015, sr, hubs=1)
        B = rand_csr(rng, 300, 300, 0.015, sr)
        Am, Bm = dsg.Matrix.from_csr(ctx, A, sr), dsg.Matrix.from_csr(ctx, B, sr)
        mats += [Am, Bm]
        prods.append(dsg.Product(ctx, Am, Bm, trans_a=ta, trans_b=tb))
        host.append([oracle.Csr.of(A), oracle.Csr.of(B)])
    for direct_log2 in (24, 0):
        t = ctx.get_tuning()
        t.batch_direct_log2 = direct_log2
        ctx.set_tuning(t)
        bx = dsg.Batch(ctx, prods)
        for rnd in range(3):
            sets = []
            for j, (ta, tb) in enumerate(specs):
                ba = random_batch(sr, 300, 300, 50 * (rnd + 1), rng)
                bb = random_batch(sr, 300, 300, 20 * (rnd + 1), rng)
                sets += [(mats[2 * j], *to_dev(ba)), (mats[2 * j + 1], *to_dev(bb))]
                host[j][0], _ = oracle.apply(sr, host[j][0], ba.rows, ba.cols, ba.vals, ba.ops)
                host[j][1], _ = oracle.apply(sr, host[j][1], bb.rows, bb.cols, bb.vals, bb.ops)
            bx.run(sets)
            for j, (ta, tb) in enumerate(specs):
                want = want_product(sr, host[j][0], host[j][1], ta, tb)
                assert_same_csr(sr, prods[j].export(), want, f"log2 {direct_log2} round {rnd} product {j}")
        bx.destroy()
        ctx.set_tuning(None)
    for P in prods:
        P.destroy()
    for M in mats:
        M.destroy()


def test_transposed_argument_errors(ctx):
    say("transposed errors")
    rng = np.random.default_rng(600)
    sr = I.PLUS_TIMES_I64
    A = dsg.Matrix.from_csr(ctx, rand_csr(rng, 20, 30, 0.1, sr), sr)
    B = dsg.Matrix.from_csr(ctx, rand_csr(rng, 20, 40, 0.1, sr), sr)
    with pytest.raises(dsg.DsgError) as e:
        dsg.Product(ctx, A, B)                      # 30 != 20
    assert e.value.status == dsg.E_STATE
    P = dsg.Product(ctx, A, B, trans_a=True)        # (30 x 20)(20 x 40)
    assert (P.nrows, P.ncols) == (30, 40)
    with pytest.raises(dsg.DsgError) as e:
        dsg.Product(ctx, A, B, trans_b=True)        # (20 x 30)(40 x 20)
    assert e.value.status == dsg.E_STATE
    h = dsg.P()
    st = ctx.L.dsg_prod_create(ctx.h, A.h, B.h, 0x8, dsg.ctypes.byref(h))
    assert st == dsg.E_ARG
    P.destroy()
    A.destroy()
    B.destroy()
