"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Structure and int64 / min-plus values must match bit for bit; fp64 values
must match bit for bit or stay inside the tolerance of ``assert_same_csr``.
Each case prints its name first so that a failing run names it.
"""
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


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return dsg.Context(0)


@pytest.fixture
def tuned(ctx):
    """Restore the default tuning after a test that changes it."""
    yield ctx
    ctx.set_tuning(None)


def rand_csr(rng, nr, nc, density, sr, row_skew=False):
    """Random CSR; with row_skew some rows are much denser than others."""
    if row_skew:
        dens = np.minimum(1.0, density * rng.pareto(1.2, nr) + density / 4)
    else:
        dens = np.full(nr, density)
    rows, cols = [], []
    for i in range(nr):
        k = rng.binomial(nc, dens[i])
        c = np.sort(rng.choice(nc, k, replace=False)) if k else np.zeros(0, np.int64)
        rows.append(np.full(c.size, i, np.int64))
        cols.append(c)
    r = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    c = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    if sr == I.MIN_PLUS_F32:
        vals = rng.integers(-5, 100, r.size).astype(np.float32)
    elif sr == I.OR_AND_U32:
        vals = I.draw_values(sr, r.size, rng, 0, (1 << 32) - 1)   # full 32-bit words
    else:
        vals = I.draw_values(sr, r.size, rng, 1, 9)
    return I.csr_from_keys(nr, nc, r * nc + c, vals)


def gpu_product(ctx, sr, A, B=None):
    Am = dsg.Matrix.from_csr(ctx, A, sr)
    Bm = Am if B is None else dsg.Matrix.from_csr(ctx, B, sr)
    return Am, Bm, dsg.Product(ctx, Am, Bm)


def check_product(sr, prod, A, B, what):
    got = prod.export()
    want = oracle.spgemm(sr, oracle.Csr.of(A), oracle.Csr.of(B), nthreads=THREADS)
    assert_same_csr(sr, got, want, what, A=oracle.Csr.of(A), B=oracle.Csr.of(B))
    return want


def destroy(*objs):
    for o in objs:
        o.destroy()


# ---------------------------------------------------------------------------

@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
@pytest.mark.parametrize("shape", [(1, 1, 1), (7, 5, 3), (64, 64, 64), (300, 200, 500), (513, 1000, 257)])
def test_static_random(ctx, sr, shape):
    say(f"static random {SR_ID[sr]} {shape}")
    rng = np.random.default_rng(hash(shape) % 1000 + sr)
    nr, nk, nc = shape
    for dens in (0.0, 0.02, 0.2):
        A = rand_csr(rng, nr, nk, dens, sr, row_skew=True)
        B = rand_csr(rng, nk, nc, dens, sr, row_skew=True)
        Am, Bm, P = gpu_product(ctx, sr, A, B)
        check_product(sr, P, A, B, f"{shape} d={dens}")
        destroy(P, Am, Bm)


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
@pytest.mark.parametrize("force", list(range(10)))
def test_static_forced_bin(tuned, sr, force):
    """Every accumulator gives the same product (rows that do not fit a
    forced group bin go to the next bin that fits)."""
    ctx = tuned
    say(f"static forced bin {force} {SR_ID[sr]}")
    t = ctx.get_tuning()
    t.force_bin = force
    ctx.set_tuning(t)
    rng = np.random.default_rng(100 + force + 10 * sr)
    A = rand_csr(rng, 150, 1200, 0.01, sr, row_skew=True)
    B = rand_csr(rng, 1200, 6000, 0.004, sr, row_skew=True)
    Am, Bm, P = gpu_product(ctx, sr, A, B)
    check_product(sr, P, A, B, f"bin {force}")
    st = P.stats()
    assert sum(st["bin_rows"]) == A.nrows
    destroy(P, Am, Bm)


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
def test_apply_matches_oracle(ctx, sr):
    """Batches with repeated keys, deletes of absent entries, inserts over
    present ones and ADD chains, applied in sequence."""
    say(f"apply {SR_ID[sr]}")
    rng = np.random.default_rng(7 + sr)
    A = rand_csr(rng, 90, 70, 0.1, sr)
    Am = dsg.Matrix.from_csr(ctx, A, sr)
    cur = oracle.Csr.of(A)
    # sizes on both sides of the one-workgroup sorts' limits (4096, 8192)
    for t, size in enumerate([0, 1, 17, 300, 2000, 4097, 5000, 8192, 8193, 12000]):
        b = I.random_batch(90, 70, sr, size, rng, hot_rows=40 if t % 2 else None)
        Am.apply_batch(b)
        cur, _ = oracle.apply(sr, cur, b.rows, b.cols, b.vals, b.ops)
        got = Am.export()
        assert_same_csr(sr, got, cur, f"apply batch {t}")
        assert Am.nnz() == cur.nnz
    destroy(Am)


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
@pytest.mark.parametrize("with_product", [False, True], ids=["matrix", "product"])
def test_apply_growth_across_compaction(ctx, sr, with_product):
    """A row that shrank keeps its old capacity; a later batch grows it again
    (in place by that capacity) while another row's move forces a pool
    compaction, which trims every capacity to the slack of its length.  The
    grown row must not spill into its neighbours."""
    say(f"apply growth across compaction {SR_ID[sr]} {with_product}")
    rng = np.random.default_rng(31 + sr)
    n = nc = 2048
    keys = np.concatenate([np.arange(40), (np.arange(1, 64)[:, None] * nc + np.array([[7, 9]])).ravel()])
    keys = np.sort(keys.astype(np.int64))
    A = I.csr_from_keys(n, nc, keys, I.draw_values(sr, keys.size, rng, 1, 9))
    Am = dsg.Matrix.from_csr(ctx, A, sr)
    P = dsg.Product(ctx, Am, Am) if with_product else None
    cur = oracle.Csr.of(A)
    # 1: row 0 shrinks from 40 to 4 entries
    dels = np.arange(4, 40, dtype=np.int32)
    b1 = I.Batch(np.zeros(dels.size, np.int32), dels, I.draw_values(sr, dels.size, rng, 1, 9),
                 np.full(dels.size, I.OP_DELETE, np.uint8))
    # 2: row 0 grows to 34 entries; rows 1 and 2 to 2002 each (moves larger
    # than the free part of the pool)
    r = np.concatenate([np.zeros(30, np.int32), np.full(2000, 1, np.int32), np.full(2000, 2, np.int32)])
    c = np.concatenate([np.arange(100, 130), np.arange(20, 2020), np.arange(20, 2020)]).astype(np.int32)
    b2 = I.Batch(r, c, I.draw_values(sr, r.size, rng, 1, 9), np.full(r.size, I.OP_SET, np.uint8))
    for t, b in enumerate((b1, b2)):
        Am.apply_batch(b)
        cur, _ = oracle.apply(sr, cur, b.rows, b.cols, b.vals, b.ops)
        assert_same_csr(sr, Am.export(), cur, f"after batch {t}")
        if P is not None:
            P.update()
            want = oracle.spgemm(sr, cur, cur, nthreads=THREADS)
            assert_same_csr(sr, P.export(), want, f"product after batch {t}", A=cur, B=cur)
    if P is not None:
        P.destroy()
    destroy(Am)


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
@pytest.mark.parametrize("with_product", [False, True], ids=["matrix", "product"])
def test_apply_heavy_rows(ctx, sr, with_product):
    """Rows that receive thousands of updates in one batch (the workgroup
    paths of the apply): inserts only (moved rows), overwrites only (in
    place), a mix with deletions, and more updates than one LDS hash holds."""
    say(f"apply heavy rows {SR_ID[sr]} {with_product}")
    rng = np.random.default_rng(51 + sr)
    n = 25000
    keys = I.er_keys(n, 3 * n, rng)
    keys = np.unique(np.concatenate([keys, np.arange(3000, dtype=np.int64) + n]))  # row 1: 3000 entries
    A = I.csr_from_keys(n, n, keys, I.draw_values(sr, keys.size, rng, 1, 9))
    Am = dsg.Matrix.from_csr(ctx, A, sr)
    P = dsg.Product(ctx, Am, Am) if with_product else None
    cur = oracle.Csr.of(A)

    def batch(rows, cols, ops):
        return I.Batch(np.asarray(rows, np.int32), np.asarray(cols, np.int32),
                       I.draw_values(sr, len(rows), rng, 1, 9), np.asarray(ops, np.uint8))

    r0 = np.zeros(5000, np.int32)
    c0 = rng.choice(n, 5000, replace=False)
    r1 = np.ones(3000, np.int32)
    c1 = np.arange(3000)
    r2 = np.full(4000, 2, np.int32)
    c2 = rng.integers(0, n, 4000)
    o2 = rng.choice(3, 4000, p=[0.5, 0.3, 0.2])
    r3 = np.full(20000, 3, np.int32)
    c3 = rng.choice(n, 20000, replace=False)
    b = batch(np.concatenate([r0, r1, r2, r3]), np.concatenate([c0, c1, c2, c3]),
              np.concatenate([np.zeros(5000), np.zeros(3000), o2, np.zeros(20000)]))
    b2 = batch(np.concatenate([r3[:9000], r0[:100]]), np.concatenate([c3[:9000], c0[:100]]),
               np.concatenate([np.full(9000, I.OP_DELETE), np.full(100, I.OP_ADD)]))
    for t, bb in enumerate((b, b2)):
        Am.apply_batch(bb)
        cur, _ = oracle.apply(sr, cur, bb.rows, bb.cols, bb.vals, bb.ops)
        assert_same_csr(sr, Am.export(), cur, f"after batch {t}")
        if P is not None:
            P.update()
            want = oracle.spgemm(sr, cur, cur, nthreads=THREADS)
            assert_same_csr(sr, P.export(), want, f"product after batch {t}", A=cur, B=cur)
    if P is not None:
        P.destroy()
    destroy(Am)


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
@pytest.mark.parametrize("with_product", [False, True], ids=["matrix", "product"])
def test_apply_row_crosses_heavy_length(ctx, sr, with_product):
    """A row planned as light (2040 entries, few updates) that grows past the
    heavy-row length in the same batch is committed exactly once (the light
    and workgroup commits split rows by the plan, not by the changed length)."""
    say(f"apply row crosses heavy length {SR_ID[sr]} {with_product}")
    rng = np.random.default_rng(91 + sr)
    n = 6000
    row0 = np.sort(rng.choice(n, 2040, replace=False)).astype(np.int64)
    rest = I.er_keys(n, 4 * n, rng)
    keys = np.unique(np.concatenate([row0, rest[rest >= n]]))
    A = I.csr_from_keys(n, n, keys, I.draw_values(sr, keys.size, rng, 1, 9))
    Am = dsg.Matrix.from_csr(ctx, A, sr)
    P = dsg.Product(ctx, Am, Am) if with_product else None
    cur = oracle.Csr.of(A)
    absent = np.setdiff1d(np.arange(n), row0)
    ins = rng.choice(absent, 30, replace=False).astype(np.int32)
    other = I.random_batch(n, n, sr, 500, rng, op_probs=(0.5, 0.3, 0.2), value_lo=1, value_hi=9)
    keep = other.rows != 0  # row 0 gets inserts only (the no-delete commit)
    other = I.Batch(other.rows[keep], other.cols[keep], other.vals[keep], other.ops[keep])
    b = I.Batch(np.concatenate([np.zeros(30, np.int32), other.rows]), np.concatenate([ins, other.cols]),
                np.concatenate([I.draw_values(sr, 30, rng, 1, 9), other.vals]),
                np.concatenate([np.full(30, I.OP_SET, np.uint8), other.ops]))
    for t in range(2):
        Am.apply_batch(b)
        cur, _ = oracle.apply(sr, cur, b.rows, b.cols, b.vals, b.ops)
        assert_same_csr(sr, Am.export(), cur, f"after batch {t}")
        if P is not None:
            P.update()
            assert_same_csr(sr, P.export(), oracle.spgemm(sr, cur, cur, nthreads=THREADS), f"product {t}",
                            A=cur, B=cur)
        b = I.random_batch(n, n, sr, 300, rng, op_probs=(0.6, 0.2, 0.2), value_lo=1, value_hi=9)
    if P is not None:
        P.destroy()
    destroy(Am)


def test_dense_row_outgrows_its_hash(ctx):
    """(min,+) rows of the dense bin are first tried in a single pass with an
    LDS hash sized from the old row; a row that grows past it is redone with
    the column passes.  Row 0 grows from ~20 entries to more than the table
    holds, shrinks back, then changes a little (the hash path again); C and
    the reported rows match the oracle at every step."""
    sr = I.MIN_PLUS_F32
    say("dense row outgrows its hash")
    rng = np.random.default_rng(71)
    n = 30000
    keys = I.er_keys(n, 10 * n, rng)
    keys = keys[(keys // n != 0) | (np.arange(keys.size) < 2)]  # row 0 starts with two entries
    A = I.csr_from_keys(n, n, keys, I.draw_values(sr, keys.size, rng, 1, 100))
    Am, _, P = gpu_product(ctx, sr, A)
    cur = oracle.Csr.of(A)
    C = oracle.spgemm(sr, cur, cur, nthreads=THREADS)
    grow = rng.choice(np.arange(1, n), 2600, replace=False).astype(np.int32)
    batches = [
        I.Batch(np.zeros(2600, np.int32), grow, I.draw_values(sr, 2600, rng, 1, 100),
                np.full(2600, I.OP_SET, np.uint8)),
        I.Batch(np.zeros(2500, np.int32), grow[:2500], np.zeros(2500, np.float32),
                np.full(2500, I.OP_DELETE, np.uint8)),
        I.Batch(np.zeros(20, np.int32), grow[2500:2520], I.draw_values(sr, 20, rng, 1, 100),
                np.full(20, I.OP_SET, np.uint8)),
    ]
    for t, b in enumerate(batches):
        Am.apply_batch(b)
        rs = P.update()
        cur, _ = oracle.apply(sr, cur, b.rows, b.cols, b.vals, b.ops)
        want = oracle.spgemm(sr, cur, cur, nthreads=THREADS)
        assert_same_csr(sr, P.export(), want, f"step {t}", A=cur, B=cur)
        assert np.array_equal(rs.row_ids(), changed_rows(C, want)), f"step {t}: reported rows"
        if t == 0:
            assert want.row_ptr[1] - want.row_ptr[0] > 16384  # more than the table's slots
        C = want
    destroy(P, Am)


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
def test_dense_passes_split_b(tuned, sr):
    """Every row in the dense bin with C 70,000 columns wide: 3 column passes
    for 4-byte values, 5 for 8-byte ones, each streaming its own part of the
    split copy of B, which is rebuilt for every update of A and B."""
    ctx = tuned
    say(f"dense passes over split B {SR_ID[sr]}")
    t = ctx.get_tuning()
    t.force_bin = 8
    t.dense_max_passes = 8
    ctx.set_tuning(t)
    rng = np.random.default_rng(90 + sr)
    A = rand_csr(rng, 120, 2500, 0.012, sr, row_skew=True)
    B = rand_csr(rng, 2500, 70000, 0.0003, sr, row_skew=True)
    Am, Bm, P = gpu_product(ctx, sr, A, B)
    a, b = oracle.Csr.of(A), oracle.Csr.of(B)
    C = check_product(sr, P, A, B, "initial")
    for k, size in enumerate([30, 600]):
        ba = I.random_batch(120, 2500, sr, size, rng)
        bb = I.random_batch(2500, 70000, sr, 4 * size, rng)
        Am.apply_batch(ba)
        Bm.apply_batch(bb)
        a, _ = oracle.apply(sr, a, ba.rows, ba.cols, ba.vals, ba.ops)
        b, _ = oracle.apply(sr, b, bb.rows, bb.cols, bb.vals, bb.ops)
        rs = P.update()
        want = oracle.spgemm(sr, a, b, nthreads=THREADS)
        assert_same_csr(sr, P.export(), want, f"batch {k}", A=a, B=b)
        truth = changed_rows(C, want)
        if sr != I.PLUS_TIMES_F64:
            assert np.array_equal(rs.row_ids(), truth), f"batch {k}: reported rows"
        C = want
    assert P.stats()["bin_rows"][8] > 0
    destroy(P, Am, Bm)


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
@pytest.mark.parametrize("square", [True, False], ids=["AxA", "AxB"])
def test_dynamic_sequence(ctx, sr, square):
    """D1 (dynamic result = static recompute of the updated operands) and D5
    (reported rows = rows whose content changed) over a sequence of batches."""
    say(f"dynamic {SR_ID[sr]} {'AxA' if square else 'AxB'}")
    rng = np.random.default_rng(11 + sr + 3 * square)
    n = 400
    A = rand_csr(rng, n, n, 0.01, sr, row_skew=True)
    B = None if square else rand_csr(rng, n, 350, 0.015, sr, row_skew=True)
    Am, Bm, P = gpu_product(ctx, sr, A, B)
    a, b = oracle.Csr.of(A), oracle.Csr.of(A if square else B)
    C = check_product(sr, P, A, A if square else B, "initial")
    for t in range(5):
        size = [1, 10, 100, 1000, 4000][t]
        ba = I.random_batch(n, n, sr, size, rng)
        Am.apply_batch(ba)
        a, _ = oracle.apply(sr, a, ba.rows, ba.cols, ba.vals, ba.ops)
        if square:
            b = a
        else:
            bb = I.random_batch(n, 350, sr, size // 2 + 1, rng)
            Bm.apply_batch(bb)
            b, _ = oracle.apply(sr, b, bb.rows, bb.cols, bb.vals, bb.ops)
        rs = P.update()
        got = P.export()
        want = oracle.spgemm(sr, a, b, nthreads=THREADS)
        assert_same_csr(sr, got, want, f"batch {t}", A=a, B=b)
        reported = rs.row_ids()
        truth = changed_rows(C, want)
        if sr != I.PLUS_TIMES_F64:
            assert np.array_equal(reported, truth), f"batch {t}: reported rows differ"
        else:
            assert set(truth.tolist()) <= set(reported.tolist())
        C = want
    destroy(P, Am)
    if not square:
        destroy(Bm)


@pytest.mark.parametrize("sr", [I.PLUS_TIMES_I64, I.MIN_PLUS_F32], ids=lambda s: SR_ID[s])
def test_inverse_batch_restores(ctx, sr):
    """D2: a batch followed by its inverse restores C bit for bit."""
    say(f"inverse batch {SR_ID[sr]}")
    rng = np.random.default_rng(21 + sr)
    A = rand_csr(rng, 300, 300, 0.02, sr, row_skew=True)
    Am, _, P = gpu_product(ctx, sr, A)
    C0 = P.export()
    bs = I.disjoint_batches(A, sr, [200], stream=77)[0]
    Am.apply_batch(bs)
    P.update()
    # inverse: delete what was inserted, re-insert deleted / changed entries with old values
    old = {(int(i), int(j)): v for i, j, v in zip(A.row_of_entry(), A.col, A.val)}
    inv_r, inv_c, inv_v, inv_o = [], [], [], []
    for i, j, o in zip(bs.rows, bs.cols, bs.ops):
        key = (int(i), int(j))
        inv_r.append(i)
        inv_c.append(j)
        if key in old:
            inv_v.append(old[key])
            inv_o.append(I.OP_SET)
        else:
            inv_v.append(0)
            inv_o.append(I.OP_DELETE)
    Am.apply(np.array(inv_r, np.int32), np.array(inv_c, np.int32), np.array(inv_v, I.VALUE_DTYPE[sr]),
             np.array(inv_o, np.uint8))
    P.update()
    C1 = P.export()
    assert_same_csr(sr, C1, C0, "restored")
    destroy(P, Am)


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
def test_split_batch_same_result(ctx, sr):
    """D3: one batch, or the same batch in consecutive pieces with an update
    after each, give the same final C."""
    say(f"split batch {SR_ID[sr]}")
    rng = np.random.default_rng(31 + sr)
    A = rand_csr(rng, 250, 250, 0.02, sr, row_skew=True)
    b = I.random_batch(250, 250, sr, 900, rng)
    A1, _, P1 = gpu_product(ctx, sr, A)
    A1.apply_batch(b)
    P1.update()
    A2, _, P2 = gpu_product(ctx, sr, A)
    for lo in range(0, 900, 250):
        A2.apply(b.rows[lo:lo + 250].copy(), b.cols[lo:lo + 250].copy(), b.vals[lo:lo + 250].copy(),
                 b.ops[lo:lo + 250].copy())
        P2.update()
    assert_same_csr(sr, P2.export(), P1.export(), "split vs whole")
    destroy(P1, A1, P2, A2)


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
def test_empty_and_noop_batches(ctx, sr):
    """D6: an empty batch, or one that changes nothing (deletes of absent
    entries, SET to the stored value), reports no rows and leaves C as is."""
    say(f"noop batches {SR_ID[sr]}")
    rng = np.random.default_rng(41 + sr)
    A = rand_csr(rng, 120, 120, 0.05, sr)
    Am, _, P = gpu_product(ctx, sr, A)
    C0 = P.export()
    assert P.update().n == 0
    Am.apply(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, I.VALUE_DTYPE[sr]), np.zeros(0, np.uint8))
    assert P.update().n == 0
    absent = I.sample_absent(120, 120, A.keys(), 30, rng)
    keys = A.keys()[:30]
    rows = np.concatenate([absent // 120, keys // 120]).astype(np.int32)
    cols = np.concatenate([absent % 120, keys % 120]).astype(np.int32)
    vals = np.concatenate([np.zeros(30, I.VALUE_DTYPE[sr]), A.val[:30]])
    ops = np.concatenate([np.full(30, I.OP_DELETE, np.uint8), np.full(30, I.OP_SET, np.uint8)])
    Am.apply(rows, cols, vals, ops)
    assert P.update().n == 0
    assert_same_csr(sr, P.export(), C0, "after no-op batch")
    destroy(P, Am)


def test_report_affected_superset(ctx):
    say("report affected")
    sr = I.PLUS_TIMES_I64
    rng = np.random.default_rng(5)
    A = rand_csr(rng, 200, 200, 0.03, sr)
    Am, _, P = gpu_product(ctx, sr, A)
    C0 = P.export()
    b = I.random_batch(200, 200, sr, 50, rng)
    Am.apply_batch(b)
    aff = P.update(report_affected=True).row_ids()
    a, _ = oracle.apply(sr, oracle.Csr.of(A), b.rows, b.cols, b.vals, b.ops)
    want = oracle.spgemm(sr, a, a)
    assert_same_csr(sr, P.export(), want, "after update")
    assert set(changed_rows(C0, want).tolist()) <= set(aff.tolist())
    destroy(P, Am)


def test_autotune_keeps_results(tuned, tmp_path):
    """The autotuner's trials and its chosen tuning never change C; a second
    call with the cache file reuses the choice without trials."""
    ctx = tuned
    say("autotune")
    sr = I.MIN_PLUS_F32
    A = I.rmat_csr(11, 16, sr, stream=55, lo=1, hi=100)
    Am, _, P = gpu_product(ctx, sr, A)
    cache = str(tmp_path / "tune.json")
    r1 = P.autotune(reps=1, cache_path=cache)
    assert not r1["cached"] and len(r1["trials"]) >= 8
    check_product(sr, P, A, A, "after autotune")
    r2 = P.autotune(reps=1, cache_path=cache)
    assert r2["cached"] and r2["group_ub"] == r1["group_ub"]
    b = I.disjoint_batches(A, sr, [500], stream=56, value_lo=1, value_hi=100)[0]
    Am.apply_batch(b)
    P.update()
    a, _ = oracle.apply(sr, oracle.Csr.of(A), b.rows, b.cols, b.vals, b.ops)
    assert_same_csr(sr, P.export(), oracle.spgemm(sr, a, a, nthreads=THREADS), "update after autotune")
    destroy(P, Am)


def test_config1_rmat12_int64(ctx):
    """R-MAT scale 12, edge factor 8, int64 plus-times, one batch of 100
    insertions: dynamic C' equals the oracle's static recompute."""
    say("config rmat12 int64")
    w = I.workload_rmat12_i64()
    sr = w.semiring
    Am, _, P = gpu_product(ctx, sr, w.A)
    C0 = check_product(sr, P, w.A, w.A, "static")
    b = w.batches_A[0]
    Am.apply_batch(b)
    rs = P.update()
    a, _ = oracle.apply(sr, oracle.Csr.of(w.A), b.rows, b.cols, b.vals, b.ops)
    want = oracle.spgemm(sr, a, a, nthreads=THREADS)
    assert_same_csr(sr, P.export(), want, "dynamic")
    assert np.array_equal(rs.row_ids(), changed_rows(C0, want))
    destroy(P, Am)
