"""GPU: the entry-granular dynamic update of C = A*A and A*B ((min,+) fp32,
int64 (+,x) and bitwise (or, and)) gives the oracle's C bit for bit and reports exactly the rows whose
content changed, like the row path; it takes over only when C reflects
every apply but the last one."""
import sys

import numpy as np
import pytest

import oracle
from gpu_util import THREADS, assert_same_csr, changed_rows
from paper_2202_08808_amd import dsg
from paper_2202_08808_amd import inputs as I

pytestmark = pytest.mark.gpu

SRS = [I.PLUS_TIMES_I64, I.MIN_PLUS_F32, I.OR_AND_U32]
SR_ID = {I.PLUS_TIMES_I64: "i64", I.MIN_PLUS_F32: "minplus", I.OR_AND_U32: "orand"}


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = dsg.Context(0)
    yield c
    c.set_tuning(None)


def row_path(ctx, on):
    """on: whole affected rows only; off: entry-granular whenever it applies."""
    t = ctx.get_tuning()
    t.update_path = 1 if on else 2
    ctx.set_tuning(t)


def run(ctx, sr, A, batches, use_row_path=False, expect_entry=True, auto=False, row_index=1):
    """Apply each batch then update; check C and the reported rows against
    the oracle after every step (auto: the library chooses the path;
    row_index 0: no per-row column index on C and A)."""
    if auto:
        ctx.set_tuning(None)
    else:
        row_path(ctx, use_row_path)
    t = ctx.get_tuning()
    t.row_index = row_index
    ctx.set_tuning(t)
    m = dsg.Matrix.from_csr(ctx, A, sr)
    P = dsg.Product(ctx, m, m)
    a = oracle.Csr.of(A)
    C = oracle.spgemm(sr, a, a, nthreads=THREADS)
    stats = []
    for t, b in enumerate(batches):
        m.apply_batch(b)
        rs = P.update()
        a, _ = oracle.apply(sr, a, b.rows, b.cols, b.vals, b.ops)
        want = oracle.spgemm(sr, a, a, nthreads=THREADS)
        assert_same_csr(sr, P.export(), want, f"step {t}")
        assert np.array_equal(rs.row_ids(), changed_rows(C, want)), f"step {t}: reported rows"
        st = P.stats()
        stats.append(st)
        if expect_entry and not use_row_path:
            assert st["path"] == 1, f"step {t}: row path taken"
        C = want
    P.destroy()
    m.destroy()
    ctx.set_tuning(None)
    return stats


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
def test_entry_matches_oracle(ctx, sr):
    say(f"entry path R-MAT {SR_ID[sr]}")
    hi = 9 if sr == I.PLUS_TIMES_I64 else 100
    A = I.rmat_csr(10, 8, sr, stream=801, lo=1, hi=hi)
    bs = I.disjoint_batches(A, sr, [1, 10, 100, 1000, 3000], stream=802, value_lo=1, value_hi=hi)
    st = run(ctx, sr, A, bs)
    assert sum(s["lost"] for s in st) > 0  # deletions hit stored minima / contributors
    run(ctx, sr, A, bs, use_row_path=True)


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
def test_entry_without_row_index(ctx, sr):
    """Regression: the entry path on C and A without their per-row column
    indexes (as when there is no room for them): the applies stream the
    touched rows and the lost entries scan rows of A'.  R-MAT s12 with rows
    over 2048 entries in C, batches up to 3000 updates, against the oracle."""
    say(f"entry path without row index {SR_ID[sr]}")
    hi = 9 if sr == I.PLUS_TIMES_I64 else 100
    A = I.rmat_csr(12, 16, sr, stream=811, lo=1, hi=hi)
    bs = I.disjoint_batches(A, sr, [10, 300, 3000], stream=812, value_lo=1, value_hi=hi)
    st = run(ctx, sr, A, bs, row_index=0)
    assert sum(s["lost"] for s in st) > 0


def test_row_index_switch_is_checked(ctx):
    t = ctx.get_tuning()
    assert t.row_index == 1
    t.row_index = 2
    with pytest.raises(dsg.DsgError):
        ctx.set_tuning(t)
    ctx.set_tuning(None)


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
def test_entry_unconstrained_batches(ctx, sr):
    """Repeated keys, deletes of absent entries, SET over present entries and
    ADD chains in one batch."""
    say(f"entry path unconstrained {SR_ID[sr]}")
    rng = np.random.default_rng(31 + sr)
    keys = I.er_keys(300, 1500, rng)
    A = I.csr_from_keys(300, 300, keys, I.draw_values(sr, keys.size, rng, 1, 9))
    bs = [I.random_batch(300, 300, sr, sz, rng, op_probs=(0.4, 0.3, 0.3), hot_rows=40, hot_cols=60)
          for sz in (5, 50, 400, 2000)]
    run(ctx, sr, A, bs)


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
def test_entry_vanishing_entries(ctx, sr):
    """Deleting the only product of an entry removes the entry; deleting one
    of two keeps it with the other's value."""
    say(f"entry path vanishing {SR_ID[sr]}")
    n = 8
    # 0->1->2 (one path), 3->4->5 and 3->6->5 (two paths)
    edges = {(0, 1): 2, (1, 2): 3, (3, 4): 1, (4, 5): 1, (3, 6): 5, (6, 5): 5}
    keys = np.array(sorted(i * n + j for i, j in edges), np.int64)
    vdt = I.VALUE_DTYPE[sr]
    vals = np.array([edges[(int(k) // n, int(k) % n)] for k in keys]).astype(vdt)
    A = I.csr_from_keys(n, n, keys, vals)
    dels = I.Batch(np.array([0, 4], np.int32), np.array([1, 5], np.int32),
                   np.zeros(2, vdt), np.full(2, I.OP_DELETE, np.uint8))
    st = run(ctx, sr, A, [dels])
    assert st[0]["lost"] >= 1


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
@pytest.mark.parametrize("long_row", [3000, 9500])
def test_entry_long_rows(ctx, sr, long_row):
    """Lost entries in a row of A longer than the small LDS hash (and, at
    9500, longer than one chunk of the large one)."""
    say(f"entry path long rows {SR_ID[sr]} {long_row}")
    rng = np.random.default_rng(41 + long_row + sr)
    n = 12000
    hi = 9 if sr == I.PLUS_TIMES_I64 else 100
    row0 = np.sort(rng.choice(n, long_row, replace=False)).astype(np.int64)
    rest = I.er_keys(n, 3 * n, rng)
    keys = np.unique(np.concatenate([row0, rest]))
    A = I.csr_from_keys(n, n, keys, I.draw_values(sr, keys.size, rng, 1, hi))
    # delete / change entries of the long row, insert elsewhere
    k0 = keys[keys < n]
    pick = rng.choice(k0.size, 400, replace=False)
    rows = np.zeros(400, np.int32)
    cols = (k0[pick] % n).astype(np.int32)
    ops = np.where(np.arange(400) < 250, I.OP_DELETE, I.OP_SET).astype(np.uint8)
    vals = I.draw_values(sr, 400, rng, 1, hi)
    b1 = I.Batch(rows, cols, vals, ops)
    b2 = I.random_batch(n, n, sr, 2000, rng, op_probs=(0.5, 0.5, 0.0), value_lo=1, value_hi=hi)
    st = run(ctx, sr, A, [b1, b2])
    assert st[0]["lost"] > 0


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
def test_entry_needs_every_apply_logged(ctx, sr):
    """Two applies before an update: only the last one is logged, so the row
    path runs; the next single apply goes entry-granular again."""
    say(f"entry path fallback {SR_ID[sr]}")
    row_path(ctx, False)
    hi = 9 if sr == I.PLUS_TIMES_I64 else 100
    A = I.rmat_csr(9, 8, sr, stream=811, lo=1, hi=hi)
    bs = I.disjoint_batches(A, sr, [50, 50, 50], stream=812, value_lo=1, value_hi=hi)
    m = dsg.Matrix.from_csr(ctx, A, sr)
    P = dsg.Product(ctx, m, m)
    a = oracle.Csr.of(A)
    m.apply_batch(bs[0])
    m.apply_batch(bs[1])
    P.update()
    for b in bs[:2]:
        a, _ = oracle.apply(sr, a, b.rows, b.cols, b.vals, b.ops)
    assert P.stats()["path"] == 0
    assert_same_csr(sr, P.export(), oracle.spgemm(sr, a, a, nthreads=THREADS), "after two applies")
    m.apply_batch(bs[2])
    P.update()
    a, _ = oracle.apply(sr, a, bs[2].rows, bs[2].cols, bs[2].vals, bs[2].ops)
    assert P.stats()["path"] == 1
    assert_same_csr(sr, P.export(), oracle.spgemm(sr, a, a, nthreads=THREADS), "after one apply")
    # an update with nothing applied since reports no rows
    assert P.update().n == 0
    P.destroy()
    m.destroy()
    ctx.set_tuning(None)


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
def test_automatic_path_choice(ctx, sr):
    """The automatic choice follows the cost rule (entry-granular while the
    affected rows' products exceed entry_fixed + entry_per_term per changed
    product) and gives the row path's C bit for bit.  R-MAT s15, batches of
    200 and 30000 updates: with entry_per_term between the two batches'
    products-per-term ratios, the first goes entry-granular and the second
    to the row path."""
    say(f"automatic path {SR_ID[sr]}")
    d = ctx.get_tuning()
    assert (d.entry_fixed, d.entry_per_term) == (1e8, 70.0)
    hi = 9 if sr == I.PLUS_TIMES_I64 else 100
    A = I.rmat_csr(15, 16, sr, stream=821, lo=1, hi=hi)
    bs = I.disjoint_batches(A, sr, [200, 30000], stream=822, value_lo=1, value_hi=hi)

    def run_mode(mode, fixed=None, per_term=None):
        t = ctx.get_tuning()
        t.update_path = mode
        if fixed is not None:
            t.entry_fixed, t.entry_per_term = fixed, per_term
        ctx.set_tuning(t)
        m = dsg.Matrix.from_csr(ctx, A, sr)
        P = dsg.Product(ctx, m, m)
        st, Cs = [], []
        for b in bs:
            m.apply_batch(b)
            P.update()
            st.append(P.stats())
            Cs.append(P.export())
        P.destroy()
        m.destroy()
        ctx.set_tuning(None)
        return st, Cs

    rows = run_mode(1)
    entries = run_mode(2)
    ratio = [rows[0][k]["flops"] / entries[0][k]["terms"] for k in range(len(bs))]
    assert ratio[0] > ratio[1]
    per_term = (ratio[0] * ratio[1]) ** 0.5
    auto = run_mode(0, 0.0, per_term)
    chosen = [s["path"] for s in auto[0]]
    for k in range(len(bs)):
        # same inputs, so the forced runs' products and terms are the automatic run's
        want_entry = rows[0][k]["flops"] > per_term * entries[0][k]["terms"]
        assert chosen[k] == (1 if want_entry else 0), f"batch {k}"
        for other in (entries, auto):
            x, y = other[1][k], rows[1][k]
            assert np.array_equal(x.row_ptr, y.row_ptr) and np.array_equal(x.col, y.col)
            assert np.asarray(x.val).tobytes() == np.asarray(y.val).tobytes(), f"batch {k}"
    assert chosen == [1, 0]


def run_ab(ctx, sr, A, B, steps, use_row_path=False, trans_a=False, trans_b=False, same=False):
    """C = op(A)*op(B) (same: B is A, one matrix): each step applies a batch
    to A, to B or to both, then updates; C and the reported rows against the
    oracle after every step."""
    row_path(ctx, use_row_path)
    ma = dsg.Matrix.from_csr(ctx, A, sr)
    mb = ma if same else dsg.Matrix.from_csr(ctx, B, sr)
    P = dsg.Product(ctx, ma, mb, trans_a=trans_a, trans_b=trans_b)
    a, b = oracle.Csr.of(A), oracle.Csr.of(B)

    def want_of(a, b):
        x = oracle.transpose(a) if trans_a else a
        y = oracle.transpose(b) if trans_b else b
        return oracle.spgemm(sr, x, y, nthreads=THREADS)

    C = want_of(a, a if same else b)
    stats = []
    for t, (ba, bb) in enumerate(steps):
        if ba is not None:
            ma.apply_batch(ba)
            a, _ = oracle.apply(sr, a, ba.rows, ba.cols, ba.vals, ba.ops)
        if bb is not None:
            mb.apply_batch(bb)
            b, _ = oracle.apply(sr, b, bb.rows, bb.cols, bb.vals, bb.ops)
        rs = P.update()
        want = want_of(a, a if same else b)
        assert_same_csr(sr, P.export(), want, f"step {t}")
        assert np.array_equal(rs.row_ids(), changed_rows(C, want)), f"step {t}: reported rows"
        st = P.stats()
        stats.append(st)
        if not use_row_path:
            assert st["path"] == 1, f"step {t}: row path taken"
        C = want
    P.destroy()
    ma.destroy()
    if not same:
        mb.destroy()
    ctx.set_tuning(None)
    return stats


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
def test_entry_a_times_b(ctx, sr):
    """C = A*B on the entry path (Eq. 1 with both operands changing): batches
    to A alone, to B alone and to both, on R-MAT operands of different shapes
    (B's valued transpose and both column indexes built on first use), and
    the same steps on the row path."""
    say(f"entry path A*B {SR_ID[sr]}")
    hi = 9 if sr == I.PLUS_TIMES_I64 else 100
    A = I.rmat_csr(11, 8, sr, stream=821, lo=1, hi=hi)
    rng = np.random.default_rng(822)
    n, m = A.nrows, A.nrows + A.nrows // 2  # B is n x 1.5n: its keys take one more column bit than A's
    keys = np.unique(rng.integers(0, n, 12 * n, dtype=np.int64) * m + rng.integers(0, m, 12 * n, dtype=np.int64))
    B = I.csr_from_keys(n, m, keys, I.draw_values(sr, keys.size, rng, 1, hi))
    ba = I.disjoint_batches(A, sr, [10, 300, 2000, 50], stream=823, value_lo=1, value_hi=hi)
    bb = I.disjoint_batches(B, sr, [20, 500, 40, 1500], stream=824, value_lo=1, value_hi=hi)
    steps = [(ba[0], None), (None, bb[0]), (ba[1], bb[1]), (ba[2], None), (None, bb[2]), (ba[3], bb[3])]
    st = run_ab(ctx, sr, A, B, steps)
    assert sum(s["lost"] for s in st) > 0
    run_ab(ctx, sr, A, B, steps, use_row_path=True)


@pytest.mark.parametrize("sr", SRS, ids=lambda s: SR_ID[s])
def test_entry_transposed_operands(ctx, sr):
    """The entry path on transposed operands (each operand's changes read
    from its transpose index's log): C = A^T*B with batches to A alone, B
    alone and both; C = A*A^T and C = A^T*A^T with batches to A; the row path
    on the first for comparison."""
    say(f"entry path transposed {SR_ID[sr]}")
    hi = 9 if sr == I.PLUS_TIMES_I64 else 100
    A = I.rmat_csr(10, 8, sr, stream=831, lo=1, hi=hi)
    rng = np.random.default_rng(832)
    n, m = A.nrows, A.nrows + A.nrows // 2
    keys = np.unique(rng.integers(0, n, 10 * n, dtype=np.int64) * m + rng.integers(0, m, 10 * n, dtype=np.int64))
    B = I.csr_from_keys(n, m, keys, I.draw_values(sr, keys.size, rng, 1, hi))
    ba = I.disjoint_batches(A, sr, [20, 400, 1500, 60], stream=833, value_lo=1, value_hi=hi)
    bb = I.disjoint_batches(B, sr, [30, 300, 50, 900], stream=834, value_lo=1, value_hi=hi)
    steps = [(ba[0], None), (None, bb[0]), (ba[1], bb[1]), (ba[2], None), (None, bb[2]), (ba[3], bb[3])]
    st = run_ab(ctx, sr, A, B, steps, trans_a=True)
    assert sum(s["lost"] for s in st) > 0
    run_ab(ctx, sr, A, B, steps, trans_a=True, use_row_path=True)
    only_a = [(b, None) for b in ba]
    run_ab(ctx, sr, A, A, only_a, trans_b=True, same=True)
    run_ab(ctx, sr, A, A, only_a, trans_a=True, trans_b=True, same=True)
