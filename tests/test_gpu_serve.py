"""GPU: the served form (request loop with continuous batching) gives every
request the result it gets alone -- updates applied one at a time in arrival
order, each query answered from the state after the updates submitted before
it -- and matches the oracle."""
import sys

import numpy as np
import pytest

import oracle
from gpu_util import THREADS, assert_same_csr, rows_of
from paper_2202_08808_amd import dsg
from paper_2202_08808_amd import inputs as I

pytestmark = pytest.mark.gpu

SR = I.MIN_PLUS_F32


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return dsg.Context(0)


def er(n, seed):
    keys = I.er_keys(n, 8 * n, I.rng_for(seed, 0))
    return I.csr_from_keys(n, n, keys, I.draw_values(SR, keys.size, I.rng_for(seed, 1), 1, 100))


def small_trace(A, n_requests, seed):
    return I.serve_trace(A, SR, n_requests, 1000.0, stream=seed, size_mu=1.6, size_sigma=0.6, size_hi=2.7,
                         max_query_rows=64)


def oracle_answers(A, trace):
    """Query answers and final C of the trace applied one request at a time."""
    a = oracle.Csr.of(A)
    C = oracle.spgemm(SR, a, a, nthreads=THREADS)
    answers = []
    for r in trace:
        if r.kind == "update":
            b = r.batch
            a, _ = oracle.apply(SR, a, b.rows, b.cols, b.vals, b.ops)
            C = None
        else:
            if C is None:
                C = oracle.spgemm(SR, a, a, nthreads=THREADS)
            answers.append(rows_of(C, r.rows))
    if C is None:
        C = oracle.spgemm(SR, a, a, nthreads=THREADS)
    return answers, C


def run_served(ctx, A, trace, alone=False, **cfg):
    """Submit the trace (all at once, or each request after the previous one
    completed) and return (query answers, final C, per-request results, stats)."""
    m = dsg.Matrix.from_csr(ctx, A, SR)
    P = dsg.Product(ctx, m, m)
    S = dsg.Server(ctx, P, **cfg)
    tickets = []
    for r in trace:
        if r.kind == "update":
            t = S.submit_batch(m, r.batch)
        else:
            t = S.submit_query(r.rows)
        tickets.append(t)
        if alone:
            S.poll(t, wait=True)
    S.drain()
    results = [S.poll(t) for t in tickets]
    answers = [S.query_result(t) for t, r in zip(tickets, trace) if r.kind == "query"]
    stats = S.stats()
    for t in tickets:
        S.release(t)
    S.destroy()
    C = P.export()
    P.destroy()
    m.destroy()
    return answers, C, results, stats


def same_rows(x, y, what):
    assert np.array_equal(x.row_ptr, y.row_ptr), f"{what}: row pointers differ"
    assert np.array_equal(x.col, y.col), f"{what}: columns differ"
    assert np.asarray(x.val).tobytes() == np.asarray(y.val).tobytes(), f"{what}: values differ"


def test_served_equals_alone_and_oracle(ctx):
    say("served mix vs alone vs oracle")
    A = er(4096, 11)
    trace = small_trace(A, 80, 611)
    want_answers, want_C = oracle_answers(A, trace)
    mix = run_served(ctx, A, trace)
    alone = run_served(ctx, A, trace, alone=True)
    for name, (answers, C, results, stats) in (("mix", mix), ("alone", alone)):
        assert all(r["status"] == dsg.OK for r in results), name
        assert len(answers) == len(want_answers)
        for k, (got, want) in enumerate(zip(answers, want_answers)):
            assert_same_csr(SR, got, want, f"{name} query {k}")
        assert_same_csr(SR, C, want_C, f"{name} final C")
        assert stats["update_requests"] + stats["query_requests"] == len(trace)
    # each result the same alone and in the mix, bit for bit
    for k, (x, y) in enumerate(zip(mix[0], alone[0])):
        same_rows(x, y, f"query {k}")
    same_rows(mix[1], alone[1], "final C")
    # alone, no group carries more than one request
    assert all(r["group_requests"] == 1 for r in alone[2])
    say(f"mix: {mix[3]['update_groups']} update groups for {mix[3]['update_requests']} update requests, "
        f"{mix[3]['query_groups']} query groups for {mix[3]['query_requests']} queries")


def test_served_memory_budget_admits_one_at_a_time(ctx):
    """A budget smaller than any group: every group holds one request (each
    runs alone) and the results still match the oracle."""
    say("served tiny budget")
    A = er(2048, 12)
    trace = small_trace(A, 40, 621)
    want_answers, want_C = oracle_answers(A, trace)
    answers, C, results, stats = run_served(ctx, A, trace, mem_budget=1)
    assert all(r["group_requests"] == 1 for r in results)
    assert stats["update_groups"] == stats["update_requests"]
    for k, (got, want) in enumerate(zip(answers, want_answers)):
        assert_same_csr(SR, got, want, f"query {k}")
    assert_same_csr(SR, C, want_C, "final C")


def test_served_coalesces_queued_updates(ctx):
    """Updates queued behind a long-running group are merged (coalescing
    limit respected) and give the same C as one at a time."""
    say("served coalescing")
    A = er(4096, 13)
    bs = I.disjoint_batches(A, SR, [3000] + [20] * 30, stream=631, value_lo=1, value_hi=100)
    trace = [I.Request(0.0, "update", batch=b) for b in bs]
    _, want_C = oracle_answers(A, trace)
    answers, C, results, stats = run_served(ctx, A, trace, max_coalesce=100, slots=1)
    assert_same_csr(SR, C, want_C, "final C")
    assert max(r["group_requests"] for r in results) <= 5  # 20-entry requests, at most 100 entries per group
    assert stats["update_entries"] == sum(len(b.ops) for b in bs)


def test_served_product_of_two_operands(ctx):
    """A*B served, updates alternating between A and B."""
    say("served A*B")
    A = er(2048, 14)
    B = er(2048, 15)
    ba = I.disjoint_batches(A, SR, [50] * 6, stream=641, value_lo=1, value_hi=100)
    bb = I.disjoint_batches(B, SR, [50] * 6, stream=642, value_lo=1, value_hi=100)
    ma, mb = dsg.Matrix.from_csr(ctx, A, SR), dsg.Matrix.from_csr(ctx, B, SR)
    P = dsg.Product(ctx, ma, mb)
    S = dsg.Server(ctx, P)
    a, b = oracle.Csr.of(A), oracle.Csr.of(B)
    qt, want = [], []
    rng = np.random.default_rng(5)
    for x, y in zip(ba, bb):
        S.submit_batch(ma, x)
        S.submit_batch(mb, y)
        a, _ = oracle.apply(SR, a, x.rows, x.cols, x.vals, x.ops)
        b, _ = oracle.apply(SR, b, y.rows, y.cols, y.vals, y.ops)
        rows = np.sort(rng.choice(2048, 50, replace=False)).astype(np.int32)
        qt.append(S.submit_query(rows))
        want.append(rows_of(oracle.spgemm(SR, a, b, nthreads=THREADS), rows))
    S.drain()
    for k, (t, w) in enumerate(zip(qt, want)):
        assert_same_csr(SR, S.query_result(t), w, f"query {k}")
    S.destroy()
    assert_same_csr(SR, P.export(), oracle.spgemm(SR, a, b, nthreads=THREADS), "final C")
    P.destroy()
    ma.destroy()
    mb.destroy()


@pytest.mark.parametrize("sr,ta,tb", [(I.MIN_PLUS_F32, True, False), (I.MIN_PLUS_F32, False, True),
                                       (I.OR_AND_U32, True, False)], ids=["AtB", "ABt", "orand-AtB"])
def test_served_transposed_product(ctx, sr, ta, tb):
    """A served product with a transposed operand (and the bitwise (or, and)
    semiring): updates go to the caller's matrices, queries read op(A) op(B)."""
    say(f"served transposed {sr} {ta} {tb}")
    n = 1500
    lo, hi = (0, (1 << 32) - 1) if sr == I.OR_AND_U32 else (1, 100)

    def mat(seed):
        keys = I.er_keys(n, 8 * n, I.rng_for(seed, 0))
        return I.csr_from_keys(n, n, keys, I.draw_values(sr, keys.size, I.rng_for(seed, 1), lo, hi))
    A, B = mat(16), mat(17)
    ba = I.disjoint_batches(A, sr, [40] * 5, stream=651, value_lo=lo, value_hi=hi)
    bb = I.disjoint_batches(B, sr, [40] * 5, stream=652, value_lo=lo, value_hi=hi)
    ma, mb = dsg.Matrix.from_csr(ctx, A, sr), dsg.Matrix.from_csr(ctx, B, sr)
    P = dsg.Product(ctx, ma, mb, trans_a=ta, trans_b=tb)
    S = dsg.Server(ctx, P)
    a, b = oracle.Csr.of(A), oracle.Csr.of(B)

    def want_c():
        return oracle.spgemm(sr, oracle.transpose(a) if ta else a, oracle.transpose(b) if tb else b,
                             nthreads=THREADS)
    qt, want = [], []
    rng = np.random.default_rng(6)
    for x, y in zip(ba, bb):
        S.submit_batch(ma, x)
        S.submit_batch(mb, y)
        a, _ = oracle.apply(sr, a, x.rows, x.cols, x.vals, x.ops)
        b, _ = oracle.apply(sr, b, y.rows, y.cols, y.vals, y.ops)
        rows = np.sort(rng.choice(n, 40, replace=False)).astype(np.int32)
        qt.append(S.submit_query(rows))
        want.append(rows_of(want_c(), rows))
    S.drain()
    for k, (t, w) in enumerate(zip(qt, want)):
        assert_same_csr(sr, S.query_result(t), w, f"query {k}")
    S.destroy()
    assert_same_csr(sr, P.export(), want_c(), "final C")
    P.destroy()
    ma.destroy()
    mb.destroy()


def test_served_errors_and_ownership(ctx):
    say("served errors")
    A = er(1024, 16)
    m = dsg.Matrix.from_csr(ctx, A, SR)
    P = dsg.Product(ctx, m, m)
    S = dsg.Server(ctx, P)
    with pytest.raises(dsg.DsgError) as e:
        S.submit_update(m, np.array([5000], np.int32), np.array([0], np.int32), np.array([1], np.float32),
                        np.array([0], np.uint8))
    assert e.value.status == dsg.E_RANGE
    with pytest.raises(dsg.DsgError) as e:
        S.submit_query(np.array([-1], np.int32))
    assert e.value.status == dsg.E_RANGE
    # while served, the context's objects are the server's
    with pytest.raises(dsg.DsgError) as e:
        P.update()
    assert e.value.status == dsg.E_STATE
    with pytest.raises(dsg.DsgError) as e:
        dsg.Server(ctx, P)
    assert e.value.status == dsg.E_STATE
    t = S.submit_query(np.arange(10, dtype=np.int32))
    assert S.poll(t, wait=True)["status"] == dsg.OK
    S.destroy()
    # returned to the caller
    P.update()
    P.destroy()
    m.destroy()


@pytest.mark.timeout(600)
def test_served_config5_scale(ctx):
    """The serving workload at full size: Erdos-Renyi with 2^21 rows and mean
    degree 8 (16.8M entries), C = A A over (min,+) resident in HBM, a Poisson
    trace of update batches of floor(10^X) entries (X ~ N(3, 0.67) on [1, 5],
    mix 50/25/25) and queries of 1..1024 rows.  Every query answer and the
    final C equal the oracle's, both when the whole trace is queued at once
    (continuous batching) and when each request runs alone, and the two runs
    agree bit for bit."""
    say("served at full size: ER 2^21")
    n = 1 << 21
    A = er(n, 501)
    trace = I.serve_trace(A, SR, 24, 1e9, stream=681)
    say(f"trace: {sum(r.kind == 'update' for r in trace)} updates "
        f"({sum(len(r.batch.ops) for r in trace if r.kind == 'update')} entries), "
        f"{sum(r.kind == 'query' for r in trace)} queries")
    a = oracle.Csr.of(A)
    want_answers = []
    for r in trace:
        if r.kind == "update":
            b = r.batch
            a, _ = oracle.apply(SR, a, b.rows, b.cols, b.vals, b.ops)
        else:
            want_answers.append(oracle.spgemm(SR, a, a, rows=r.rows, nthreads=THREADS))
    want_C = oracle.spgemm(SR, a, a, nthreads=THREADS)
    mix = run_served(ctx, A, trace, mem_budget=4 << 30)
    say(f"mix: {mix[3]['update_groups']} update groups for {mix[3]['update_requests']} updates")
    alone = run_served(ctx, A, trace, alone=True, mem_budget=4 << 30)
    for name, (answers, C, results, stats) in (("mix", mix), ("alone", alone)):
        assert all(r["status"] == dsg.OK for r in results), name
        assert len(answers) == len(want_answers)
        for k, (got, want) in enumerate(zip(answers, want_answers)):
            assert_same_csr(SR, got, want, f"{name} query {k}")
        assert_same_csr(SR, C, want_C, f"{name} final C")
    for k, (x, y) in enumerate(zip(mix[0], alone[0])):
        same_rows(x, y, f"query {k}")
    same_rows(mix[1], alone[1], "final C")
