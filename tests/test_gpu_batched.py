"""GPU: the batched form (one hipGraph replay for many instances) gives the
same C, bit for bit, and the same reported rows as the plain per-instance
loop, and matches the oracle."""
import sys

import numpy as np
import pytest

import oracle
from gpu_util import assert_same_csr, changed_rows
from paper_2202_08808_amd import dsg
from paper_2202_08808_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return dsg.Context(0)


def instances(count, seed, scales=(8, 11)):
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        sr = I.PLUS_TIMES_I64 if t % 2 == 0 else I.MIN_PLUS_F32
        scale = int(rng.integers(scales[0], scales[1] + 1))
        ef = int(rng.choice([4, 8, 16]))
        A = I.rmat_csr(scale, ef, sr, stream=700 + t, lo=1, hi=9 if sr == I.PLUS_TIMES_I64 else 100)
        out.append((sr, A, int(10 ** rng.uniform(1, 3))))
    return out


def to_dev(b):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (b.rows, b.cols, b.vals, b.ops)]


@pytest.mark.parametrize("direct_log2", [24, 16, 0], ids=["graph", "mixed", "direct"])
def test_batched_equals_plain_loop(ctx, direct_log2):
    """All instances in the graph (C under 2^24 slots), a mix (the three with
    C over 2^16 slots take the plain path beside the replay), and none."""
    import torch
    say(f"batched vs plain loop, direct from 2^{direct_log2}")
    tu = ctx.get_tuning()
    tu.batch_direct_log2 = direct_log2
    ctx.set_tuning(tu)
    inst = instances(6, 3)
    plain, batched, oracles = [], [], []
    for sr, A, _ in inst:
        a1 = dsg.Matrix.from_csr(ctx, A, sr)
        plain.append((a1, dsg.Product(ctx, a1, a1)))
        a2 = dsg.Matrix.from_csr(ctx, A, sr)
        batched.append((a2, dsg.Product(ctx, a2, a2)))
        oracles.append(oracle.Csr.of(A))
    B = dsg.Batch(ctx, [p for _, p in batched])
    # fixed device buffers, refilled each round, so the graph is replayed
    rng = np.random.default_rng(9)
    bufs = None
    for rnd in range(3):
        batches = [I.random_batch(A.nrows, A.ncols, sr, nb, rng, value_lo=1, value_hi=9)
                   for (sr, A, nb) in inst]
        dev = [to_dev(b) for b in batches]
        if bufs is None:
            bufs = dev
        else:
            for d, s in zip(bufs, dev):
                for x, y in zip(d, s):
                    x.copy_(y)
        torch.cuda.synchronize()
        counts = B.run([(batched[t][0], *bufs[t]) for t in range(len(inst))])
        for t, ((sr, A, _), (a1, p1), (a2, p2)) in enumerate(zip(inst, plain, batched)):
            C_before = p1.export()
            a1.apply_batch(batches[t])
            rs = p1.update()
            got_plain, got_batch = p1.export(), p2.export()
            assert_same_csr(sr, got_batch, got_plain, f"round {rnd} instance {t}")
            assert counts[t] == rs.n
            assert np.array_equal(B.rows(t).row_ids(), rs.row_ids())
            b = batches[t]
            oracles[t], _ = oracle.apply(sr, oracles[t], b.rows, b.cols, b.vals, b.ops)
            want = oracle.spgemm(sr, oracles[t], oracles[t])
            assert_same_csr(sr, got_batch, want, f"oracle round {rnd} instance {t}")
            assert np.array_equal(rs.row_ids(), changed_rows(C_before, want))
    info = B.info()
    if direct_log2 == 24:
        assert info["replays"] == 3 and info["captures"] >= 1 and info["direct"] == 0
    elif direct_log2 == 0:
        assert info["replays"] == 0 and info["direct"] == 3 * len(inst)
    else:
        assert info["replays"] == 3 and 0 < info["direct"] < 3 * len(inst)
    ctx.set_tuning(None)
    B.destroy()
    for a, p in plain + batched:
        p.destroy()
        a.destroy()


def test_batched_defers_when_room_is_short(ctx):
    """An instance whose C grows far beyond the room set aside is completed
    by the plain path with the same result."""
    import torch
    say("batched deferral")
    sr = I.PLUS_TIMES_I64
    A = I.csr_from_keys(300, 300, np.array([5], np.int64), np.array([1], np.int64))
    a = dsg.Matrix.from_csr(ctx, A, sr)
    p = dsg.Product(ctx, a, a)
    B = dsg.Batch(ctx, [p])
    rng = np.random.default_rng(1)
    b = I.random_batch(300, 300, sr, 20000, rng, op_probs=(1, 0, 0))
    counts = B.run([(a, *to_dev(b))])
    assert B.info()["deferred"] == 1
    want_a, _ = oracle.apply(sr, oracle.Csr.of(A), b.rows, b.cols, b.vals, b.ops)
    want = oracle.spgemm(sr, want_a, want_a)
    assert_same_csr(sr, p.export(), want, "after deferral")
    assert counts[0] == len(changed_rows(oracle.spgemm(sr, oracle.Csr.of(A), oracle.Csr.of(A)), want))
    B.destroy()
    p.destroy()
    a.destroy()
    torch.cuda.synchronize()


def to_dev_bits(b):
    """Device copies of a batch; 32-bit words travel as int32 (same bits)."""
    import torch
    vals = np.ascontiguousarray(b.vals)
    if vals.dtype == np.uint32:
        vals = vals.view(np.int32)
    return [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (b.rows, b.cols, vals, b.ops)]


@pytest.mark.parametrize("direct_log2", [24, 0], ids=["graph", "direct"])
def test_batched_boolean_and_fp64(ctx, direct_log2):
    """Bitwise (or, and) products (A A and A^T A) and an fp64 A B in one batch,
    in the graph and on the plain path, against the oracle and the reported
    rows against the changed rows."""
    import torch
    say(f"batched boolean and fp64, direct from 2^{direct_log2}")
    tu = ctx.get_tuning()
    tu.batch_direct_log2 = direct_log2
    ctx.set_tuning(tu)
    try:
        rng = np.random.default_rng(77)
        specs = [(I.OR_AND_U32, False, True), (I.OR_AND_U32, True, True), (I.PLUS_TIMES_F64, False, False)]
        objs, host = [], []
        for t, (sr, ta, square) in enumerate(specs):
            lo, hi = (0, (1 << 32) - 1) if sr == I.OR_AND_U32 else (1, 9)
            A = I.rmat_csr(10, 8, sr, stream=760 + t, lo=lo, hi=hi)
            a = dsg.Matrix.from_csr(ctx, A, sr)
            if square:
                b, B = a, A
            else:
                B = I.rmat_csr(10, 8, sr, stream=770 + t, lo=lo, hi=hi)
                b = dsg.Matrix.from_csr(ctx, B, sr)
            p = dsg.Product(ctx, a, b, trans_a=ta)
            objs.append((a, b, p))
            host.append([oracle.Csr.of(A), oracle.Csr.of(B), None])
        for j, (sr, ta, square) in enumerate(specs):
            ha = host[j]
            ha[2] = oracle.spgemm(sr, oracle.transpose(ha[0]) if ta else ha[0], ha[0] if square else ha[1])
        bx = dsg.Batch(ctx, [p for _, _, p in objs])
        for rnd in range(3):
            sets, keep = [], []
            for j, (sr, ta, square) in enumerate(specs):
                a, b, p = objs[j]
                ba = I.random_batch(1024, 1024, sr, 60 * (rnd + 1), rng)
                dev = to_dev_bits(ba)
                keep.append(dev)
                sets.append((a, *dev))
                host[j][0], _ = oracle.apply(sr, host[j][0], ba.rows, ba.cols, ba.vals, ba.ops)
                if not square:
                    bb = I.random_batch(1024, 1024, sr, 30 * (rnd + 1), rng)
                    dev = to_dev_bits(bb)
                    keep.append(dev)
                    sets.append((b, *dev))
                    host[j][1], _ = oracle.apply(sr, host[j][1], bb.rows, bb.cols, bb.vals, bb.ops)
            counts = bx.run(sets)
            for j, (sr, ta, square) in enumerate(specs):
                ha = host[j]
                lhs = oracle.transpose(ha[0]) if ta else ha[0]
                rhs = ha[0] if square else ha[1]
                want = oracle.spgemm(sr, lhs, rhs)
                assert_same_csr(sr, objs[j][2].export(), want, f"round {rnd} product {j}", A=lhs, B=rhs)
                if sr != I.PLUS_TIMES_F64:
                    assert counts[j] == len(changed_rows(ha[2], want)), f"round {rnd} product {j}: row count"
                ha[2] = want
        bx.destroy()
        for a, b, p in objs:
            p.destroy()
        for a, b, p in objs:
            if b is not a:
                b.destroy()
            a.destroy()
        torch.cuda.synchronize()
    finally:
        ctx.set_tuning(None)
