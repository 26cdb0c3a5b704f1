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


@pytest.mark.parametrize("force_bin", [8, 9], ids=["dense", "global"])
def test_batched_forced_long_bins_in_graph(ctx, force_bin):
    """Every row of every instance in the dense (8) or global-hash (9) bin,
    all instances inside the captured graph (whose persistent grids read the
    bin sizes on the device), over two replays: bitwise equal to the plain
    loop under the same tuning, and to the oracle."""
    import torch
    say(f"batched, every row forced to bin {force_bin}, all in the graph")
    tu = ctx.get_tuning()
    tu.batch_direct_log2 = 62
    tu.force_bin = force_bin
    tu.update_path = 1  # the plain copy takes the row path, as the graph does
    ctx.set_tuning(tu)
    try:
        inst = instances(4, 17, scales=(9, 12))
        plain, batched, oracles = [], [], []
        for sr, A, _ in inst:
            a1 = dsg.Matrix.from_csr(ctx, A, sr)
            plain.append((a1, dsg.Product(ctx, a1, a1)))
            a2 = dsg.Matrix.from_csr(ctx, A, sr)
            batched.append((a2, dsg.Product(ctx, a2, a2)))
            oracles.append(oracle.Csr.of(A))
        B = dsg.Batch(ctx, [p for _, p in batched])
        rng = np.random.default_rng(21)
        bufs = None
        for rnd in range(2):
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
                got_batch = p2.export()
                assert_same_csr(sr, got_batch, p1.export(), f"round {rnd} instance {t}")
                assert counts[t] == rs.n
                b = batches[t]
                oracles[t], _ = oracle.apply(sr, oracles[t], b.rows, b.cols, b.vals, b.ops)
                want = oracle.spgemm(sr, oracles[t], oracles[t])
                assert_same_csr(sr, got_batch, want, f"oracle round {rnd} instance {t}")
                assert np.array_equal(B.rows(t).row_ids(), changed_rows(C_before, want))
            # the plain copy runs under the same tuning as the captured graph
            st = plain[0][1].stats()
            assert st["bin_rows"][force_bin] == st["affected_rows"] > 0, "rows left the forced bin"
        info = B.info()
        assert info["replays"] == 2 and info["direct"] == 0
        B.destroy()
        for a, p in plain + batched:
            p.destroy()
            a.destroy()
        torch.cuda.synchronize()
    finally:
        ctx.set_tuning(None)


@pytest.mark.timeout(600)
def test_batched_config4_shape(ctx):
    """The batched workload's own instances (R-MAT scales 10..16, edge factors
    {4, 8, 16, 32}, int64 plus-times and min-plus alternating, batches of
    floor(10^U(1, 4)) entries, mix 50/25/25) with the default tuning, so that
    small products run in the captured graph -- rows wider than 4096 columns
    reach the dense bin there -- and large ones on the plain path beside it.
    Two rounds; every instance's C equals the oracle's static recompute, and
    its reported rows are the rows whose content changed.  The seven scale-16
    instances of edge factor 16 and 32 (C of 1.6e8..3.6e8 entries) stay out:
    the oracle alone would take minutes on them."""
    import torch
    say("batched, config-4 instances")
    desc = [(t, d) for t, d in enumerate(I.batched_instances(64)) if not (d[0] == 16 and d[1] >= 16)]
    objs, host, prev, rounds = [], [], [], []
    for t, (scale, ef, sr, b) in desc:
        lo, hi = (1, 9) if sr == I.PLUS_TIMES_I64 else (1, 100)
        A = I.rmat_csr(scale, ef, sr, stream=1000 + t, lo=lo, hi=hi)
        try:
            bs = I.disjoint_batches(A, sr, [b] * 2, stream=2000 + t, value_lo=lo, value_hi=hi)
        except ValueError:
            rng = I.rng_for(2000 + t, 1)
            bs = [I.random_batch(A.nrows, A.ncols, sr, b, rng, op_probs=(0.75, 0.25, 0.0), value_lo=lo,
                                 value_hi=hi) for _ in range(2)]
        a = dsg.Matrix.from_csr(ctx, A, sr)
        objs.append((a, dsg.Product(ctx, a, a)))
        host.append(oracle.Csr.of(A))
        rounds.append(bs)
        prev.append(None)
    say(f"{len(desc)} instances set up")
    B = dsg.Batch(ctx, [p for _, p in objs])
    bufs = [to_dev(rounds[q][0]) for q in range(len(desc))]
    for rnd in range(2):
        if rnd:
            for q in range(len(desc)):
                for x, y in zip(bufs[q], to_dev(rounds[q][rnd])):
                    x.copy_(y)
        torch.cuda.synchronize()
        counts = B.run([(objs[q][0], *bufs[q]) for q in range(len(desc))])
        for q, (t, (scale, ef, sr, b)) in enumerate(desc):
            bt = rounds[q][rnd]
            before = prev[q] if prev[q] is not None else oracle.spgemm(sr, host[q], host[q], nthreads=8)
            host[q], _ = oracle.apply(sr, host[q], bt.rows, bt.cols, bt.vals, bt.ops)
            want = oracle.spgemm(sr, host[q], host[q], nthreads=8)
            got = objs[q][1].export()
            assert_same_csr(sr, got, want, f"round {rnd} instance {t} (s{scale} ef{ef} b{b})")
            truth = changed_rows(before, want)
            assert counts[q] == truth.size, f"round {rnd} instance {t}: reported row count"
            assert np.array_equal(B.rows(q).row_ids(), truth), f"round {rnd} instance {t}: reported rows"
            prev[q] = want
        say(f"round {rnd} checked")
    info = B.info()
    assert info["replays"] == 2 and 0 < info["direct"] < 2 * len(desc)
    B.destroy()
    for a, p in objs:
        p.destroy()
        a.destroy()
    torch.cuda.synchronize()


def test_batch_rejects_shared_operands(ctx):
    """Two products over one matrix, or one product listed twice, cannot be
    batched (each matrix takes its updates in one product's chain)."""
    say("batched operand sharing rejected")
    sr = I.MIN_PLUS_F32
    A = I.rmat_csr(8, 4, sr, stream=790, lo=1, hi=100)
    a = dsg.Matrix.from_csr(ctx, A, sr)
    b = dsg.Matrix.from_csr(ctx, A, sr)
    p1 = dsg.Product(ctx, a, a)
    p2 = dsg.Product(ctx, a, a)
    p3 = dsg.Product(ctx, b, a)
    p4 = dsg.Product(ctx, b, b)
    for prods in ([p1, p2], [p1, p1], [p1, p3], [p4, p3]):
        with pytest.raises(dsg.DsgError) as e:
            dsg.Batch(ctx, prods)
        assert e.value.status == dsg.E_STATE
    ok = dsg.Batch(ctx, [p1, p4])  # disjoint operands, each product A A
    ok.destroy()
    for p in (p1, p2, p3, p4):
        p.destroy()
    a.destroy()
    b.destroy()
