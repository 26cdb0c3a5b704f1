"""GPU: dsg_rows_export_noalloc (the row export for callers that cannot
allocate device memory) gives what dsg_rows_export gives, allocates nothing
on the context, and rejects views beyond its fixed staging."""
import sys

import numpy as np
import pytest

from paper_2202_08808_amd import dsg
from paper_2202_08808_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def same(x, y, what):
    for a, b, name in zip(x, y, ("rows", "row_ptr", "col", "val")):
        assert np.asarray(a).tobytes() == np.asarray(b).tobytes(), f"{what}: {name} differ"


@pytest.mark.parametrize("sr", [I.MIN_PLUS_F32, I.PLUS_TIMES_I64, I.PLUS_TIMES_F64], ids=["minplus", "i64", "f64"])
def test_noalloc_export_matches_export(sr):
    """Two calls in a row, the second on a smaller view: the changed rows of an
    update, then a few listed rows (with repeats); each equals
    dsg_rows_export bit for bit, and the context holds the same device bytes
    before and after."""
    say(f"no-alloc row export, semiring {sr}")
    ctx = dsg.Context(0)
    lo, hi = (1, 100) if sr == I.MIN_PLUS_F32 else (1, 9)
    A = I.rmat_csr(12, 8, sr, stream=900 + sr, lo=lo, hi=hi)
    m = dsg.Matrix.from_csr(ctx, A, sr)
    P = dsg.Product(ctx, m, m)
    b = I.disjoint_batches(A, sr, [300], stream=910 + sr, value_lo=lo, value_hi=hi)[0]
    m.apply_batch(b)
    rs = P.update()
    assert rs.n > 100
    first = rs.to_host()
    held = ctx.memory()
    got = rs.to_host_noalloc()
    assert ctx.memory() == held, "the allocation-free export changed the context's device memory"
    same(got, first, "changed rows")
    assert first[2].size > 0
    rows = np.array([5, 0, 4095, 5, 77], np.int32)
    small = P.rows(rows)
    want = small.to_host()
    held = ctx.memory()
    got = small.to_host_noalloc()
    assert ctx.memory() == held
    same(got, want, "listed rows")
    assert got[2].size < first[2].size
    P.destroy()
    m.destroy()
    ctx.close()


def test_noalloc_export_limits():
    """Views beyond the staging array's rows or entries, and too little room,
    give DSG_E_ARG; a view at the row limit still works."""
    say("no-alloc row export limits")
    sr = I.MIN_PLUS_F32
    ctx = dsg.Context(0)
    A = I.rmat_csr(12, 8, sr, stream=920, lo=1, hi=100)
    m = dsg.Matrix.from_csr(ctx, A, sr)
    P = dsg.Product(ctx, m, m)
    lens = np.diff(P.export().row_ptr)
    short = int(np.argmin(lens))  # at most 8 entries, so the row limit stays within the entry limit
    assert lens[short] <= 8
    ok = P.rows(np.full(1 << 18, short, np.int32))
    same(ok.to_host_noalloc(), ok.to_host(), "view at the row limit")
    with pytest.raises(dsg.DsgError) as e:
        P.rows(np.full((1 << 18) + 1, short, np.int32)).to_host_noalloc()
    assert e.value.status == dsg.E_ARG
    longest = int(np.argmax(lens))
    reps = (1 << 21) // int(lens[longest]) + 1
    with pytest.raises(dsg.DsgError) as e:
        P.rows(np.full(reps, longest, np.int32)).to_host_noalloc()
    assert e.value.status == dsg.E_ARG
    with pytest.raises(dsg.DsgError) as e:
        P.rows(np.array([longest], np.int32)).to_host_noalloc(cap=int(lens[longest]) - 1)
    assert e.value.status == dsg.E_ARG
    # still usable after the refusals
    v = P.rows(np.array([longest, short], np.int32))
    same(v.to_host_noalloc(), v.to_host(), "after refusals")
    P.destroy()
    m.destroy()
    ctx.close()
