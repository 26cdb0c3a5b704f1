"""GPU: a context whose device memory comes from the caller's allocator
(dsg_ctx_set_allocator; here PyTorch's caching allocator) gives the same
results, holds its blocks in that allocator while it lives and returns all
of them; an allocator that refuses gives DSG_E_OOM."""
import sys

import numpy as np
import pytest

import oracle
from gpu_util import assert_same_csr
from paper_2202_08808_amd import dsg
from paper_2202_08808_amd import inputs as I

pytestmark = pytest.mark.gpu

SR = I.MIN_PLUS_F32


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def test_torch_allocator_holds_and_returns_every_block():
    import torch
    say("torch caching allocator")
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    ctx = dsg.Context(0, stream=torch.cuda.current_stream(), allocator="torch")
    A0 = I.rmat_csr(11, 8, SR, stream=1300, lo=1, hi=100)
    a = dsg.Matrix.from_csr(ctx, A0, SR)
    P = dsg.Product(ctx, a, a)
    h = oracle.Csr.of(A0)
    for b in I.disjoint_batches(A0, SR, [50, 500, 2000], stream=1301, value_lo=1, value_hi=100):
        a.apply_batch(b)
        P.update()
        h, _ = oracle.apply(SR, h, b.rows, b.cols, b.vals, b.ops)
        assert_same_csr(SR, P.export(), oracle.spgemm(SR, h, h), "with the torch allocator")
    held = ctx.memory()
    assert held > 0
    assert torch.cuda.memory_allocated() - base >= held, "the context's blocks are not in torch's allocator"
    # the served form allocates from its own threads
    e = a.export()
    cur = I.Csr(e.nrows, e.ncols, e.row_ptr, e.col, e.val)
    S = dsg.Server(ctx, P)
    for b in I.disjoint_batches(cur, SR, [300, 300], stream=1302, value_lo=1, value_hi=100):
        S.submit_batch(a, b)
        h, _ = oracle.apply(SR, h, b.rows, b.cols, b.vals, b.ops)
    S.drain()
    S.destroy()
    assert_same_csr(SR, P.export(), oracle.spgemm(SR, h, h), "served, with the torch allocator")
    assert ctx.L.dsg_ctx_set_allocator(ctx.h, None) == dsg.E_STATE  # not while it holds memory
    P.destroy()
    a.destroy()
    ctx.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base, "blocks left in torch's allocator"


def test_refusing_allocator_gives_oom():
    say("refusing allocator")
    calls = {"n": 0}

    def alloc(nbytes, stream, user):
        calls["n"] += 1
        return None

    def free(ptr, nbytes, stream, user):
        raise AssertionError("nothing was allocated")
    al = dsg.Allocator(dsg._ALLOC_FN(alloc), dsg._FREE_FN(free), None)
    ctx = dsg.Context(0, allocator=al)
    A0 = I.rmat_csr(8, 4, SR, stream=1310, lo=1, hi=100)
    with pytest.raises(dsg.DsgError) as e:
        dsg.Matrix.from_csr(ctx, A0, SR)
    assert e.value.status == dsg.E_OOM
    assert calls["n"] >= 1 and ctx.memory() == 0
    ctx.close()


def test_allocator_only_before_the_first_allocation():
    say("allocator set late")
    ctx = dsg.Context(0)
    a = dsg.Matrix.from_csr(ctx, I.rmat_csr(8, 4, SR, stream=1320, lo=1, hi=100), SR)
    st = ctx.L.dsg_ctx_set_allocator(ctx.h, dsg.ctypes.byref(dsg.torch_allocator(0)))
    assert st == dsg.E_STATE
    a.destroy()
    ctx.close()
