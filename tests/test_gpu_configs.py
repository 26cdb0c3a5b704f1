"""GPU parity at the full sizes of the evaluation workloads, in the launch
configuration the benchmark uses (default tuning, one product per workload).

Every check compares the whole product C' exported from the GPU with the
oracle's static recompute of the updated operands, plus the reported
changed rows against the rows whose content really changed.
"""
import sys

import numpy as np
import pytest

import oracle
from gpu_util import THREADS, assert_same_csr, changed_rows
from paper_2202_08808_amd import dsg
from paper_2202_08808_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return dsg.Context(0)


class Tracker:
    """GPU objects plus the oracle's copy of the operands and of C."""

    def __init__(self, ctx, w):
        self.w = w
        self.sr = w.semiring
        self.Am = dsg.Matrix.from_csr(ctx, w.A, self.sr)
        self.Bm = self.Am if w.B is None else dsg.Matrix.from_csr(ctx, w.B, self.sr)
        self.P = dsg.Product(ctx, self.Am, self.Bm)
        self.a = oracle.Csr.of(w.A)
        self.b = None if w.B is None else oracle.Csr.of(w.B)
        self.C = None

    def right(self):
        return self.a if self.b is None else self.b

    def check_full(self, what):
        want = oracle.spgemm(self.sr, self.a, self.right(), nthreads=THREADS)
        got = self.P.export()
        assert_same_csr(self.sr, got, want, what, A=self.a, B=self.right())
        return want

    def step(self, t, what):
        ba = self.w.batches_A[t]
        self.Am.apply_batch(ba)
        self.a, _ = oracle.apply(self.sr, self.a, ba.rows, ba.cols, ba.vals, ba.ops)
        if self.b is not None:
            bb = self.w.batches_B[t]
            self.Bm.apply_batch(bb)
            self.b, _ = oracle.apply(self.sr, self.b, bb.rows, bb.cols, bb.vals, bb.ops)
        rs = self.P.update()
        want = self.check_full(what)
        truth = changed_rows(self.C, want)
        got_rows = rs.row_ids()
        if self.sr != I.PLUS_TIMES_F64:
            assert np.array_equal(got_rows, truth), f"{what}: reported rows differ"
        else:
            assert set(truth.tolist()) <= set(got_rows.tolist()), f"{what}: a changed row was not reported"
        self.C = want
        return rs

    def close(self):
        self.P.destroy()
        if self.Bm is not self.Am:
            self.Bm.destroy()
        self.Am.destroy()


@pytest.mark.parametrize("batch", [100, 1000, 10000, 100000])
def test_rmat16_minplus(ctx, batch):
    """R-MAT scale 16, edge factor 16, min-plus fp32, batches mixed 50/25/25."""
    say(f"rmat16 min-plus batch {batch}")
    w = I.workload_rmat16_minplus(batch=batch, n_batches=2)
    tr = Tracker(ctx, w)
    tr.C = tr.check_full("static")
    for t in range(2):
        tr.step(t, f"batch {t} of {batch}")
    tr.close()


def test_stencil_fp64(ctx):
    """9-point stencil 1024^2 times random 8-per-row, fp64; each batch holds
    1e4 value changes and 1e3 insertions in each of A and B."""
    say("stencil fp64")
    w = I.workload_stencil_f64(n_batches=2)
    tr = Tracker(ctx, w)
    tr.C = tr.check_full("static")
    for t in range(2):
        tr.step(t, f"batch {t}")
    tr.close()


def test_er2m_minplus(ctx):
    """Erdos-Renyi, 2^21 rows, mean degree 8, min-plus fp32."""
    say("er 2M min-plus")
    w = I.workload_er_minplus(n_batches=2, batch=3000)
    tr = Tracker(ctx, w)
    tr.C = tr.check_full("static")
    for t in range(2):
        tr.step(t, f"batch {t}")
    tr.close()
