"""Seeded synthetic inputs for batch-dynamic SpGEMM.

This module only draws numbers: graph structures (R-MAT, Erdos-Renyi, 9-point
stencil, k-per-row random), values and update batches.  It contains none of
the method's arithmetic (no semiring, no product, no update semantics), so
both the CPU oracle and the GPU path may consume what it produces.

Every generator is deterministic in its seed: ``numpy.random.Generator(PCG64)``
seeded from ``SeedSequence([2202, 8808, stream, index])``.

The workloads stand in for the paper's real-world graphs (Section 7.1,
Table I), which are not available; the paper itself uses R-MAT graphs with the
Graph500 parameters for its synthetic scaling runs (Section 7.2, "Scalability
on Synthetic Graphs"), permuting vertex labels (Section 7.1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence

import numpy as np

# Update operation codes (same numbering as the C ABI).
OP_SET = 0      # insert-or-overwrite ("merge", Section 4.1)
OP_DELETE = 1   # remove if present ("mask", Section 4.1)
OP_ADD = 2      # a <- a (+) x, insert x if absent (algebraic update, Section 4.1)

# Semiring ids (same numbering as the C ABI); they fix the value dtype.
PLUS_TIMES_I64 = 0
MIN_PLUS_F32 = 1
PLUS_TIMES_F64 = 2
OR_AND_U32 = 3

VALUE_DTYPE = {PLUS_TIMES_I64: np.int64, MIN_PLUS_F32: np.float32,
               PLUS_TIMES_F64: np.float64, OR_AND_U32: np.uint32}


def rng_for(stream: int, index: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([2202, 8808, stream, index])))


@dataclasses.dataclass
class Csr:
    """Host CSR with rows sorted by column and no duplicate keys."""
    nrows: int
    ncols: int
    row_ptr: np.ndarray  # int64[nrows+1]
    col: np.ndarray      # int32[nnz]
    val: np.ndarray      # dtype by semiring

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row_of_entry(self) -> np.ndarray:
        return np.repeat(np.arange(self.nrows, dtype=np.int32), np.diff(self.row_ptr))

    def keys(self) -> np.ndarray:
        return self.row_of_entry().astype(np.int64) * self.ncols + self.col.astype(np.int64)


@dataclasses.dataclass
class Batch:
    """One update batch as structure-of-arrays, in batch order."""
    rows: np.ndarray  # int32[b]
    cols: np.ndarray  # int32[b]
    vals: np.ndarray  # value dtype [b]
    ops: np.ndarray   # uint8[b]

    def __len__(self) -> int:
        return int(self.rows.shape[0])


def csr_from_keys(nrows: int, ncols: int, keys: np.ndarray, vals: np.ndarray) -> Csr:
    """Build a CSR from unique int64 keys (row*ncols+col) sorted ascending."""
    keys = np.asarray(keys, np.int64)
    rows = keys // ncols
    cols = (keys % ncols).astype(np.int32)
    counts = np.bincount(rows, minlength=nrows).astype(np.int64)
    rp = np.zeros(nrows + 1, np.int64)
    np.cumsum(counts, out=rp[1:])
    return Csr(nrows, ncols, rp, cols, np.ascontiguousarray(vals))


# ----------------------------------------------------------------------------
# Structures
# ----------------------------------------------------------------------------

def rmat_keys(scale: int, edge_factor: int, rng: np.random.Generator,
              a: float = 0.57, b: float = 0.19, c: float = 0.19) -> np.ndarray:
    """R-MAT edge keys with the Graph500 quadrant probabilities.

    Draws ``edge_factor * 2**scale`` directed edges; at each of ``scale`` bit
    levels a quadrant is chosen with probabilities (a, b, c, 1-a-b-c).  No
    noise.  Vertex labels are relabelled by a seeded random permutation.
    Duplicates are removed, self-loops kept.  Returns sorted unique keys.
    """
    n = 1 << scale
    m = edge_factor << scale
    r = np.zeros(m, np.int64)
    s = np.zeros(m, np.int64)
    for bit in range(scale):
        u = rng.random(m)
        rbit = u >= a + b                       # quadrants c, d: lower half
        cbit = ((u >= a) & (u < a + b)) | (u >= a + b + c)  # quadrants b, d
        r |= rbit.astype(np.int64) << bit
        s |= cbit.astype(np.int64) << bit
    perm = rng.permutation(n).astype(np.int64)
    return np.unique(perm[r] * n + perm[s])


def er_keys(n: int, m: int, rng: np.random.Generator) -> np.ndarray:
    """G(n, m): m uniform directed pairs (self-loops allowed), deduplicated."""
    r = rng.integers(0, n, m, dtype=np.int64)
    s = rng.integers(0, n, m, dtype=np.int64)
    return np.unique(r * n + s)


def stencil9_keys(side: int) -> np.ndarray:
    """9-point stencil (3x3 neighbourhood incl. centre) on a non-periodic grid.

    Row/column r = y*side + x.  nnz = (3*side - 2)**2.
    """
    n = side * side
    y, x = np.divmod(np.arange(n, dtype=np.int64), side)
    out = []
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            yy, xx = y + dy, x + dx
            ok = (yy >= 0) & (yy < side) & (xx >= 0) & (xx < side)
            out.append(np.arange(n, dtype=np.int64)[ok] * n + (yy * side + xx)[ok])
    return np.sort(np.concatenate(out))


def k_per_row_keys(nrows: int, ncols: int, k: int, rng: np.random.Generator) -> np.ndarray:
    """Exactly k distinct uniformly random columns per row."""
    # rejection in vectorised rounds: redraw every row that holds a duplicate
    need = np.arange(nrows)
    cols = rng.integers(0, ncols, (nrows, k), dtype=np.int64)
    while True:
        srt = np.sort(cols[need], axis=1)
        dup = (srt[:, 1:] == srt[:, :-1]).any(axis=1)
        need = need[dup]
        if need.size == 0:
            break
        cols[need] = rng.integers(0, ncols, (need.size, k), dtype=np.int64)
    keys = np.arange(nrows, dtype=np.int64)[:, None] * ncols + cols
    return np.sort(keys.ravel())


# ----------------------------------------------------------------------------
# Values
# ----------------------------------------------------------------------------

def draw_values(semiring: int, count: int, rng: np.random.Generator,
                lo: int = 1, hi: int = 9) -> np.ndarray:
    """Values by workload family: uniform integers in [lo, hi] for int64,
    min-plus fp32 (stored as float32) and 32-bit words (uint32), N(0, 1) for
    fp64."""
    if semiring == PLUS_TIMES_I64:
        return rng.integers(lo, hi + 1, count, dtype=np.int64)
    if semiring == MIN_PLUS_F32:
        return rng.integers(lo, hi + 1, count, dtype=np.int64).astype(np.float32)
    if semiring == PLUS_TIMES_F64:
        return rng.standard_normal(count)
    if semiring == OR_AND_U32:
        return rng.integers(lo, hi + 1, count, dtype=np.uint64).astype(np.uint32)
    raise ValueError(semiring)


# ----------------------------------------------------------------------------
# Update batches
# ----------------------------------------------------------------------------

def sample_absent(keyspace_rows: int, ncols: int, present: np.ndarray, count: int,
                  rng: np.random.Generator,
                  accept: Optional[Callable[[np.ndarray], np.ndarray]] = None) -> np.ndarray:
    """``count`` distinct keys drawn uniformly from positions not in ``present``
    (sorted int64 keys), by rejection.  ``accept`` may narrow the positions."""
    got = np.empty(0, np.int64)
    total = keyspace_rows * ncols
    while got.size < count:
        want = int((count - got.size) * 1.2) + 16
        cand = rng.integers(0, total, want, dtype=np.int64)
        pos = np.searchsorted(present, cand)
        pos = np.minimum(pos, max(present.size - 1, 0))
        ok = (present[pos] != cand) if present.size else np.ones(cand.size, bool)
        if accept is not None:
            ok &= accept(cand)
        cand = cand[ok]
        # keep first occurrence only, preserve draw order
        allk = np.concatenate([got, cand])
        _, first = np.unique(allk, return_index=True)
        got = allk[np.sort(first)]
    return got[:count]


def disjoint_batches(base: Csr, semiring: int, sizes: Sequence[int], mix=(0.5, 0.25, 0.25),
                     stream: int = 0, value_lo: int = 1, value_hi: int = 9,
                     accept_insert: Optional[Callable[[np.ndarray], np.ndarray]] = None
                     ) -> List[Batch]:
    """A sequence of update batches whose touched positions are pairwise
    disjoint over the whole sequence.

    Inserts (op SET) go to positions absent from ``base`` (uniform, rejection);
    deletes (op DELETE) and value changes (op SET with a fresh value) go to
    entries present in ``base``, uniform without replacement.  Because no
    position is touched twice, each insert lands on a position that is absent
    when its batch is applied and each delete/change on one that is present,
    whatever the order of application.  Ops are shuffled within a batch.
    """
    rng = rng_for(stream, 0)
    sizes = list(sizes)
    n_ins = [int(round(s * mix[0])) for s in sizes]
    n_del = [int(round(s * mix[1])) for s in sizes]
    n_chg = [s - a - d for s, a, d in zip(sizes, n_ins, n_del)]
    present = base.keys()
    ins_all = sample_absent(base.nrows, base.ncols, present, sum(n_ins), rng, accept_insert)
    need_present = sum(n_del) + sum(n_chg)
    if need_present > present.size:
        raise ValueError("not enough present entries for disjoint deletes/changes")
    pick = rng.choice(present.size, need_present, replace=False)
    pres_all = present[pick]
    out = []
    io = po = 0
    for t, s in enumerate(sizes):
        brng = rng_for(stream, t + 1)
        ins = ins_all[io:io + n_ins[t]]; io += n_ins[t]
        dele = pres_all[po:po + n_del[t]]; po += n_del[t]
        chg = pres_all[po:po + n_chg[t]]; po += n_chg[t]
        keys = np.concatenate([ins, dele, chg])
        ops = np.concatenate([np.full(ins.size, OP_SET, np.uint8),
                              np.full(dele.size, OP_DELETE, np.uint8),
                              np.full(chg.size, OP_SET, np.uint8)])
        vals = draw_values(semiring, keys.size, brng, value_lo, value_hi)
        vals[ins.size:ins.size + dele.size] = 0
        order = brng.permutation(keys.size)
        keys, ops, vals = keys[order], ops[order], vals[order]
        out.append(Batch((keys // base.ncols).astype(np.int32),
                         (keys % base.ncols).astype(np.int32),
                         np.ascontiguousarray(vals), ops))
    return out


def random_batch(nrows: int, ncols: int, semiring: int, size: int, rng: np.random.Generator,
                 op_probs=(0.5, 0.3, 0.2), hot_rows: Optional[int] = None,
                 hot_cols: Optional[int] = None, value_lo: int = 1, value_hi: int = 9) -> Batch:
    """An unconstrained batch: ops drawn with ``op_probs`` over (SET, DELETE,
    ADD), positions uniform in a (hot_rows x hot_cols) corner so that repeated
    keys, deletes of absent entries and inserts over present ones all occur."""
    hr = nrows if hot_rows is None else min(hot_rows, nrows)
    hc = ncols if hot_cols is None else min(hot_cols, ncols)
    rows = rng.integers(0, hr, size, dtype=np.int64).astype(np.int32)
    cols = rng.integers(0, hc, size, dtype=np.int64).astype(np.int32)
    ops = rng.choice(3, size, p=np.asarray(op_probs) / sum(op_probs)).astype(np.uint8)
    vals = draw_values(semiring, size, rng, value_lo, value_hi)
    return Batch(rows, cols, np.ascontiguousarray(vals), ops)


# ----------------------------------------------------------------------------
# Workloads (shapes of the five evaluation configurations)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    semiring: int
    A: Csr
    B: Optional[Csr]          # None means C = A*A
    batches_A: List[Batch]
    batches_B: List[Batch]    # empty unless B is a separate operand


def rmat_csr(scale: int, edge_factor: int, semiring: int, stream: int,
             lo: int = 1, hi: int = 9) -> Csr:
    rng = rng_for(stream, 0)
    keys = rmat_keys(scale, edge_factor, rng)
    n = 1 << scale
    vals = draw_values(semiring, keys.size, rng_for(stream, 1), lo, hi)
    return csr_from_keys(n, n, keys, vals)


def workload_rmat12_i64(n_batches: int = 1, batch: int = 100) -> Workload:
    """R-MAT scale 12, edge factor 8, plus-times int64, values 1..9, C = A*A;
    batches of uniformly random insertions at absent positions."""
    A = rmat_csr(12, 8, PLUS_TIMES_I64, stream=101)
    bs = disjoint_batches(A, PLUS_TIMES_I64, [batch] * n_batches, mix=(1.0, 0.0, 0.0), stream=102)
    return Workload("rmat12_ef8_plus_times_i64", PLUS_TIMES_I64, A, None, bs, [])


def workload_rmat16_minplus(batch: int = 10000, n_batches: int = 10, scale: int = 16,
                            edge_factor: int = 16) -> Workload:
    """R-MAT scale 16, edge factor 16, min-plus fp32 with integer weights in
    [1, 100], C = A*A; batches mixed 50% inserts, 25% deletes, 25% changes."""
    A = rmat_csr(scale, edge_factor, MIN_PLUS_F32, stream=201, lo=1, hi=100)
    bs = disjoint_batches(A, MIN_PLUS_F32, [batch] * n_batches, stream=202 + batch % 997,
                          value_lo=1, value_hi=100)
    return Workload(f"rmat{scale}_ef{edge_factor}_min_plus_f32_b{batch}", MIN_PLUS_F32, A, None, bs, [])


def workload_stencil_f64(side: int = 1024, n_batches: int = 10, n_change: int = 10000,
                         n_insert: int = 1000) -> Workload:
    """A = 9-point stencil on side x side grid, B = 8 random distinct columns per
    row, both N(0,1), fp64 plus-times, C = A*B.  Each batch: n_change value
    changes plus n_insert new entries in each of A (off-stencil) and B."""
    n = side * side
    ka = stencil9_keys(side)
    A = csr_from_keys(n, n, ka, draw_values(PLUS_TIMES_F64, ka.size, rng_for(301, 1)))
    kb = k_per_row_keys(n, n, 8, rng_for(302, 0))
    B = csr_from_keys(n, n, kb, draw_values(PLUS_TIMES_F64, kb.size, rng_for(302, 1)))
    tot = n_change + n_insert
    mix = (n_insert / tot, 0.0, n_change / tot)

    def off_stencil(keys):
        r, c = np.divmod(keys, n)
        ry, rx = np.divmod(r, side)
        cy, cx = np.divmod(c, side)
        return (np.abs(ry - cy) > 1) | (np.abs(rx - cx) > 1)

    ba = disjoint_batches(A, PLUS_TIMES_F64, [tot] * n_batches, mix=mix, stream=303,
                          accept_insert=off_stencil)
    bb = disjoint_batches(B, PLUS_TIMES_F64, [tot] * n_batches, mix=mix, stream=304)
    return Workload(f"stencil{side}_x_rand8_plus_times_f64", PLUS_TIMES_F64, A, B, ba, bb)


def workload_er_minplus(n: int = 1 << 21, mean_degree: int = 8, n_batches: int = 1,
                        batch: int = 1000) -> Workload:
    """Erdos-Renyi G(n, m = mean_degree*n), min-plus fp32 weights in [1, 100], C = A*A."""
    keys = er_keys(n, mean_degree * n, rng_for(501, 0))
    A = csr_from_keys(n, n, keys, draw_values(MIN_PLUS_F32, keys.size, rng_for(501, 1), 1, 100))
    bs = disjoint_batches(A, MIN_PLUS_F32, [batch] * n_batches, stream=502, value_lo=1, value_hi=100)
    return Workload(f"er{n}_d{mean_degree}_min_plus_f32", MIN_PLUS_F32, A, None, bs, [])


def batched_instances(count: int = 64, stream: int = 401, max_scale: int = 16):
    """Descriptors of the batched-form instances: scale ~ U{10..max_scale},
    edge factor ~ U{4, 8, 16, 32}, semiring alternating (even index int64
    plus-times, odd index min-plus fp32), batch size floor(10**U(1, 4))."""
    rng = rng_for(stream, 0)
    out = []
    for t in range(count):
        scale = int(rng.integers(10, max_scale + 1))
        ef = int(rng.choice([4, 8, 16, 32]))
        sr = PLUS_TIMES_I64 if t % 2 == 0 else MIN_PLUS_F32
        b = int(math.floor(10 ** rng.uniform(1, 4)))
        out.append((scale, ef, sr, b))
    return out


@dataclasses.dataclass
class Request:
    """One request of a serving trace."""
    t: float                        # arrival time in seconds from the start
    kind: str                       # "update" or "query"
    batch: Optional[Batch] = None   # update entries
    rows: Optional[np.ndarray] = None  # query rows (int32, distinct)


def serve_trace(base: Csr, semiring: int, n_requests: int, rate: float, stream: int = 601,
                query_frac: float = 0.5, size_mu: float = 3.0, size_sigma: float = 0.67,
                size_lo: float = 1.0, size_hi: float = 5.0, max_query_rows: int = 1024,
                value_lo: int = 1, value_hi: int = 100) -> List[Request]:
    """Poisson arrivals at ``rate`` requests/s.  A request is a query with
    probability ``query_frac`` (1..max_query_rows distinct uniform rows), else
    an update batch of floor(10**X) entries, X ~ N(size_mu, size_sigma)
    truncated to [size_lo, size_hi], mix 50/25/25, positions disjoint over the
    whole trace (see disjoint_batches)."""
    rng = rng_for(stream, 0)
    t = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    is_query = rng.random(n_requests) < query_frac
    n_upd = int((~is_query).sum())
    x = np.clip(rng.normal(size_mu, size_sigma, n_upd), size_lo, size_hi)
    sizes = np.floor(10.0 ** x).astype(np.int64)
    batches = disjoint_batches(base, semiring, sizes, stream=stream + 1, value_lo=value_lo, value_hi=value_hi)
    qn = rng.integers(1, max_query_rows + 1, n_requests - n_upd)
    out, u, q = [], 0, 0
    for k in range(n_requests):
        if is_query[k]:
            rows = np.sort(rng.choice(base.nrows, min(int(qn[q]), base.nrows), replace=False)).astype(np.int32)
            out.append(Request(float(t[k]), "query", rows=rows))
            q += 1
        else:
            out.append(Request(float(t[k]), "update", batch=batches[u]))
            u += 1
    return out
