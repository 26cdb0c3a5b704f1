"""Thin Python binding of ``libdsg.so`` (declared in ``include/dsg.h``).

Argument marshalling only: every step of the update and multiply path runs in
the library's HIP kernels.  Arrays may be numpy arrays (host memory) or torch
tensors on the GPU (device memory, passed with DSG_INPUT_DEVICE).  The
library is required: importing this module fails loudly if it is missing.
"""
from __future__ import annotations

import ctypes
import json
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdsg.so")

OK, E_ARG, E_RANGE, E_OOM, E_DEVICE, E_STATE, E_UNSUPPORTED = range(7)
PLUS_TIMES_I64, MIN_PLUS_F32, PLUS_TIMES_F64, OR_AND_U32 = 0, 1, 2, 3
OP_SET, OP_DELETE, OP_ADD = 0, 1, 2
INPUT_DEVICE, SYNC, REPORT_AFFECTED = 0x1, 0x2, 0x4
TRANS_A, TRANS_B, GENERAL_BLOOM = 0x1, 0x2, 0x4
DTYPE = {PLUS_TIMES_I64: np.int64, MIN_PLUS_F32: np.float32, PLUS_TIMES_F64: np.float64,
         OR_AND_U32: np.uint32}
NAMES = {OK: "DSG_OK", E_ARG: "DSG_E_ARG", E_RANGE: "DSG_E_RANGE", E_OOM: "DSG_E_OOM",
         E_DEVICE: "DSG_E_DEVICE", E_STATE: "DSG_E_STATE", E_UNSUPPORTED: "DSG_E_UNSUPPORTED"}

P = ctypes.c_void_p


class DsgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{NAMES.get(status, status)}: {msg}")
        self.status = status


class Rows(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("rows", P), ("row_off", P), ("row_len", P), ("col", P),
                ("val", P)]


class Tuning(ctypes.Structure):
    _fields_ = [("group_ub", ctypes.c_int32 * 8), ("dense_max_passes", ctypes.c_int32),
                ("force_bin", ctypes.c_int32), ("update_path", ctypes.c_int32), ("batch_direct_log2", ctypes.c_int32),
                ("entry_fixed", ctypes.c_double), ("entry_per_term", ctypes.c_double),
                ("row_index", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("affected_rows", ctypes.c_int64), ("changed_rows", ctypes.c_int64),
                ("a_entries", ctypes.c_int64), ("flops", ctypes.c_int64),
                ("nnz_new", ctypes.c_int64), ("nnz_old", ctypes.c_int64),
                ("bin_rows", ctypes.c_int64 * 10), ("bin_flops", ctypes.c_int64 * 10),
                ("path", ctypes.c_int32), ("pad", ctypes.c_int32), ("terms", ctypes.c_int64),
                ("entries", ctypes.c_int64), ("lost", ctypes.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if not k.startswith("bin_") and k != "pad"}
        d["bin_rows"] = list(self.bin_rows)
        d["bin_flops"] = list(self.bin_flops)
        return d


class BatchStats(ctypes.Structure):
    _fields_ = [("captures", ctypes.c_int64), ("replays", ctypes.c_int64), ("deferred", ctypes.c_int64),
                ("prepare_ms", ctypes.c_double), ("capture_ms", ctypes.c_double),
                ("replay_ms", ctypes.c_double), ("finish_ms", ctypes.c_double), ("direct", ctypes.c_int64),
                ("direct_ms", ctypes.c_double)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("mem_budget", ctypes.c_size_t), ("max_coalesce", ctypes.c_int64),
                ("max_query_rows", ctypes.c_int32), ("slots", ctypes.c_int32)]


class ServerResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("kind", ctypes.c_int32), ("latency_ms", ctypes.c_double),
                ("group", ctypes.c_int64), ("group_requests", ctypes.c_int32), ("changed_rows", ctypes.c_int32),
                ("nq", ctypes.c_int32), ("nnz", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("update_requests", ctypes.c_int64), ("query_requests", ctypes.c_int64),
                ("update_entries", ctypes.c_int64), ("update_groups", ctypes.c_int64),
                ("query_groups", ctypes.c_int64), ("update_p50_ms", ctypes.c_double),
                ("update_p99_ms", ctypes.c_double), ("update_mean_ms", ctypes.c_double),
                ("query_p50_ms", ctypes.c_double), ("query_p99_ms", ctypes.c_double),
                ("query_mean_ms", ctypes.c_double), ("busy_ms", ctypes.c_double),
                ("updates_per_s", ctypes.c_double), ("peak_inflight_bytes", ctypes.c_size_t)]


PENDING = -1

_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", ctypes.c_void_p)]


def torch_allocator(device: int = 0) -> Allocator:
    """dsg_allocator callbacks on PyTorch's caching allocator: blocks come from
    torch.cuda.caching_allocator_alloc on the context's stream."""
    import torch

    def alloc(nbytes, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device=device, stream=int(stream or 0))
        except RuntimeError:
            return None

    def free(ptr, nbytes, stream, user):
        torch.cuda.caching_allocator_delete(ptr)
    return Allocator(_ALLOC_FN(alloc), _FREE_FN(free), None)

SIGNATURES = {
    "dsg_ctx_create": [ctypes.c_int, P, ctypes.c_size_t, P],
    "dsg_ctx_destroy": [P],
    "dsg_ctx_set_allocator": [P, P],
    "dsg_ctx_synchronize": [P],
    "dsg_ctx_memory": [P, P],
    "dsg_ctx_set_timing": [P, ctypes.c_int],
    "dsg_ctx_set_timing_phase": [P, ctypes.c_char_p],
    "dsg_ctx_timing_report": [P, ctypes.c_char_p, ctypes.c_size_t],
    "dsg_ctx_get_tuning": [P, P],
    "dsg_ctx_set_tuning": [P, P],
    "dsg_mat_create": [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, P, P, P, ctypes.c_uint32, P],
    "dsg_mat_apply": [P, P, P, P, P, ctypes.c_int64, ctypes.c_uint32],
    "dsg_mat_nnz": [P, P],
    "dsg_mat_shape": [P, P, P, P],
    "dsg_mat_export": [P, P, P, P, ctypes.c_int64, P],
    "dsg_mat_destroy": [P],
    "dsg_prod_create_static": [P, P, P, P],
    "dsg_prod_create": [P, P, P, ctypes.c_uint32, P],
    "dsg_prod_scale_add": [P, P, P, P, P],
    "dsg_prod_recompute_static": [P, ctypes.c_uint32],
    "dsg_prod_update": [P, ctypes.c_uint32, P],
    "dsg_prod_rows": [P, P, ctypes.c_int32, ctypes.c_uint32, P],
    "dsg_rows_export": [P, P, P, P, P, ctypes.c_int64, P],
    "dsg_rows_export_noalloc": [P, P, P, P, P, ctypes.c_int64, P],
    "dsg_prod_nnz": [P, P],
    "dsg_prod_export": [P, P, P, P, ctypes.c_int64, P],
    "dsg_prod_export_bloom": [P, P, P, P, ctypes.c_int64, P],
    "dsg_prod_stats": [P, P],
    "dsg_prod_autotune": [P, ctypes.c_int32, P, P, ctypes.c_char_p, ctypes.c_size_t],
    "dsg_prod_destroy": [P],
    "dsg_batch_create": [P, P, ctypes.c_int32, P],
    "dsg_batch_run": [P, P, ctypes.c_int32, ctypes.c_uint32, P],
    "dsg_batch_rows": [P, ctypes.c_int32, P],
    "dsg_batch_info": [P, P],
    "dsg_batch_destroy": [P],
    "dsg_server_create": [P, P, P, P],
    "dsg_server_submit_update": [P, P, P, P, P, P, ctypes.c_int64, P],
    "dsg_server_submit_query": [P, P, ctypes.c_int32, P],
    "dsg_server_poll": [P, ctypes.c_uint64, ctypes.c_int32, P],
    "dsg_server_query_result": [P, ctypes.c_uint64, P, P, P, ctypes.c_int64, P],
    "dsg_server_release": [P, ctypes.c_uint64],
    "dsg_server_drain": [P],
    "dsg_server_stats_get": [P, P],
    "dsg_server_destroy": [P],
}


class UpdateSet(ctypes.Structure):
    _fields_ = [("mat", P), ("rows", P), ("cols", P), ("vals", P), ("ops", P), ("n", ctypes.c_int64)]


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`"
                          " (the GPU path has no fallback)")
    # PyTorch-ROCm ships its own HIP runtime under the same soname as the
    # system one.  Loading torch first makes the library bind to that copy, so
    # the process holds one HIP runtime and torch's buffers and streams are
    # usable by the library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(path)
    for name, args in SIGNATURES.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.dsg_last_error.argtypes = [P]
    L.dsg_last_error.restype = ctypes.c_char_p
    return L


_L: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _L
    if _L is None:
        _L = load()
    return _L


def _ptr(a):
    """(pointer, is_device) of a numpy array or a torch tensor."""
    if a is None:
        return None, False
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be contiguous")
        return a.ctypes.data_as(P), False
    if hasattr(a, "data_ptr") and hasattr(a, "is_cuda"):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return P(a.data_ptr()), bool(a.is_cuda)
    raise TypeError(f"unsupported array type {type(a)}")


class Context:
    def __init__(self, device: int = 0, stream=None, budget: int = 0, allocator=None):
        """stream: a torch.cuda.Stream (or None for the library's own).
        allocator: None (hipMalloc), "torch" (PyTorch's caching allocator)
        or an Allocator."""
        self.L = lib()
        h = P()
        s = None if stream is None else P(stream.cuda_stream)
        self._check(self.L.dsg_ctx_create(device, s, budget, ctypes.byref(h)), None)
        self.h = h
        self._allocator = None
        if allocator is not None:
            a = torch_allocator(device) if allocator == "torch" else allocator
            self._check(self.L.dsg_ctx_set_allocator(self.h, ctypes.byref(a)))
            self._allocator = a  # the callbacks live as long as the context

    def _check(self, st, h="self"):
        if st != OK:
            hh = self.h if h == "self" else h
            msg = self.L.dsg_last_error(hh)
            raise DsgError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None):
            self._check(self.L.dsg_ctx_destroy(self.h))
            self.h = None

    def synchronize(self):
        self._check(self.L.dsg_ctx_synchronize(self.h))

    def memory(self) -> int:
        v = ctypes.c_size_t()
        self._check(self.L.dsg_ctx_memory(self.h, ctypes.byref(v)))
        return v.value

    def set_timing(self, on: bool, phase: Optional[str] = None):
        """Per-phase HIP-event timing; with phase, only phases of that name."""
        self._check(self.L.dsg_ctx_set_timing_phase(self.h, phase.encode() if phase else None))
        self._check(self.L.dsg_ctx_set_timing(self.h, 1 if on else 0))

    def timing_report(self) -> dict:
        buf = ctypes.create_string_buffer(1 << 16)
        self._check(self.L.dsg_ctx_timing_report(self.h, buf, len(buf)))
        return json.loads(buf.value.decode())

    def get_tuning(self) -> Tuning:
        t = Tuning()
        self._check(self.L.dsg_ctx_get_tuning(self.h, ctypes.byref(t)))
        return t

    def set_tuning(self, t: Optional[Tuning]):
        self._check(self.L.dsg_ctx_set_tuning(self.h, None if t is None else ctypes.byref(t)))


class Matrix:
    def __init__(self, ctx: Context, nrows: int, ncols: int, semiring: int, row_ptr=None, col=None, val=None):
        self.ctx, self.L = ctx, ctx.L
        self.nrows, self.ncols, self.semiring = int(nrows), int(ncols), int(semiring)
        h = P()
        flags = 0
        prp, dev = _ptr(row_ptr)
        pci, _ = _ptr(col)
        pv, _ = _ptr(val)
        if dev:
            flags |= INPUT_DEVICE
        ctx._check(self.L.dsg_mat_create(ctx.h, self.nrows, self.ncols, self.semiring, prp, pci, pv, flags,
                                         ctypes.byref(h)))
        self.h = h

    @classmethod
    def _wrap(cls, ctx: Context, h, nrows: int, ncols: int, semiring: int):
        """A Matrix around a handle the library created."""
        m = cls.__new__(cls)
        m.ctx, m.L = ctx, ctx.L
        m.nrows, m.ncols, m.semiring = int(nrows), int(ncols), int(semiring)
        m.h = h
        return m

    @classmethod
    def from_csr(cls, ctx: Context, csr, semiring: int):
        return cls(ctx, csr.nrows, csr.ncols, semiring, np.ascontiguousarray(csr.row_ptr, np.int64),
                   np.ascontiguousarray(csr.col, np.int32),
                   np.ascontiguousarray(csr.val, DTYPE[semiring]))

    def apply(self, rows, cols, vals, ops, sync: bool = False):
        n = int(rows.shape[0])
        pr, dev = _ptr(rows)
        pc, _ = _ptr(cols)
        pv, _ = _ptr(vals)
        po, _ = _ptr(ops)
        flags = (INPUT_DEVICE if dev else 0) | (SYNC if sync else 0)
        self.ctx._check(self.L.dsg_mat_apply(self.h, pr, pc, pv, po, n, flags))

    def apply_batch(self, b, sync: bool = False):
        self.apply(b.rows, b.cols, b.vals, b.ops, sync)

    def nnz(self) -> int:
        v = ctypes.c_int64()
        self.ctx._check(self.L.dsg_mat_nnz(self.h, ctypes.byref(v)))
        return v.value

    def export(self):
        return _export(self.ctx, self.L.dsg_mat_export, self.h, self.nrows, self.ncols, self.semiring)

    def destroy(self):
        if self.h:
            self.ctx._check(self.L.dsg_mat_destroy(self.h))
            self.h = None


class Csr:
    def __init__(self, nrows, ncols, row_ptr, col, val):
        self.nrows, self.ncols = nrows, ncols
        self.row_ptr, self.col, self.val = row_ptr, col, val

    @property
    def nnz(self):
        return int(self.row_ptr[-1])


def _export(ctx, fn, h, nrows, ncols, semiring):
    nnz = ctypes.c_int64()
    rp = np.zeros(nrows + 1, np.int64)
    ctx._check(fn(h, rp.ctypes.data_as(P), None, None, 0, ctypes.byref(nnz)))
    col = np.zeros(max(nnz.value, 1), np.int32)
    val = np.zeros(max(nnz.value, 1), DTYPE[semiring])
    ctx._check(fn(h, rp.ctypes.data_as(P), col.ctypes.data_as(P), val.ctypes.data_as(P), col.size,
                  ctypes.byref(nnz)))
    return Csr(nrows, ncols, rp, col[:nnz.value], val[:nnz.value])


class RowSet:
    """Device views returned by Product.update / Product.rows."""

    def __init__(self, prod: "Product", v: Rows):
        self.prod, self.v = prod, v

    @property
    def n(self) -> int:
        return int(self.v.n)

    def to_host(self):
        """(rows, row_ptr, col, val) with each row sorted by column."""
        p = self.prod
        L = p.L
        nnz = ctypes.c_int64()
        rp = np.zeros(self.n + 1, np.int64)
        p.ctx._check(L.dsg_rows_export(p.h, ctypes.byref(self.v), rp.ctypes.data_as(P), None, None, 0,
                                       ctypes.byref(nnz)))
        col = np.zeros(max(nnz.value, 1), np.int32)
        val = np.zeros(max(nnz.value, 1), DTYPE[p.semiring])
        p.ctx._check(L.dsg_rows_export(p.h, ctypes.byref(self.v), rp.ctypes.data_as(P), col.ctypes.data_as(P),
                                       val.ctypes.data_as(P), col.size, ctypes.byref(nnz)))
        return self.row_ids(), rp, col[:nnz.value], val[:nnz.value]

    def to_host_noalloc(self, cap: Optional[int] = None):
        """As to_host, through dsg_rows_export_noalloc (no device allocation;
        cap: room of the entry arrays, default the view's entry count)."""
        p = self.prod
        L = p.L
        nnz = ctypes.c_int64()
        rp = np.zeros(self.n + 1, np.int64)
        p.ctx._check(L.dsg_rows_export_noalloc(p.h, ctypes.byref(self.v), rp.ctypes.data_as(P), None, None, 0,
                                               ctypes.byref(nnz)))
        room = nnz.value if cap is None else cap
        col = np.zeros(max(room, 1), np.int32)
        val = np.zeros(max(room, 1), DTYPE[p.semiring])
        p.ctx._check(L.dsg_rows_export_noalloc(p.h, ctypes.byref(self.v), rp.ctypes.data_as(P),
                                               col.ctypes.data_as(P), val.ctypes.data_as(P), room,
                                               ctypes.byref(nnz)))
        return self.row_ids(), rp, col[:nnz.value], val[:nnz.value]

    def row_ids(self) -> np.ndarray:
        """The view's row list, copied from device memory."""
        out = np.zeros(self.n, np.int32)
        if self.n:
            self.prod.ctx.synchronize()
            st = _hip().hipMemcpy(out.ctypes.data_as(P), self.v.rows, self.n * 4, 2)  # device to host
            if st != 0:
                raise DsgError(E_DEVICE, f"hipMemcpy failed ({st})")
        return out


_HIP = None


def _arch() -> str:
    try:
        import torch
        return str(torch.cuda.get_device_properties(0).gcnArchName).split(":")[0]
    except Exception:
        return "unknown"


def _hip():
    global _HIP
    if _HIP is None:
        _HIP = ctypes.CDLL("libamdhip64.so")
        _HIP.hipMemcpy.argtypes = [P, P, ctypes.c_size_t, ctypes.c_int]
        _HIP.hipMemcpy.restype = ctypes.c_int
    return _HIP


class Product:
    """C = op(A) op(B), op(X) = X^T when trans_a / trans_b is set."""

    def __init__(self, ctx: Context, A: Matrix, B: Matrix, trans_a: bool = False, trans_b: bool = False,
                 bloom: bool = False):
        self.ctx, self.L = ctx, ctx.L
        self.A, self.B = A, B
        self.trans_a, self.trans_b = bool(trans_a), bool(trans_b)
        self.semiring = A.semiring
        self.nrows = A.ncols if trans_a else A.nrows
        self.ncols = B.nrows if trans_b else B.ncols
        h = P()
        ops = (TRANS_A if trans_a else 0) | (TRANS_B if trans_b else 0) | (GENERAL_BLOOM if bloom else 0)
        ctx._check(self.L.dsg_prod_create(ctx.h, A.h, B.h, ops, ctypes.byref(h)))
        self.h = h

    def update(self, report_affected: bool = False) -> RowSet:
        v = Rows()
        self.ctx._check(self.L.dsg_prod_update(self.h, REPORT_AFFECTED if report_affected else 0,
                                               ctypes.byref(v)))
        return RowSet(self, v)

    def recompute_static(self):
        self.ctx._check(self.L.dsg_prod_recompute_static(self.h, 0))

    def scale_add(self, alpha, X: Optional["Matrix"] = None, beta=None) -> "Matrix":
        """A new Matrix (alpha (x) C) (+) (beta (x) X) from the current C."""
        dt = DTYPE[self.semiring]
        a = np.array([alpha], dt)
        b = np.array([0 if beta is None else beta], dt)
        h = P()
        self.ctx._check(self.L.dsg_prod_scale_add(self.h, a.ctypes.data_as(P), X.h if X is not None else None,
                                                  b.ctypes.data_as(P) if X is not None else None,
                                                  ctypes.byref(h)))
        return Matrix._wrap(self.ctx, h, self.nrows, self.ncols, self.semiring)

    def rows(self, rows) -> RowSet:
        v = Rows()
        pr, dev = _ptr(rows)
        n = int(rows.shape[0])
        self.ctx._check(self.L.dsg_prod_rows(self.h, pr, n, INPUT_DEVICE if dev else 0, ctypes.byref(v)))
        return RowSet(self, v)

    def nnz(self) -> int:
        v = ctypes.c_int64()
        self.ctx._check(self.L.dsg_prod_nnz(self.h, ctypes.byref(v)))
        return v.value

    def export(self):
        return _export(self.ctx, self.L.dsg_prod_export, self.h, self.nrows, self.ncols, self.semiring)

    def export_bloom(self):
        """Canonical CSR of the Bloom matrix F (uint64 bit fields), for a
        product created with bloom=True."""
        nnz = ctypes.c_int64()
        rp = np.zeros(self.nrows + 1, np.int64)
        fn = self.L.dsg_prod_export_bloom
        self.ctx._check(fn(self.h, rp.ctypes.data_as(P), None, None, 0, ctypes.byref(nnz)))
        col = np.zeros(max(nnz.value, 1), np.int32)
        val = np.zeros(max(nnz.value, 1), np.uint64)
        self.ctx._check(fn(self.h, rp.ctypes.data_as(P), col.ctypes.data_as(P), val.ctypes.data_as(P), col.size,
                           ctypes.byref(nnz)))
        return Csr(self.nrows, self.ncols, rp, col[:nnz.value], val[:nnz.value])

    def stats(self) -> dict:
        s = Stats()
        self.ctx._check(self.L.dsg_prod_stats(self.h, ctypes.byref(s)))
        return s.as_dict()

    def autotune(self, reps: int = 3, cache_path: Optional[str] = None) -> dict:
        """Pick the row-kernel tuning for this product (timed trials in the
        library).  With cache_path, results are stored in a JSON file keyed by
        (device arch, semiring, shape, nnz(A) and nnz(C) to two significant
        digits) and reused without trials."""
        key = json.dumps([_arch(), self.semiring, self.trans_a, self.trans_b, self.nrows, self.ncols,
                          float(f"{self.A.nnz():.2g}"), float(f"{self.nnz():.2g}")])
        cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        if key in cache:
            t = self.ctx.get_tuning()
            ent = cache[key]
            for b in range(8):
                t.group_ub[b] = ent["group_ub"][b]
            t.dense_max_passes = ent["dense_max_passes"]
            t.force_bin = -1
            t.update_path = 0
            self.ctx.set_tuning(t)
            return dict(ent, cached=True)
        best = Tuning()
        ms = ctypes.c_double()
        buf = ctypes.create_string_buffer(1 << 16)
        self.ctx._check(self.L.dsg_prod_autotune(self.h, reps, ctypes.byref(best), ctypes.byref(ms), buf,
                                                 len(buf)))
        ent = {"group_ub": list(best.group_ub), "dense_max_passes": best.dense_max_passes,
               "ms": ms.value, "trials": json.loads(buf.value.decode())}
        if cache_path:
            cache[key] = {k: v for k, v in ent.items() if k != "trials"}
            with open(cache_path, "w") as f:
                json.dump(cache, f, indent=1)
        return dict(ent, cached=False)

    def destroy(self):
        if self.h:
            self.ctx._check(self.L.dsg_prod_destroy(self.h))
            self.h = None


class Batch:
    """Batched executor: many independent products, one hipGraph replay per run."""

    def __init__(self, ctx: Context, prods):
        self.ctx, self.L = ctx, ctx.L
        self.prods = list(prods)
        arr = (P * max(len(self.prods), 1))(*[p.h for p in self.prods])
        h = P()
        ctx._check(self.L.dsg_batch_create(ctx.h, arr, len(self.prods), ctypes.byref(h)))
        self.h = h

    def run(self, sets):
        """sets: list of (Matrix, rows, cols, vals, ops) with device tensors.
        Returns the reported-row count of every product."""
        arr = (UpdateSet * max(len(sets), 1))()
        for k, (m, rows, cols, vals, ops) in enumerate(sets):
            arr[k].mat = m.h
            arr[k].rows = _ptr(rows)[0]
            arr[k].cols = _ptr(cols)[0]
            arr[k].vals = _ptr(vals)[0]
            arr[k].ops = _ptr(ops)[0]
            arr[k].n = int(rows.shape[0])
        counts = (ctypes.c_int32 * max(len(self.prods), 1))()
        self.ctx._check(self.L.dsg_batch_run(self.h, arr, len(sets), 0, counts))
        return [int(counts[i]) for i in range(len(self.prods))]

    def rows(self, i: int) -> RowSet:
        v = Rows()
        self.ctx._check(self.L.dsg_batch_rows(self.h, i, ctypes.byref(v)))
        return RowSet(self.prods[i], v)

    def info(self) -> dict:
        st = BatchStats()
        self.ctx._check(self.L.dsg_batch_info(self.h, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in BatchStats._fields_}

    def destroy(self):
        if self.h:
            self.ctx._check(self.L.dsg_batch_destroy(self.h))
            self.h = None


class Server:
    """Served form: a request loop (library threads) over a product's
    resident operands and result.  Requests are host arrays; results are
    polled by ticket.  While the server lives, the context is its own."""

    def __init__(self, ctx: Context, prod: Product, mem_budget: int = 0, max_coalesce: int = 0,
                 max_query_rows: int = 0, slots: int = 0):
        self.ctx, self.L, self.prod = ctx, ctx.L, prod
        cfg = ServerCfg(mem_budget, max_coalesce, max_query_rows, slots)
        h = P()
        ctx._check(self.L.dsg_server_create(ctx.h, prod.h, ctypes.byref(cfg), ctypes.byref(h)))
        self.h = h

    def _check(self, st):
        self.ctx._check(st, h=None)

    def submit_update(self, mat: Matrix, rows, cols, vals, ops) -> int:
        rows = np.ascontiguousarray(rows, np.int32)
        cols = np.ascontiguousarray(cols, np.int32)
        vals = np.ascontiguousarray(vals, DTYPE[mat.semiring])
        ops = np.ascontiguousarray(ops, np.uint8)
        t = ctypes.c_uint64()
        self._check(self.L.dsg_server_submit_update(self.h, mat.h, rows.ctypes.data_as(P), cols.ctypes.data_as(P),
                                                    vals.ctypes.data_as(P), ops.ctypes.data_as(P), rows.size,
                                                    ctypes.byref(t)))
        return t.value

    def submit_batch(self, mat: Matrix, b) -> int:
        return self.submit_update(mat, b.rows, b.cols, b.vals, b.ops)

    def submit_query(self, rows) -> int:
        rows = np.ascontiguousarray(rows, np.int32)
        t = ctypes.c_uint64()
        self._check(self.L.dsg_server_submit_query(self.h, rows.ctypes.data_as(P), rows.size, ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int, wait: bool = False) -> dict:
        r = ServerResult()
        self._check(self.L.dsg_server_poll(self.h, ticket, 1 if wait else 0, ctypes.byref(r)))
        return {name: getattr(r, name) for name, _ in ServerResult._fields_}

    def query_result(self, ticket: int) -> Csr:
        info = self.poll(ticket, wait=True)
        if info["status"] != OK:
            raise DsgError(info["status"], "query failed")
        nq = info["nq"]
        nnz = ctypes.c_int64()
        rp = np.zeros(nq + 1, np.int64)
        col = np.zeros(max(info["nnz"], 1), np.int32)
        val = np.zeros(max(info["nnz"], 1), DTYPE[self.prod.semiring])
        self._check(self.L.dsg_server_query_result(self.h, ticket, rp.ctypes.data_as(P), col.ctypes.data_as(P),
                                                   val.ctypes.data_as(P), col.size, ctypes.byref(nnz)))
        return Csr(nq, self.prod.ncols, rp, col[:nnz.value], val[:nnz.value])

    def release(self, ticket: int):
        self._check(self.L.dsg_server_release(self.h, ticket))

    def drain(self):
        self._check(self.L.dsg_server_drain(self.h))

    def stats(self) -> dict:
        st = ServerStats()
        self._check(self.L.dsg_server_stats_get(self.h, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in ServerStats._fields_}

    def destroy(self):
        if self.h:
            self._check(self.L.dsg_server_destroy(self.h))
            self.h = None
