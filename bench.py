"""Benchmark of batch-dynamic SpGEMM on one MI355X.

One step = the whole hot path over one update batch: ingest the batch into
the dynamic operand (sort, fold, apply, transpose index), find the affected
rows, recompute them with the binned row kernels, and merge them into C.
Batches are uploaded to HBM before the timed region.

Prints one JSON line (metric: dynamic-SpGEMM updates/s) with the speedup over
a static recompute on the same GPU, the p99 batch latency, the roofline of
the dominant row kernel (algorithmic bytes / measured time, HIP events on the
library's stream) and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
EXTRA = 3  # steps after the timed ones, every phase timed, for the per-phase breakdown


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name: str, batch: int, count: int):
    from paper_2202_08808_amd import inputs as I
    if name == "rmat16":
        return I.workload_rmat16_minplus(batch=batch, n_batches=count)
    if name == "rmat12":
        return I.workload_rmat12_i64(n_batches=count, batch=batch)
    if name == "stencil":
        return I.workload_stencil_f64(n_batches=count)
    if name == "er":
        return I.workload_er_minplus(n_batches=count, batch=batch)
    raise SystemExit(f"unknown workload {name}")


KERNEL_SOURCES = ["paper_2202_08808_amd/csrc/spgemm.hip", "paper_2202_08808_amd/csrc/kernel_common.h"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str, batch: int):
    """HBM bytes per launch of the row kernel, from the committed PMC summary
    (FETCH_SIZE and WRITE_SIZE scaled by a copy kernel of known size), when
    it was taken on the same kernel source and workload; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if "```json" not in text:
        return None
    rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    if rec.get("source_sha256") != kernel_source_hash() or rec.get("updates_per_batch") != batch:
        return None
    return rec.get("traffic_bytes_per_launch")


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, n_batches: int, budget_s: float = 12.0):
    """The oracle as it stands: apply the batch, recompute C' = A'B' from
    scratch; timed on this host's cores (OpenMP over rows, every thread the
    host gives this process) and on one thread, each on a bounded number of
    batches (the first that end past budget_s seconds)."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = max(1, min(threads, os.cpu_count() or 1))

    def leg(nthreads):
        A = oracle.Csr.of(w.A)
        B = None if w.B is None else oracle.Csr.of(w.B)
        done = updates = 0
        t0 = time.perf_counter()
        for t in range(n_batches):
            b = w.batches_A[t]
            A, _ = oracle.apply(w.semiring, A, b.rows, b.cols, b.vals, b.ops)
            updates += len(b)
            if B is not None:
                bb = w.batches_B[t]
                B, _ = oracle.apply(w.semiring, B, bb.rows, bb.cols, bb.vals, bb.ops)
                updates += len(bb)
            oracle.spgemm(w.semiring, A, A if B is None else B, nthreads=nthreads)
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
        return updates / (time.perf_counter() - t0), done, time.perf_counter() - t0
    v, done, dt = leg(threads)
    v1, done1, dt1 = leg(1)
    return {"value": v, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} batch(es) of the same workload: sequential apply + full static "
                      f"recompute of C' ({dt:.1f} s on {threads} threads); {done1} batch(es) on one "
                      f"thread ({dt1:.1f} s)",
            "single_thread_value": v1, "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


OTHER_CONFIGS = [("rmat12", 100), ("stencil", 0), ("er", 1000), ("er", 10000)]


def bench_other_configs(steps: int = 5, warmup: int = 1):
    """The other evaluation workloads, briefly, on the same GPU: median ms of
    apply + update per batch (every phase on the context's stream, batches
    resident in HBM), the static recompute of the same product, and the path
    the update took.  R-MAT scale 12 int64 with 100 insertions, the stencil
    fp64 A B with 1e4 changes + 1e3 insertions in each operand, the
    Erdos-Renyi 2^21 min-plus product at 1e3 and 1e4 updates."""
    import torch
    from paper_2202_08808_amd import dsg
    dev = torch.device("cuda:0")
    out = []
    for name, b in OTHER_CONFIGS:
        t0 = time.perf_counter()
        w = make_workload(name, b, steps + warmup)
        gen_s = time.perf_counter() - t0
        ctx = dsg.Context(0, stream=torch.cuda.current_stream(dev))
        A = dsg.Matrix.from_csr(ctx, w.A, w.semiring)
        B = A if w.B is None else dsg.Matrix.from_csr(ctx, w.B, w.semiring)
        P = dsg.Product(ctx, A, B)

        def dev_batch(q):
            return [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (q.rows, q.cols, q.vals, q.ops)]
        ba = [dev_batch(q) for q in w.batches_A]
        bb = [dev_batch(q) for q in w.batches_B] if w.B is not None else None
        per = len(w.batches_A[0]) + (len(w.batches_B[0]) if w.B is not None else 0)
        ts, paths = [], []
        for k in range(warmup + steps):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            A.apply(*ba[k])
            if bb is not None:
                B.apply(*bb[k])
            P.update()
            torch.cuda.synchronize()
            if k >= warmup:
                ts.append(time.perf_counter() - t1)
                paths.append(P.stats()["path"])
        st = []
        for _ in range(2):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            P.recompute_static()
            torch.cuda.synchronize()
            st.append(time.perf_counter() - t1)
        ms = float(np.median(ts)) * 1e3
        sms = float(np.median(st)) * 1e3
        rec = {"workload": w.name, "n": w.A.nrows, "nnz_A": w.A.nnz, "nnz_B": None if w.B is None else w.B.nnz,
               "nnz_C": P.nnz(), "updates_per_batch": per, "ms_per_step": round(ms, 4),
               "updates_per_s": round(per / ms * 1e3, 1), "static_recompute_ms": round(sms, 4),
               "speedup_vs_static_gpu_recompute": round(sms / ms, 3),
               "paths": sorted(set({0: "rows", 1: "entries", 2: "bloom"}[x] for x in paths)), "steps": steps}
        log(f"[bench] {json.dumps(rec)} (inputs in {gen_s:.1f}s)")
        out.append(rec)
        P.destroy()
        if B is not A:
            B.destroy()
        A.destroy()
        ctx.close()
    return out


def bench_batched(args):
    """Batched form: independent R-MAT instances (scale ~ U{10..16}, edge
    factor ~ U{4,8,16,32}, int64 plus-times and min-plus alternating, one
    batch of size floor(10^U(1,4)) each per round, mix 50/25/25).  Two equal
    copies of every instance: one brought up to date by the plain
    per-instance loop (apply + update), one by one batched graph replay; both
    timed over the same rounds, both outside the timed region fed from
    device-resident batches."""
    import torch
    from paper_2202_08808_amd import dsg
    from paper_2202_08808_amd import inputs as I

    K, W = args.steps, args.warmup
    desc = I.batched_instances(args.instances, max_scale=args.max_scale)
    ctx = dsg.Context(0, stream=torch.cuda.current_stream())
    plain, batched, rounds = [], [], []
    t0 = time.perf_counter()
    total_updates = 0
    for t, (scale, ef, sr, b) in enumerate(desc):
        lo, hi = (1, 9) if sr == I.PLUS_TIMES_I64 else (1, 100)
        A = I.rmat_csr(scale, ef, sr, stream=1000 + t, lo=lo, hi=hi)
        try:
            bs = I.disjoint_batches(A, sr, [b] * (K + W), stream=2000 + t, value_lo=lo, value_hi=hi)
        except ValueError:
            # too few entries for pairwise-distinct deletes/changes over all rounds:
            # uniform positions, 75% SET (insert or change) and 25% DELETE
            rng = I.rng_for(2000 + t, 1)
            bs = [I.random_batch(A.nrows, A.ncols, sr, b, rng, op_probs=(0.75, 0.25, 0.0), value_lo=lo,
                                 value_hi=hi) for _ in range(K + W)]
        a1 = dsg.Matrix.from_csr(ctx, A, sr)
        a2 = dsg.Matrix.from_csr(ctx, A, sr)
        plain.append((a1, dsg.Product(ctx, a1, a1)))
        batched.append((a2, dsg.Product(ctx, a2, a2)))
        rounds.append([[torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (q.rows, q.cols, q.vals, q.ops)]
                       for q in bs])
        total_updates += b
    log(f"[bench] {len(desc)} instances, {total_updates} updates per round, set up in "
        f"{time.perf_counter() - t0:.1f}s")
    B = dsg.Batch(ctx, [p for _, p in batched])
    bufs = [[x.clone() for x in rounds[t][0]] for t in range(len(desc))]

    def fill(r):
        for t in range(len(desc)):
            for x, y in zip(bufs[t], rounds[t][r]):
                x.copy_(y)
        torch.cuda.synchronize()

    t_plain, t_batch = [], []
    for r in range(W + K):
        fill(r)
        # plain loop: apply + update, instance after instance
        t1 = time.perf_counter()
        for t, (a, p) in enumerate(plain):
            a.apply(*bufs[t])
            p.update()
        torch.cuda.synchronize()
        dt_plain = time.perf_counter() - t1
        # batched: every instance in one graph replay
        t1 = time.perf_counter()
        counts = B.run([(batched[t][0], *bufs[t]) for t in range(len(desc))])
        torch.cuda.synchronize()
        dt_batch = time.perf_counter() - t1
        if r >= W:
            t_plain.append(dt_plain)
            t_batch.append(dt_batch)
        log(f"[bench] round {r}: plain loop {dt_plain * 1e3:.2f} ms, batched {dt_batch * 1e3:.2f} ms, "
            f"{sum(counts)} rows reported")
    # the two copies must agree bit for bit: canonical row pointers, columns
    # and value bits of every instance's C (one instance at a time on the host)
    for t in range(len(desc)):
        x, y = plain[t][1].export(), batched[t][1].export()
        same = (np.array_equal(x.row_ptr, y.row_ptr) and np.array_equal(x.col, y.col)
                and np.ascontiguousarray(x.val).tobytes() == np.ascontiguousarray(y.val).tobytes())
        assert same, f"instance {t}: batched C differs from the plain loop's"
        del x, y
    log(f"[bench] all {len(desc)} instances: batched C equals the plain loop's bit for bit")
    info = B.info()
    tp, tb = float(np.sum(t_plain)), float(np.sum(t_batch))
    out = {
        "metric": "batched dynamic SpGEMM updates/s",
        "value": round(total_updates * K / tb, 2),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(tb / K * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64+f32",
        "data": "synthetic",
        "config": {"workload": f"batched_{len(desc)}_rmat_instances", "instances": len(desc),
                   "scales": [d[0] for d in desc], "edge_factors": [d[1] for d in desc],
                   "batch_sizes": [d[3] for d in desc], "updates_per_round": total_updates},
        "plain_loop_ms_per_round": round(tp / K * 1e3, 4),
        "speedup_vs_plain_loop": round(tp / tb, 4),
        "graph": info,
    }
    B.destroy()
    for a, p in plain + batched:
        p.destroy()
        a.destroy()
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Served form on the Erdos-Renyi n=2^21, mean degree 8, min-plus product
    (C = A*A resident in HBM).  One Poisson trace per offered load (a
    multiple of the measured synchronous capacity): update batches of
    floor(10**X) entries, X ~ N(3, 0.67) on [1, 5], mix 50/25/25, and queries
    of 1..1024 random rows, half and half.  The same trace is run by the
    plain synchronous path (one request at a time: apply + update, or row
    query) and by the server (continuous batching); both from host arrays,
    latency = completion - scheduled arrival."""
    import torch
    from paper_2202_08808_amd import dsg
    from paper_2202_08808_amd import inputs as I

    n = 1 << args.serve_scale
    t0 = time.perf_counter()
    keys = I.er_keys(n, 8 * n, I.rng_for(501, 0))
    A = I.csr_from_keys(n, n, keys, I.draw_values(I.MIN_PLUS_F32, keys.size, I.rng_for(501, 1), 1, 100))
    sr = I.MIN_PLUS_F32
    log(f"[serve] ER n={n} nnz={A.nnz} ({time.perf_counter() - t0:.1f}s)")
    ctx = dsg.Context(0, stream=torch.cuda.current_stream())

    def fresh():
        m = dsg.Matrix.from_csr(ctx, A, sr)
        return m, dsg.Product(ctx, m, m)

    def wait_until(t):
        while True:
            d = t - time.perf_counter()
            if d <= 0:
                return
            time.sleep(min(d, 2e-4) if d > 2e-4 else 0)

    def run_sync(trace):
        m, P = fresh()
        torch.cuda.synchronize()
        lat_u, lat_q, entries = [], [], 0
        start = time.perf_counter() + 0.05
        last = start
        for r in trace:
            target = start + r.t
            wait_until(target)
            if r.kind == "update":
                m.apply_batch(r.batch)
                P.update()
                entries += len(r.batch.ops)
            else:
                P.rows(r.rows).to_host()
            last = time.perf_counter()
            (lat_u if r.kind == "update" else lat_q).append((last - target) * 1e3)
        busy = last - (start + trace[0].t)
        P.destroy()
        m.destroy()
        return {"update_p50_ms": float(np.percentile(lat_u, 50)), "update_p99_ms": float(np.percentile(lat_u, 99)),
                "query_p50_ms": float(np.percentile(lat_q, 50)), "query_p99_ms": float(np.percentile(lat_q, 99)),
                "updates_per_s": entries / busy, "busy_s": busy}

    def run_served(trace):
        m, P = fresh()
        torch.cuda.synchronize()
        S = dsg.Server(ctx, P, mem_budget=args.serve_budget << 20)
        tickets, late = [], []
        start = time.perf_counter() + 0.05
        for r in trace:
            target = start + r.t
            wait_until(target)
            late.append((time.perf_counter() - target) * 1e3)
            tickets.append(S.submit_batch(m, r.batch) if r.kind == "update" else S.submit_query(r.rows))
        S.drain()
        res = [S.poll(t) for t in tickets]
        st = S.stats()
        S.destroy()
        P.destroy()
        m.destroy()
        assert all(x["status"] == dsg.OK for x in res)
        lat_u = [x["latency_ms"] + lt for x, lt in zip(res, late) if x["kind"] == 0]
        lat_q = [x["latency_ms"] + lt for x, lt in zip(res, late) if x["kind"] == 1]
        return {"update_p50_ms": float(np.percentile(lat_u, 50)), "update_p99_ms": float(np.percentile(lat_u, 99)),
                "query_p50_ms": float(np.percentile(lat_q, 50)), "query_p99_ms": float(np.percentile(lat_q, 99)),
                "updates_per_s": st["updates_per_s"], "busy_s": st["busy_ms"] * 1e-3,
                "update_groups": st["update_groups"], "update_requests": st["update_requests"],
                "query_groups": st["query_groups"], "query_requests": st["query_requests"],
                "peak_inflight_MiB": round(st["peak_inflight_bytes"] / 2**20, 1),
                "max_submit_lateness_ms": float(np.max(late))}

    # synchronous capacity: a calibration trace served back to back
    cal = I.serve_trace(A, sr, args.serve_calib, 1e9, stream=611)
    c = run_sync(cal)
    capacity = args.serve_calib / c["busy_s"]
    log(f"[serve] synchronous capacity ~{capacity:.0f} requests/s ({c['updates_per_s']:.0f} updates/s back to back)")
    loads = []
    for load in args.serve_loads:
        rate = load * capacity
        t0 = time.perf_counter()
        trace = I.serve_trace(A, sr, args.serve_requests, rate, stream=621)
        log(f"[serve] load {load}: {len(trace)} requests at {rate:.0f}/s over {trace[-1].t:.1f}s "
            f"(trace in {time.perf_counter() - t0:.1f}s)")
        sy = run_sync(trace)
        log(f"[serve]   synchronous: {json.dumps({k: round(v, 3) for k, v in sy.items()})}")
        sv = run_served(trace)
        log(f"[serve]   served:      {json.dumps({k: round(v, 3) for k, v in sv.items()})}")
        loads.append({"load": load, "rate_per_s": round(rate, 1), "synchronous": sy, "served": sv})
    top = loads[-1]
    out = {
        "metric": "served dynamic SpGEMM updates/s",
        "value": round(top["served"]["updates_per_s"], 2),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.serve_requests,
        "warmup": args.serve_calib,
        "ms_per_step": round(top["served"]["busy_s"] * 1e3 / args.serve_requests, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"er{n}_d8_min_plus_f32_serving", "n": n, "nnz_A": A.nnz,
                   "requests": args.serve_requests, "query_fraction": 0.5,
                   "batch_size": "floor(10**X), X~N(3,0.67) on [1,5]", "query_rows": "U{1..1024}",
                   "mem_budget_MiB": args.serve_budget},
        "synchronous_capacity_req_per_s": round(capacity, 1),
        "speedup_vs_synchronous": round(top["served"]["updates_per_s"] / top["synchronous"]["updates_per_s"], 4),
        "p99_batch_latency_ms": round(top["served"]["update_p99_ms"], 4),
        "loads": loads,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_sweep(args):
    """Per batch size on the default workload: ms per step of the row path,
    of the entry-granular path, of the automatic choice between them, of the
    general-update algorithm with the Bloom matrix, and of a static
    recompute, same GPU."""
    import torch
    from paper_2202_08808_amd import dsg
    from paper_2202_08808_amd import inputs as I
    out = []
    for b in args.sweep:
        w = make_workload(args.workload, b, args.steps + args.warmup)
        dev = torch.device("cuda:0")
        batches = [tuple(torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (q.rows, q.cols, q.vals, q.ops))
                   for q in w.batches_A]
        rec = {"batch": b}
        for path in args.sweep_paths:
            ctx = dsg.Context(0, stream=torch.cuda.current_stream(dev))
            t = ctx.get_tuning()
            t.update_path = {"row": 1, "entry": 2, "auto": 0, "bloom": 0}[path]
            ctx.set_tuning(t)
            A = dsg.Matrix.from_csr(ctx, w.A, w.semiring)
            P = dsg.Product(ctx, A, A, bloom=path == "bloom")
            ts = []
            for k in range(args.warmup + args.steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                A.apply(*batches[k])
                P.update()
                torch.cuda.synchronize()
                if k >= args.warmup:
                    ts.append(time.perf_counter() - t0)
            st = P.stats()
            rec[path + "_ms"] = round(float(np.median(ts)) * 1e3, 4)
            if path == "row":
                rec["row_flops"] = st["flops"]
            if path == "auto":
                rec["auto_took_entry"] = bool(st["path"] == 1)
            if path == "bloom":
                # Algorithm 2: entries and rows of C*, the columns of A' the
                # row filter kept, the products the masked multiply walked
                # plus the b'_kj it probed, and its parts that walked / probed
                rec["bloom_taken"] = bool(st["path"] == 2)
                rec["bloom_cstar_entries"] = st["entries"]
                rec["bloom_cstar_rows"] = st["affected_rows"]
                rec["bloom_kept_a_entries"] = st["a_entries"]
                rec["bloom_masked_products"] = st["flops"]
                rec["bloom_parts_walked"], rec["bloom_parts_probed"] = st["bin_rows"][0], st["bin_rows"][1]
            if path == "entry":
                rec["entry_taken"] = bool(st["path"] == 1)
                rec["lost_per_batch"] = st["lost"]
                rec["terms_per_batch"] = st["terms"]
            # the static recompute on a product without the Bloom matrix (which
            # would also rebuild F)
            if path == next((x for x in args.sweep_paths if x != "bloom"), None):
                ts = []
                for _ in range(3):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    P.recompute_static()
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                rec["static_ms"] = round(float(np.median(ts)) * 1e3, 4)
            P.destroy()
            A.destroy()
            ctx.close()
        if "static_ms" not in rec:
            rec["static_ms"] = None
        for path in args.sweep_paths:
            if path != "auto" and rec["static_ms"]:
                rec[f"speedup_{path}"] = round(rec["static_ms"] / rec[path + "_ms"], 3)
        log(f"[sweep] {json.dumps(rec)}")
        out.append(rec)
    print(json.dumps({"workload": args.workload, "sweep": out}), flush=True)


FORMS = [("minplus", False, False), ("minplus", True, False), ("minplus", False, True),
         ("orand", False, False), ("orand", True, False)]


def bench_forms(args):
    """Operand forms and semirings on one R-MAT graph (scale 16, edge factor
    16, the default workload's structure and batch recipe): per batch size,
    ms per step of the dynamic update (apply + update) on the row path and
    with the automatic path choice (entry-granular where the cost rule takes
    it), and of a static recompute, for C = A A, A^T A and A A^T over (min,+)
    and the bitwise (or, and) semiring on 32-bit words."""
    import torch
    from paper_2202_08808_amd import dsg
    from paper_2202_08808_amd import inputs as I
    sr_of = {"minplus": (I.MIN_PLUS_F32, 1, 100), "orand": (I.OR_AND_U32, 0, (1 << 32) - 1)}
    dev = torch.device("cuda:0")
    out = []
    for b in args.sweep or [args.batch]:
        for name, ta, tb in FORMS:
            sr, lo, hi = sr_of[name]
            A0 = I.rmat_csr(16, 16, sr, stream=201, lo=lo, hi=hi)
            bs = I.disjoint_batches(A0, sr, [b] * (args.steps + args.warmup), stream=202 + b % 997,
                                    value_lo=lo, value_hi=hi)
            batches = [tuple(torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (q.rows, q.cols, q.vals, q.ops))
                       for q in bs]
            rec = {"batch": b, "semiring": name, "form": ("At" if ta else "A") + ("At" if tb else "A")}
            for mode, key in ((1, "ms"), (0, "auto_ms")):
                ctx = dsg.Context(0, stream=torch.cuda.current_stream(dev))
                t = ctx.get_tuning()
                t.update_path = mode
                ctx.set_tuning(t)
                A = dsg.Matrix.from_csr(ctx, A0, sr)
                P = dsg.Product(ctx, A, A, trans_a=ta, trans_b=tb)
                ts, paths = [], []
                for k in range(args.warmup + args.steps):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    A.apply(*batches[k])
                    P.update()
                    torch.cuda.synchronize()
                    if k >= args.warmup:
                        ts.append(time.perf_counter() - t0)
                        paths.append(P.stats()["path"])
                rec[key] = round(float(np.median(ts)) * 1e3, 4)
                if mode == 1:
                    st = P.stats()
                    rec.update({"updates_per_s": round(b / float(np.median(ts)), 1),
                                "affected_rows": st["affected_rows"], "flops": st["flops"], "nnz_c": P.nnz()})
                    ts = []
                    for _ in range(3):
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        P.recompute_static()
                        torch.cuda.synchronize()
                        ts.append(time.perf_counter() - t0)
                    rec["static_ms"] = round(float(np.median(ts)) * 1e3, 4)
                else:
                    rec["auto_entry_steps"] = int(sum(1 for x in paths if x == 1))
                P.destroy()
                A.destroy()
                ctx.close()
            rec["speedup"] = round(rec["static_ms"] / rec["ms"], 3)
            rec["speedup_auto"] = round(rec["static_ms"] / rec["auto_ms"], 3)
            log(f"[forms] {json.dumps(rec)}")
            out.append(rec)
    print(json.dumps({"workload": "forms", "sweep": out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat16", choices=["rmat16", "rmat12", "stencil", "er", "batched", "serve", "forms"])
    ap.add_argument("--instances", type=int, default=64, help="batched workload: number of instances")
    ap.add_argument("--max-scale", type=int, default=16, help="batched workload: largest R-MAT scale")
    ap.add_argument("--batch", type=int, default=10000)
    ap.add_argument("--sweep", type=int, nargs="*", default=None,
                    help="time the row and entry-granular paths and a static recompute at these batch sizes")
    ap.add_argument("--sweep-paths", nargs="+", default=["row", "entry", "auto", "bloom"],
                    choices=["row", "entry", "auto", "bloom"], help="paths the sweep times")
    ap.add_argument("--serve-scale", type=int, default=21, help="serve workload: log2 of the ER rows")
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--serve-calib", type=int, default=300)
    ap.add_argument("--serve-loads", type=float, nargs="+", default=[0.9, 1.5],
                    help="offered loads as multiples of the synchronous capacity")
    ap.add_argument("--serve-budget", type=int, default=4096, help="serve workload: memory budget in MiB")
    ap.add_argument("--static-reps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other-configs", action="store_true",
                    help="skip the short runs of the other evaluation workloads")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first copy a buffer of this many MiB device to device three times (reference "
                         "dispatches for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}): the whole problem lives on one "
              "MI355X and the library has no multi-GPU path", file=sys.stderr)
        raise SystemExit(2)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "forms":
        return bench_forms(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.sweep:
        return bench_sweep(args)

    import torch
    from paper_2202_08808_amd import dsg
    from paper_2202_08808_amd import inputs as I

    K, W = args.steps, args.warmup
    if args.calibrate_copy:
        x = torch.ones(args.calibrate_copy << 20, dtype=torch.uint8, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: 3 x {args.calibrate_copy} MiB device to device")
        del x, y
    t0 = time.perf_counter()
    w = make_workload(args.workload, args.batch, K + W + EXTRA)
    log(f"[bench] workload {w.name}: n={w.A.nrows} nnz(A)={w.A.nnz} batches={K + W + EXTRA} "
        f"({time.perf_counter() - t0:.1f}s to generate)")
    sr = w.semiring
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    ctx = dsg.Context(0, stream=stream)
    A = dsg.Matrix.from_csr(ctx, w.A, sr)
    B = A if w.B is None else dsg.Matrix.from_csr(ctx, w.B, sr)
    t0 = time.perf_counter()
    P = dsg.Product(ctx, A, B)
    ctx.synchronize()
    log(f"[bench] initial product: nnz(C)={P.nnz()} in {time.perf_counter() - t0:.2f}s")

    def dev_batch(b):
        return (torch.from_numpy(b.rows).to(dev), torch.from_numpy(b.cols).to(dev),
                torch.from_numpy(np.ascontiguousarray(b.vals)).to(dev), torch.from_numpy(b.ops).to(dev))
    batches = [(dev_batch(w.batches_A[t]), dev_batch(w.batches_B[t]) if w.B is not None else None)
               for t in range(K + W + EXTRA)]
    per_step_updates = len(w.batches_A[0]) + (len(w.batches_B[0]) if w.B is not None else 0)
    torch.cuda.synchronize()

    def step(t):
        ba, bb = batches[t]
        A.apply(*ba)
        if bb is not None:
            B.apply(*bb)
        return P.update()

    # warmup, every phase timed: names the dominant kernel
    ctx.set_timing(True)
    for t in range(W):
        step(t)
    torch.cuda.synchronize()
    warm = ctx.timing_report()["kernels"]
    dom_name = max(warm, key=lambda k: warm[k]["ms"]) if warm else None
    log(f"[bench] warmup done; dominant kernel {dom_name}")

    # timed steps: HIP events around the dominant kernel's launches only
    ctx.set_timing(True, phase=dom_name)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    stops = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    affected = changed = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        starts[k].record(stream)
        rs = step(W + k)
        stops[k].record(stream)
        st = P.stats()
        affected += st["affected_rows"]
        changed += rs.n
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    report = ctx.timing_report()
    if dom_name is None and report["kernels"]:   # no warmup: every phase was timed
        dom_name = max(report["kernels"], key=lambda k: report["kernels"][k]["ms"])
    lat = np.array([starts[k].elapsed_time(stops[k]) for k in range(K)])
    log(f"[bench] timed {K} steps in {wall:.3f}s; per-step ms: {np.round(lat, 3).tolist()}")
    # untimed extra steps with every phase timed: the per-phase breakdown
    ctx.set_timing(True)
    for t in range(W + K, W + K + EXTRA):
        step(t)
    breakdown = ctx.timing_report()["kernels"]
    ctx.set_timing(False)

    # static recompute on the same GPU, same kernels, full C written
    torch.cuda.synchronize()
    ts = []
    for _ in range(args.static_reps):
        t1 = time.perf_counter()
        P.recompute_static()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t1)
    t_static = float(np.median(ts)) if ts else None
    log(f"[bench] static recompute: {np.round(np.array(ts) * 1e3, 3).tolist()} ms")

    ms_per_step = wall / K * 1e3
    apply_ms = breakdown["apply"]["ms"] / EXTRA if "apply" in breakdown else 0.0
    kern = report["kernels"]
    roof = None
    if dom_name and dom_name in kern:
        d = kern[dom_name]
        gbs = d["bytes"] / (d["ms"] * 1e-3) / 1e9 if d["ms"] > 0 else 0.0
        traffic = measured_traffic(dom_name, w.name, per_step_updates)
        roof = {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_unit": "bytes/launch",
                "kernel": dom_name,
                "launches": d["launches"], "avg_launch_ms": round(d["ms"] / max(d["launches"], 1), 4),
                "bytes_per_launch": round(d["bytes"] / max(d["launches"], 1), 1)}
    others = None
    if not args.no_other_configs:
        log("[bench] other evaluation workloads ...")
        others = bench_other_configs()
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline ...")
        cpu = cpu_baseline(w, K + W)
        log(f"[bench] CPU oracle: {cpu['value']:.1f} updates/s on {cpu['cores']} threads, "
            f"{cpu['single_thread_value']:.1f} on one ({cpu['cpu_model']})")
    out = {
        "metric": "dynamic SpGEMM updates/s",
        "value": round(per_step_updates * K / wall, 2),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {0: "int64", 1: "f32", 2: "f64"}[sr],
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.A.nrows, "nnz_A": w.A.nnz,
                   "nnz_B": None if w.B is None else w.B.nnz, "nnz_C": P.nnz(),
                   "updates_per_batch": per_step_updates, "mix_insert_delete_change": "50/25/25"
                   if args.workload in ("rmat16", "er") else None, "parallelism": "single-gpu"},
        "speedup_vs_static_gpu_recompute": round(t_static * 1e3 / ms_per_step, 4) if t_static else None,
        "static_recompute_ms": round(t_static * 1e3, 4) if t_static else None,
        # a static system ingests the batch too: the same apply (its HIP-event
        # time per step in the breakdown) followed by a full recompute
        "static_step_ms": round(t_static * 1e3 + apply_ms, 4) if t_static else None,
        "speedup_vs_static_step": round((t_static * 1e3 + apply_ms) / ms_per_step, 4) if t_static else None,
        "p99_batch_latency_ms": round(float(np.percentile(lat, 99)), 4),
        "p50_batch_latency_ms": round(float(np.percentile(lat, 50)), 4),
        "affected_rows_per_batch": affected / K,
        "changed_rows_per_batch": changed / K,
        "recomputed_rows_per_s": round(affected / wall, 1),
        # per-phase HIP-event times of EXTRA steps after the timed ones
        "kernels": {k: {"launches": v["launches"], "ms": round(v["ms"], 4),
                        "GB/s": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] else None}
                    for k, v in breakdown.items()},
        "kernels_steps": EXTRA,
        "roofline": roof,
        "cpu_baseline": cpu,
        "other_configs": others,
    }
    P.destroy()
    if B is not A:
        B.destroy()
    A.destroy()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
