// Batched form: many independent products, each with its own update sets,
// brought up to date by one hipGraph replay.
//
// Each product's chain (apply its operands' sets, then the dynamic update)
// is captured on a stream of its own, forked from and joined to the
// context's stream, so independent instances overlap on the device.  The
// chains make no host round trip: operand pools hold the worst-case room a
// set can take (apply_headroom); rows of C that find no room in C or in the
// staging arena write nothing and are recomputed after the replay, once the
// room has grown by exactly what they asked for.  The graph is captured on the first run and
// replayed while every pointer and size it baked in is unchanged.
#include <algorithm>
#include <chrono>

#include "internal.h"

namespace {

constexpr int OUT_WORDS = 8;  // per product: k_publish's 6 words, apply error flags, spare

__global__ void k_or_flags(const int* a, const int* b, int64_t* out) {
  int v = a ? *a : 0;
  if (b) v |= *b;
  *out |= (int64_t)v;
}

__global__ void k_clear_out(int64_t* out, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) out[i] = 0;
}

__global__ void k_gather_tops(int64_t* const* tops, int n, int64_t* out) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) out[i] = *tops[i];
}

__global__ void k_zero_ints(int* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

}  // namespace

struct DBatch {
  Ctx* c = nullptr;
  std::vector<DProd*> prods;
  std::vector<DMat*> mats;          // every matrix the graph may touch (operands, indexes, products)
  hipGraphExec_t exec = nullptr;
  std::vector<uintptr_t> signature; // what the captured graph baked in
  // workspaces: per set (apply, transpose index) and per product
  std::vector<void*> aw, awt;
  std::vector<size_t> aw_bytes, awt_bytes;
  std::vector<void*> pw;
  std::vector<size_t> pw_bytes;
  int64_t* d_out = nullptr;
  int64_t* d_tops = nullptr;
  int64_t** d_top_ptrs = nullptr;
  int* d_valid = nullptr;
  std::vector<hipStream_t> streams;
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join;
  int64_t captures = 0, replays = 0, deferred = 0;
  double prepare_ms = 0, capture_ms = 0, replay_ms = 0, finish_ms = 0;
};

static double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

static void free_ws(Ctx* c, std::vector<void*>& v, std::vector<size_t>& b) {
  for (size_t i = 0; i < v.size(); ++i) ctx_free(c, v[i], b[i]);
  v.clear();
  b.clear();
}

static void drop_graph(DBatch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  b->exec = nullptr;
  b->signature.clear();
}

DBatch* batch_create(Ctx* c, const std::vector<DProd*>& prods) {
  DBatch* b = new DBatch();
  b->c = c;
  b->prods = prods;
  for (DProd* p : prods) p->refs++;  // released by batch_destroy
  try {
    for (DProd* p : prods) {
      for (DMat* m : {p->A, p->B, p->A->tidx, p->C})
        if (m && std::find(b->mats.begin(), b->mats.end(), m) == b->mats.end()) b->mats.push_back(m);
    }
    const size_t np = prods.size() ? prods.size() : 1;
    b->d_out = (int64_t*)ctx_alloc(c, np * OUT_WORDS * 8);
    b->d_tops = (int64_t*)ctx_alloc(c, b->mats.size() * 8 + 8);
    b->d_top_ptrs = (int64_t**)ctx_alloc(c, b->mats.size() * 8 + 8);
    b->d_valid = (int*)ctx_alloc(c, 4 * (np * 2 + 1));
    const int nstreams = (int)std::min<size_t>(prods.size(), 8);
    for (int i = 0; i < nstreams; ++i) {
      hipStream_t s;
      DSG_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      b->streams.push_back(s);
    }
    DSG_HIP(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    b->ev_join.resize(prods.size());
    for (auto& e : b->ev_join) DSG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  } catch (...) {
    batch_destroy(b);
    throw;
  }
  return b;
}

void batch_destroy(DBatch* b) {
  if (!b) return;
  Ctx* c = b->c;
  (void)hipStreamSynchronize(c->stream);
  drop_graph(b);
  free_ws(c, b->aw, b->aw_bytes);
  free_ws(c, b->awt, b->awt_bytes);
  free_ws(c, b->pw, b->pw_bytes);
  const size_t np = b->prods.size() ? b->prods.size() : 1;
  ctx_free(c, b->d_out, np * OUT_WORDS * 8);
  ctx_free(c, b->d_tops, b->mats.size() * 8 + 8);
  ctx_free(c, b->d_top_ptrs, b->mats.size() * 8 + 8);
  ctx_free(c, b->d_valid, 4 * (np * 2 + 1));
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  for (auto& e : b->ev_join)
    if (e) (void)hipEventDestroy(e);
  for (DProd* p : b->prods) p->refs--;
  delete b;
}

DProd* batch_prod(DBatch* b, int i) { return b->prods[(size_t)i]; }

void batch_info(const DBatch* b, dsg_batch_stats* out) {
  out->captures = b->captures;
  out->replays = b->replays;
  out->deferred = b->deferred;
  out->prepare_ms = b->prepare_ms;
  out->capture_ms = b->capture_ms;
  out->replay_ms = b->replay_ms;
  out->finish_ms = b->finish_ms;
}

static void ensure_ws(Ctx* c, std::vector<void*>& v, std::vector<size_t>& have, size_t i, size_t bytes,
                      bool& changed) {
  if (v.size() <= i) {
    v.resize(i + 1, nullptr);
    have.resize(i + 1, 0);
  }
  if (bytes <= have[i]) return;
  ctx_free(c, v[i], have[i]);
  v[i] = nullptr;
  have[i] = 0;
  v[i] = ctx_alloc(c, bytes);
  have[i] = bytes;
  changed = true;
}

dsg_status batch_run(DBatch* b, const std::vector<DBatchSet>& sets, std::vector<int32_t>& counts) {
  Ctx* c = b->c;
  const hipStream_t main = c->stream;
  const size_t np = b->prods.size();
  counts.assign(np, 0);
  auto t0 = std::chrono::steady_clock::now();
  // which product each set belongs to (sets name operands of one product)
  std::vector<int> owner(sets.size(), -1);
  for (size_t k = 0; k < sets.size(); ++k) {
    for (size_t j = 0; j < np; ++j)
      if (sets[k].m == b->prods[j]->A || sets[k].m == b->prods[j]->B) owner[k] = (int)j;
    if (owner[k] < 0) throw DsgError{DSG_E_ARG, "update set names a matrix outside the batch"};
    for (size_t k2 = 0; k2 < k; ++k2)
      if (sets[k2].m == sets[k].m) throw DsgError{DSG_E_ARG, "two update sets name the same matrix"};
  }
  // ---- validate every set before anything runs: one round trip ----
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, main, b->d_valid, (int)sets.size() + 1);
  for (size_t k = 0; k < sets.size(); ++k)
    validate_batch_async(sets[k].m, sets[k].rows, sets[k].cols, sets[k].ops, sets[k].n, b->d_valid + k);
  if (!sets.empty()) {
    int* h = (int*)c->pinned;
    DSG_HIP(hipMemcpyAsync(h, b->d_valid, sets.size() * 4, hipMemcpyDeviceToHost, main));
    DSG_HIP(hipStreamSynchronize(main));
    for (size_t k = 0; k < sets.size(); ++k) {
      if (h[k] & 1) return DSG_E_RANGE;
      if (h[k] & 2) return DSG_E_ARG;
    }
  }
  // ---- room: worst case for operands, last need plus margin for C ----
  bool ws_changed = false;
  for (size_t k = 0; k < sets.size(); ++k) {
    DMat* m = sets[k].m;
    // (a compaction makes room for about four rounds: each one changes the
    // pools the graph bakes in)
    const int64_t hm = apply_headroom(m, sets[k].n);
    mat_reserve(m, hm, 4 * hm);
    if (m->tidx) {
      const int64_t ht = apply_headroom(m->tidx, sets[k].n);
      mat_reserve(m->tidx, ht, 4 * ht);
    }
    ensure_ws(c, b->aw, b->aw_bytes, k, apply_work_bytes(sets[k].n, m->tidx != nullptr), ws_changed);
    ensure_ws(c, b->awt, b->awt_bytes, k, apply_work_bytes(sets[k].n, false), ws_changed);
  }
  std::vector<int64_t> c_top_before(np);
  for (size_t j = 0; j < np; ++j) {
    DProd* p = b->prods[j];
    // room for C: twice what the last run took, at least 1/64 of its pool;
    // rows that need still more are completed after the replay.  (A
    // compaction leaves a third of the new pool free, so a floor this low
    // makes C's pool, and the graph that bakes it in, change only every few
    // dozen rounds.)
    const int64_t c_room = std::max<int64_t>(p->C->h_top_ub / 64, 2 * p->last_c_growth) + 4096;
    const size_t arena = std::max<size_t>(p->arena_bytes, (size_t)1 << 20);
    prod_prepare_graph(p, c_room, arena, 4 * c_room);
    ensure_ws(c, b->pw, b->pw_bytes, j, prod_graph_work_bytes(p), ws_changed);
    c_top_before[j] = p->C->h_top_ub;
  }
  // ---- the signature of what a graph bakes in ----
  std::vector<uintptr_t> sig;
  for (size_t k = 0; k < sets.size(); ++k) {
    const DBatchSet& s = sets[k];
    for (uintptr_t x : {(uintptr_t)s.m, (uintptr_t)s.rows, (uintptr_t)s.cols, (uintptr_t)s.vals, (uintptr_t)s.ops,
                        (uintptr_t)s.n, (uintptr_t)b->aw[k], (uintptr_t)b->awt[k]})
      sig.push_back(x);
  }
  for (DMat* m : b->mats)
    for (uintptr_t x : {(uintptr_t)m->col, (uintptr_t)m->val, (uintptr_t)m->pool_cap, (uintptr_t)m->version})
      sig.push_back(x);
  for (size_t j = 0; j < np; ++j) {
    DProd* p = b->prods[j];
    for (uintptr_t x : {(uintptr_t)p->changed_rows, (uintptr_t)p->arena, (uintptr_t)p->arena_bytes,
                        (uintptr_t)p->arena_top, (uintptr_t)b->pw[j]})
      sig.push_back(x);
  }
  const dsg_tuning& t = c->tuning;
  for (int x = 0; x < 8; ++x) sig.push_back((uintptr_t)t.group_ub[x]);
  sig.push_back((uintptr_t)t.dense_max_passes);
  sig.push_back((uintptr_t)(t.force_bin + 1));
  b->prepare_ms += ms_since(t0);
  if (!b->exec || sig != b->signature) {
    t0 = std::chrono::steady_clock::now();
    drop_graph(b);
    // device table of the pool tops the graph reports back
    std::vector<int64_t*> tops;
    for (DMat* m : b->mats) tops.push_back(m->d_top);
    DSG_HIP(hipMemcpyAsync(b->d_top_ptrs, tops.data(), tops.size() * 8, hipMemcpyHostToDevice, main));
    DSG_HIP(hipStreamSynchronize(main));
    hipGraph_t graph = nullptr;
    DSG_HIP(hipStreamBeginCapture(main, hipStreamCaptureModeThreadLocal));
    try {
      hipLaunchKernelGGL(k_clear_out, dim3(1), dim3(256), 0, main, b->d_out, (int)(np * OUT_WORDS));
      DSG_HIP(hipEventRecord(b->ev_fork, main));
      for (size_t j = 0; j < np; ++j) {
        hipStream_t sj = b->streams[j % b->streams.size()];
        DSG_HIP(hipStreamWaitEvent(sj, b->ev_fork, 0));
        c->stream = sj;
        int slot = 6;
        for (size_t k = 0; k < sets.size(); ++k) {
          if (owner[k] != (int)j) continue;
          const DBatchSet& s = sets[k];
          mat_apply_graph(s.m, s.rows, s.cols, s.vals, s.ops, s.n, b->aw[k], b->awt[k]);
          if (s.n > 0) {
            const int* e1 = apply_err_ptr(b->aw[k], s.n, s.m->tidx != nullptr);
            const int* e2 = s.m->tidx ? apply_err_ptr(b->awt[k], s.n, false) : nullptr;
            hipLaunchKernelGGL(k_or_flags, dim3(1), dim3(1), 0, sj, e1, e2, b->d_out + j * OUT_WORDS + slot);
          }
          slot = 7;
        }
        prod_update_graph(b->prods[j], b->pw[j], b->d_out + j * OUT_WORDS);
        DSG_HIP(hipEventRecord(b->ev_join[j], sj));
      }
      c->stream = main;
      for (size_t j = 0; j < np; ++j) DSG_HIP(hipStreamWaitEvent(main, b->ev_join[j], 0));
      hipLaunchKernelGGL(k_gather_tops, dim3(1), dim3(256), 0, main, (int64_t* const*)b->d_top_ptrs,
                         (int)b->mats.size(), b->d_tops);
      DSG_HIP(hipGetLastError());
    } catch (...) {
      c->stream = main;
      (void)hipStreamEndCapture(main, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      throw;
    }
    DSG_HIP(hipStreamEndCapture(main, &graph));
    hipError_t e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    DSG_HIP(e);
    b->signature = sig;
    b->captures++;
    b->capture_ms += ms_since(t0);
  }
  // ---- one replay for every product ----
  t0 = std::chrono::steady_clock::now();
  DSG_HIP(hipGraphLaunch(b->exec, main));
  b->replays++;
  std::vector<int64_t> out(np * OUT_WORDS), tops(b->mats.size());
  DSG_HIP(hipMemcpyAsync(out.data(), b->d_out, out.size() * 8, hipMemcpyDeviceToHost, main));
  DSG_HIP(hipMemcpyAsync(tops.data(), b->d_tops, tops.size() * 8, hipMemcpyDeviceToHost, main));
  DSG_HIP(hipStreamSynchronize(main));
  for (size_t i = 0; i < b->mats.size(); ++i) b->mats[i]->h_top_ub = tops[i];
  // these applies keep no log: the entry-granular update does not follow them
  for (const DBatchSet& st : sets)
    if (st.n > 0) st.m->apply_seq++;
  b->replay_ms += ms_since(t0);
  t0 = std::chrono::steady_clock::now();
  for (size_t j = 0; j < np; ++j) {
    const int64_t* o = &out[j * OUT_WORDS];
    DSG_REQUIRE(o[2] == 0 && o[6] == 0 && o[7] == 0, DSG_E_DEVICE,
                "internal: device error flags " + std::to_string(o[2]) + "/" + std::to_string(o[6]) + "/" +
                    std::to_string(o[7]) + " in batched product " + std::to_string(j));
    DProd* p = b->prods[j];
    // slots taken (a pool top that ran past the end also counts what the
    // rows without room asked for)
    p->last_c_growth = std::max<int64_t>(0, p->C->h_top_ub - c_top_before[j]) + o[4];
    if (o[3]) {
      // some rows found no room (they wrote nothing): grow C / the arena by
      // exactly what they asked for and recompute them
      counts[j] = prod_finish_graph(p, b->pw[j]);
      b->deferred++;
    } else {
      counts[j] = (int32_t)o[0];
    }
    p->a_seq = p->A->apply_seq;
    p->b_seq = p->B->apply_seq;
  }
  b->finish_ms += ms_since(t0);
  return DSG_OK;
}
