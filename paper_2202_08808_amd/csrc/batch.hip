// Batched form: many independent products, each with its own update sets,
// brought up to date together.  Products whose C is large (at least
// 2^batch_direct_log2 slots, a tuning field) take the plain path on the context's stream, with its host
// round trips, which their kernel time hides, and with everything it offers
// (the split copy of B, the entry-granular choice, room sized from the
// plan); so do products with the Bloom matrix, whose general update sizes
// its pattern on the host.  The others are brought up to date by one
// hipGraph replay on a stream of its own, which runs meanwhile.
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
#include <array>
#include <chrono>

#include "internal.h"

namespace {

constexpr int OUT_WORDS = 8;  // per product: k_publish's 6 words, apply error flags, spare
// Rounds of worst-case growth a compaction of a graphed product's pools
// leaves room for.  Graphed products are the small ones (C below
// 2^batch_direct_log2 slots), so the room costs little memory, and fewer
// compactions mean fewer captures.
constexpr int64_t ROOM_ROUNDS = 16;

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
  hipGraphExec_t exec = nullptr;
  std::vector<uintptr_t> signature; // what the captured graph baked in
  // workspaces: per set (apply, transpose index) and per product
  std::vector<void*> aw, awt;
  std::vector<size_t> aw_bytes, awt_bytes;
  std::vector<void*> pw;
  std::vector<size_t> pw_bytes;
  int64_t* d_out = nullptr;
  size_t ntop = 0;                  // room of the two tables below: 5 matrices per product (prod_matrices)
  int64_t* d_tops = nullptr;
  int64_t** d_top_ptrs = nullptr;
  int* d_valid = nullptr;
  std::vector<hipStream_t> streams;
  hipStream_t replay_stream = nullptr;  // the graph's replay runs here, beside the direct products
  hipEvent_t ev_ready = nullptr;        // preparation on the context's stream done
  std::vector<uint8_t> graphed;         // per product: in the graph (else the plain path)
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join;
  int64_t captures = 0, replays = 0, deferred = 0, direct = 0;
  double prepare_ms = 0, capture_ms = 0, replay_ms = 0, finish_ms = 0, direct_ms = 0;
};

// Every matrix a product's update chain may touch: the caller's operands
// and their transposes (an apply writes both), and C.
static std::array<DMat*, 5> prod_matrices(const DProd* p) {
  return {p->src_a, p->src_a->tidx, p->src_b, p->src_b->tidx, p->C};
}

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
    const size_t np = prods.size() ? prods.size() : 1;
    b->d_out = (int64_t*)ctx_alloc(c, np * OUT_WORDS * 8);
    b->ntop = 5 * np + 1;
    b->d_tops = (int64_t*)ctx_alloc(c, b->ntop * 8);
    b->d_top_ptrs = (int64_t**)ctx_alloc(c, b->ntop * 8);
    b->d_valid = (int*)ctx_alloc(c, 4 * (np * 2 + 1));
    const int nstreams = (int)std::min<size_t>(prods.size(), 8);
    for (int i = 0; i < nstreams; ++i) {
      hipStream_t s;
      DSG_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      b->streams.push_back(s);
    }
    DSG_HIP(hipStreamCreateWithFlags(&b->replay_stream, hipStreamNonBlocking));
    DSG_HIP(hipEventCreateWithFlags(&b->ev_ready, hipEventDisableTiming));
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
  ctx_free(c, b->d_tops, b->ntop * 8);
  ctx_free(c, b->d_top_ptrs, b->ntop * 8);
  ctx_free(c, b->d_valid, 4 * (np * 2 + 1));
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  if (b->replay_stream) {
    (void)hipStreamSynchronize(b->replay_stream);
    (void)hipStreamDestroy(b->replay_stream);
  }
  if (b->ev_ready) (void)hipEventDestroy(b->ev_ready);
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
  out->direct = b->direct;
  out->direct_ms = b->direct_ms;
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
      if (sets[k].m == b->prods[j]->src_a || sets[k].m == b->prods[j]->src_b) owner[k] = (int)j;
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
  // ---- which products the graph takes: the ones whose C is small ----
  std::vector<uint8_t> graphed(np, 0);
  std::vector<DMat*> gmats;  // the matrices the graph touches
  size_t ng = 0;
  for (size_t j = 0; j < np; ++j) {
    DProd* p = b->prods[j];
    graphed[j] = !p->bloom && p->C->h_top_ub < (int64_t(1) << c->tuning.batch_direct_log2) ? 1 : 0;
    if (!graphed[j]) continue;
    ++ng;
    for (DMat* m : prod_matrices(p))
      if (m && std::find(gmats.begin(), gmats.end(), m) == gmats.end()) gmats.push_back(m);
  }
  // ---- room for the graph: worst case for operands, last need plus margin for C ----
  bool ws_changed = false;
  for (size_t k = 0; k < sets.size(); ++k) {
    if (!graphed[(size_t)owner[k]]) continue;
    DMat* m = sets[k].m;
    // (a compaction makes room for about ROOM_ROUNDS rounds: each one
    // changes the pools the graph bakes in, and so forces a new capture)
    const int64_t hm = apply_headroom(m, sets[k].n);
    mat_reserve(m, hm, ROOM_ROUNDS * hm);
    if (m->tidx) {
      const int64_t ht = apply_headroom(m->tidx, sets[k].n);
      mat_reserve(m->tidx, ht, ROOM_ROUNDS * ht);
    }
    ensure_ws(c, b->aw, b->aw_bytes, k, apply_work_bytes(sets[k].n, m->tidx != nullptr), ws_changed);
    ensure_ws(c, b->awt, b->awt_bytes, k, apply_work_bytes(sets[k].n, false), ws_changed);
  }
  std::vector<int64_t> c_top_before(np);
  for (size_t j = 0; j < np; ++j) {
    if (!graphed[j]) continue;
    DProd* p = b->prods[j];
    // room for C: twice what the last run took, at least 1/64 of its pool;
    // rows that need still more are completed after the replay.  (A
    // compaction leaves a third of the new pool free, so a floor this low
    // makes C's pool, and the graph that bakes it in, change only every few
    // dozen rounds.)
    const int64_t c_room = std::max<int64_t>(p->C->h_top_ub / 64, 2 * p->last_c_growth) + 4096;
    const size_t arena = std::max<size_t>(p->arena_bytes, (size_t)1 << 20);
    prod_prepare_graph(p, c_room, arena, ROOM_ROUNDS * c_room);
    ensure_ws(c, b->pw, b->pw_bytes, j, prod_graph_work_bytes(p), ws_changed);
    c_top_before[j] = p->C->h_top_ub;
  }
  // ---- the signature of what a graph bakes in ----
  std::vector<uintptr_t> sig(graphed.begin(), graphed.end());
  for (size_t k = 0; k < sets.size(); ++k) {
    if (!graphed[(size_t)owner[k]]) continue;
    const DBatchSet& st = sets[k];
    // (the transpose too: one built later, for another product, must be
    // updated by this set's apply as well)
    for (uintptr_t x : {(uintptr_t)st.m, (uintptr_t)st.m->tidx, (uintptr_t)st.rows, (uintptr_t)st.cols,
                        (uintptr_t)st.vals, (uintptr_t)st.ops, (uintptr_t)st.n, (uintptr_t)b->aw[k],
                        (uintptr_t)b->awt[k]})
      sig.push_back(x);
  }
  for (DMat* m : gmats)
    for (uintptr_t x : {(uintptr_t)m->col, (uintptr_t)m->val, (uintptr_t)m->pool_cap, (uintptr_t)m->version})
      sig.push_back(x);
  for (size_t j = 0; j < np; ++j) {
    if (!graphed[j]) continue;
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
  if (ng > 0 && (!b->exec || sig != b->signature)) {
    t0 = std::chrono::steady_clock::now();
    drop_graph(b);
    // device table of the pool tops the graph reports back (device addresses
    // of each touched matrix's top)
    std::vector<int64_t*> top_ptrs;
    for (DMat* m : gmats) top_ptrs.push_back(m->d_top);
    DSG_REQUIRE(top_ptrs.size() <= b->ntop, DSG_E_DEVICE, "internal: pool-top table too small");
    DSG_HIP(hipMemcpyAsync(b->d_top_ptrs, top_ptrs.data(), top_ptrs.size() * 8, hipMemcpyHostToDevice, main));
    DSG_HIP(hipStreamSynchronize(main));
    hipGraph_t graph = nullptr;
    DSG_HIP(hipStreamBeginCapture(main, hipStreamCaptureModeThreadLocal));
    try {
      hipLaunchKernelGGL(k_clear_out, dim3(1), dim3(256), 0, main, b->d_out, (int)(np * OUT_WORDS));
      DSG_HIP(hipEventRecord(b->ev_fork, main));
      size_t lane = 0;
      for (size_t j = 0; j < np; ++j) {
        if (!graphed[j]) continue;
        hipStream_t sj = b->streams[lane++ % b->streams.size()];
        DSG_HIP(hipStreamWaitEvent(sj, b->ev_fork, 0));
        c->stream = sj;
        int slot = 6;
        for (size_t k = 0; k < sets.size(); ++k) {
          if (owner[k] != (int)j) continue;
          const DBatchSet& st = sets[k];
          mat_apply_graph(st.m, st.rows, st.cols, st.vals, st.ops, st.n, b->aw[k], b->awt[k]);
          if (st.n > 0) {
            const int* e1 = apply_err_ptr(b->aw[k], st.n, st.m->tidx != nullptr);
            const int* e2 = st.m->tidx ? apply_err_ptr(b->awt[k], st.n, false) : nullptr;
            hipLaunchKernelGGL(k_or_flags, dim3(1), dim3(1), 0, sj, e1, e2, b->d_out + j * OUT_WORDS + slot);
          }
          slot = 7;
        }
        prod_update_graph(b->prods[j], b->pw[j], b->d_out + j * OUT_WORDS);
        DSG_HIP(hipEventRecord(b->ev_join[j], sj));
      }
      c->stream = main;
      for (size_t j = 0; j < np; ++j)
        if (graphed[j]) DSG_HIP(hipStreamWaitEvent(main, b->ev_join[j], 0));
      hipLaunchKernelGGL(k_gather_tops, dim3(1), dim3(256), 0, main, (int64_t* const*)b->d_top_ptrs,
                         (int)gmats.size(), b->d_tops);
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
  // ---- the replay, on its own stream once the preparation is done ----
  t0 = std::chrono::steady_clock::now();
  if (ng > 0) {
    DSG_HIP(hipEventRecord(b->ev_ready, main));
    DSG_HIP(hipStreamWaitEvent(b->replay_stream, b->ev_ready, 0));
    // the graph's applies and row writes keep no column index
    for (DMat* m : gmats) mat_index_invalidate(m);
    DSG_HIP(hipGraphLaunch(b->exec, b->replay_stream));
    b->replays++;
  }
  // ---- meanwhile the large products, plain path, on the context's stream ----
  const auto td = std::chrono::steady_clock::now();
  for (size_t j = 0; j < np; ++j) {
    if (graphed[j]) continue;
    for (size_t k = 0; k < sets.size(); ++k)
      if (owner[k] == (int)j) mat_apply_device(sets[k].m, sets[k].rows, sets[k].cols, sets[k].vals, sets[k].ops,
                                               sets[k].n);
    counts[j] = prod_run(b->prods[j], 0, false);
    b->direct++;
  }
  b->direct_ms += ms_since(td);
  if (ng == 0) return DSG_OK;
  // ---- the graph's results ----
  std::vector<int64_t> out(np * OUT_WORDS), tops(gmats.size());
  DSG_HIP(hipMemcpyAsync(out.data(), b->d_out, out.size() * 8, hipMemcpyDeviceToHost, b->replay_stream));
  DSG_HIP(hipMemcpyAsync(tops.data(), b->d_tops, tops.size() * 8, hipMemcpyDeviceToHost, b->replay_stream));
  DSG_HIP(hipStreamSynchronize(b->replay_stream));
  for (size_t i = 0; i < gmats.size(); ++i) gmats[i]->h_top_ub = tops[i];
  // these applies keep no log: the entry-granular update does not follow them
  for (size_t k = 0; k < sets.size(); ++k)
    if (graphed[(size_t)owner[k]] && sets[k].n > 0) sets[k].m->apply_seq++;
  b->replay_ms += ms_since(t0);
  t0 = std::chrono::steady_clock::now();
  for (size_t j = 0; j < np; ++j) {
    if (!graphed[j]) continue;
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
    p->a_seq = p->src_a->apply_seq;
    p->b_seq = p->src_b->apply_seq;
  }
  b->finish_ms += ms_since(t0);
  return DSG_OK;
}
