// Served form: a request loop that keeps A, B and C resident in device memory
// and answers update batches and row queries in arrival order.
//
// Two host threads share the work.  The stager admits requests from the
// arrival queue as staging slots and the memory budget allow.  It merges
// consecutive update requests on one operand into one batch.  Their entries
// keep arrival order, so the merged batch has the effect of the sequence:
// within a batch, later entries of a key win or fold after earlier ones.  It
// also merges consecutive queries into one gather.  Each group is packed into
// pinned host memory and copied to the device on a stream of its own.  The
// executor takes the groups in order: ingest plus the dynamic update for an
// update group (context's stream), a row gather for a query group (a query
// stream).  Results are those of the arrival order, and device work overlaps:
//   - the copy of the next group overlaps the device work of the current one;
//   - a query's gather overlaps the ingest of the update after it (which
//     changes only the operand): the gather starts after the update before
//     it (an event), and the next update's product step waits for the gather
//     (another event), since only that step changes C.
// Requests that arrive meanwhile join the next group.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "internal.h"

namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct SReq {
  uint64_t ticket = 0;
  int kind = 0;                     // 0: update, 1: query
  DMat* target = nullptr;           // update: the operand
  std::vector<int32_t> rows, cols;  // update entries, or the query's rows
  std::vector<char> vals;
  std::vector<uint8_t> ops;
  double t_submit = 0, t_done = 0;
  int status = DSG_PENDING;
  int64_t group = -1;
  int32_t group_requests = 0;
  int32_t changed = 0;
  RowsHost answer;
  int64_t size() const { return kind == 0 ? (int64_t)ops.size() : (int64_t)rows.size(); }
};

struct Slot {
  void* host = nullptr;  // pinned staging
  size_t host_bytes = 0;
  void* dev = nullptr;
  size_t dev_bytes = 0;
  hipEvent_t copied = nullptr;
  bool busy = false;
};

struct Group {
  int kind = 0;
  int64_t id = 0;
  DMat* target = nullptr;
  std::vector<SReq*> reqs;
  int slot = -1;
  int64_t n = 0;   // entries (update) or rows (query)
  size_t est = 0;  // bytes it holds against the budget
  int32_t* d_rows = nullptr;
  int32_t* d_cols = nullptr;
  void* d_vals = nullptr;
  uint8_t* d_ops = nullptr;
};

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q * (double)(v.size() - 1);
  const size_t lo = (size_t)pos;
  const size_t hi = std::min(lo + 1, v.size() - 1);
  return v[lo] + (v[hi] - v[lo]) * (pos - (double)lo);
}

}  // namespace

struct DServer {
  Ctx* c = nullptr;
  DProd* p = nullptr;
  dsg_server_cfg cfg{};
  std::mutex mu;
  std::condition_variable cv_arrive;  // stager: requests arrived, or stop
  std::condition_variable cv_ready;   // executor: a group is staged, or the stager ended
  std::condition_variable cv_free;    // stager: a slot or memory was released
  std::condition_variable cv_done;    // clients: requests completed
  std::deque<SReq*> arrivals;
  std::deque<Group*> ready;
  std::unordered_map<uint64_t, SReq*> reqs;
  std::vector<Slot> slots;
  uint64_t next_ticket = 1;
  int64_t submitted = 0, completed = 0, next_group = 0;
  size_t inflight = 0, peak_inflight = 0;
  bool stop = false, stager_done = false;
  dsg_status failed = DSG_OK;
  std::string failure;
  hipStream_t copy = nullptr;
  hipStream_t qstream = nullptr;  // query gathers
  hipEvent_t c_ready = nullptr;   // on the context's stream: C after the last update
  hipEvent_t q_done = nullptr;    // on the query stream: the gather in flight read C
  void* q_col_h = nullptr;        // pinned: the gathered entries
  size_t q_col_bytes = 0;
  void* q_val_h = nullptr;
  size_t q_val_bytes = 0;
  std::thread stager, executor;
  GatherBufs gather;
  // admission estimates, refreshed by the executor after each group
  double ws_per_entry = 64.0;   // product workspace bytes per update entry
  double row_bytes = 64.0;      // bytes of an average row of C
  // statistics
  std::vector<double> lat_update, lat_query;
  int64_t n_update = 0, n_query = 0, update_entries = 0, update_groups = 0, query_groups = 0;
  double first_submit = -1.0, last_done = 0.0;
};

namespace {

// bytes an update group of n entries holds: its staged entries plus an
// estimate of the ingest and product workspaces it needs
size_t update_bytes(const DServer* s, DMat* m, int64_t n) {
  const bool deltas = m->tidx != nullptr;
  return (size_t)n * (9 + (size_t)m->vsz) + apply_work_bytes(n, deltas) + (deltas ? apply_work_bytes(n, false) : 0) +
         (size_t)(s->ws_per_entry * (double)n);
}

size_t query_bytes(const DServer* s, int64_t nq) {
  return (size_t)nq * 20 + (size_t)(s->row_bytes * (double)nq) + 4096;
}

size_t group_bytes(const DServer* s, const SReq* head, int64_t n) {
  return head->kind == 0 ? update_bytes(s, head->target, n) : query_bytes(s, n);
}

int free_slot(const DServer* s) {
  for (size_t i = 0; i < s->slots.size(); ++i)
    if (!s->slots[i].busy) return (int)i;
  return -1;
}

// complete a request (lock held)
void finish(DServer* s, SReq* r, int status, double t) {
  r->status = status;
  r->t_done = t;
  if (status == DSG_OK) {
    const double lat = t - r->t_submit;
    if (r->kind == 0) {
      s->lat_update.push_back(lat);
      s->n_update++;
      s->update_entries += r->size();
    } else {
      s->lat_query.push_back(lat);
      s->n_query++;
    }
  }
  s->completed++;
  s->last_done = std::max(s->last_done, t);
  // a finished request's input is no longer needed
  std::vector<int32_t>().swap(r->cols);
  std::vector<char>().swap(r->vals);
  std::vector<uint8_t>().swap(r->ops);
  if (r->kind == 0) std::vector<int32_t>().swap(r->rows);
}

void grow_slot(DServer* s, Slot& sl, size_t bytes) {
  if (sl.host_bytes < bytes) {
    if (sl.host) (void)hipHostFree(sl.host);
    sl.host = nullptr;
    sl.host_bytes = 0;
    const size_t nb = bytes + bytes / 2 + 65536;
    DSG_HIP(hipHostMalloc(&sl.host, nb, hipHostMallocDefault));
    sl.host_bytes = nb;
  }
  if (sl.dev_bytes < bytes) {
    ctx_free(s->c, sl.dev, sl.dev_bytes);
    sl.dev = nullptr;
    sl.dev_bytes = 0;
    const size_t nb = bytes + bytes / 2 + 65536;
    sl.dev = ctx_alloc(s->c, nb);
    sl.dev_bytes = nb;
  }
}

// Pack a group into its slot's pinned buffer and start the copy to the device.
void stage(DServer* s, Group* g) {
  Slot& sl = s->slots[(size_t)g->slot];
  if (g->kind == 0) {
    const size_t vsz = (size_t)g->target->vsz;
    const size_t n = (size_t)g->n;
    const size_t o_cols = align256(n * 4), o_vals = o_cols + align256(n * 4), o_ops = o_vals + align256(n * vsz);
    const size_t total = o_ops + align256(n);
    grow_slot(s, sl, total);
    char* h = (char*)sl.host;
    size_t at = 0;
    for (SReq* r : g->reqs) {
      const size_t k = r->ops.size();
      if (k) {
        memcpy(h + at * 4, r->rows.data(), k * 4);
        memcpy(h + o_cols + at * 4, r->cols.data(), k * 4);
        if (vsz) memcpy(h + o_vals + at * vsz, r->vals.data(), k * vsz);
        memcpy(h + o_ops + at, r->ops.data(), k);
      }
      at += k;
    }
    char* d = (char*)sl.dev;
    g->d_rows = (int32_t*)d;
    g->d_cols = (int32_t*)(d + o_cols);
    g->d_vals = vsz ? (void*)(d + o_vals) : nullptr;
    g->d_ops = (uint8_t*)(d + o_ops);
    if (total) DSG_HIP(hipMemcpyAsync(d, h, total, hipMemcpyHostToDevice, s->copy));
  } else {
    const size_t total = align256((size_t)g->n * 4);
    grow_slot(s, sl, total);
    size_t at = 0;
    for (SReq* r : g->reqs) {
      if (!r->rows.empty()) memcpy((char*)sl.host + at * 4, r->rows.data(), r->rows.size() * 4);
      at += r->rows.size();
    }
    g->d_rows = (int32_t*)sl.dev;
    if (total) DSG_HIP(hipMemcpyAsync(sl.dev, sl.host, total, hipMemcpyHostToDevice, s->copy));
  }
  DSG_HIP(hipEventRecord(sl.copied, s->copy));
}

void stager_main(DServer* s) {
  (void)hipSetDevice(s->c->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_arrive.wait(lk, [&] { return s->stop || !s->arrivals.empty(); });
    if (s->arrivals.empty()) break;
    if (s->failed != DSG_OK) {
      // the executor failed: nothing more runs
      const double t = now_ms();
      while (!s->arrivals.empty()) {
        finish(s, s->arrivals.front(), s->failed, t);
        s->arrivals.pop_front();
      }
      s->cv_done.notify_all();
      continue;
    }
    // a slot first; requests that arrive meanwhile join the group
    s->cv_free.wait(lk, [&] { return free_slot(s) >= 0; });
    SReq* head = s->arrivals.front();
    const int64_t cap = head->kind == 0 ? s->cfg.max_coalesce : (int64_t)s->cfg.max_query_rows;
    size_t k = 0;
    int64_t n = 0;
    while (k < s->arrivals.size()) {
      SReq* r = s->arrivals[k];
      if (r->kind != head->kind || r->target != head->target) break;
      const int64_t rn = r->size();
      if (k > 0 && (n + rn > cap || s->inflight + group_bytes(s, head, n + rn) > s->cfg.mem_budget)) break;
      n += rn;
      ++k;
    }
    const size_t est = group_bytes(s, head, n);
    // memory: wait for groups in flight to finish (a group larger than the
    // whole budget runs alone)
    s->cv_free.wait(lk, [&] { return s->inflight == 0 || s->inflight + est <= s->cfg.mem_budget; });
    Group* g = new Group();
    g->kind = head->kind;
    g->target = head->target;
    g->n = n;
    g->est = est;
    g->id = s->next_group++;
    g->slot = free_slot(s);
    for (size_t t = 0; t < k; ++t) {
      g->reqs.push_back(s->arrivals.front());
      s->arrivals.pop_front();
    }
    s->slots[(size_t)g->slot].busy = true;
    s->inflight += est;
    s->peak_inflight = std::max(s->peak_inflight, s->inflight);
    lk.unlock();
    int st = DSG_OK;
    std::string msg;
    try {
      stage(s, g);
    } catch (const DsgError& e) {
      st = e.code;
      msg = e.msg;
    } catch (...) {
      st = DSG_E_DEVICE;
      msg = "staging failed";
    }
    lk.lock();
    if (st != DSG_OK) {
      const double t = now_ms();
      for (SReq* r : g->reqs) finish(s, r, st, t);
      s->slots[(size_t)g->slot].busy = false;
      s->inflight -= g->est;
      if (s->failed == DSG_OK) {
        s->failed = (dsg_status)st;
        s->failure = msg;
      }
      delete g;
      s->cv_done.notify_all();
      continue;
    }
    s->ready.push_back(g);
    s->cv_ready.notify_one();
  }
  s->stager_done = true;
  s->cv_ready.notify_all();
}

// A query group whose gather is in flight on the query stream.
struct PendingQuery {
  Group* g = nullptr;
  std::vector<int64_t> row_ptr;  // the gathered rows' pointers
  int64_t nnz = 0;
  int status = DSG_OK;
  std::string msg;
};

void ensure_dev(Ctx* c, void*& p, size_t& have, size_t bytes) {
  if (have >= bytes) return;
  ctx_free(c, p, have);
  p = nullptr;
  have = 0;
  const size_t nb = bytes + bytes / 2 + 4096;
  p = ctx_alloc(c, nb);
  have = nb;
}

void ensure_pinned(void*& p, size_t& have, size_t bytes) {
  if (have >= bytes) return;
  if (p) (void)hipHostFree(p);
  p = nullptr;
  have = 0;
  const size_t nb = bytes + bytes / 2 + 4096;
  DSG_HIP(hipHostMalloc(&p, nb, hipHostMallocDefault));
  have = nb;
}

// Start a query group's gather on the query stream, after its rows are
// staged and after the last update: row lengths and pointers (read back),
// then the entries into pinned memory; q_done marks the end.
void query_begin(DServer* s, Group* g, PendingQuery& pq) {
  Ctx* c = s->c;
  DMat* C = s->p->C;
  hipStream_t q = s->qstream;
  pq = PendingQuery();
  pq.g = g;
  const int32_t n = (int32_t)g->n;
  DSG_HIP(hipStreamWaitEvent(q, s->slots[(size_t)g->slot].copied, 0));
  DSG_HIP(hipStreamWaitEvent(q, s->c_ready, 0));
  GatherBufs& b = s->gather;
  ensure_dev(c, b.lens, b.lens_bytes, ((size_t)n + 1) * 8);
  ensure_dev(c, b.rp, b.rp_bytes, ((size_t)n + 1) * 8);
  ensure_dev(c, b.scan, b.scan_bytes, scan_scratch_bytes(n) + 64);
  gather_row_ptr(C, g->d_rows, n, (int64_t*)b.lens, (int64_t*)b.rp, b.scan, q);
  pq.row_ptr.assign((size_t)n + 1, 0);
  DSG_HIP(hipMemcpyAsync(pq.row_ptr.data(), b.rp, pq.row_ptr.size() * 8, hipMemcpyDeviceToHost, q));
  DSG_HIP(hipStreamSynchronize(q));
  pq.nnz = pq.row_ptr[(size_t)n];
  const size_t vs = (size_t)C->vsz;
  if (pq.nnz > 0) {
    ensure_dev(c, b.col, b.col_bytes, (size_t)pq.nnz * 4);
    ensure_dev(c, b.val, b.val_bytes, (size_t)pq.nnz * (vs ? vs : 1));
    ensure_pinned(s->q_col_h, s->q_col_bytes, (size_t)pq.nnz * 4);
    if (vs) ensure_pinned(s->q_val_h, s->q_val_bytes, (size_t)pq.nnz * vs);
    gather_row_entries(C, g->d_rows, n, (const int64_t*)b.rp, (int32_t*)b.col, b.val, q);
    DSG_HIP(hipMemcpyAsync(s->q_col_h, b.col, (size_t)pq.nnz * 4, hipMemcpyDeviceToHost, q));
    if (vs) DSG_HIP(hipMemcpyAsync(s->q_val_h, b.val, (size_t)pq.nnz * vs, hipMemcpyDeviceToHost, q));
  }
  DSG_HIP(hipEventRecord(s->q_done, q));
}

// Complete the query in flight: wait for its gather, sort each row by column,
// split the answer per request, release its slot.
void query_finish(DServer* s, PendingQuery& pq) {
  Group* g = pq.g;
  int st = pq.status;
  std::string msg = pq.msg;
  if (st == DSG_OK) {
    try {
      DSG_HIP(hipEventSynchronize(s->q_done));
      const size_t vs = (size_t)s->p->C->vsz;
      const int32_t* hc = (const int32_t*)s->q_col_h;
      const char* hv = (const char*)s->q_val_h;
      std::vector<int64_t> perm;
      size_t q0 = 0;
      for (SReq* r : g->reqs) {
        const size_t nq = r->rows.size();
        const int64_t e0 = pq.row_ptr[q0], e1 = pq.row_ptr[q0 + nq];
        r->answer.row_ptr.resize(nq + 1);
        for (size_t q = 0; q <= nq; ++q) r->answer.row_ptr[q] = pq.row_ptr[q0 + q] - e0;
        r->answer.col.resize((size_t)(e1 - e0));
        r->answer.val.resize((size_t)(e1 - e0) * vs);
        // rows are stored in no particular column order: sort each one
        for (size_t q = 0; q < nq; ++q) {
          const int64_t a = pq.row_ptr[q0 + q], b = pq.row_ptr[q0 + q + 1];
          perm.resize((size_t)(b - a));
          for (int64_t e = a; e < b; ++e) perm[(size_t)(e - a)] = e;
          std::sort(perm.begin(), perm.end(), [&](int64_t x, int64_t y) { return hc[x] < hc[y]; });
          for (int64_t e = a; e < b; ++e) {
            const int64_t src = perm[(size_t)(e - a)];
            r->answer.col[(size_t)(e - e0)] = hc[src];
            if (vs) memcpy(r->answer.val.data() + (size_t)(e - e0) * vs, hv + (size_t)src * vs, vs);
          }
        }
        q0 += nq;
      }
    } catch (const DsgError& e) {
      st = e.code;
      msg = e.msg;
    }
  }
  // (a gather that failed part way may still be reading the slot)
  if (st != DSG_OK) (void)hipStreamSynchronize(s->qstream);
  const double t = now_ms();
  std::lock_guard<std::mutex> lk(s->mu);
  for (SReq* r : g->reqs) {
    r->group = g->id;
    r->group_requests = (int32_t)g->reqs.size();
    finish(s, r, st, t);
  }
  if (st == DSG_OK) s->query_groups++;
  else if (s->failed == DSG_OK) {
    s->failed = (dsg_status)st;
    s->failure = msg;
  }
  s->slots[(size_t)g->slot].busy = false;
  s->inflight -= g->est;
  delete g;
  pq.g = nullptr;
  s->cv_free.notify_all();
  s->cv_done.notify_all();
  if (s->failed != DSG_OK) s->cv_arrive.notify_all();
}

void executor_main(DServer* s) {
  (void)hipSetDevice(s->c->device);
  Ctx* c = s->c;
  PendingQuery pq;
  for (;;) {
    Group* g = nullptr;
    dsg_status failed;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (pq.g && s->ready.empty()) {
        // nothing to overlap the gather with: complete the query now
        lk.unlock();
        query_finish(s, pq);
        continue;
      }
      s->cv_ready.wait(lk, [&] { return !s->ready.empty() || s->stager_done; });
      if (s->ready.empty()) break;
      g = s->ready.front();
      s->ready.pop_front();
      failed = s->failed;
    }
    if (g->kind == 1) {
      if (pq.g) query_finish(s, pq);  // one gather in flight at a time
      PendingQuery next;
      next.g = g;
      next.status = failed;
      if (failed == DSG_OK) {
        try {
          query_begin(s, g, next);
        } catch (const DsgError& e) {
          next.g = g;
          next.status = e.code;
          next.msg = e.msg;
        }
      }
      pq = std::move(next);
      continue;
    }
    int st = failed;
    std::string msg;
    int32_t changed = 0;
    double ws = -1.0, rb = -1.0;
    if (st == DSG_OK) {
      try {
        DSG_HIP(hipStreamWaitEvent(c->stream, s->slots[(size_t)g->slot].copied, 0));
        if (g->n > 0) mat_apply_device(g->target, g->d_rows, g->d_cols, g->d_vals, g->d_ops, g->n);
        if (pq.g) {
          // the product step changes C: after the gather before it
          DSG_HIP(hipStreamWaitEvent(c->stream, s->q_done, 0));
          query_finish(s, pq);
        }
        changed = prod_run(s->p, 0, false);
        DSG_HIP(hipEventRecord(s->c_ready, c->stream));
        if (g->n > 0) {
          // workspace the update took: products and entry updates on the
          // entry-granular path, staging and new C space on the row path
          const dsg_update_stats& st = s->p->stats;
          const double sz = 4.0 + (double)s->p->C->vsz;
          const double bytes = st.path == 1 ? 32.0 * (double)st.terms + 64.0 * (double)st.entries
                                            : (double)s->p->last_arena_demand + sz * (double)s->p->last_c_demand;
          ws = std::min(std::max(bytes / (double)g->n, 16.0), 65536.0);
        }
        rb = (4.0 + (double)s->p->C->vsz) * (double)s->p->C->h_top_ub / (double)std::max<int32_t>(s->p->C->nrows, 1);
      } catch (const DsgError& e) {
        st = e.code;
        msg = e.msg;
      } catch (...) {
        st = DSG_E_DEVICE;
        msg = "unexpected internal error";
      }
    }
    if (pq.g) query_finish(s, pq);  // (an update that failed before its product step)
    const double t = now_ms();
    std::lock_guard<std::mutex> lk(s->mu);
    for (SReq* r : g->reqs) {
      r->group = g->id;
      r->group_requests = (int32_t)g->reqs.size();
      r->changed = changed;
      finish(s, r, st, t);
    }
    if (st == DSG_OK) {
      s->update_groups++;
      if (ws >= 0) s->ws_per_entry = 0.5 * s->ws_per_entry + 0.5 * ws;
      if (rb >= 0) s->row_bytes = rb;
    } else if (s->failed == DSG_OK) {
      s->failed = (dsg_status)st;
      s->failure = msg;
    }
    s->slots[(size_t)g->slot].busy = false;
    s->inflight -= g->est;
    delete g;
    s->cv_free.notify_all();
    s->cv_done.notify_all();
    if (s->failed != DSG_OK) s->cv_arrive.notify_all();
  }
  if (pq.g) query_finish(s, pq);
}

void check_entries(const DMat* m, const int32_t* rows, const int32_t* cols, const uint8_t* ops, int64_t n) {
  for (int64_t t = 0; t < n; ++t) {
    if (rows[t] < 0 || rows[t] >= m->nrows || cols[t] < 0 || cols[t] >= m->ncols)
      throw DsgError{DSG_E_RANGE, "update entry " + std::to_string(t) + " out of range"};
    if (ops[t] > DSG_OP_ADD) throw DsgError{DSG_E_ARG, "bad op code at entry " + std::to_string(t)};
  }
}

SReq* find_req(DServer* s, uint64_t ticket) {
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) throw DsgError{DSG_E_ARG, "unknown ticket"};
  return it->second;
}

uint64_t enqueue(DServer* s, SReq* r) {
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) {
    delete r;
    throw DsgError{DSG_E_STATE, "server is stopping"};
  }
  r->ticket = s->next_ticket++;
  r->t_submit = now_ms();
  if (s->first_submit < 0) s->first_submit = r->t_submit;
  s->reqs[r->ticket] = r;
  s->arrivals.push_back(r);
  s->submitted++;
  s->cv_arrive.notify_one();
  return r->ticket;
}

}  // namespace

DServer* server_create(Ctx* c, DProd* p, const dsg_server_cfg* cfg) {
  DServer* s = new DServer();
  s->c = c;
  s->p = p;
  if (cfg) s->cfg = *cfg;
  if (s->cfg.mem_budget == 0) s->cfg.mem_budget = (size_t)4 << 30;
  if (s->cfg.max_coalesce <= 0) s->cfg.max_coalesce = (int64_t)1 << 20;
  if (s->cfg.max_query_rows <= 0) s->cfg.max_query_rows = 65536;
  if (s->cfg.slots <= 0) s->cfg.slots = 2;
  s->cfg.slots = std::min(s->cfg.slots, 8);
  try {
    DSG_HIP(hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking));
    DSG_HIP(hipStreamCreateWithFlags(&s->qstream, hipStreamNonBlocking));
    DSG_HIP(hipEventCreateWithFlags(&s->c_ready, hipEventDisableTiming));
    DSG_HIP(hipEventCreateWithFlags(&s->q_done, hipEventDisableTiming));
    DSG_HIP(hipEventRecord(s->c_ready, c->stream));
    s->slots.resize((size_t)s->cfg.slots);
    for (Slot& sl : s->slots) DSG_HIP(hipEventCreateWithFlags(&sl.copied, hipEventDisableTiming));
    // the product's workspaces at their largest before requests arrive
    ctx_sync(c);
    p->refs++;
    s->stager = std::thread(stager_main, s);
    s->executor = std::thread(executor_main, s);
  } catch (...) {
    for (Slot& sl : s->slots)
      if (sl.copied) (void)hipEventDestroy(sl.copied);
    if (s->copy) (void)hipStreamDestroy(s->copy);
    if (s->qstream) (void)hipStreamDestroy(s->qstream);
    if (s->c_ready) (void)hipEventDestroy(s->c_ready);
    if (s->q_done) (void)hipEventDestroy(s->q_done);
    delete s;
    throw;
  }
  return s;
}

void server_destroy(DServer* s) {
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->completed == s->submitted; });
    s->stop = true;
  }
  s->cv_arrive.notify_all();
  s->cv_free.notify_all();
  s->stager.join();
  s->executor.join();
  (void)hipStreamSynchronize(s->c->stream);
  (void)hipStreamSynchronize(s->copy);
  (void)hipStreamSynchronize(s->qstream);
  for (Slot& sl : s->slots) {
    if (sl.host) (void)hipHostFree(sl.host);
    ctx_free(s->c, sl.dev, sl.dev_bytes);
    if (sl.copied) (void)hipEventDestroy(sl.copied);
  }
  gather_bufs_free(s->c, s->gather);
  if (s->q_col_h) (void)hipHostFree(s->q_col_h);
  if (s->q_val_h) (void)hipHostFree(s->q_val_h);
  (void)hipStreamDestroy(s->copy);
  (void)hipStreamDestroy(s->qstream);
  (void)hipEventDestroy(s->c_ready);
  (void)hipEventDestroy(s->q_done);
  for (auto& kv : s->reqs) delete kv.second;
  s->p->refs--;
  delete s;
}

uint64_t server_submit_update(DServer* s, DMat* m, const int32_t* rows, const int32_t* cols, const void* vals,
                              const uint8_t* ops, int64_t n) {
  DSG_REQUIRE(m == s->p->src_a || m == s->p->src_b, DSG_E_ARG, "matrix is not an operand of the served product");
  check_entries(m, rows, cols, ops, n);
  SReq* r = new SReq();
  r->kind = 0;
  r->target = m;
  r->rows.assign(rows, rows + n);
  r->cols.assign(cols, cols + n);
  r->ops.assign(ops, ops + n);
  if (m->vsz) r->vals.assign((const char*)vals, (const char*)vals + (size_t)n * m->vsz);
  return enqueue(s, r);
}

uint64_t server_submit_query(DServer* s, const int32_t* rows, int32_t nq) {
  const int32_t nr = s->p->C->nrows;
  for (int32_t t = 0; t < nq; ++t)
    if (rows[t] < 0 || rows[t] >= nr) throw DsgError{DSG_E_RANGE, "query row " + std::to_string(t) + " out of range"};
  SReq* r = new SReq();
  r->kind = 1;
  r->rows.assign(rows, rows + nq);
  return enqueue(s, r);
}

void server_poll(DServer* s, uint64_t ticket, bool wait, dsg_server_result* out) {
  std::unique_lock<std::mutex> lk(s->mu);
  SReq* r = find_req(s, ticket);
  if (wait) s->cv_done.wait(lk, [&] { return r->status != DSG_PENDING; });
  *out = dsg_server_result{};
  out->status = r->status;
  out->kind = r->kind;
  out->latency_ms = r->status == DSG_PENDING ? 0.0 : r->t_done - r->t_submit;
  out->group = r->group;
  out->group_requests = r->group_requests;
  out->changed_rows = r->changed;
  out->nq = r->kind == 1 ? (int32_t)r->rows.size() : 0;
  out->nnz = r->kind == 1 && !r->answer.row_ptr.empty() ? r->answer.row_ptr.back() : 0;
}

void server_query_result(DServer* s, uint64_t ticket, int64_t* row_ptr, int32_t* col, void* val, int64_t cap,
                         int64_t* nnz_out) {
  std::lock_guard<std::mutex> lk(s->mu);
  SReq* r = find_req(s, ticket);
  DSG_REQUIRE(r->kind == 1, DSG_E_ARG, "not a query");
  DSG_REQUIRE(r->status == DSG_OK, DSG_E_STATE, "query has not completed successfully");
  const int64_t nnz = r->answer.row_ptr.back();
  *nnz_out = nnz;
  if (row_ptr) memcpy(row_ptr, r->answer.row_ptr.data(), r->answer.row_ptr.size() * 8);
  if (!col) return;
  DSG_REQUIRE(cap >= nnz, DSG_E_ARG, "capacity < nnz");
  if (nnz == 0) return;
  memcpy(col, r->answer.col.data(), (size_t)nnz * 4);
  memcpy(val, r->answer.val.data(), r->answer.val.size());
}

void server_release(DServer* s, uint64_t ticket) {
  std::lock_guard<std::mutex> lk(s->mu);
  SReq* r = find_req(s, ticket);
  DSG_REQUIRE(r->status != DSG_PENDING, DSG_E_STATE, "request still pending");
  s->reqs.erase(ticket);
  delete r;
}

void server_drain(DServer* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->completed == s->submitted; });
}

void server_stats(DServer* s, dsg_server_stats* out) {
  std::lock_guard<std::mutex> lk(s->mu);
  *out = dsg_server_stats{};
  out->update_requests = s->n_update;
  out->query_requests = s->n_query;
  out->update_entries = s->update_entries;
  out->update_groups = s->update_groups;
  out->query_groups = s->query_groups;
  out->update_p50_ms = percentile(s->lat_update, 0.5);
  out->update_p99_ms = percentile(s->lat_update, 0.99);
  out->query_p50_ms = percentile(s->lat_query, 0.5);
  out->query_p99_ms = percentile(s->lat_query, 0.99);
  double a = 0, b = 0;
  for (double x : s->lat_update) a += x;
  for (double x : s->lat_query) b += x;
  out->update_mean_ms = s->lat_update.empty() ? 0.0 : a / (double)s->lat_update.size();
  out->query_mean_ms = s->lat_query.empty() ? 0.0 : b / (double)s->lat_query.size();
  out->busy_ms = s->first_submit < 0 ? 0.0 : std::max(0.0, s->last_done - s->first_submit);
  out->updates_per_s = out->busy_ms > 0 ? (double)s->update_entries / (out->busy_ms * 1e-3) : 0.0;
  out->peak_inflight_bytes = s->peak_inflight;
}

std::string server_failure(DServer* s) {
  std::lock_guard<std::mutex> lk(s->mu);
  return s->failure;
}
