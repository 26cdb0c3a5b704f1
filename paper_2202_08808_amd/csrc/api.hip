// C ABI of the dsg library: argument checks, host/device marshalling, error
// mapping.  All numeric work happens in the HIP kernels of the other files.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>

#include "internal.h"

struct dsg_ctx {
  Ctx c;
};
struct dsg_mat {
  DMat* m;
  dsg_ctx* owner;
  bool alive;
};
struct dsg_prod {
  DProd* p;
  dsg_ctx* owner;
  dsg_mat* A;
  dsg_mat* B;
};

// ---------------------------------------------------------------------------
// context services used by the rest of the library
// ---------------------------------------------------------------------------

void* ctx_alloc(Ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 1;
  std::lock_guard<std::mutex> lk(c->alloc_mu);
  if (c->budget && c->held + bytes > c->budget)
    throw DsgError{DSG_E_OOM, "memory budget exceeded (" + std::to_string(c->held + bytes) + " > " +
                                  std::to_string(c->budget) + " bytes)"};
  void* p = nullptr;
  if (c->allocator.alloc) {
    p = c->allocator.alloc(bytes, (void*)c->stream, c->allocator.user);
    if (!p) throw DsgError{DSG_E_OOM, "the caller's allocator refused " + std::to_string(bytes) + " bytes"};
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      throw DsgError{DSG_E_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
    }
  }
  c->held += bytes;
  return p;
}

void ctx_free(Ctx* c, void* p, size_t bytes) {
  if (!p) return;
  if (bytes == 0) bytes = 1;
  std::lock_guard<std::mutex> lk(c->alloc_mu);
  if (c->allocator.alloc) c->allocator.free(p, bytes, (void*)c->stream, c->allocator.user);
  else (void)hipFree(p);
  c->held -= std::min(c->held, bytes);
}

static void* grow_scratch(Ctx* c, void*& buf, size_t& have, size_t bytes) {
  if (bytes <= have) return buf;
  DSG_HIP(hipStreamSynchronize(c->stream));
  ctx_free(c, buf, have);
  buf = nullptr;
  have = 0;
  size_t nb = bytes + bytes / 4 + (1 << 20);
  buf = ctx_alloc(c, nb);
  have = nb;
  return buf;
}

void* ctx_scratch(Ctx* c, size_t bytes) { return grow_scratch(c, c->scratch, c->scratch_bytes, bytes); }
void* ctx_scratch2(Ctx* c, size_t bytes) { return grow_scratch(c, c->scratch2, c->scratch2_bytes, bytes); }

void ctx_sync(Ctx* c) { DSG_HIP(hipStreamSynchronize(c->stream)); }

// Timing events come from a pool filled when timing is switched on, so that
// a timed phase costs two event records and no event creation.
static hipEvent_t take_event(Ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  DSG_HIP(hipEventCreate(&e));
  return e;
}

bool ctx_timing_begin(Ctx* c, const char* name, double bytes, hipEvent_t* start, hipEvent_t* stop,
                      hipStream_t on) {
  if (!c->timing_phase.empty() && c->timing_phase != name) {
    *start = *stop = nullptr;
    return false;
  }
  KernelTiming t;
  t.name = name;
  t.bytes = bytes;
  t.start = take_event(c);
  t.stop = take_event(c);
  DSG_HIP(hipEventRecord(t.start, on ? on : c->stream));
  *start = t.start;
  *stop = t.stop;
  c->timings.push_back(t);
  return true;
}

void ctx_timing_end(Ctx* c, hipEvent_t stop, hipStream_t on) {
  if (stop) DSG_HIP(hipEventRecord(stop, on ? on : c->stream));
}

hipStream_t ctx_side_stream(Ctx* c) {
  if (!c->side) {
    DSG_HIP(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
    DSG_HIP(hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming));
    DSG_HIP(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
  }
  return c->side;
}

static void clear_timings(Ctx* c) {
  for (auto& t : c->timings) {
    c->event_pool.push_back(t.start);
    c->event_pool.push_back(t.stop);
  }
  c->timings.clear();
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

static thread_local std::string g_create_error;

static dsg_status fail(dsg_ctx* ctx, dsg_status code, const std::string& msg) {
  if (ctx) ctx->c.last_error = msg;
  else g_create_error = msg;
  return code;
}

#define API_BEGIN(ctxp)                                                            \
  dsg_ctx* ctx__ = (ctxp);                                                         \
  if (ctx__ && ctx__->c.served) return fail(ctx__, DSG_E_STATE, "context is served"); \
  try {
#define API_END                                                   \
  }                                                               \
  catch (const DsgError& e) {                                     \
    return fail(ctx__, e.code, e.msg);                            \
  }                                                               \
  catch (const std::bad_alloc&) {                                 \
    return fail(ctx__, DSG_E_OOM, "host allocation failed");      \
  }                                                               \
  catch (...) {                                                   \
    return fail(ctx__, DSG_E_DEVICE, "unexpected internal error"); \
  }                                                               \
  return DSG_OK;

static int value_size(int sr) { return sr == DSG_MIN_PLUS_F32 || sr == DSG_OR_AND_U32 ? 4 : 8; }

static void set_device(dsg_ctx* ctx) { DSG_HIP(hipSetDevice(ctx->c.device)); }

// device copy of a host array (or a device alias when flags say so)
struct DevArray {
  Ctx* c = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  bool owned = false;
  DevArray() = default;
  DevArray(const DevArray&) = delete;
  ~DevArray() {
    if (owned && c) ctx_free(c, p, bytes);
  }
  void host(Ctx* cc, const void* src, size_t b) {
    c = cc;
    bytes = b;
    p = ctx_alloc(c, b ? b : 1);
    owned = true;
    if (b) DSG_HIP(hipMemcpyAsync(p, src, b, hipMemcpyHostToDevice, c->stream));
  }
  void device(const void* src) { p = const_cast<void*>(src); }
};

static void default_tuning(dsg_tuning* t) {
  for (int b = 0; b < 8; ++b) t->group_ub[b] = 32 << b;
  t->dense_max_passes = 4;
  t->force_bin = -1;
  t->update_path = 0;
  t->batch_direct_log2 = 24;
  t->entry_fixed = 1e8;
  t->entry_per_term = 70.0;
  t->row_index = 1;
}

// host-side check of a CSR: row_ptr monotone from 0, columns in range, no
// repeated column inside a row
static dsg_status check_csr(int32_t nrows, int32_t ncols, const int64_t* rp, const int32_t* ci,
                            std::string& msg) {
  if (rp[0] != 0) {
    msg = "row_ptr[0] must be 0";
    return DSG_E_ARG;
  }
  std::vector<int32_t> mark((size_t)std::max(ncols, 1), -1);
  for (int32_t i = 0; i < nrows; ++i) {
    if (rp[i + 1] < rp[i]) {
      msg = "row_ptr is not monotone at row " + std::to_string(i);
      return DSG_E_ARG;
    }
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      int32_t j = ci[e];
      if (j < 0 || j >= ncols) {
        msg = "column index out of range in row " + std::to_string(i);
        return DSG_E_RANGE;
      }
      if (mark[j] == i) {
        msg = "repeated column " + std::to_string(j) + " in row " + std::to_string(i);
        return DSG_E_ARG;
      }
      mark[j] = i;
    }
  }
  return DSG_OK;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------

extern "C" dsg_status dsg_ctx_create(int device, void* hip_stream, size_t mem_budget, dsg_ctx** out) {
  if (!out) return fail(nullptr, DSG_E_ARG, "out is NULL");
  *out = nullptr;
  dsg_ctx* ctx = nullptr;
  try {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
      (void)hipGetLastError();
      return fail(nullptr, DSG_E_DEVICE, "no HIP device available");
    }
    if (device < 0 || device >= count) return fail(nullptr, DSG_E_ARG, "bad device index");
    DSG_HIP(hipSetDevice(device));
    ctx = new dsg_ctx();
    Ctx& c = ctx->c;
    c.device = device;
    c.budget = mem_budget;
    int cus = 0;
    DSG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    c.num_cus = cus > 0 ? cus : 1;
    default_tuning(&c.tuning);
    if (hip_stream) {
      c.stream = (hipStream_t)hip_stream;
    } else {
      DSG_HIP(hipStreamCreate(&c.stream));
      c.own_stream = true;
    }
    DSG_HIP(hipHostMalloc(&c.pinned, 4096, hipHostMallocDefault));
    DSG_HIP(hipHostGetDevicePointer(&c.pinned_dev, c.pinned, 0));
    noalloc_init(device);  // the allocation-free row export's staging array on this device
  } catch (const DsgError& e) {
    if (ctx) {
      if (ctx->c.own_stream) (void)hipStreamDestroy(ctx->c.stream);
      delete ctx;
    }
    return fail(nullptr, e.code, e.msg);
  } catch (...) {
    delete ctx;
    return fail(nullptr, DSG_E_DEVICE, "context creation failed");
  }
  *out = ctx;
  return DSG_OK;
}

extern "C" dsg_status dsg_ctx_destroy(dsg_ctx* ctx) {
  if (!ctx) return fail(nullptr, DSG_E_ARG, "ctx is NULL");
  Ctx& c = ctx->c;
  if (c.objects > 0) return fail(ctx, DSG_E_STATE, "context still owns matrices or products");
  (void)hipSetDevice(c.device);
  (void)hipStreamSynchronize(c.stream);
  clear_timings(&c);
  for (hipEvent_t e : c.event_pool) (void)hipEventDestroy(e);
  c.event_pool.clear();
  ctx_free(&c, c.scratch, c.scratch_bytes);
  ctx_free(&c, c.scratch2, c.scratch2_bytes);
  if (c.pinned) (void)hipHostFree(c.pinned);
  if (c.side) {
    (void)hipStreamSynchronize(c.side);
    (void)hipStreamDestroy(c.side);
  }
  if (c.fork_ev) (void)hipEventDestroy(c.fork_ev);
  if (c.join_ev) (void)hipEventDestroy(c.join_ev);
  if (c.own_stream) (void)hipStreamDestroy(c.stream);
  delete ctx;
  return DSG_OK;
}

extern "C" dsg_status dsg_ctx_set_allocator(dsg_ctx* ctx, const dsg_allocator* a) {
  if (!ctx) return fail(nullptr, DSG_E_ARG, "ctx is NULL");
  if (a && (!a->alloc || !a->free)) return fail(ctx, DSG_E_ARG, "allocator without alloc or free");
  std::lock_guard<std::mutex> lk(ctx->c.alloc_mu);
  if (ctx->c.held > 0) return fail(ctx, DSG_E_STATE, "the context already holds device memory");
  if (a) ctx->c.allocator = *a;
  else ctx->c.allocator = dsg_allocator{};
  return DSG_OK;
}

extern "C" const char* dsg_last_error(const dsg_ctx* ctx) {
  return ctx ? ctx->c.last_error.c_str() : g_create_error.c_str();
}

extern "C" dsg_status dsg_ctx_synchronize(dsg_ctx* ctx) {
  if (!ctx) return fail(nullptr, DSG_E_ARG, "ctx is NULL");
  API_BEGIN(ctx)
  set_device(ctx);
  ctx_sync(&ctx->c);
  API_END
}

extern "C" dsg_status dsg_ctx_memory(const dsg_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return fail(const_cast<dsg_ctx*>(ctx), DSG_E_ARG, "NULL argument");
  *bytes = ctx->c.held;
  return DSG_OK;
}

extern "C" dsg_status dsg_ctx_set_timing(dsg_ctx* ctx, int on) {
  if (!ctx) return fail(nullptr, DSG_E_ARG, "ctx is NULL");
  API_BEGIN(ctx)
  set_device(ctx);
  ctx_sync(&ctx->c);
  clear_timings(&ctx->c);
  ctx->c.timing = on != 0;
  // enough events for many timed calls (more are created when these run out)
  while (ctx->c.timing && ctx->c.event_pool.size() < 1024) {
    hipEvent_t e;
    DSG_HIP(hipEventCreate(&e));
    ctx->c.event_pool.push_back(e);
  }
  API_END
}

extern "C" dsg_status dsg_ctx_set_timing_phase(dsg_ctx* ctx, const char* phase) {
  if (!ctx) return fail(nullptr, DSG_E_ARG, "ctx is NULL");
  API_BEGIN(ctx)
  ctx->c.timing_phase = phase ? phase : "";
  API_END
}

extern "C" dsg_status dsg_ctx_timing_report(dsg_ctx* ctx, char* buf, size_t cap) {
  if (!ctx || !buf || cap == 0) return fail(ctx, DSG_E_ARG, "NULL argument");
  API_BEGIN(ctx)
  set_device(ctx);
  ctx_sync(&ctx->c);
  struct Agg {
    long n = 0;
    double ms = 0, bytes = 0;
  };
  std::map<std::string, Agg> agg;
  for (auto& t : ctx->c.timings) {
    float ms = 0;
    DSG_HIP(hipEventElapsedTime(&ms, t.start, t.stop));
    Agg& a = agg[t.name];
    a.n++;
    a.ms += ms;
    a.bytes += t.bytes;
  }
  std::string s = "{\"kernels\": {";
  bool first = true;
  for (auto& kv : agg) {
    char tmp[256];
    snprintf(tmp, sizeof tmp, "%s\"%s\": {\"launches\": %ld, \"ms\": %.6f, \"bytes\": %.1f}", first ? "" : ", ",
             kv.first.c_str(), kv.second.n, kv.second.ms, kv.second.bytes);
    s += tmp;
    first = false;
  }
  s += "}}";
  size_t n = std::min(cap - 1, s.size());
  memcpy(buf, s.data(), n);
  buf[n] = 0;
  API_END
}

extern "C" dsg_status dsg_ctx_get_tuning(const dsg_ctx* ctx, dsg_tuning* t) {
  if (!ctx || !t) return fail(const_cast<dsg_ctx*>(ctx), DSG_E_ARG, "NULL argument");
  *t = ctx->c.tuning;
  return DSG_OK;
}

extern "C" dsg_status dsg_ctx_set_tuning(dsg_ctx* ctx, const dsg_tuning* t) {
  if (!ctx) return fail(nullptr, DSG_E_ARG, "ctx is NULL");
  if (!t) {
    default_tuning(&ctx->c.tuning);
    return DSG_OK;
  }
  int prev = 0;
  for (int b = 0; b < 8; ++b) {
    if (t->group_ub[b] < 0 || t->group_ub[b] > (32 << b))
      return fail(ctx, DSG_E_ARG, "group_ub[" + std::to_string(b) + "] outside [0, " + std::to_string(32 << b) + "]");
    if (t->group_ub[b] && t->group_ub[b] < prev) return fail(ctx, DSG_E_ARG, "group_ub must ascend");
    if (t->group_ub[b]) prev = t->group_ub[b];
  }
  if (t->dense_max_passes < 0) return fail(ctx, DSG_E_ARG, "dense_max_passes < 0");
  if (t->force_bin < -1 || t->force_bin > 9) return fail(ctx, DSG_E_ARG, "force_bin outside [-1, 9]");
  if (t->update_path < 0 || t->update_path > 2) return fail(ctx, DSG_E_ARG, "update_path outside [0, 2]");
  if (t->batch_direct_log2 < 0 || t->batch_direct_log2 > 62)
    return fail(ctx, DSG_E_ARG, "batch_direct_log2 outside [0, 62]");
  if (!(t->entry_fixed >= 0.0 && t->entry_fixed < 1e300) || !(t->entry_per_term >= 0.0 && t->entry_per_term < 1e300))
    return fail(ctx, DSG_E_ARG, "entry_fixed and entry_per_term must be finite and >= 0");
  if (t->row_index != 0 && t->row_index != 1) return fail(ctx, DSG_E_ARG, "row_index must be 0 or 1");
  ctx->c.tuning = *t;
  return DSG_OK;
}

// ---------------------------------------------------------------------------
// matrices
// ---------------------------------------------------------------------------

extern "C" dsg_status dsg_mat_create(dsg_ctx* ctx, int32_t nrows, int32_t ncols, dsg_semiring sr,
                                     const int64_t* row_ptr, const int32_t* col, const void* val, uint32_t flags,
                                     dsg_mat** out) {
  if (!ctx) return fail(nullptr, DSG_E_ARG, "ctx is NULL");
  if (!out) return fail(ctx, DSG_E_ARG, "out is NULL");
  *out = nullptr;
  if (nrows < 0 || ncols < 0) return fail(ctx, DSG_E_ARG, "negative shape");
  if (sr < DSG_PLUS_TIMES_I64 || sr > DSG_OR_AND_U32) return fail(ctx, DSG_E_ARG, "unknown semiring");
  if (flags & ~(uint32_t)(DSG_INPUT_DEVICE | DSG_SYNC)) return fail(ctx, DSG_E_ARG, "unknown flag");
  API_BEGIN(ctx)
  set_device(ctx);
  Ctx* c = &ctx->c;
  const int vs = value_size(sr);
  DevArray drp, dci, dv;
  std::vector<int64_t> hrp;
  std::vector<int32_t> hci;
  std::vector<char> hv;
  const int64_t* rp_h = row_ptr;
  const int32_t* ci_h = col;
  if (row_ptr) {
    if (flags & DSG_INPUT_DEVICE) {
      hrp.resize((size_t)nrows + 1);
      DSG_HIP(hipMemcpy(hrp.data(), row_ptr, hrp.size() * 8, hipMemcpyDeviceToHost));
      rp_h = hrp.data();
    }
    int64_t nnz = rp_h[nrows];
    if (nnz < 0) throw DsgError{DSG_E_ARG, "negative nnz"};
    if (nnz > 0 && (!col || !val)) throw DsgError{DSG_E_ARG, "col/val NULL with nnz > 0"};
    if (flags & DSG_INPUT_DEVICE) {
      hci.resize((size_t)nnz);
      if (nnz) DSG_HIP(hipMemcpy(hci.data(), col, (size_t)nnz * 4, hipMemcpyDeviceToHost));
      ci_h = hci.data();
    }
    std::string msg;
    dsg_status st = check_csr(nrows, ncols, rp_h, ci_h, msg);
    if (st != DSG_OK) throw DsgError{st, msg};
    if (flags & DSG_INPUT_DEVICE) {
      drp.device(row_ptr);
      dci.device(col);
      dv.device(val);
    } else {
      drp.host(c, row_ptr, ((size_t)nrows + 1) * 8);
      dci.host(c, col, (size_t)nnz * 4);
      dv.host(c, val, (size_t)nnz * vs);
    }
  }
  DMat* m = mat_create(c, nrows, ncols, (int)sr, row_ptr ? (const int64_t*)drp.p : nullptr,
                       (const int32_t*)dci.p, dv.p);
  ctx_sync(c);
  *out = new dsg_mat{m, ctx, true};
  API_END
}

extern "C" dsg_status dsg_mat_apply(dsg_mat* mh, const int32_t* rows, const int32_t* cols, const void* vals,
                                    const uint8_t* ops, int64_t n, uint32_t flags) {
  if (!mh || !mh->alive) return fail(nullptr, DSG_E_ARG, "matrix is NULL or destroyed");
  dsg_ctx* ctx = mh->owner;
  if (n < 0) return fail(ctx, DSG_E_ARG, "negative batch size");
  if (n > 0 && (!rows || !cols || !vals || !ops)) return fail(ctx, DSG_E_ARG, "NULL batch array");
  if (n > (int64_t)0x7fffffff) return fail(ctx, DSG_E_ARG, "batch larger than 2^31-1");
  if (flags & ~(uint32_t)(DSG_INPUT_DEVICE | DSG_SYNC)) return fail(ctx, DSG_E_ARG, "unknown flag");
  API_BEGIN(ctx)
  set_device(ctx);
  DMat* m = mh->m;
  Ctx* c = &ctx->c;
  if (n == 0) return DSG_OK;
  DevArray dr, dcol, dval, dop;
  if (flags & DSG_INPUT_DEVICE) {
    dsg_status st = validate_batch_device(m, rows, cols, ops, n);
    if (st == DSG_E_RANGE) throw DsgError{st, "update index out of range"};
    if (st != DSG_OK) throw DsgError{st, "unknown update op code"};
    dr.device(rows);
    dcol.device(cols);
    dval.device(vals);
    dop.device(ops);
  } else {
    for (int64_t t = 0; t < n; ++t) {
      if (rows[t] < 0 || rows[t] >= m->nrows || cols[t] < 0 || cols[t] >= m->ncols)
        throw DsgError{DSG_E_RANGE, "update " + std::to_string(t) + " index out of range"};
      if (ops[t] > DSG_OP_ADD) throw DsgError{DSG_E_ARG, "update " + std::to_string(t) + " unknown op"};
    }
    dr.host(c, rows, (size_t)n * 4);
    dcol.host(c, cols, (size_t)n * 4);
    dval.host(c, vals, (size_t)n * value_size(m->sr));
    dop.host(c, ops, (size_t)n);
  }
  mat_apply_device(m, (const int32_t*)dr.p, (const int32_t*)dcol.p, dval.p, (const uint8_t*)dop.p, n);
  if ((flags & DSG_SYNC) || !(flags & DSG_INPUT_DEVICE)) ctx_sync(c);
  API_END
}

extern "C" dsg_status dsg_mat_nnz(dsg_mat* mh, int64_t* nnz) {
  if (!mh || !mh->alive || !nnz) return fail(mh ? mh->owner : nullptr, DSG_E_ARG, "NULL argument");
  API_BEGIN(mh->owner)
  set_device(ctx__);
  *nnz = mat_nnz(mh->m);
  API_END
}

extern "C" dsg_status dsg_mat_shape(const dsg_mat* mh, int32_t* nrows, int32_t* ncols, dsg_semiring* sr) {
  if (!mh || !mh->alive) return fail(nullptr, DSG_E_ARG, "matrix is NULL or destroyed");
  if (nrows) *nrows = mh->m->nrows;
  if (ncols) *ncols = mh->m->ncols;
  if (sr) *sr = (dsg_semiring)mh->m->sr;
  return DSG_OK;
}

static void export_impl(DMat* m, int64_t* row_ptr, int32_t* col, void* val, int64_t cap, int64_t* nnz_out) {
  Ctx* c = m->ctx;
  const int32_t n = m->nrows;
  DevArray drp;
  drp.c = c;
  drp.bytes = ((size_t)n + 1) * 8;
  drp.p = ctx_alloc(c, drp.bytes);
  drp.owned = true;
  mat_export_device(m, (int64_t*)drp.p, nullptr, nullptr, nullptr, c->stream);
  int64_t nnz = 0;
  DSG_HIP(hipMemcpy(&nnz, (int64_t*)drp.p + n, 8, hipMemcpyDeviceToHost));
  *nnz_out = nnz;
  if (row_ptr) DSG_HIP(hipMemcpy(row_ptr, drp.p, drp.bytes, hipMemcpyDeviceToHost));
  if (!col) return;
  if (cap < nnz) throw DsgError{DSG_E_ARG, "capacity " + std::to_string(cap) + " < nnz " + std::to_string(nnz)};
  if (nnz == 0) return;
  const int vs = m->vsz ? m->vsz : 4;
  DevArray dc, dv;
  dc.c = dv.c = c;
  dc.bytes = (size_t)nnz * 4;
  dv.bytes = (size_t)nnz * vs;
  dc.p = ctx_alloc(c, dc.bytes);
  dc.owned = true;
  dv.p = ctx_alloc(c, dv.bytes);
  dv.owned = true;
  mat_export_device(m, (int64_t*)drp.p, (int32_t*)dc.p, dv.p, nullptr, c->stream);
  ctx_sync(c);
  DSG_HIP(hipMemcpy(col, dc.p, dc.bytes, hipMemcpyDeviceToHost));
  if (val && m->vsz) DSG_HIP(hipMemcpy(val, dv.p, dv.bytes, hipMemcpyDeviceToHost));
}

extern "C" dsg_status dsg_mat_export(dsg_mat* mh, int64_t* row_ptr, int32_t* col, void* val, int64_t cap,
                                     int64_t* nnz_out) {
  if (!mh || !mh->alive || !nnz_out) return fail(mh ? mh->owner : nullptr, DSG_E_ARG, "NULL argument");
  if (col && !val) return fail(mh->owner, DSG_E_ARG, "val is NULL");
  API_BEGIN(mh->owner)
  set_device(ctx__);
  export_impl(mh->m, row_ptr, col, val, cap, nnz_out);
  API_END
}

extern "C" dsg_status dsg_mat_destroy(dsg_mat* mh) {
  if (!mh || !mh->alive) return fail(nullptr, DSG_E_ARG, "matrix is NULL or destroyed");
  dsg_ctx* ctx = mh->owner;
  if (mh->m->refs > 0) return fail(ctx, DSG_E_STATE, "matrix is used by a product");
  API_BEGIN(ctx)
  set_device(ctx);
  ctx_sync(&ctx->c);
  mat_destroy(mh->m);
  mh->m = nullptr;
  mh->alive = false;
  delete mh;
  API_END
}

// ---------------------------------------------------------------------------
// products
// ---------------------------------------------------------------------------

static void fill_rows(DProd* p, const int32_t* rows, int32_t n, dsg_rows* out) {
  out->n = n;
  out->rows = rows;
  out->row_off = p->C->row_off;
  out->row_len = p->C->row_len;
  out->col = p->C->col;
  out->val = p->C->val;
}

extern "C" dsg_status dsg_prod_create(dsg_ctx* ctx, dsg_mat* A, dsg_mat* B, uint32_t ops, dsg_prod** out) {
  if (!ctx) return fail(nullptr, DSG_E_ARG, "ctx is NULL");
  if (!out || !A || !B || !A->alive || !B->alive) return fail(ctx, DSG_E_ARG, "NULL or destroyed argument");
  *out = nullptr;
  if (ops & ~(uint32_t)(DSG_TRANS_A | DSG_TRANS_B | DSG_GENERAL_BLOOM)) return fail(ctx, DSG_E_ARG, "unknown operand flag");
  if (A->owner != ctx || B->owner != ctx) return fail(ctx, DSG_E_STATE, "operands belong to another context");
  if (A->m->sr != B->m->sr) return fail(ctx, DSG_E_STATE, "semiring mismatch");
  const int32_t inner_a = (ops & DSG_TRANS_A) ? A->m->nrows : A->m->ncols;
  const int32_t inner_b = (ops & DSG_TRANS_B) ? B->m->ncols : B->m->nrows;
  if (inner_a != inner_b) return fail(ctx, DSG_E_STATE, "shape mismatch: inner dimensions of op(A) and op(B) differ");
  API_BEGIN(ctx)
  set_device(ctx);
  DProd* p = prod_create(&ctx->c, A->m, B->m, ops);
  *out = new dsg_prod{p, ctx, A, B};
  API_END
}

extern "C" dsg_status dsg_prod_create_static(dsg_ctx* ctx, dsg_mat* A, dsg_mat* B, dsg_prod** out) {
  return dsg_prod_create(ctx, A, B, 0, out);
}

extern "C" dsg_status dsg_prod_scale_add(dsg_prod* ph, const void* alpha, dsg_mat* X, const void* beta,
                                         dsg_mat** out) {
  if (!ph) return fail(nullptr, DSG_E_ARG, "product is NULL");
  dsg_ctx* ctx = ph->owner;
  if (!out || !alpha || (X && !beta)) return fail(ctx, DSG_E_ARG, "NULL argument");
  *out = nullptr;
  const DMat* C = ph->p->C;
  if (X) {
    if (!X->alive) return fail(ctx, DSG_E_ARG, "X is destroyed");
    if (X->owner != ctx) return fail(ctx, DSG_E_STATE, "X belongs to another context");
    if (X->m->sr != C->sr) return fail(ctx, DSG_E_STATE, "semiring mismatch");
    if (X->m->nrows != C->nrows || X->m->ncols != C->ncols) return fail(ctx, DSG_E_STATE, "shape of X differs from C");
  }
  API_BEGIN(ctx)
  set_device(ctx);
  DMat* d = prod_scale_add(ph->p, alpha, X ? X->m : nullptr, beta);
  *out = new dsg_mat{d, ctx, true};
  API_END
}

extern "C" dsg_status dsg_prod_recompute_static(dsg_prod* ph, uint32_t flags) {
  if (!ph) return fail(nullptr, DSG_E_ARG, "product is NULL");
  if (flags & ~(uint32_t)DSG_SYNC) return fail(ph->owner, DSG_E_ARG, "unknown flag");
  API_BEGIN(ph->owner)
  set_device(ctx__);
  prod_run(ph->p, 1, true);
  API_END
}

extern "C" dsg_status dsg_prod_update(dsg_prod* ph, uint32_t flags, dsg_rows* changed) {
  if (!ph) return fail(nullptr, DSG_E_ARG, "product is NULL");
  if (flags & ~(uint32_t)(DSG_SYNC | DSG_REPORT_AFFECTED)) return fail(ph->owner, DSG_E_ARG, "unknown flag");
  API_BEGIN(ph->owner)
  set_device(ctx__);
  int32_t n = prod_run(ph->p, 0, (flags & DSG_REPORT_AFFECTED) != 0);
  if (changed) fill_rows(ph->p, ph->p->changed_rows, n, changed);
  API_END
}

__global__ static void k_check_rows(const int32_t* rows, int32_t n, int32_t nrows, int* bad) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n && (rows[t] < 0 || rows[t] >= nrows)) atomicOr(bad, 1);
}

extern "C" dsg_status dsg_prod_rows(dsg_prod* ph, const int32_t* rows, int32_t nq, uint32_t flags,
                                    dsg_rows* out) {
  if (!ph || !out) return fail(ph ? ph->owner : nullptr, DSG_E_ARG, "NULL argument");
  if (nq < 0 || (nq > 0 && !rows)) return fail(ph->owner, DSG_E_ARG, "bad row list");
  if (flags & ~(uint32_t)(DSG_INPUT_DEVICE | DSG_SYNC)) return fail(ph->owner, DSG_E_ARG, "unknown flag");
  API_BEGIN(ph->owner)
  set_device(ctx__);
  DProd* p = ph->p;
  Ctx* c = p->ctx;
  const int32_t nrows = p->C->nrows;
  if (nq > p->query_cap) {
    if (p->query_rows) ctx_free(c, p->query_rows, (size_t)p->query_cap * 4);
    p->query_rows = nullptr;
    p->query_cap = 0;
    int64_t cap = std::max<int64_t>(nq, 1024);
    p->query_rows = (int32_t*)ctx_alloc(c, (size_t)cap * 4);
    p->query_cap = cap;
  }
  if (flags & DSG_INPUT_DEVICE) {
    if (nq > 0) {
      int* bad = (int*)ctx_scratch(c, 64);
      DSG_HIP(hipMemsetAsync(bad, 0, 4, c->stream));
      hipLaunchKernelGGL(k_check_rows, dim3((nq + 255) / 256), dim3(256), 0, c->stream, rows, nq, nrows, bad);
      int* h = (int*)c->pinned;
      DSG_HIP(hipMemcpyAsync(h, bad, 4, hipMemcpyDeviceToHost, c->stream));
      DSG_HIP(hipStreamSynchronize(c->stream));
      if (h[0]) throw DsgError{DSG_E_RANGE, "row index out of range"};
      DSG_HIP(hipMemcpyAsync(p->query_rows, rows, (size_t)nq * 4, hipMemcpyDeviceToDevice, c->stream));
    }
  } else {
    for (int32_t t = 0; t < nq; ++t)
      if (rows[t] < 0 || rows[t] >= nrows) throw DsgError{DSG_E_RANGE, "row index out of range"};
    if (nq > 0) DSG_HIP(hipMemcpyAsync(p->query_rows, rows, (size_t)nq * 4, hipMemcpyHostToDevice, c->stream));
  }
  if (flags & DSG_SYNC || !(flags & DSG_INPUT_DEVICE)) ctx_sync(c);
  fill_rows(p, p->query_rows, nq, out);
  API_END
}

extern "C" dsg_status dsg_rows_export(dsg_prod* ph, const dsg_rows* v, int64_t* row_ptr, int32_t* col,
                                      void* val, int64_t cap, int64_t* nnz_out) {
  if (!ph || !v || !nnz_out) return fail(ph ? ph->owner : nullptr, DSG_E_ARG, "NULL argument");
  if (col && !val) return fail(ph->owner, DSG_E_ARG, "val is NULL");
  if (v->n < 0 || (v->n > 0 && !v->rows)) return fail(ph->owner, DSG_E_ARG, "bad view");
  API_BEGIN(ph->owner)
  set_device(ctx__);
  DProd* p = ph->p;
  Ctx* c = p->ctx;
  GatherBufs g;
  RowsHost h;
  try {
    mat_gather_rows(p->C, v->rows, v->n, g, h, c->stream, col != nullptr);
  } catch (...) {
    gather_bufs_free(c, g);
    throw;
  }
  gather_bufs_free(c, g);
  const int64_t nnz = h.row_ptr[(size_t)v->n];
  *nnz_out = nnz;
  if (row_ptr) memcpy(row_ptr, h.row_ptr.data(), h.row_ptr.size() * 8);
  if (!col) return DSG_OK;
  if (cap < nnz) throw DsgError{DSG_E_ARG, "capacity < nnz"};
  if (nnz == 0) return DSG_OK;
  memcpy(col, h.col.data(), (size_t)nnz * 4);
  memcpy(val, h.val.data(), h.val.size());
  API_END
}

extern "C" dsg_status dsg_rows_export_noalloc(dsg_prod* ph, const dsg_rows* v, int64_t* row_ptr, int32_t* col,
                                              void* val, int64_t cap, int64_t* nnz_out) {
  if (!ph || !v || !nnz_out) return fail(ph ? ph->owner : nullptr, DSG_E_ARG, "NULL argument");
  if (col && (!val || !row_ptr)) return fail(ph->owner, DSG_E_ARG, "val or row_ptr is NULL");
  if (v->n < 0 || (v->n > 0 && !v->rows)) return fail(ph->owner, DSG_E_ARG, "bad view");
  API_BEGIN(ph->owner)
  set_device(ctx__);
  *nnz_out = rows_export_noalloc(ph->p->C, v->rows, v->n, row_ptr, col, val, cap);
  API_END
}

extern "C" dsg_status dsg_prod_nnz(dsg_prod* ph, int64_t* nnz) {
  if (!ph || !nnz) return fail(ph ? ph->owner : nullptr, DSG_E_ARG, "NULL argument");
  API_BEGIN(ph->owner)
  set_device(ctx__);
  *nnz = mat_nnz(ph->p->C);
  API_END
}

extern "C" dsg_status dsg_prod_export(dsg_prod* ph, int64_t* row_ptr, int32_t* col, void* val, int64_t cap,
                                      int64_t* nnz_out) {
  if (!ph || !nnz_out) return fail(ph ? ph->owner : nullptr, DSG_E_ARG, "NULL argument");
  if (col && !val) return fail(ph->owner, DSG_E_ARG, "val is NULL");
  API_BEGIN(ph->owner)
  set_device(ctx__);
  export_impl(ph->p->C, row_ptr, col, val, cap, nnz_out);
  API_END
}

extern "C" dsg_status dsg_prod_export_bloom(dsg_prod* ph, int64_t* row_ptr, int32_t* col, uint64_t* val, int64_t cap,
                                            int64_t* nnz_out) {
  if (!ph || !nnz_out) return fail(ph ? ph->owner : nullptr, DSG_E_ARG, "NULL argument");
  if (col && !val) return fail(ph->owner, DSG_E_ARG, "val is NULL");
  if (!ph->p->F) return fail(ph->owner, DSG_E_STATE, "product keeps no Bloom matrix");
  API_BEGIN(ph->owner)
  set_device(ctx__);
  export_impl(ph->p->F, row_ptr, col, val, cap, nnz_out);
  API_END
}

extern "C" dsg_status dsg_prod_stats(const dsg_prod* ph, dsg_update_stats* s) {
  if (!ph || !s) return fail(ph ? ph->owner : nullptr, DSG_E_ARG, "NULL argument");
  *s = ph->p->stats;
  return DSG_OK;
}

// Candidate tunings: bin thresholds at full or half capacity, small bins on
// or off, and the pass limit of the dense accumulator.
static std::vector<dsg_tuning> tuning_candidates() {
  std::vector<dsg_tuning> out;
  for (int half = 0; half < 2; ++half)
    for (int skip_small = 0; skip_small < 2; ++skip_small)
      for (int passes : {1, 2, 4, 8}) {
        dsg_tuning t;
        default_tuning(&t);
        for (int b = 0; b < 8; ++b) t.group_ub[b] = half ? (16 << b) : (32 << b);
        if (skip_small) t.group_ub[0] = t.group_ub[1] = 0;
        t.dense_max_passes = passes;
        t.force_bin = -1;
        t.update_path = 0;
        out.push_back(t);
      }
  return out;
}

extern "C" dsg_status dsg_prod_autotune(dsg_prod* ph, int32_t reps, dsg_tuning* best, double* best_ms,
                                        char* report, size_t cap) {
  if (!ph || !best || !best_ms) return fail(ph ? ph->owner : nullptr, DSG_E_ARG, "NULL argument");
  if (reps < 1 || reps > 100) return fail(ph->owner, DSG_E_ARG, "reps outside [1, 100]");
  API_BEGIN(ph->owner)
  set_device(ctx__);
  Ctx* c = &ctx__->c;
  const dsg_tuning saved = c->tuning;
  hipEvent_t e0, e1;
  DSG_HIP(hipEventCreate(&e0));
  DSG_HIP(hipEventCreate(&e1));
  std::string js = "[";
  double best_t = 1e300;
  dsg_tuning best_tu = saved;
  const bool timing = c->timing;
  c->timing = false;
  try {
    for (dsg_tuning t : tuning_candidates()) {
      // the trials vary the row kernels only; the path choice stays as set
      t.update_path = saved.update_path;
      t.entry_fixed = saved.entry_fixed;
      t.entry_per_term = saved.entry_per_term;
      t.row_index = saved.row_index;
      c->tuning = t;
      prod_run(ph->p, 1, true);  // warm: sizes the pools and the arena for this setting
      std::vector<float> ms;
      for (int r = 0; r < reps; ++r) {
        DSG_HIP(hipEventRecord(e0, c->stream));
        prod_run(ph->p, 1, true);
        DSG_HIP(hipEventRecord(e1, c->stream));
        DSG_HIP(hipEventSynchronize(e1));
        float x = 0;
        DSG_HIP(hipEventElapsedTime(&x, e0, e1));
        ms.push_back(x);
      }
      std::sort(ms.begin(), ms.end());
      const double med = ms[ms.size() / 2];
      char tmp[256];
      snprintf(tmp, sizeof tmp, "%s{\"group_ub\": [%d,%d,%d,%d,%d,%d,%d,%d], \"dense_max_passes\": %d, \"ms\": %.4f}",
               js.size() > 1 ? ", " : "", t.group_ub[0], t.group_ub[1], t.group_ub[2], t.group_ub[3],
               t.group_ub[4], t.group_ub[5], t.group_ub[6], t.group_ub[7], t.dense_max_passes, med);
      js += tmp;
      if (med < best_t) {
        best_t = med;
        best_tu = t;
      }
    }
  } catch (...) {
    c->tuning = saved;
    c->timing = timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  js += "]";
  c->timing = timing;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->tuning = best_tu;
  *best = best_tu;
  *best_ms = best_t;
  if (report && cap) {
    size_t n = std::min(cap - 1, js.size());
    memcpy(report, js.data(), n);
    report[n] = 0;
  }
  API_END
}

struct dsg_batch {
  DBatch* b;
  dsg_ctx* owner;
  std::vector<dsg_prod*> prods;
  std::vector<int32_t> counts;
};

extern "C" dsg_status dsg_batch_create(dsg_ctx* ctx, dsg_prod* const* prods, int32_t nprod, dsg_batch** out) {
  if (!ctx) return fail(nullptr, DSG_E_ARG, "ctx is NULL");
  if (!out || (nprod > 0 && !prods) || nprod < 0) return fail(ctx, DSG_E_ARG, "bad arguments");
  *out = nullptr;
  // Every matrix belongs to one product only: a product may name one matrix
  // twice (C = A A), but no matrix -- and so no product -- may appear in two
  // entries of the list, since each matrix takes its updates inside its own
  // product's chain.
  std::vector<DMat*> seen;
  for (int32_t i = 0; i < nprod; ++i) {
    if (!prods[i] || prods[i]->owner != ctx) return fail(ctx, DSG_E_STATE, "product of another context");
    DMat* mine[2] = {prods[i]->p->src_a, prods[i]->p->src_b};
    for (DMat* m : mine)
      if (std::find(seen.begin(), seen.end(), m) != seen.end())
        return fail(ctx, DSG_E_STATE, "products of a batch must not share operands");
    seen.push_back(mine[0]);
    if (mine[1] != mine[0]) seen.push_back(mine[1]);
  }
  API_BEGIN(ctx)
  set_device(ctx);
  std::vector<DProd*> ps;
  for (int32_t i = 0; i < nprod; ++i) ps.push_back(prods[i]->p);
  DBatch* b = batch_create(&ctx->c, ps);
  dsg_batch* h = new dsg_batch();
  h->b = b;
  h->owner = ctx;
  h->prods.assign(prods, prods + nprod);
  h->counts.assign((size_t)nprod, 0);
  *out = h;
  API_END
}

extern "C" dsg_status dsg_batch_run(dsg_batch* bh, const dsg_update_set* sets, int32_t nsets, uint32_t flags,
                                    int32_t* changed_counts) {
  if (!bh) return fail(nullptr, DSG_E_ARG, "batch is NULL");
  if (nsets < 0 || (nsets > 0 && !sets)) return fail(bh->owner, DSG_E_ARG, "bad set list");
  if (flags & ~(uint32_t)DSG_SYNC) return fail(bh->owner, DSG_E_ARG, "unknown flag");
  std::vector<DBatchSet> ss;
  for (int32_t k = 0; k < nsets; ++k) {
    const dsg_update_set& s = sets[k];
    if (!s.mat || !s.mat->alive || s.mat->owner != bh->owner) return fail(bh->owner, DSG_E_ARG, "bad matrix in set");
    if (s.n < 0 || (s.n > 0 && (!s.rows || !s.cols || !s.vals || !s.ops)))
      return fail(bh->owner, DSG_E_ARG, "bad set arrays");
    ss.push_back(DBatchSet{s.mat->m, s.rows, s.cols, s.vals, s.ops, s.n});
  }
  API_BEGIN(bh->owner)
  set_device(ctx__);
  dsg_status st = batch_run(bh->b, ss, bh->counts);
  if (st == DSG_E_RANGE) throw DsgError{st, "update index out of range in a set"};
  if (st != DSG_OK) throw DsgError{st, "unknown update op code in a set"};
  if (changed_counts)
    for (size_t j = 0; j < bh->counts.size(); ++j) changed_counts[j] = bh->counts[j];
  API_END
}

extern "C" dsg_status dsg_batch_rows(dsg_batch* bh, int32_t i, dsg_rows* out) {
  if (!bh || !out) return fail(bh ? bh->owner : nullptr, DSG_E_ARG, "NULL argument");
  if (i < 0 || i >= (int32_t)bh->prods.size()) return fail(bh->owner, DSG_E_ARG, "product index out of range");
  DProd* p = batch_prod(bh->b, i);
  fill_rows(p, p->changed_rows, bh->counts[(size_t)i], out);
  return DSG_OK;
}

extern "C" dsg_status dsg_batch_info(const dsg_batch* bh, dsg_batch_stats* out) {
  if (!bh || !out) return fail(nullptr, DSG_E_ARG, "batch or output is NULL");
  batch_info(bh->b, out);
  return DSG_OK;
}

extern "C" dsg_status dsg_batch_destroy(dsg_batch* bh) {
  if (!bh) return fail(nullptr, DSG_E_ARG, "batch is NULL");
  API_BEGIN(bh->owner)
  set_device(ctx__);
  batch_destroy(bh->b);
  delete bh;
  API_END
}

extern "C" dsg_status dsg_prod_destroy(dsg_prod* ph) {
  if (!ph) return fail(nullptr, DSG_E_ARG, "product is NULL");
  if (ph->p->refs > 0) return fail(ph->owner, DSG_E_STATE, "product is used by a batched executor or server");
  API_BEGIN(ph->owner)
  set_device(ctx__);
  ctx_sync(&ctx__->c);
  prod_destroy(ph->p);
  delete ph;
  API_END
}

// ---------------------------------------------------------------------------
// served form
// ---------------------------------------------------------------------------

struct dsg_server {
  DServer* s;
  dsg_ctx* owner;
  dsg_prod* prod;
};

// Server calls may come from several client threads: their failures go to the
// calling thread's message (dsg_last_error(NULL)), not to the context.
#define SERVER_BEGIN(sh)                                        \
  if (!(sh)) return fail(nullptr, DSG_E_ARG, "server is NULL"); \
  dsg_ctx* ctx__ = nullptr;                                     \
  try {

extern "C" dsg_status dsg_server_create(dsg_ctx* ctx, dsg_prod* ph, const dsg_server_cfg* cfg, dsg_server** out) {
  if (!ctx) return fail(nullptr, DSG_E_ARG, "ctx is NULL");
  if (!ph || !out) return fail(ctx, DSG_E_ARG, "NULL argument");
  if (ph->owner != ctx) return fail(ctx, DSG_E_STATE, "product of another context");
  if (cfg && (cfg->slots < 0 || cfg->slots > 8)) return fail(ctx, DSG_E_ARG, "slots must be 0..8");
  *out = nullptr;
  API_BEGIN(ctx)
  set_device(ctx);
  if (ph->p->refs > 0) throw DsgError{DSG_E_STATE, "product is used by a batched executor or server"};
  DServer* s = server_create(&ctx->c, ph->p, cfg);
  dsg_server* h = new dsg_server();
  h->s = s;
  h->owner = ctx;
  h->prod = ph;
  ctx->c.served = true;
  *out = h;
  API_END
}

extern "C" dsg_status dsg_server_submit_update(dsg_server* sh, dsg_mat* mh, const int32_t* rows, const int32_t* cols,
                                               const void* vals, const uint8_t* ops, int64_t n, uint64_t* ticket) {
  SERVER_BEGIN(sh)
  if (!mh || !ticket || n < 0 || (n > 0 && (!rows || !cols || !ops || (mh->m->vsz && !vals))))
    throw DsgError{DSG_E_ARG, "bad arguments"};
  *ticket = server_submit_update(sh->s, mh->m, rows, cols, vals, ops, n);
  API_END
}

extern "C" dsg_status dsg_server_submit_query(dsg_server* sh, const int32_t* rows, int32_t nq, uint64_t* ticket) {
  SERVER_BEGIN(sh)
  if (!ticket || nq < 0 || (nq > 0 && !rows)) throw DsgError{DSG_E_ARG, "bad arguments"};
  *ticket = server_submit_query(sh->s, rows, nq);
  API_END
}

extern "C" dsg_status dsg_server_poll(dsg_server* sh, uint64_t ticket, int32_t wait, dsg_server_result* out) {
  SERVER_BEGIN(sh)
  if (!out) throw DsgError{DSG_E_ARG, "out is NULL"};
  server_poll(sh->s, ticket, wait != 0, out);
  API_END
}

extern "C" dsg_status dsg_server_query_result(dsg_server* sh, uint64_t ticket, int64_t* row_ptr, int32_t* col,
                                              void* val, int64_t cap, int64_t* nnz_out) {
  SERVER_BEGIN(sh)
  if (!nnz_out || (col && !val)) throw DsgError{DSG_E_ARG, "bad arguments"};
  server_query_result(sh->s, ticket, row_ptr, col, val, cap, nnz_out);
  API_END
}

extern "C" dsg_status dsg_server_release(dsg_server* sh, uint64_t ticket) {
  SERVER_BEGIN(sh)
  server_release(sh->s, ticket);
  API_END
}

extern "C" dsg_status dsg_server_drain(dsg_server* sh) {
  SERVER_BEGIN(sh)
  server_drain(sh->s);
  API_END
}

extern "C" dsg_status dsg_server_stats_get(dsg_server* sh, dsg_server_stats* out) {
  SERVER_BEGIN(sh)
  if (!out) throw DsgError{DSG_E_ARG, "out is NULL"};
  server_stats(sh->s, out);
  API_END
}

extern "C" dsg_status dsg_server_destroy(dsg_server* sh) {
  SERVER_BEGIN(sh)
  dsg_ctx* ctx = sh->owner;
  server_destroy(sh->s);
  ctx->c.served = false;
  delete sh;
  API_END
}
