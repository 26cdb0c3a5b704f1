// Per-row column index of a dynamic matrix (host side and the builders).
//
// The tables are described in rowindex.h.  A matrix gets an index on demand
// (the entry-granular product path asks for one on C and on A); every apply
// of a matrix with an index builds the missing tables of the rows it touches
// before planning, plans those rows by lookups instead of streaming them,
// and keeps the tables of the rows it changes (rowindex.h: which writers
// keep and which invalidate).
#include <algorithm>

#include "internal.h"
#include "kernel_common.h"

namespace {

unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

constexpr int32_t IX_LIGHT_MAX = 2048;  // longer rows are built by a whole workgroup
constexpr int IX_HEAVY_WG = 512;

__device__ inline int32_t table_size(int32_t len) { return 2 * len + 16; }

// one wavefront per listed row of at most IX_LIGHT_MAX entries without a
// usable table (rows taken in turn): take a table from the pool top, clear
// it, record every entry
// (b: the block's index among the nb blocks that build light rows)
__device__ inline void ix_build_light(const int64_t* row_off, const int32_t* row_len, const int32_t* col,
                                      const RowIx& X, const int32_t* rows, int64_t n, int fresh, int64_t b,
                                      int64_t nb) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (nb * blockDim.x) >> 6;
  for (int64_t r = (b * blockDim.x + threadIdx.x) >> 6; r < n; r += nw) {
    const int32_t i = rows ? rows[r] : (int32_t)r;
    if (!fresh && X.stamp[i] == X.gen) continue;
    const int32_t len = row_len[i];
    if (len > IX_LIGHT_MAX) continue;
    int32_t sz;
    unsigned long long base = 0;
    if (fresh) {
      sz = X.sz[i];
      base = (unsigned long long)X.off[i];
    } else {
      sz = table_size(len);
      if (lane == 0) base = atomicAdd(X.top, (unsigned long long)sz);
      base = __shfl(base, 0, 64);
    }
    if ((int64_t)base + sz > X.cap) continue;  // pool full: the row stays without a table
    uint64_t* t = X.tab + base;
    for (int32_t x = lane; x < sz; x += 64) t[x] = IX_EMPTY;
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    const int64_t off = row_off[i];
    for (int32_t p = lane; p < len; p += 64) ix_put(t, (uint32_t)sz, col[off + p], p);
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
      X.off[i] = (int64_t)base;
      X.sz[i] = sz;
      X.used[i] = len;
      X.stamp[i] = X.gen;
    }
  }
}

// the longer rows: one workgroup per row, rows taken in turn (b: the block's
// index among the nb blocks that build them)
__device__ inline void ix_build_heavy(const int64_t* row_off, const int32_t* row_len, const int32_t* col,
                                      const RowIx& X, const int32_t* rows, int64_t n, int fresh, int64_t b,
                                      int64_t nb) {
  __shared__ unsigned long long base_s;
  __shared__ int32_t wc[IX_HEAVY_WG / 64];
  __shared__ int32_t picked[IX_HEAVY_WG];
  const int tid = threadIdx.x;
  // this workgroup's share of the listed rows, scanned IX_HEAVY_WG at a time
  // by every thread at once; the long rows without a table are then built in
  // turn
  const int64_t per = (n + nb - 1) / nb;
  const int64_t rb = b * per, re = min(n, rb + per);
  for (int64_t c0 = rb; c0 < re; c0 += IX_HEAVY_WG) {
    int32_t npick;
    {
      const int64_t rr = c0 + tid;
      bool f = false;
      if (rr < re) {
        const int32_t ii = rows ? rows[rr] : (int32_t)rr;
        f = row_len[ii] > IX_LIGHT_MAX && (fresh || X.stamp[ii] != X.gen);
      }
      const int32_t q = block_flag_prefix<IX_HEAVY_WG>(f, wc, npick);
      if (f) picked[q] = rows ? rows[rr] : (int32_t)rr;
      __syncthreads();
    }
    for (int32_t pq = 0; pq < npick; ++pq) {
      const int32_t i = picked[pq];
      const int32_t len = row_len[i];
      int32_t sz;
      unsigned long long base;
      if (fresh) {
        sz = X.sz[i];
        base = (unsigned long long)X.off[i];
      } else {
        sz = table_size(len);
        if (tid == 0) base_s = atomicAdd(X.top, (unsigned long long)sz);
        __syncthreads();
        base = base_s;
        __syncthreads();
      }
      if ((int64_t)base + sz > X.cap) continue;
      uint64_t* t = X.tab + base;
      for (int32_t x = tid; x < sz; x += IX_HEAVY_WG) t[x] = IX_EMPTY;
      __threadfence_block();
      __syncthreads();
      const int64_t off = row_off[i];
      for (int32_t p = tid; p < len; p += IX_HEAVY_WG) ix_put(t, (uint32_t)sz, col[off + p], p);
      __threadfence_block();
      __syncthreads();
      if (tid == 0) {
        X.off[i] = (int64_t)base;
        X.sz[i] = sz;
        X.used[i] = len;
        X.stamp[i] = X.gen;
      }
    }
    __syncthreads();  // before the next share overwrites the picked rows
  }
}

// Tables of the listed rows (all rows when rows is null; their count on the
// device, or n_all) that have none: blocks [0, nl) take the short rows a
// wavefront each, the others the long rows a workgroup each.
__global__ __launch_bounds__(IX_HEAVY_WG) void k_ix_build(const int64_t* row_off, const int32_t* row_len,
                                                          const int32_t* col, RowIx X, const int32_t* rows,
                                                          const int64_t* d_n, int64_t n_all, int fresh, int64_t nl) {
  const int64_t n = d_n ? *d_n : n_all;
  const int64_t b = blockIdx.x;
  if (b < nl) ix_build_light(row_off, row_len, col, X, rows, n, fresh, b, nl);
  else ix_build_heavy(row_off, row_len, col, X, rows, n, fresh, b - nl, (int64_t)gridDim.x - nl);
}

// block counts of k_ix_build for n listed rows
void ix_build_grid(Ctx* c, int64_t n, int64_t& nl, int64_t& nh) {
  nl = std::max<int64_t>(1, std::min<int64_t>(blocks_for(n * 64, IX_HEAVY_WG), 8 * (int64_t)c->num_cus));
  nh = std::max<int64_t>(1, std::min<int64_t>(n, 2 * (int64_t)c->num_cus));
}

// table sizes of every row (a fresh build: offsets by a scan of these)
__global__ void k_ix_sizes(const int32_t* row_len, int32_t n, int32_t* sz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) sz[i] = table_size(row_len[i]);
}

__global__ void k_ix_set_top(unsigned long long* top, const int64_t* total) { *top = (unsigned long long)*total; }

__global__ void k_ix_zero_stamps(uint32_t* stamp, int32_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) stamp[i] = 0;
}

void free_index(DMat* m) {
  Ctx* c = m->ctx;
  const size_t n = (size_t)std::max<int32_t>(m->nrows, 1);
  ctx_free(c, m->ix_tab, (size_t)m->ix_cap * 8);
  c->ix_held -= std::min(c->ix_held, (size_t)m->ix_cap * 8);
  ctx_free(c, m->ix_off, n * 8);
  ctx_free(c, m->ix_sz, n * 4);
  ctx_free(c, m->ix_used, n * 4);
  ctx_free(c, m->ix_stamp, n * 4);
  ctx_free(c, m->ix_top, 64);
  m->ix_tab = nullptr;
  m->ix_off = nullptr;
  m->ix_sz = nullptr;
  m->ix_used = nullptr;
  m->ix_stamp = nullptr;
  m->ix_top = nullptr;
  m->ix_cap = 0;
}

}  // namespace

RowIx mat_index_view(const DMat* m) {
  RowIx X;
  if (!m->ix_tab) return X;
  X.tab = m->ix_tab;
  X.off = m->ix_off;
  X.sz = m->ix_sz;
  X.used = m->ix_used;
  X.stamp = m->ix_stamp;
  X.top = m->ix_top;
  X.cap = m->ix_cap;
  X.gen = m->ix_gen;
  return X;
}

namespace {

// Whether an index pool of `bytes` (replacing one of `old` bytes) may be
// taken: under a memory budget at most half of what is left; the pools of a
// context together at most 1/8 of the device; and of the device memory free
// now, a small pool (up to 1/256 of the device) at most half, a larger one
// at most a quarter of what lies beyond a reserve of a quarter of the
// device.  Indexes are an accelerator: they never crowd out the matrices,
// workspaces and exports.
bool room_for(Ctx* c, size_t bytes, size_t old) {
  if (c->budget && c->held - std::min(c->held, old) + 2 * bytes > c->budget) return false;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (c->ix_held - std::min(c->ix_held, old) + bytes > total_b / 8) return false;
  const size_t avail = free_b + old, reserve = total_b / 4;
  if (bytes <= total_b / 256) return bytes <= avail / 2;
  return avail > reserve && bytes <= (avail - reserve) / 4;
}

// Every row's table at once: sizes, offsets by a scan (no contended
// counter), a pool of 5/4 of their sum (grown if needed), then every row
// built.  Returns false when the pool cannot be had.
bool build_all(DMat* m) {
  Ctx* c = m->ctx;
  hipStream_t s = c->stream;
  const int32_t n = m->nrows;
  if (n == 0) return true;
  const size_t sb = scan_scratch_bytes(n) + 64;
  void* scr = ctx_alloc(c, sb);
  int64_t* d_total = (int64_t*)((char*)scr + scan_scratch_bytes(n));
  int64_t total = 0;
  try {
    hipLaunchKernelGGL(k_ix_sizes, dim3(blocks_for(n, 256)), dim3(256), 0, s, (const int32_t*)m->row_len, n,
                       m->ix_sz);
    exclusive_scan_i32_to_i64(m->ix_sz, m->ix_off, n, d_total, scr, s);
    hipLaunchKernelGGL(k_ix_set_top, dim3(1), dim3(1), 0, s, m->ix_top, (const int64_t*)d_total);
    int64_t* h = (int64_t*)c->pinned;
    DSG_HIP(hipMemcpyAsync(h, d_total, 8, hipMemcpyDeviceToHost, s));
    DSG_HIP(hipStreamSynchronize(s));
    total = *h;
  } catch (...) {
    ctx_free(c, scr, sb);
    throw;
  }
  ctx_free(c, scr, sb);
  // room for rebuilt tables until the pool is rebuilt as a whole
  const int64_t want = total + total / 4 + 65536;
  if (m->ix_cap < total + total / 8) {
    const size_t bytes = (size_t)want * 8;
    if (!room_for(c, bytes, (size_t)m->ix_cap * 8)) return false;
    ctx_free(c, m->ix_tab, (size_t)m->ix_cap * 8);
    c->ix_held -= std::min(c->ix_held, (size_t)m->ix_cap * 8);
    m->ix_tab = nullptr;
    m->ix_cap = 0;
    try {
      m->ix_tab = (uint64_t*)ctx_alloc(c, bytes);
    } catch (const DsgError& e) {
      if (e.code != DSG_E_OOM) throw;
      return false;
    }
    m->ix_cap = want;
    c->ix_held += bytes;
  }
  const RowIx X = mat_index_view(m);
  int64_t nl, nh;
  ix_build_grid(c, n, nl, nh);
  hipLaunchKernelGGL(k_ix_build, dim3((unsigned)(nl + nh)), dim3(IX_HEAVY_WG), 0, s, (const int64_t*)m->row_off,
                     (const int32_t*)m->row_len, (const int32_t*)m->col, X, (const int32_t*)nullptr,
                     (const int64_t*)nullptr, (int64_t)n, 1, nl);
  DSG_HIP(hipGetLastError());
  return true;
}

}  // namespace

bool mat_index_enable(DMat* m) {
  if (m->ix_tab) return true;
  if (m->ix_refused) return false;
  Ctx* c = m->ctx;
  const size_t n = (size_t)std::max<int32_t>(m->nrows, 1);
  // tables take about twice the entries, and the pool a quarter more
  if (!room_for(c, (size_t)(2 * m->h_top_ub + 16 * (int64_t)n) * 10 + n * 20, 0)) {
    m->ix_refused = true;
    return false;
  }
  bool ok = false;
  try {
    m->ix_off = (int64_t*)ctx_alloc(c, n * 8);
    m->ix_sz = (int32_t*)ctx_alloc(c, n * 4);
    m->ix_used = (int32_t*)ctx_alloc(c, n * 4);
    m->ix_stamp = (uint32_t*)ctx_alloc(c, n * 4);
    m->ix_top = (unsigned long long*)ctx_alloc(c, 64);
    m->ix_gen = 1;
    ok = build_all(m);
  } catch (const DsgError& e) {
    if (e.code != DSG_E_OOM) throw;
    ok = false;
  }
  if (!ok || !m->ix_tab) {
    free_index(m);
    m->ix_refused = true;
    return false;
  }
  return true;
}

void mat_index_free(DMat* m) {
  if (m->ix_tab) free_index(m);
}

void mat_index_invalidate(DMat* m) {
  if (!m->ix_tab) return;
  if (++m->ix_gen == 0) {
    // the stamps would meet old values again: clear them
    if (m->nrows > 0)
      hipLaunchKernelGGL(k_ix_zero_stamps, dim3(blocks_for(m->nrows, 256)), dim3(256), 0, m->ctx->stream,
                         m->ix_stamp, m->nrows);
    m->ix_gen = 1;
  }
}

void mat_index_build(DMat* m, const int32_t* d_rows, const int64_t* d_n, int64_t n_max) {
  if (!m->ix_tab || n_max <= 0) return;
  Ctx* c = m->ctx;
  hipStream_t s = c->stream;
  const RowIx X = mat_index_view(m);
  // a bounded grid: the listed rows are taken in turn
  int64_t nl, nh;
  ix_build_grid(c, n_max, nl, nh);
  hipLaunchKernelGGL(k_ix_build, dim3((unsigned)(nl + nh)), dim3(IX_HEAVY_WG), 0, s, (const int64_t*)m->row_off,
                     (const int32_t*)m->row_len, (const int32_t*)m->col, X, d_rows, d_n, n_max, 0, nl);
  DSG_HIP(hipGetLastError());
}

void mat_index_note_top(DMat* m, uint64_t top) {
  if (!m->ix_tab) return;
  if ((int64_t)top * 10 > m->ix_cap * 9) {
    // the pool is nearly taken (tables of rows since rebuilt included):
    // every table again, at fresh offsets
    if (!build_all(m)) {
      free_index(m);
      m->ix_refused = true;
    }
  }
}
