// Dynamic matrix storage on the device: creation, pool compaction, canonical
// export and the transpose index.
//
// The paper's dynamic matrix keeps an adjacency array per row plus a per-row
// hash table from column to slot so that a single update costs O(1) expected
// time (Section 4).  On the GPU a batch is sorted first (ingest.hip), so one
// wavefront streams a whole row once and matches it against that row's
// updates; no per-row hash table is kept.  Rows keep slack capacity so that
// most insertions need no move.
#include <algorithm>
#include <cstring>

#include "internal.h"
#include "kernel_common.h"

namespace {

int bits_for(int64_t n) {
  int b = 0;
  while ((int64_t(1) << b) < n) ++b;
  return b;
}

__global__ void k_caps_from_csr(const int64_t* rp, int32_t n, int32_t* len, int32_t* cap) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    int32_t l = (int32_t)(rp[i + 1] - rp[i]);
    len[i] = l;
    cap[i] = slack_cap(l);
  }
}

__global__ void k_zero_rows(int32_t n, int32_t* len, int32_t* cap, int64_t* off, uint32_t* ep) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    len[i] = 0;
    cap[i] = 0;
    off[i] = 0;
    ep[i] = 0;
  }
}

// one wavefront per row: copy CSR row i to its pool slots
template <int VSZ>
__global__ __launch_bounds__(256) void k_copy_from_csr(const int64_t* rp, const int32_t* ci, const char* cv,
                                                       int32_t n, const int64_t* off, int32_t* col,
                                                       char* val) {
  int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (i >= n) return;
  int64_t s = rp[i], e = rp[i + 1], o = off[i];
  for (int64_t t = s + lane; t < e; t += 64) {
    col[o + (t - s)] = ci[t];
    if constexpr (VSZ == 8) ((uint64_t*)val)[o + (t - s)] = ((const uint64_t*)cv)[t];
    if constexpr (VSZ == 4) ((uint32_t*)val)[o + (t - s)] = ((const uint32_t*)cv)[t];
  }
}

// one wavefront per row: copy row i from the old pool to the new one
template <int VSZ>
__global__ __launch_bounds__(256) void k_move_rows(int32_t n, const int64_t* old_off, const int64_t* new_off,
                                                   const int32_t* len, const int32_t* ocol, const char* oval,
                                                   int32_t* ncol, char* nval) {
  int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (i >= n) return;
  int64_t so = old_off[i], dn = new_off[i];
  int32_t l = len[i];
  for (int32_t t = lane; t < l; t += 64) {
    ncol[dn + t] = ocol[so + t];
    if constexpr (VSZ == 8) ((uint64_t*)nval)[dn + t] = ((const uint64_t*)oval)[so + t];
    if constexpr (VSZ == 4) ((uint32_t*)nval)[dn + t] = ((const uint32_t*)oval)[so + t];
  }
}

__global__ void k_slack_of_len(int32_t n, const int32_t* len, int32_t* cap) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cap[i] = slack_cap(len[i]);
}

__global__ void k_sum_len(int32_t n, const int32_t* len, unsigned long long* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long v = i < n ? (unsigned long long)len[i] : 0ull;
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(out, v);
}

// export of rows [r0, r1): one wavefront per row writes (row - r0, col) keys
// and compact values at the row's place relative to the first row's
template <int VSZ>
__global__ __launch_bounds__(256) void k_export_keys(int32_t r0, int32_t r1, const int64_t* off, const int32_t* len,
                                                     const int32_t* col, const char* val,
                                                     const int64_t* rp, int cbits, uint64_t* keys,
                                                     uint32_t* pos, char* vtmp) {
  int64_t i = r0 + (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  int lane = threadIdx.x & 63;
  if (i >= r1) return;
  int64_t o = off[i], d = rp[i] - rp[r0];
  int32_t l = len[i];
  for (int32_t t = lane; t < l; t += 64) {
    keys[d + t] = ((uint64_t)(i - r0) << cbits) | (uint64_t)(uint32_t)col[o + t];
    pos[d + t] = (uint32_t)(d + t);
    if constexpr (VSZ == 8) ((uint64_t*)vtmp)[d + t] = ((const uint64_t*)val)[o + t];
    if constexpr (VSZ == 4) ((uint32_t*)vtmp)[d + t] = ((const uint32_t*)val)[o + t];
  }
}

template <int VSZ>
__global__ void k_export_gather(int64_t nnz, const uint64_t* keys, const uint32_t* pos, const char* vtmp,
                                uint64_t cmask, int32_t* ocol, char* oval) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nnz) return;
  ocol[q] = (int32_t)(keys[q] & cmask);
  if constexpr (VSZ == 8) ((uint64_t*)oval)[q] = ((const uint64_t*)vtmp)[pos[q]];
  if constexpr (VSZ == 4) ((uint32_t*)oval)[q] = ((const uint32_t*)vtmp)[pos[q]];
}

// transpose index: count entries per column
__global__ __launch_bounds__(256) void k_col_counts(int32_t n, const int64_t* off, const int32_t* len,
                                                    const int32_t* col, int32_t* cnt) {
  int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (i >= n) return;
  int64_t o = off[i];
  for (int32_t t = lane; t < len[i]; t += 64) atomicAdd(&cnt[col[o + t]], 1);
}

template <int VSZ>
__global__ __launch_bounds__(256) void k_fill_transpose(int32_t n, const int64_t* off, const int32_t* len,
                                                        const int32_t* col, const char* val, const int64_t* toff,
                                                        int32_t* tlen, int32_t* tcol, char* tval) {
  int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (i >= n) return;
  int64_t o = off[i];
  for (int32_t t = lane; t < len[i]; t += 64) {
    int32_t j = col[o + t];
    int32_t p = atomicAdd(&tlen[j], 1);
    tcol[toff[j] + p] = (int32_t)i;
    if constexpr (VSZ == 8) ((uint64_t*)tval)[toff[j] + p] = ((const uint64_t*)val)[o + t];
    else if constexpr (VSZ == 4) ((uint32_t*)tval)[toff[j] + p] = ((const uint32_t*)val)[o + t];
  }
}

unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

void set_top(DMat* m, int64_t top) {
  DSG_HIP(hipMemcpyAsync(m->d_top, &top, sizeof(int64_t), hipMemcpyHostToDevice, m->ctx->stream));
  m->h_top_ub = top;
}

int64_t read_i64(Ctx* c, const int64_t* d) {
  int64_t* h = (int64_t*)c->pinned;
  DSG_HIP(hipMemcpyAsync(h, d, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  DSG_HIP(hipStreamSynchronize(c->stream));
  return *h;
}

}  // namespace

DMat* mat_create(Ctx* c, int32_t nrows, int32_t ncols, int sr, const int64_t* d_rp, const int32_t* d_col,
                 const void* d_val) {
  DMat* m = new DMat();
  m->ctx = c;
  m->nrows = nrows;
  m->ncols = ncols;
  m->sr = sr;
  m->vsz = sr < 0 ? 0 : (sr == 1 || sr == 3 ? 4 : 8);
  hipStream_t s = c->stream;
  try {
    size_t n = (size_t)(nrows > 0 ? nrows : 1);
    m->row_off = (int64_t*)ctx_alloc(c, n * 8);
    m->row_len = (int32_t*)ctx_alloc(c, n * 4);
    m->row_cap = (int32_t*)ctx_alloc(c, n * 4);
    m->row_epoch = (uint32_t*)ctx_alloc(c, n * 4);
    m->d_top = (int64_t*)ctx_alloc(c, 16);
    m->d_epoch = (uint32_t*)(m->d_top + 1);
    {
      const uint32_t one = 1;
      DSG_HIP(hipMemcpyAsync(m->d_epoch, &one, 4, hipMemcpyHostToDevice, s));
      DSG_HIP(hipStreamSynchronize(s));
    }
    hipLaunchKernelGGL(k_zero_rows, dim3(blocks_for(nrows, 256) + 1), dim3(256), 0, s, nrows, m->row_len,
                       m->row_cap, m->row_off, m->row_epoch);
    int64_t total = 0;
    if (d_rp && nrows > 0) {
      hipLaunchKernelGGL(k_caps_from_csr, dim3(blocks_for(nrows, 256)), dim3(256), 0, s, d_rp, nrows,
                         m->row_len, m->row_cap);
      void* scr = ctx_scratch(c, scan_scratch_bytes(nrows) + 64);
      int64_t* d_total = (int64_t*)((char*)scr + scan_scratch_bytes(nrows));
      exclusive_scan_i32_to_i64(m->row_cap, m->row_off, nrows, d_total, scr, s);
      total = read_i64(c, d_total);
    }
    m->pool_cap = total + total / 4 + 1024;
    m->col = (int32_t*)ctx_alloc(c, pool_bytes(m->pool_cap, 4));
    if (m->vsz) m->val = ctx_alloc(c, pool_bytes(m->pool_cap, m->vsz));
    if (d_rp && nrows > 0) {
      unsigned nb = blocks_for((int64_t)nrows * 64, 256);
      if (m->vsz == 8)
        hipLaunchKernelGGL(k_copy_from_csr<8>, dim3(nb), dim3(256), 0, s, d_rp, d_col, (const char*)d_val,
                           nrows, m->row_off, m->col, (char*)m->val);
      else if (m->vsz == 4)
        hipLaunchKernelGGL(k_copy_from_csr<4>, dim3(nb), dim3(256), 0, s, d_rp, d_col, (const char*)d_val,
                           nrows, m->row_off, m->col, (char*)m->val);
      else
        hipLaunchKernelGGL(k_copy_from_csr<0>, dim3(nb), dim3(256), 0, s, d_rp, d_col, (const char*)d_val,
                           nrows, m->row_off, m->col, (char*)m->val);
    }
    set_top(m, total);
    DSG_HIP(hipGetLastError());
  } catch (...) {
    mat_destroy(m);
    throw;
  }
  c->objects++;
  m->counted = true;
  return m;
}

void mat_destroy(DMat* m) {
  if (!m) return;
  Ctx* c = m->ctx;
  size_t n = (size_t)(m->nrows > 0 ? m->nrows : 1);
  if (m->tidx) mat_destroy(m->tidx);
  ctx_free(c, m->row_off, n * 8);
  ctx_free(c, m->row_len, n * 4);
  ctx_free(c, m->row_cap, n * 4);
  ctx_free(c, m->row_epoch, n * 4);
  ctx_free(c, m->d_top, 16);
  ctx_free(c, m->col, pool_bytes(m->pool_cap, 4));
  if (m->val) ctx_free(c, m->val, pool_bytes(m->pool_cap, m->vsz));
  ctx_free(c, m->log_key, (size_t)m->log_cap * 8);
  ctx_free(c, m->log_old, (size_t)m->log_cap * 8);
  ctx_free(c, m->log_new, (size_t)m->log_cap * 8);
  ctx_free(c, m->log_code, (size_t)m->log_cap);
  ctx_free(c, m->d_log_n, 64);
  mat_index_free(m);
  if (m->counted) c->objects--;
  delete m;
}

void mat_compact(DMat* m, int64_t extra) {
  Ctx* c = m->ctx;
  hipStream_t s = c->stream;
  int32_t n = m->nrows;
  size_t nn = (size_t)(n > 0 ? n : 1);
  int64_t* new_off = (int64_t*)ctx_alloc(c, nn * 8);
  int64_t total = 0;
  try {
    if (n > 0) {
      hipLaunchKernelGGL(k_slack_of_len, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, m->row_len,
                         m->row_cap);
      size_t sb = scan_scratch_bytes(n) + 64;
      void* scr = ctx_alloc(c, sb);
      int64_t* d_total = (int64_t*)((char*)scr + scan_scratch_bytes(n));
      exclusive_scan_i32_to_i64(m->row_cap, new_off, n, d_total, scr, s);
      total = read_i64(c, d_total);
      ctx_free(c, scr, sb);
    }
    int64_t cap = total + extra + (total + extra) / 2 + 1024;
    int32_t* ncol = (int32_t*)ctx_alloc(c, pool_bytes(cap, 4));
    void* nval = nullptr;
    if (m->vsz) {
      try {
        nval = ctx_alloc(c, pool_bytes(cap, m->vsz));
      } catch (...) {
        ctx_free(c, ncol, pool_bytes(cap, 4));
        throw;
      }
    }
    if (n > 0) {
      unsigned nb = blocks_for((int64_t)n * 64, 256);
      if (m->vsz == 8)
        hipLaunchKernelGGL(k_move_rows<8>, dim3(nb), dim3(256), 0, s, n, m->row_off, new_off, m->row_len,
                           m->col, (const char*)m->val, ncol, (char*)nval);
      else if (m->vsz == 4)
        hipLaunchKernelGGL(k_move_rows<4>, dim3(nb), dim3(256), 0, s, n, m->row_off, new_off, m->row_len,
                           m->col, (const char*)m->val, ncol, (char*)nval);
      else
        hipLaunchKernelGGL(k_move_rows<0>, dim3(nb), dim3(256), 0, s, n, m->row_off, new_off, m->row_len,
                           m->col, (const char*)m->val, ncol, (char*)nval);
      DSG_HIP(hipMemcpyAsync(m->row_off, new_off, nn * 8, hipMemcpyDeviceToDevice, s));
    }
    DSG_HIP(hipStreamSynchronize(s));
    ctx_free(c, m->col, pool_bytes(m->pool_cap, 4));
    if (m->val) ctx_free(c, m->val, pool_bytes(m->pool_cap, m->vsz));
    m->col = ncol;
    m->val = nval;
    m->pool_cap = cap;
    m->version++;
    set_top(m, total);
  } catch (...) {
    ctx_free(c, new_off, nn * 8);
    throw;
  }
  ctx_free(c, new_off, nn * 8);
}

void mat_reserve(DMat* m, int64_t extra) { mat_reserve(m, extra, extra); }

void mat_reserve(DMat* m, int64_t extra, int64_t want) {
  if (m->pool_cap - m->h_top_ub >= extra) return;
  m->h_top_ub = read_i64(m->ctx, m->d_top);
  if (m->pool_cap - m->h_top_ub >= extra) return;
  mat_compact(m, std::max(extra, want));
}

int64_t mat_nnz(DMat* m) {
  Ctx* c = m->ctx;
  unsigned long long* d = (unsigned long long*)ctx_scratch(c, 64);
  DSG_HIP(hipMemsetAsync(d, 0, 8, c->stream));
  if (m->nrows > 0)
    hipLaunchKernelGGL(k_sum_len, dim3(blocks_for(m->nrows, 256)), dim3(256), 0, c->stream, m->nrows,
                       m->row_len, d);
  return read_i64(c, (const int64_t*)d);
}

void mat_export_device(DMat* m, int64_t* d_rp, int32_t* d_col, void* d_val, void* /*unused*/,
                       hipStream_t s) {
  Ctx* c = m->ctx;
  int32_t n = m->nrows;
  if (n == 0) {
    DSG_HIP(hipMemsetAsync(d_rp, 0, 8, s));
    return;
  }
  // row pointers
  {
    void* scr = ctx_scratch(c, scan_scratch_bytes(n) + 64);
    exclusive_scan_i32_to_i64(m->row_len, d_rp, n, d_rp + n, scr, s);
  }
  int64_t nnz = read_i64(c, d_rp + n);
  if (!d_col || nnz == 0) return;
  // rows in chunks of at most EXPORT_CHUNK entries (a longer row is a chunk
  // of its own), each sorted by (row, column) on its own: the scratch stays
  // bounded whatever the matrix's size
  constexpr int64_t EXPORT_CHUNK = int64_t(1) << 25;
  std::vector<int64_t> hrp((size_t)n + 1);
  DSG_HIP(hipMemcpyAsync(hrp.data(), d_rp, ((size_t)n + 1) * 8, hipMemcpyDeviceToHost, s));
  DSG_HIP(hipStreamSynchronize(s));
  int64_t most = 0;
  for (int32_t i = 0; i < n; ++i) most = std::max<int64_t>(most, hrp[i + 1] - hrp[i]);
  const int64_t cap = std::max<int64_t>(std::min<int64_t>(nnz, EXPORT_CHUNK), most);
  int cbits = bits_for(m->ncols);
  size_t vs = (size_t)(m->vsz ? m->vsz : 4);
  size_t need = Carve::need({(size_t)cap * 8, (size_t)cap * 4, (size_t)cap * vs, radix_scratch_bytes(cap), 64});
  Carve cv(ctx_scratch(c, need), need);
  uint64_t* keys = cv.take<uint64_t>(cap);
  uint32_t* pos = cv.take<uint32_t>(cap);
  char* vtmp = cv.take<char>((size_t)cap * vs);
  void* rs = cv.take<char>(radix_scratch_bytes(cap));
  int* d_err = cv.take<int>(16);  // the sorts' error flag
  DSG_HIP(hipMemsetAsync(d_err, 0, 4, s));
  uint64_t cmask = cbits >= 64 ? ~0ull : ((1ull << cbits) - 1);
  for (int32_t r0 = 0; r0 < n;) {
    int32_t r1 = r0 + 1;
    while (r1 < n && hrp[r1 + 1] - hrp[r0] <= cap) ++r1;
    const int64_t base = hrp[r0], e = hrp[r1] - base;
    if (e > 0) {
      unsigned nb = blocks_for((int64_t)(r1 - r0) * 64, 256);
      if (m->vsz == 8)
        hipLaunchKernelGGL(k_export_keys<8>, dim3(nb), dim3(256), 0, s, r0, r1, m->row_off, m->row_len, m->col,
                           (const char*)m->val, d_rp, cbits, keys, pos, vtmp);
      else if (m->vsz == 4)
        hipLaunchKernelGGL(k_export_keys<4>, dim3(nb), dim3(256), 0, s, r0, r1, m->row_off, m->row_len, m->col,
                           (const char*)m->val, d_rp, cbits, keys, pos, vtmp);
      else
        hipLaunchKernelGGL(k_export_keys<0>, dim3(nb), dim3(256), 0, s, r0, r1, m->row_off, m->row_len, m->col,
                           (const char*)m->val, d_rp, cbits, keys, pos, vtmp);
      radix_sort_pairs(keys, pos, e, cbits + bits_for(r1 - r0), rs, s, d_err);
      unsigned gb = blocks_for(e, 256);
      char* ov = d_val ? (char*)d_val + (size_t)base * vs : nullptr;
      if (m->vsz == 8)
        hipLaunchKernelGGL(k_export_gather<8>, dim3(gb), dim3(256), 0, s, e, keys, pos, vtmp, cmask, d_col + base,
                           ov);
      else if (m->vsz == 4)
        hipLaunchKernelGGL(k_export_gather<4>, dim3(gb), dim3(256), 0, s, e, keys, pos, vtmp, cmask, d_col + base,
                           ov);
      else
        hipLaunchKernelGGL(k_export_gather<0>, dim3(gb), dim3(256), 0, s, e, keys, pos, vtmp, cmask, d_col + base,
                           ov);
    }
    r0 = r1;
  }
  DSG_HIP(hipGetLastError());
  int* h = (int*)c->pinned;
  DSG_HIP(hipMemcpyAsync(h, d_err, 4, hipMemcpyDeviceToHost, s));
  DSG_HIP(hipStreamSynchronize(s));
  DSG_REQUIRE(h[0] == 0, DSG_E_DEVICE, "internal: the export's sort could not complete");
}

void mat_build_transpose(DMat* m) {
  if (m->tidx) return;
  Ctx* c = m->ctx;
  hipStream_t s = c->stream;
  // the transpose carries the values too: columns of m with their entries
  DMat* t = mat_create(c, m->ncols, m->nrows, m->sr, nullptr, nullptr, nullptr);
  try {
    int32_t nt = t->nrows;
    if (nt > 0 && m->nrows > 0) {
      int32_t* cnt = (int32_t*)ctx_scratch(c, (size_t)nt * 4 + scan_scratch_bytes(nt) + 64);
      void* scr = (char*)cnt + (size_t)nt * 4;
      int64_t* d_total = (int64_t*)((char*)scr + scan_scratch_bytes(nt));
      DSG_HIP(hipMemsetAsync(cnt, 0, (size_t)nt * 4, s));
      unsigned nb = blocks_for((int64_t)m->nrows * 64, 256);
      hipLaunchKernelGGL(k_col_counts, dim3(nb), dim3(256), 0, s, m->nrows, m->row_off, m->row_len, m->col,
                         cnt);
      hipLaunchKernelGGL(k_slack_of_len, dim3(blocks_for(nt, 256)), dim3(256), 0, s, nt, cnt, t->row_cap);
      exclusive_scan_i32_to_i64(t->row_cap, t->row_off, nt, d_total, scr, s);
      int64_t total = read_i64(c, d_total);
      ctx_free(c, t->col, pool_bytes(t->pool_cap, 4));
      if (t->val) ctx_free(c, t->val, pool_bytes(t->pool_cap, t->vsz));
      t->col = nullptr;
      t->val = nullptr;
      t->pool_cap = total + total / 4 + 1024;
      t->version++;
      t->col = (int32_t*)ctx_alloc(c, pool_bytes(t->pool_cap, 4));
      if (t->vsz) t->val = ctx_alloc(c, pool_bytes(t->pool_cap, t->vsz));
      DSG_HIP(hipMemsetAsync(t->row_len, 0, (size_t)nt * 4, s));
      if (t->vsz == 8)
        hipLaunchKernelGGL(k_fill_transpose<8>, dim3(nb), dim3(256), 0, s, m->nrows, m->row_off, m->row_len,
                           m->col, (const char*)m->val, t->row_off, t->row_len, t->col, (char*)t->val);
      else if (t->vsz == 4)
        hipLaunchKernelGGL(k_fill_transpose<4>, dim3(nb), dim3(256), 0, s, m->nrows, m->row_off, m->row_len,
                           m->col, (const char*)m->val, t->row_off, t->row_len, t->col, (char*)t->val);
      else
        hipLaunchKernelGGL(k_fill_transpose<0>, dim3(nb), dim3(256), 0, s, m->nrows, m->row_off, m->row_len,
                           m->col, (const char*)m->val, t->row_off, t->row_len, t->col, (char*)t->val);
      set_top(t, total);
      DSG_HIP(hipGetLastError());
    }
  } catch (...) {
    mat_destroy(t);
    throw;
  }
  m->tidx = t;
}

// ---------------------------------------------------------------------------
// row gather: listed rows of a matrix, canonical, into host memory
// ---------------------------------------------------------------------------

namespace {

__global__ void k_gather_lens(const int32_t* rows, int32_t n, const int32_t* row_len, int64_t* lens) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) lens[q] = row_len[rows[q]];
}

// one wavefront per listed row: its entries into a compact buffer
template <int VSZ>
__global__ __launch_bounds__(256) void k_gather_rows(const int32_t* rows, int32_t n, const int64_t* off,
                                                     const int32_t* len, const int32_t* col, const char* val,
                                                     const int64_t* rp, int32_t* ocol, char* oval) {
  const int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (q >= n) return;
  const int32_t i = rows[q];
  const int64_t o = off[i], d = rp[q];
  for (int32_t t = lane; t < len[i]; t += 64) {
    ocol[d + t] = col[o + t];
    if constexpr (VSZ == 8) ((uint64_t*)oval)[d + t] = ((const uint64_t*)val)[o + t];
    else if constexpr (VSZ == 4) ((uint32_t*)oval)[d + t] = ((const uint32_t*)val)[o + t];
  }
}

void ensure_buf(Ctx* c, void*& p, size_t& have, size_t bytes) {
  if (bytes <= have) return;
  ctx_free(c, p, have);
  p = nullptr;
  have = 0;
  const size_t nb = bytes + bytes / 2 + 4096;
  p = ctx_alloc(c, nb);
  have = nb;
}

}  // namespace

void gather_bufs_free(Ctx* c, GatherBufs& g) {
  ctx_free(c, g.lens, g.lens_bytes);
  ctx_free(c, g.rp, g.rp_bytes);
  ctx_free(c, g.scan, g.scan_bytes);
  ctx_free(c, g.col, g.col_bytes);
  ctx_free(c, g.val, g.val_bytes);
  g = GatherBufs{};
}

void gather_row_ptr(DMat* m, const int32_t* d_rows, int32_t n, int64_t* d_lens, int64_t* d_rp, void* d_scan,
                    hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_gather_lens, dim3(blocks_for(n, 256)), dim3(256), 0, s, d_rows, n, m->row_len, d_lens);
  exclusive_scan_i64(d_lens, d_rp, n, d_rp + n, d_scan, s);
}

void gather_row_entries(DMat* m, const int32_t* d_rows, int32_t n, const int64_t* d_rp, int32_t* d_col,
                        void* d_val, hipStream_t s) {
  if (n <= 0) return;
  const unsigned nb = (unsigned)blocks_for((int64_t)n * 64, 256);
  if (m->vsz == 8)
    hipLaunchKernelGGL(k_gather_rows<8>, dim3(nb), dim3(256), 0, s, d_rows, n, m->row_off, m->row_len, m->col,
                       (const char*)m->val, d_rp, d_col, (char*)d_val);
  else if (m->vsz == 4)
    hipLaunchKernelGGL(k_gather_rows<4>, dim3(nb), dim3(256), 0, s, d_rows, n, m->row_off, m->row_len, m->col,
                       (const char*)m->val, d_rp, d_col, (char*)d_val);
  else
    hipLaunchKernelGGL(k_gather_rows<0>, dim3(nb), dim3(256), 0, s, d_rows, n, m->row_off, m->row_len, m->col,
                       (const char*)m->val, d_rp, d_col, (char*)d_val);
  DSG_HIP(hipGetLastError());
}

void mat_gather_rows(DMat* m, const int32_t* d_rows, int32_t n, GatherBufs& g, RowsHost& out, hipStream_t s,
                     bool entries) {
  Ctx* c = m->ctx;
  const int vs = m->vsz;
  ensure_buf(c, g.lens, g.lens_bytes, (size_t)(n + 1) * 8);
  ensure_buf(c, g.rp, g.rp_bytes, (size_t)(n + 1) * 8);
  ensure_buf(c, g.scan, g.scan_bytes, scan_scratch_bytes(n) + 64);
  gather_row_ptr(m, d_rows, n, (int64_t*)g.lens, (int64_t*)g.rp, g.scan, s);
  out.row_ptr.assign((size_t)n + 1, 0);
  DSG_HIP(hipMemcpyAsync(out.row_ptr.data(), g.rp, out.row_ptr.size() * 8, hipMemcpyDeviceToHost, s));
  DSG_HIP(hipStreamSynchronize(s));
  const int64_t nnz = out.row_ptr[(size_t)n];
  if (!entries) return;
  out.col.resize((size_t)nnz);
  out.val.resize((size_t)nnz * vs);
  if (nnz == 0) return;
  ensure_buf(c, g.col, g.col_bytes, (size_t)nnz * 4);
  ensure_buf(c, g.val, g.val_bytes, (size_t)nnz * (vs ? vs : 1));
  gather_row_entries(m, d_rows, n, (const int64_t*)g.rp, (int32_t*)g.col, g.val, s);
  std::vector<int32_t> hc((size_t)nnz);
  std::vector<char> hv((size_t)nnz * vs);
  DSG_HIP(hipMemcpyAsync(hc.data(), g.col, (size_t)nnz * 4, hipMemcpyDeviceToHost, s));
  if (vs) DSG_HIP(hipMemcpyAsync(hv.data(), g.val, (size_t)nnz * vs, hipMemcpyDeviceToHost, s));
  DSG_HIP(hipStreamSynchronize(s));
  // rows are stored in no particular column order: sort each one
  std::vector<int64_t> perm;
  for (int32_t q = 0; q < n; ++q) {
    const int64_t a = out.row_ptr[(size_t)q], b = out.row_ptr[(size_t)q + 1];
    perm.resize((size_t)(b - a));
    for (int64_t e = a; e < b; ++e) perm[(size_t)(e - a)] = e;
    std::sort(perm.begin(), perm.end(), [&](int64_t x, int64_t y) { return hc[(size_t)x] < hc[(size_t)y]; });
    for (int64_t e = a; e < b; ++e) {
      const int64_t src = perm[(size_t)(e - a)];
      out.col[(size_t)e] = hc[(size_t)src];
      if (vs) memcpy(out.val.data() + (size_t)e * vs, hv.data() + (size_t)src * vs, (size_t)vs);
    }
  }
}
