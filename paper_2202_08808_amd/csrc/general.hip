// Dynamic updates by the paper's algorithm for general updates (Section 5.2,
// Algorithm 2) on one GPU, with its Bloom matrix F kept beside C.
//
// F has C's structure; bit (k mod 64) of f_ij is set when a_ik b_kj is a term
// of c_ij (l = 64, the width the paper uses).  One GPU holds every block, so
// the algorithm's broadcasts, sends and aggregations are the identity; its
// local steps run here in its order:
//   computePattern  the terms of C* = A* B + A' B* (Eq. 1 in the equivalent
//                   form of the paper's footnote) with their bits, sorted by
//                   (i, j) and reduced to C* and F*.  A* holds the entries the
//                   last apply of A changed (deletions included), B* those of
//                   B; B's old row k is B' row k plus the entries of row k that
//                   apply deleted, A' column k is a row of A's transpose index
//                   (of A itself when the product reads A^T).
//                   Entries of B' row k that the apply inserted make the pattern
//                   a superset, which the masked product below resolves.
//   E, R            r_i = the bitwise or over (i, j) in C* of f*_ij | f_ij
//                   (f_ij read by streaming F's row i against a table of the
//                   row's C* columns).
//   A^R             row i of A' keeping the k whose bit is set in r_i (a
//                   filter applied while the row is read, nothing is copied).
//   Z, H            A^R B' masked at C*: a row-wise Gustavson that adds a term
//                   only when (i, j) is in C* (Section 6.2: a table of C*'s
//                   entries checked before each addition), H the new bits.
//   merges          Z into C and H into F at C*: SET where a term exists,
//                   DELETE where none does, through the ordinary apply.
// A and B above stand for op(A) and op(B) (Section 5, transposition): a
// transposed operand's rows are its transpose index's, its log is the one
// that index keeps of every apply, in the transposed coordinates, and its
// columns as rows are the source matrix itself.
// Semiring additions that are exactly associative combine with atomics in
// any order; fp64 sums take the kept k of a row one at a time in ascending k,
// so every c'_ij is summed in the order of its definition.
#include <algorithm>

#include "internal.h"
#include "kernel_common.h"

namespace {

unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

int bits_for(int64_t n) {
  int b = 0;
  while ((int64_t(1) << b) < n) ++b;
  return b;
}

__device__ inline uint64_t bloom_bit(int32_t k) { return 1ull << ((uint32_t)k & 63u); }

__device__ inline bool changed_code(uint8_t c) { return c == UPD_INS || c == UPD_DEL || c == UPD_OVR; }

struct LogView {
  const uint64_t* key;  // (row << cbits) | col, ascending
  const uint8_t* code;  // UPD_*
  int64_t n;
  int cbits;
};

struct RowsView {
  const int64_t* off;
  const int32_t* len;
  const int32_t* col;
  const void* val;
};

RowsView rows_of(const DMat* m) { return RowsView{m->row_off, m->row_len, m->col, m->val}; }

// first log index with key >= k
__device__ inline int64_t key_lower(const uint64_t* key, int64_t n, uint64_t k) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (key[mid] < k) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// ---- computePattern: terms ----

// Terms per log entry: entries [0, LA.n) are A's, [LA.n, LA.n + LB.n) B's.
//   a changed (i, k) of A: one term per entry of B' row k and per entry of B
//     row k that the apply deleted;
//   a changed (k, j) of B: one term per entry of A' column k.
__global__ void k_pat_counts(LogView LA, LogView LB, const int32_t* b_len, const int32_t* t_len, int64_t* cnt) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= LA.n + LB.n) return;
  int64_t c = 0;
  if (u < LA.n) {
    if (changed_code(LA.code[u])) {
      const int32_t k = (int32_t)(LA.key[u] & ((1ull << LA.cbits) - 1));
      const int64_t lo = key_lower(LB.key, LB.n, (uint64_t)k << LB.cbits);
      const int64_t hi = key_lower(LB.key, LB.n, ((uint64_t)k + 1) << LB.cbits);
      int64_t ndel = 0;
      for (int64_t e = lo; e < hi; ++e) ndel += LB.code[e] == UPD_DEL;
      c = (int64_t)b_len[k] + ndel;
    }
  } else {
    const int64_t v = u - LA.n;
    if (changed_code(LB.code[v])) c = t_len[(int32_t)(LB.key[v] >> LB.cbits)];
  }
  cnt[u] = c;
}

__device__ inline uint64_t term_key(int32_t i, int32_t j, int32_t k, int cb) {
  return (((((uint64_t)(uint32_t)i) << cb) | (uint64_t)(uint32_t)j) << 6) | (uint64_t)((uint32_t)k & 63u);
}

// One wavefront per log entry: its terms (i, j, k mod 64) as sort keys.
__global__ __launch_bounds__(256) void k_pat_write(LogView LA, LogView LB, RowsView B, RowsView T,
                                                   const int64_t* off, int cb, uint64_t* keys) {
  const int64_t u = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (u >= LA.n + LB.n) return;
  int64_t o = off[u];
  if (u < LA.n) {
    if (!changed_code(LA.code[u])) return;
    const int32_t i = (int32_t)(LA.key[u] >> LA.cbits);
    const int32_t k = (int32_t)(LA.key[u] & ((1ull << LA.cbits) - 1));
    const int64_t bo = B.off[k];
    const int32_t bl = B.len[k];
    for (int32_t t = lane; t < bl; t += 64) keys[o + t] = term_key(i, B.col[bo + t], k, cb);
    o += bl;
    // entries of B row k the apply deleted
    const int64_t lo = key_lower(LB.key, LB.n, (uint64_t)k << LB.cbits);
    const int64_t hi = key_lower(LB.key, LB.n, ((uint64_t)k + 1) << LB.cbits);
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (int64_t e0 = lo; e0 < hi; e0 += 64) {
      const int64_t e = e0 + lane;
      const bool del = e < hi && LB.code[e] == UPD_DEL;
      const uint64_t b = __ballot(del);
      if (del) keys[o + __popcll(b & lt)] = term_key(i, (int32_t)(LB.key[e] & ((1ull << LB.cbits) - 1)), k, cb);
      o += __popcll(b);
    }
  } else {
    const int64_t v = u - LA.n;
    if (!changed_code(LB.code[v])) return;
    const int32_t k = (int32_t)(LB.key[v] >> LB.cbits);
    const int32_t j = (int32_t)(LB.key[v] & ((1ull << LB.cbits) - 1));
    const int64_t to = T.off[k];
    const int32_t tl = T.len[k];
    for (int32_t t = lane; t < tl; t += 64) keys[o + t] = term_key(T.col[to + t], j, k, cb);
  }
}

__global__ void k_iota_u32(uint32_t* p, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = (uint32_t)t;
}

// ---- computePattern: C* and F* from the sorted terms ----

__global__ void k_pat_heads(const uint64_t* keys, int64_t n, int64_t* head) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) head[t] = (t == 0 || (keys[t] >> 6) != (keys[t - 1] >> 6)) ? 1 : 0;
}

// segid: exclusive scan of head; fstar zeroed before
__global__ void k_pat_reduce(const uint64_t* keys, int64_t n, const int64_t* head, const int64_t* segid,
                             uint64_t* cs_key, unsigned long long* fstar) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t s = segid[t] + head[t] - 1;
  if (head[t]) cs_key[s] = keys[t] >> 6;
  atomicOr(&fstar[s], (unsigned long long)bloom_bit((int32_t)(keys[t] & 63u)));
}

// columns of C* and the heads of its rows (*d_n entries of C*, a grid over
// cap >= *d_n: the heads past the entries are zero, so a scan over cap
// counts the rows)
__global__ void k_cs_rows_heads(const uint64_t* cs_key, const int64_t* d_n, int64_t cap, int cb, int32_t* cs_col,
                                int64_t* rhead) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= cap) return;
  if (s >= *d_n) {
    rhead[s] = 0;
    return;
  }
  cs_col[s] = (int32_t)(cs_key[s] & ((1ull << cb) - 1));
  rhead[s] = (s == 0 || (cs_key[s] >> cb) != (cs_key[s - 1] >> cb)) ? 1 : 0;
}

__global__ void k_cs_rows(const uint64_t* cs_key, const int64_t* d_n, int cb, const int64_t* rhead, const int64_t* rid,
                          int32_t* row_id, int64_t* row_start) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = *d_n;
  if (s >= n) return;
  if (rhead[s]) {
    row_id[rid[s]] = (int32_t)(cs_key[s] >> cb);
    row_start[rid[s]] = s;
  }
  if (s == n - 1) row_start[rid[s] + rhead[s]] = n;
}

// ---- masked rows: a row id and a run of sorted columns per mask row ----

struct Mask {
  const int32_t* row;    // [nrow]
  const int64_t* start;  // [nrow + 1]: entries [start[r], start[r+1]) of col
  const int32_t* col;    // ascending inside each row
};

constexpr int MW = 256;          // workgroup of the masked kernels
constexpr int MSLOTS = 8192;     // LDS table of a mask row's columns: rows of up to MSLOTS/2 entries
constexpr int FP64_KCAP = 4096;  // fp64: kept entries of an A row sorted in LDS

// position of column j in the sorted run [lo, hi) of col, or -1
__device__ inline int64_t run_find(const int32_t* col, int64_t lo, int64_t hi, int32_t j) {
  const int64_t end = hi;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (col[mid] < j) lo = mid + 1;
    else hi = mid;
  }
  return (lo < end && col[lo] == j) ? lo : -1;
}

// LDS table of the mask row's columns: key column -> index inside the run
__device__ inline void table_build(int32_t* hk, int32_t* hv, const int32_t* col, int64_t s0, int32_t len) {
  for (int x = threadIdx.x; x < MSLOTS; x += blockDim.x) hk[x] = -1;
  __syncthreads();
  for (int32_t t = threadIdx.x; t < len; t += blockDim.x) {
    const int32_t j = col[s0 + t];
    uint32_t h = hash_col(j) & (MSLOTS - 1);
    while (atomicCAS(&hk[h], -1, j) != -1) h = (h + 1) & (MSLOTS - 1);
    hv[h] = t;
  }
  __syncthreads();
}

__device__ inline int32_t table_find(const int32_t* hk, const int32_t* hv, int32_t j) {
  uint32_t h = hash_col(j) & (MSLOTS - 1);
  for (;;) {
    const int32_t x = hk[h];
    if (x == j) return hv[h];
    if (x == -1) return -1;
    h = (h + 1) & (MSLOTS - 1);
  }
}

__device__ inline uint64_t wg_or(uint64_t x, uint64_t* red) {
  for (int d = 32; d > 0; d >>= 1) x |= __shfl_xor(x, d, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  uint64_t r = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r |= red[w];
  return r;
}

// A probe (a lookup in a row's column table: a few dependent global reads)
// is taken to cost PROBE_COST elements of a streamed row (one coalesced read
// and an LDS lookup each).  The row filter and the masked product probe where
// that costs less than streaming, e.g. a mask row with kept k's probes every
// b'_kj when kept * len * PROBE_COST < the summed lengths of the kept rows
// of B'.
constexpr unsigned long long PROBE_COST = 8;

// E and R: r = OR over the row's C* entries of f*_ij | f_ij, with f_ij read
// from F's row i (stored entries whose column is in the row's C*): found
// through F's column index when the row's C* entries are few against F's
// row (PROBE_COST), else by streaming F's row against a table of them.
__global__ __launch_bounds__(MW) void k_row_filter(Mask M, const unsigned long long* fstar, RowsView F, RowIx XF,
                                                   uint64_t* rbits) {
  __shared__ int32_t hk[MSLOTS];
  __shared__ int32_t hv[MSLOTS];
  __shared__ uint64_t red[MW / 64];
  const int64_t r = blockIdx.x;
  const int32_t i = M.row[r];
  const int64_t s0 = M.start[r], s1 = M.start[r + 1];
  const int32_t len = (int32_t)(s1 - s0);
  uint64_t acc = 0;
  for (int64_t e = s0 + threadIdx.x; e < s1; e += MW) acc |= fstar[e];
  const int64_t fo = F.off[i];
  const int32_t fl = F.len[i];
  const uint64_t* fval = (const uint64_t*)F.val;
  if (XF.tab && XF.stamp[i] == XF.gen && (uint64_t)len * PROBE_COST < (uint64_t)fl) {
    const uint64_t* ft = XF.tab + XF.off[i];
    const uint32_t fn = (uint32_t)XF.sz[i];
    for (int32_t t = threadIdx.x; t < len; t += MW) {
      const int32_t pos = ix_find(ft, fn, M.col[s0 + t]);
      if (pos >= 0) acc |= fval[fo + pos];
    }
  } else if (len <= MSLOTS / 2) {
    table_build(hk, hv, M.col, s0, len);
    for (int32_t t = threadIdx.x; t < fl; t += MW)
      if (table_find(hk, hv, F.col[fo + t]) >= 0) acc |= fval[fo + t];
  } else {
    for (int32_t t = threadIdx.x; t < fl; t += MW)
      if (run_find(M.col, s0, s1, F.col[fo + t]) >= 0) acc |= fval[fo + t];
  }
  acc = wg_or(acc, red);
  if (threadIdx.x == 0) rbits[r] = acc;
}

template <class A>
__global__ void k_fill_acc(A* z, unsigned long long* h, int64_t n, A ident) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) {
    z[t] = ident;
    h[t] = 0ull;
  }
}

struct MaskedArgs {
  Mask M;
  const uint64_t* rbits;  // per mask row; null: keep every k
  RowsView A, B;
  RowIx XB;               // B's per-row column index (tab null: no probing)
  void* z;                // accumulator word per mask entry (Sem::Acc)
  unsigned long long* h;  // Bloom bits per mask entry
  unsigned long long* stats;  // [0] kept A entries, [1] products tried (walk) or probes,
                              // [2] rows that walked, [3] rows that probed
  int* err;
};


// position of column c in row r of B' (its table, or a scan of the row when
// the table is not usable), or -1
__device__ inline int32_t row_find(const RowIx& X, const RowsView& M, int32_t r, int32_t c) {
  if (X.tab && X.stamp[r] == X.gen) return ix_find(X.tab + X.off[r], (uint32_t)X.sz[r], c);
  const int64_t o = M.off[r];
  const int32_t n = M.len[r];
  for (int32_t t = 0; t < n; ++t)
    if (M.col[o + t] == c) return t;
  return -1;
}

// Z and H: a mask row's entries of A' (row i, read with the filter r_i) are
// cut into up to MSPLIT parts of at least MIN_SLICE entries, so that the few
// rows of C* that reach hub rows of B' do not leave one workgroup with most
// of the work; the parts combine their terms with atomics.  The parts are
// listed first ((row << 5) | part), and a bounded grid takes them in turn.
// In a part each wavefront takes one kept k at a time and its lanes walk B'
// row k, adding a term only where (i, j) is in the mask; a part whose probes
// cost less (PROBE_COST) takes every (kept k, masked j) pair to B' row k's
// column table instead.
constexpr int MSPLIT = 32;  // (the part index takes 5 bits of a list word)
constexpr int MIN_SLICE = 64;
constexpr int MASK_GRID = 8192;

__device__ inline int32_t n_parts(int32_t al) { return min(MSPLIT, max(1, (al + MIN_SLICE - 1) / MIN_SLICE)); }

// parts per mask row: none when no term can reach it
__global__ void k_part_counts(Mask M, const uint64_t* rbits, RowsView A, int64_t nrow, int64_t* cnt) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrow) return;
  const int64_t len = M.start[r + 1] - M.start[r];
  const uint64_t R = rbits ? rbits[r] : ~0ull;
  const int32_t al = A.len[M.row[r]];
  cnt[r] = (len == 0 || R == 0 || al == 0) ? 0 : n_parts(al);
}

__global__ void k_part_items(const int64_t* cnt, const int64_t* off, int64_t nrow, int64_t* items) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrow) return;
  for (int64_t y = 0; y < cnt[r]; ++y) items[off[r] + y] = (r << 5) | y;
}

template <int SR>
__global__ __launch_bounds__(MW) void k_masked(MaskedArgs P, const int64_t* items, const int64_t* d_nitems) {
  using S = Sem<SR>;
  using V = typename S::V;
  using Acc = typename S::Acc;
  __shared__ int32_t hk[MSLOTS];
  __shared__ int32_t hv[MSLOTS];
  __shared__ unsigned long long cnt[2];
  __shared__ unsigned long long pre[2];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  Acc* z = (Acc*)P.z;
  const int64_t ni = *d_nitems;
  unsigned long long sum_kept = 0, sum_tried = 0, n_walk = 0, n_probe = 0;  // (thread 0)
  for (int64_t it = blockIdx.x; it < ni; it += gridDim.x) {
    const int64_t w = items[it];
    const int64_t r = w >> 5;
    const int32_t part = (int32_t)(w & 31);
    const int32_t i = P.M.row[r];
    const int64_t s0 = P.M.start[r], s1 = P.M.start[r + 1];
    const int32_t len = (int32_t)(s1 - s0);
    const uint64_t R = P.rbits ? P.rbits[r] : ~0ull;
    const int64_t ao = P.A.off[i];
    const int32_t al = P.A.len[i];
    // this part [t0, t1) of A' row i
    const int32_t np = n_parts(al);
    const int32_t t0 = (int32_t)((int64_t)al * part / np);
    const int32_t t1 = (int32_t)((int64_t)al * (part + 1) / np);
    if (threadIdx.x < 2) {
      cnt[threadIdx.x] = 0;
      pre[threadIdx.x] = 0;
    }
    __syncthreads();
    bool probe = false;
    if (P.XB.tab) {
      // the walk's length: the rows of B' the part's kept k name
      unsigned long long nk = 0, walk = 0;
      for (int32_t t = t0 + threadIdx.x; t < t1; t += MW) {
        const int32_t k = P.A.col[ao + t];
        if (R & bloom_bit(k)) {
          ++nk;
          walk += (unsigned long long)P.B.len[k];
        }
      }
      for (int d = 32; d > 0; d >>= 1) {
        nk += __shfl_xor(nk, d, 64);
        walk += __shfl_xor(walk, d, 64);
      }
      if (lane == 0) {
        atomicAdd(&pre[0], nk);
        atomicAdd(&pre[1], walk);
      }
      __syncthreads();
      probe = pre[0] * (unsigned long long)len * PROBE_COST < pre[1];
    }
    unsigned long long kept = 0, tried = 0;
    if (probe) {
      const int64_t npair = (int64_t)(t1 - t0) * len;
      for (int64_t q = threadIdx.x; q < npair; q += MW) {
        const int32_t t = t0 + (int32_t)(q / len);
        const int32_t e = (int32_t)(q - (int64_t)(t - t0) * len);
        const int32_t k = P.A.col[ao + t];
        if (!(R & bloom_bit(k))) continue;  // not in A^R
        kept += e == 0;
        ++tried;
        const int32_t pos = row_find(P.XB, P.B, k, P.M.col[s0 + e]);
        if (pos < 0) continue;  // no b'_kj
        const V a = ((const V*)P.A.val)[ao + t];
        S::atomic_combine(&z[s0 + e], S::mul(a, ((const V*)P.B.val)[P.B.off[k] + pos]));
        atomicOr(&P.h[s0 + e], (unsigned long long)bloom_bit(k));
      }
      for (int d = 32; d > 0; d >>= 1) {
        kept += __shfl_xor(kept, d, 64);
        tried += __shfl_xor(tried, d, 64);
      }
    } else {
      const bool tab = len <= MSLOTS / 2;
      if (tab) table_build(hk, hv, P.M.col, s0, len);
      for (int32_t t = t0 + wv; t < t1; t += MW / 64) {
        const int32_t k = P.A.col[ao + t];
        if (!(R & bloom_bit(k))) continue;  // not in A^R
        const V a = ((const V*)P.A.val)[ao + t];
        const int64_t bo = P.B.off[k];
        const int32_t bl = P.B.len[k];
        const unsigned long long bit = (unsigned long long)bloom_bit(k);
        ++kept;
        tried += (unsigned long long)bl;
        for (int32_t u = lane; u < bl; u += 64) {
          const int32_t j = P.B.col[bo + u];
          const int64_t e = tab ? (int64_t)table_find(hk, hv, j) : run_find(P.M.col, s0, s1, j) - s0;
          if (e < 0) continue;  // (i, j) is not in the mask
          S::atomic_combine(&z[s0 + e], S::mul(a, ((const V*)P.B.val)[bo + u]));
          atomicOr(&P.h[s0 + e], bit);
        }
      }
    }
    if (lane == 0) {
      atomicAdd(&cnt[0], kept);
      atomicAdd(&cnt[1], tried);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      sum_kept += cnt[0];
      sum_tried += cnt[1];
      if (probe) ++n_probe;
      else ++n_walk;
    }
    __syncthreads();  // the next part resets cnt and pre and rebuilds the table
  }
  if (threadIdx.x == 0 && (n_walk | n_probe)) {
    atomicAdd(&P.stats[0], sum_kept);
    atomicAdd(&P.stats[1], sum_tried);
    atomicAdd(&P.stats[2], n_walk);
    atomicAdd(&P.stats[3], n_probe);
  }
}

// fp64: the row's kept k sorted in LDS, then one k at a time in ascending
// order; the workgroup's lanes share B' row k, whose columns are distinct, so
// each masked entry takes its terms in ascending k without atomics.  Rows
// whose probes cost less give each masked entry one lane, which probes the
// kept k in ascending order.
__global__ __launch_bounds__(MW) void k_masked_f64(MaskedArgs P) {
  __shared__ int32_t hk[MSLOTS / 2];
  __shared__ int32_t hv[MSLOTS / 2];
  __shared__ uint64_t ks[FP64_KCAP];
  __shared__ int nk;
  __shared__ unsigned long long walk;
  const int64_t r = blockIdx.x;
  const int32_t i = P.M.row[r];
  const int64_t s0 = P.M.start[r], s1 = P.M.start[r + 1];
  const int32_t len = (int32_t)(s1 - s0);
  if (len == 0) return;
  const uint64_t R = P.rbits ? P.rbits[r] : ~0ull;
  if (R == 0) return;
  constexpr int SL = MSLOTS / 2;
  const bool tab = len <= SL / 2;
  if (threadIdx.x == 0) {
    nk = 0;
    walk = 0;
  }
  if (tab) {
    for (int x = threadIdx.x; x < SL; x += MW) hk[x] = -1;
    __syncthreads();
    for (int32_t t = threadIdx.x; t < len; t += MW) {
      const int32_t j = P.M.col[s0 + t];
      uint32_t h = hash_col(j) & (SL - 1);
      while (atomicCAS(&hk[h], -1, j) != -1) h = (h + 1) & (SL - 1);
      hv[h] = t;
    }
  }
  __syncthreads();
  const int64_t ao = P.A.off[i];
  const int32_t al = P.A.len[i];
  unsigned long long wl = 0;
  for (int32_t t = threadIdx.x; t < al; t += MW) {
    const int32_t k = P.A.col[ao + t];
    if (R & bloom_bit(k)) {
      const int q = atomicAdd(&nk, 1);
      if (q < FP64_KCAP) ks[q] = ((uint64_t)(uint32_t)k << 32) | (uint32_t)t;
      wl += (unsigned long long)P.B.len[k];
    }
  }
  for (int d = 32; d > 0; d >>= 1) wl += __shfl_xor(wl, d, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(&walk, wl);
  __syncthreads();
  const int n = nk;
  if (n > FP64_KCAP) {
    if (threadIdx.x == 0) atomicOr(P.err, 16);
    return;
  }
  const bool probe = P.XB.tab && (unsigned long long)n * (unsigned long long)len * PROBE_COST < walk;
  int np2 = 1;
  while (np2 < n) np2 <<= 1;
  for (int x = n + threadIdx.x; x < np2; x += MW) ks[x] = ~0ull;
  __syncthreads();
  // bitonic sort by k (k unique within a row)
  for (int size = 2; size <= np2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int x = threadIdx.x; x < np2; x += MW) {
        const int y = x ^ stride;
        if (y > x) {
          const bool up = (x & size) == 0;
          const uint64_t a = ks[x], b = ks[y];
          if ((a > b) == up) {
            ks[x] = b;
            ks[y] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  double* z = (double*)P.z;
  if (probe) {
    for (int32_t e = threadIdx.x; e < len; e += MW) {
      const int32_t j = P.M.col[s0 + e];
      double acc = 0.0;
      unsigned long long hb = 0;
      for (int q = 0; q < n; ++q) {
        const int32_t k = (int32_t)(ks[q] >> 32);
        const int32_t pos = row_find(P.XB, P.B, k, j);
        if (pos < 0) continue;
        const int32_t t = (int32_t)(uint32_t)ks[q];
        const double p = __dmul_rn(((const double*)P.A.val)[ao + t], ((const double*)P.B.val)[P.B.off[k] + pos]);
        acc = hb ? __dadd_rn(acc, p) : p;  // the first term as it is, then ascending k
        hb |= (unsigned long long)bloom_bit(k);
      }
      if (hb) {
        z[s0 + e] = acc;
        P.h[s0 + e] = hb;
      }
    }
    if (threadIdx.x == 0) {
      atomicAdd(&P.stats[0], (unsigned long long)n);
      atomicAdd(&P.stats[1], (unsigned long long)n * (unsigned long long)len);
      atomicAdd(&P.stats[3], 1ull);
    }
    return;
  }
  unsigned long long tried = 0;
  for (int q = 0; q < n; ++q) {
    const int32_t k = (int32_t)(ks[q] >> 32);
    const int32_t t = (int32_t)(uint32_t)ks[q];
    const double a = ((const double*)P.A.val)[ao + t];
    const int64_t bo = P.B.off[k];
    const int32_t bl = P.B.len[k];
    tried += (unsigned long long)bl;
    for (int32_t u = threadIdx.x; u < bl; u += MW) {
      const int32_t j = P.B.col[bo + u];
      int64_t e;
      if (tab) {
        uint32_t h = hash_col(j) & (SL - 1);
        e = -1;
        for (;;) {
          const int32_t x = hk[h];
          if (x == j) {
            e = hv[h];
            break;
          }
          if (x == -1) break;
          h = (h + 1) & (SL - 1);
        }
      } else {
        e = run_find(P.M.col, s0, s1, j);
        if (e >= 0) e -= s0;
      }
      if (e < 0) continue;
      const double p = __dmul_rn(a, ((const double*)P.B.val)[bo + u]);
      const int64_t x = s0 + e;
      z[x] = P.h[x] ? __dadd_rn(z[x], p) : p;  // the first term as it is, then ascending k
      P.h[x] |= (unsigned long long)bloom_bit(k);
    }
    __threadfence_block();
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&P.stats[0], (unsigned long long)n);
    atomicAdd(&P.stats[1], tried);
    atomicAdd(&P.stats[2], 1ull);
  }
}

// The merge batches: SET (i, j, z) where a term exists, DELETE where none
// does; the accumulator words become values in place.
template <int SR>
__global__ void k_merge_batch(const uint64_t* cs_key, int64_t n, int cb, void* z, const unsigned long long* h,
                              int32_t* rows, int32_t* cols, uint8_t* ops) {
  using S = Sem<SR>;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  rows[e] = (int32_t)(cs_key[e] >> cb);
  cols[e] = (int32_t)(cs_key[e] & ((1ull << cb) - 1));
  ops[e] = h[e] ? (uint8_t)DSG_OP_SET : (uint8_t)DSG_OP_DELETE;
  typename S::Acc x = ((typename S::Acc*)z)[e];
  ((typename S::V*)z)[e] = S::from_acc(x);
}

__global__ void k_copy_u32(const uint32_t* src, uint32_t* dst) { *dst = *src; }

__global__ void k_rows_after(int32_t n, const uint32_t* epoch, const uint32_t* since, uint8_t* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flags[i] = epoch[i] > *since ? 1 : 0;
}

__global__ void k_set_sync2(uint32_t* sync, const uint32_t* ea, const uint32_t* eb) {
  sync[0] = *ea;
  sync[1] = *eb;
}

__global__ void k_zero_n(unsigned long long* p, int n) {
  for (int x = threadIdx.x; x < n; x += blockDim.x) p[x] = 0ull;
}

// the mask of a whole matrix in canonical form: every row, its sorted columns
__global__ void k_iota_i32(int32_t* p, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = (int32_t)t;
}

void* ensure_gws(DProd* p, size_t bytes) {
  if (bytes <= p->gws_bytes) return p->gws;
  Ctx* c = p->ctx;
  DSG_HIP(hipStreamSynchronize(c->stream));
  ctx_free(c, p->gws, p->gws_bytes);
  p->gws = nullptr;
  p->gws_bytes = 0;
  const size_t nb = bytes + bytes / 4 + (1 << 20);
  p->gws = ctx_alloc(c, nb);
  p->gws_bytes = nb;
  return p->gws;
}

int64_t read_i64(Ctx* c, const int64_t* d) {
  int64_t* h = (int64_t*)((char*)c->pinned + 3072);
  DSG_HIP(hipMemcpyAsync(h, d, 8, hipMemcpyDeviceToHost, c->stream));
  DSG_HIP(hipStreamSynchronize(c->stream));
  return *h;
}

// Z and H over a mask (z / h filled here first).  bits_only: only h is
// wanted (F from scratch), so fp64 too takes the kernel that combines in any
// order (its z is then left meaningless).
void launch_masked(DProd* p, const Mask& M, int64_t nrow, int64_t nmask, const uint64_t* rbits, void* z,
                   unsigned long long* h, unsigned long long* stats, int* err, const RowIx& XB = RowIx(),
                   bool bits_only = false) {
  Ctx* c = p->ctx;
  hipStream_t s = c->stream;
  const int sr = p->C->sr;
  const unsigned fb = blocks_for(std::max<int64_t>(nmask, 1), 256);
  switch (sr) {
    case 0: hipLaunchKernelGGL(k_fill_acc<unsigned long long>, dim3(fb), dim3(256), 0, s, (unsigned long long*)z, h, nmask, 0ull); break;
    case 1: hipLaunchKernelGGL(k_fill_acc<uint32_t>, dim3(fb), dim3(256), 0, s, (uint32_t*)z, h, nmask, 0xffffffffu); break;
    case 2: hipLaunchKernelGGL(k_fill_acc<double>, dim3(fb), dim3(256), 0, s, (double*)z, h, nmask, 0.0); break;
    default: hipLaunchKernelGGL(k_fill_acc<uint32_t>, dim3(fb), dim3(256), 0, s, (uint32_t*)z, h, nmask, 0u); break;
  }
  if (nrow == 0) return;
  MaskedArgs P;
  P.M = M;
  P.rbits = rbits;
  P.A = rows_of(p->A);
  P.B = rows_of(p->B);
  P.XB = XB;
  P.z = z;
  P.h = h;
  P.stats = stats;
  P.err = err;
  if (sr == 2 && !bits_only) {
    // fp64 keeps a row whole (its terms in ascending k)
    hipLaunchKernelGGL(k_masked_f64, dim3((unsigned)nrow), dim3(MW), 0, s, P);
    DSG_HIP(hipGetLastError());
    return;
  }
  // the list of parts (in the context's scratch, free while this runs)
  const size_t pb = Carve::need({(size_t)nrow * 8, (size_t)nrow * 8, (size_t)nrow * MSPLIT * 8,
                                 scan_scratch_bytes(nrow) + 64, 64});
  Carve cv(ctx_scratch(c, pb), pb);
  int64_t* pcnt = cv.take<int64_t>(nrow);
  int64_t* poff = cv.take<int64_t>(nrow);
  int64_t* items = cv.take<int64_t>(nrow * MSPLIT);
  void* pscan = cv.take<char>(scan_scratch_bytes(nrow) + 64);
  int64_t* d_nitems = cv.take<int64_t>(8);
  const unsigned rb = blocks_for(nrow, 256);
  hipLaunchKernelGGL(k_part_counts, dim3(rb), dim3(256), 0, s, M, rbits, P.A, nrow, pcnt);
  exclusive_scan_i64(pcnt, poff, nrow, d_nitems, pscan, s);
  hipLaunchKernelGGL(k_part_items, dim3(rb), dim3(256), 0, s, (const int64_t*)pcnt, (const int64_t*)poff, nrow, items);
  const dim3 g((unsigned)std::min<int64_t>(nrow * MSPLIT, MASK_GRID));
  const int64_t* it = items;
  const int64_t* ni = d_nitems;
  switch (sr) {
    case 0:
    case 2: hipLaunchKernelGGL(k_masked<0>, g, dim3(MW), 0, s, P, it, ni); break;  // (fp64: bits only, 8-byte words)
    case 1: hipLaunchKernelGGL(k_masked<1>, g, dim3(MW), 0, s, P, it, ni); break;
    default: hipLaunchKernelGGL(k_masked<3>, g, dim3(MW), 0, s, P, it, ni); break;
  }
  DSG_HIP(hipGetLastError());
}

// The masked product's flags: 16 when an fp64 row kept more columns of A'
// than its ascending-k sum takes (FP64_KCAP); anything else is an internal
// error.
int read_err(Ctx* c, const int* d_err) {
  int* h = (int*)((char*)c->pinned + 3328);
  DSG_HIP(hipMemcpyAsync(h, d_err, 4, hipMemcpyDeviceToHost, c->stream));
  DSG_HIP(hipStreamSynchronize(c->stream));
  DSG_REQUIRE((h[0] & ~16) == 0, DSG_E_DEVICE, "internal: masked product error " + std::to_string(h[0]));
  return h[0];
}

// op(X)'s log since the product last saw X: the log of X's last apply in
// op(X)'s coordinates (X's own, or its transpose index's), or nothing when X
// was not applied since.
bool fresh_log(const OpView& v) { return unchanged(v) || changed_once(v); }

LogView log_since(const OpView& v) {
  LogView L{v.logm->log_key, v.logm->log_code, unchanged(v) ? 0 : v.logm->h_log_n, bits_for(v.logm->ncols)};
  return L;
}

}  // namespace

bool general_eligible(const DProd* p) {
  if (!p->F) return false;
  return fresh_log(op_view(p, true)) && fresh_log(op_view(p, false));
}

// F from scratch: the masked product over C's whole structure with every k
// kept.  Its values z equal C's (the same sums in the same order); only the
// bits are kept.
void bloom_build(DProd* p) {
  Ctx* c = p->ctx;
  hipStream_t s = c->stream;
  DMat* C = p->C;
  const int32_t n = C->nrows;
  const int64_t N = std::max<int32_t>(n, 1);
  // C in canonical form: row pointers first, for the entry count
  int64_t* rp0 = (int64_t*)ensure_gws(p, (size_t)(N + 1) * 8 + 4096);
  mat_export_device(C, rp0, nullptr, nullptr, nullptr, s);
  const int64_t nnz = n > 0 ? read_i64(c, rp0 + n) : 0;
  const int64_t NZ = std::max<int64_t>(nnz, 1);
  const size_t need = Carve::need({(size_t)(N + 1) * 8, (size_t)N * 4, (size_t)NZ * 4, (size_t)NZ * 8, (size_t)NZ * 8,
                                   (size_t)NZ * 8, 64, 64});
  Carve cv(ensure_gws(p, need), need);
  int64_t* rp = cv.take<int64_t>(N + 1);
  int32_t* rid = cv.take<int32_t>(N);
  int32_t* col = cv.take<int32_t>(NZ);
  void* val = cv.take<uint64_t>(NZ);
  void* z = cv.take<uint64_t>(NZ);
  unsigned long long* h = cv.take<unsigned long long>(NZ);
  unsigned long long* stats = cv.take<unsigned long long>(8);
  int* err = cv.take<int>(16);
  mat_export_device(C, rp, nnz > 0 ? col : nullptr, nnz > 0 ? val : nullptr, nullptr, s);
  hipLaunchKernelGGL(k_zero_n, dim3(1), dim3(64), 0, s, stats, 8);
  hipLaunchKernelGGL(k_zero_n, dim3(1), dim3(64), 0, s, (unsigned long long*)err, 8);
  if (n > 0) hipLaunchKernelGGL(k_iota_i32, dim3(blocks_for(n, 256)), dim3(256), 0, s, rid, (int64_t)n);
  Mask M{rid, rp, col};
  if (nnz > 0) launch_masked(p, M, n, nnz, nullptr, z, h, stats, err, RowIx(), true);
  (void)read_err(c, err);
  DMat* F = mat_create(c, n, C->ncols, 0, rp, col, h);
  if (p->F) mat_destroy(p->F);
  p->F = F;
}

int32_t general_update(DProd* p) {
  Ctx* c = p->ctx;
  hipStream_t s = c->stream;
  DMat* A = p->A;
  DMat* B = p->B;
  DMat* C = p->C;
  const OpView l = op_view(p, true), r = op_view(p, false);
  DMat* T = l.cols;  // columns of op(A)' as rows
  DSG_REQUIRE(T && p->F, DSG_E_STATE, "internal: Bloom product without transpose index or F");
  // C and F take per-row column indexes, which the merges (ordinary applies)
  // keep current: the merges then place their entries by lookup, and R finds
  // f_ij by lookup where that is cheaper; B takes one for the masked
  // product's probes.  Where C's rows are short (under IX_MIN_ROW slots on
  // average) streaming and walking rows cost less than keeping the tables,
  // and they go without (B keeps an index some other path gave it).
  constexpr int64_t IX_MIN_ROW = 128;
  const bool long_rows = C->h_top_ub >= IX_MIN_ROW * (int64_t)C->nrows;
  if (c->tuning.row_index && long_rows) {
    mat_index_enable(C);
    mat_index_enable(p->F);
  }
  const int32_t n = C->nrows;
  const int cb = bits_for(C->ncols);
  const int rb = bits_for(n);
  dsg_update_stats& st = p->stats;
  st = dsg_update_stats{};
  st.path = 2;
  const LogView LA = log_since(l);
  const LogView LB = A == B ? LA : log_since(r);
  const int64_t nL = LA.n + LB.n;

  // ---- computePattern: count and write the terms ----
  // (the counts and offsets live in the context's second scratch, which
  // nothing else takes before the terms are written; the product's own
  // workspace is sized from their total)
  const size_t head_b = Carve::need({(size_t)(nL + 1) * 8, (size_t)(nL + 1) * 8, scan_scratch_bytes(nL + 1) + 64, 64});
  Carve ch(ctx_scratch2(c, head_b), head_b);
  int64_t* cnt = ch.take<int64_t>(nL + 1);
  int64_t* off = ch.take<int64_t>(nL + 1);
  void* scan1 = ch.take<char>(scan_scratch_bytes(nL + 1) + 64);
  int64_t* d_total = ch.take<int64_t>(8);
  int64_t nterm = 0;
  if (nL > 0) {
    hipLaunchKernelGGL(k_pat_counts, dim3(blocks_for(nL, 256)), dim3(256), 0, s, LA, LB, (const int32_t*)B->row_len,
                       (const int32_t*)T->row_len, cnt);
    exclusive_scan_i64(cnt, off, nL, d_total, scan1, s);
    nterm = read_i64(c, d_total);
  }
  st.terms = nterm;
  const int64_t NT = std::max<int64_t>(nterm, 1);
  // workspace: terms (keys, sort, heads), then C*, its rows, Z, H and the merge batch
  const size_t terms_b = Carve::need({(size_t)NT * 8, (size_t)NT * 4, radix_scratch_bytes(NT), (size_t)NT * 8,
                                      (size_t)NT * 8, scan_scratch_bytes(NT) + 64, 64});
  const size_t cs_b = Carve::need({(size_t)NT * 8, (size_t)NT * 8, (size_t)NT * 4, (size_t)NT * 8, (size_t)NT * 8,
                                   (size_t)NT * 4, (size_t)(NT + 1) * 8, (size_t)NT * 8, (size_t)NT * 8, (size_t)NT * 8,
                                   (size_t)NT * 4, (size_t)NT * 4, (size_t)NT, 64, 64,
                                   (size_t)std::max<int32_t>(n, 1) + 64,
                                   compact_scratch_bytes(std::max<int32_t>(n, 1)) + 64, 64});
  char* base = (char*)ensure_gws(p, terms_b + cs_b);
  Carve ct(base, terms_b);
  uint64_t* keys = ct.take<uint64_t>(NT);
  uint32_t* idx = ct.take<uint32_t>(NT);
  void* rscr = ct.take<char>(radix_scratch_bytes(NT));
  int64_t* head = ct.take<int64_t>(NT);
  int64_t* segid = ct.take<int64_t>(NT);
  void* scan2 = ct.take<char>(scan_scratch_bytes(NT) + 64);
  Carve cs(base + terms_b, cs_b);
  uint64_t* cs_key = cs.take<uint64_t>(NT);
  unsigned long long* fstar = cs.take<unsigned long long>(NT);
  int32_t* cs_col = cs.take<int32_t>(NT);
  int64_t* rhead = cs.take<int64_t>(NT);
  int64_t* rid = cs.take<int64_t>(NT);
  int32_t* row_id = cs.take<int32_t>(NT);
  int64_t* row_start = cs.take<int64_t>(NT + 1);
  uint64_t* rbits = cs.take<uint64_t>(NT);
  void* z = cs.take<uint64_t>(NT);
  unsigned long long* h = cs.take<unsigned long long>(NT);
  int32_t* mrows = cs.take<int32_t>(NT);
  int32_t* mcols = cs.take<int32_t>(NT);
  uint8_t* mops = cs.take<uint8_t>(NT);
  unsigned long long* stats = cs.take<unsigned long long>(8);
  int* err = cs.take<int>(16);
  uint8_t* rflags = cs.take<uint8_t>((size_t)std::max<int32_t>(n, 1) + 64);
  void* cscr = cs.take<char>(compact_scratch_bytes(std::max<int32_t>(n, 1)) + 64);
  uint32_t* ep_before = (uint32_t*)cs.take<uint64_t>(8);
  hipLaunchKernelGGL(k_zero_n, dim3(1), dim3(64), 0, s, stats, 8);
  hipLaunchKernelGGL(k_zero_n, dim3(1), dim3(64), 0, s, (unsigned long long*)err, 8);
  hipLaunchKernelGGL(k_copy_u32, dim3(1), dim3(1), 0, s, (const uint32_t*)C->d_epoch, ep_before);

  int64_t ncs = 0, nrow = 0;
  if (nterm > 0) {
    hipLaunchKernelGGL(k_pat_write, dim3(blocks_for(nL * 64, 256)), dim3(256), 0, s, LA, LB, rows_of(B), rows_of(T),
                       (const int64_t*)off, cb, keys);
    hipLaunchKernelGGL(k_iota_u32, dim3(blocks_for(nterm, 256)), dim3(256), 0, s, idx, nterm);
    radix_sort_pairs(keys, idx, nterm, rb + cb + 6, rscr, s, err);
    // C* and F*
    hipLaunchKernelGGL(k_pat_heads, dim3(blocks_for(nterm, 256)), dim3(256), 0, s, keys, nterm, head);
    // (the entry count stays on the device until the rows are counted too:
    // one round trip for both; grids over the terms, an upper bound)
    int64_t* d_ncs = d_total;
    int64_t* d_nrow = d_total + 1;
    exclusive_scan_i64(head, segid, nterm, d_ncs, scan2, s);
    hipLaunchKernelGGL(k_fill_acc<uint64_t>, dim3(blocks_for(nterm, 256)), dim3(256), 0, s, (uint64_t*)cs_key,
                       fstar, nterm, 0ull);
    hipLaunchKernelGGL(k_pat_reduce, dim3(blocks_for(nterm, 256)), dim3(256), 0, s, keys, nterm,
                       (const int64_t*)head, (const int64_t*)segid, cs_key, fstar);
    // the rows of C*
    hipLaunchKernelGGL(k_cs_rows_heads, dim3(blocks_for(nterm, 256)), dim3(256), 0, s, (const uint64_t*)cs_key,
                       (const int64_t*)d_ncs, nterm, cb, cs_col, rhead);
    exclusive_scan_i64(rhead, rid, nterm, d_nrow, scan2, s);
    hipLaunchKernelGGL(k_cs_rows, dim3(blocks_for(nterm, 256)), dim3(256), 0, s, (const uint64_t*)cs_key,
                       (const int64_t*)d_ncs, cb, (const int64_t*)rhead, (const int64_t*)rid, row_id, row_start);
    int64_t* hn = (int64_t*)((char*)c->pinned + 3072);
    DSG_HIP(hipMemcpyAsync(hn, d_total, 16, hipMemcpyDeviceToHost, s));
    DSG_HIP(hipStreamSynchronize(s));
    ncs = hn[0];
    nrow = hn[1];
  }
  st.entries = ncs;
  st.affected_rows = nrow;
  const Mask M{row_id, row_start, cs_col};
  RowIx XB;
  if (nrow > 0) {
    // E and R
    RowIx XF;
    if (p->F->ix_tab) {
      mat_index_build(p->F, nullptr, nullptr, p->F->nrows);
      XF = mat_index_view(p->F);
    }
    hipLaunchKernelGGL(k_row_filter, dim3((unsigned)nrow), dim3(MW), 0, s, M, (const unsigned long long*)fstar,
                       rows_of(p->F), XF, rbits);
    // Z and H (rows with few masked entries probe B' through its column
    // index: every row's table made usable first)
    if (c->tuning.row_index && (B->ix_tab || (long_rows && mat_index_enable(B)))) {
      mat_index_build(B, nullptr, nullptr, B->nrows);
      XB = mat_index_view(B);
    }
    launch_masked(p, M, nrow, ncs, rbits, z, h, stats, err, XB);
    if (read_err(c, err) & 16) {
      // an fp64 row kept more columns of A' than its ascending-k sum takes:
      // nothing is merged; the row path brings C up to date and F is built
      // again, as after several applies
      p->bloom = false;
      int32_t nchg = 0;
      try {
        nchg = prod_run(p, 0, false);
      } catch (...) {
        p->bloom = true;
        throw;
      }
      p->bloom = true;
      bloom_build(p);
      return nchg;
    }
    // the merges, masked at C*
    const unsigned gb = blocks_for(ncs, 256);
    switch (C->sr) {
      case 0: hipLaunchKernelGGL(k_merge_batch<0>, dim3(gb), dim3(256), 0, s, cs_key, ncs, cb, z, h, mrows, mcols, mops); break;
      case 1: hipLaunchKernelGGL(k_merge_batch<1>, dim3(gb), dim3(256), 0, s, cs_key, ncs, cb, z, h, mrows, mcols, mops); break;
      case 2: hipLaunchKernelGGL(k_merge_batch<2>, dim3(gb), dim3(256), 0, s, cs_key, ncs, cb, z, h, mrows, mcols, mops); break;
      default: hipLaunchKernelGGL(k_merge_batch<3>, dim3(gb), dim3(256), 0, s, cs_key, ncs, cb, z, h, mrows, mcols, mops); break;
    }
    DSG_HIP(hipGetLastError());
    mat_apply_device(C, mrows, mcols, z, mops, ncs);
    mat_apply_device(p->F, mrows, mcols, h, mops, ncs);
  }
  // ---- rows whose stored content changed; C reflects A's and B's epochs ----
  if (p->changed_cap < n) {
    ctx_free(c, p->changed_rows, (size_t)p->changed_cap * 4);
    p->changed_rows = nullptr;
    p->changed_cap = 0;
    p->changed_rows = (int32_t*)ctx_alloc(c, (size_t)std::max<int32_t>(n, 1024) * 4);
    p->changed_cap = std::max<int32_t>(n, 1024);
  }
  int32_t* d_nchg = (int32_t*)(stats + 4);
  if (n > 0) {
    hipLaunchKernelGGL(k_rows_after, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, (const uint32_t*)C->row_epoch,
                       (const uint32_t*)ep_before, rflags);
    compact_flags(rflags, n, p->changed_rows, d_nchg, cscr, s);
  }
  hipLaunchKernelGGL(k_set_sync2, dim3(1), dim3(1), 0, s, p->d_sync, (const uint32_t*)A->d_epoch,
                     (const uint32_t*)B->d_epoch);
  struct Tail {
    unsigned long long st[4];
    unsigned long long ix_top[3];  // index pool tops of B, C and F
    int32_t nchg;
  };
  Tail* ht = (Tail*)((char*)c->pinned + 3072);
  ht->nchg = 0;
  DSG_HIP(hipMemcpyAsync(ht->st, stats, 32, hipMemcpyDeviceToHost, s));
  if (n > 0) DSG_HIP(hipMemcpyAsync(&ht->nchg, d_nchg, 4, hipMemcpyDeviceToHost, s));
  DMat* ixm[3] = {XB.tab ? B : nullptr, C, p->F};
  for (int q = 0; q < 3; ++q)
    if (ixm[q] && ixm[q]->ix_tab) DSG_HIP(hipMemcpyAsync(&ht->ix_top[q], ixm[q]->ix_top, 8, hipMemcpyDeviceToHost, s));
  DSG_HIP(hipStreamSynchronize(s));
  for (int q = 0; q < 3; ++q)
    if (ixm[q] && ixm[q]->ix_tab) mat_index_note_top(ixm[q], ht->ix_top[q]);
  st.a_entries = (int64_t)ht->st[0];
  st.flops = (int64_t)ht->st[1];
  st.bin_rows[0] = (int64_t)ht->st[2];
  st.bin_rows[1] = (int64_t)ht->st[3];
  st.changed_rows = ht->nchg;
  return ht->nchg;
}
