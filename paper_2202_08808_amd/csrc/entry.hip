// Entry-granular dynamic update of C = A*A over (min,+) fp32 and (+,x) int64.
//
// Section 5 writes the new product as the old one combined with the products
// that involve changed entries (Eq. 1), and observes that C can change only
// where that change pattern is non-zero.  The row path recomputes every row
// the pattern reaches.  This path works one level finer: it lists every
// product a_ik * a_kj the last batch changed, with its value before and after,
// and folds those values into the stored entries of C.
//
//   (+,x) int64   c' = c + sum(new - old) over the entry's changed products
//                 (two's-complement ring, so the subtraction is exact).  An
//                 entry that lost a contributing product may vanish and is
//                 recomputed.
//   (min,+)       c' = min(c, min over the changed products' new values),
//                 unless a product that got worse (or vanished) held the old
//                 minimum and no new value reaches it.  Then the entry is
//                 recomputed.  Using the stored minimum as a witness this way
//                 is this library's addition.
//
// A recomputed entry takes the minimum (or sum) of a'_ik * a'_kj over k.  A'
// row i goes into an LDS hash; column j of A' is read from the valued
// transpose.
//
// Steps (all on the device, a few host reads of counts in between):
//   1. per changed entry (r, c) of A, count its products: as a left factor
//      (i = r, k = c) over row c of A' plus row c's deleted entries, and as a
//      right factor (k = r, j = c) over column r of A' (rows i whose entry
//      (i, r) did not change -- the others are covered as left factors);
//   2. write the products (key i<<bits | j, old value, new value, presence);
//   3. sort them by key, and reduce each key to one ADD update of C
//      (min or sum of the changes), with a guard for the witness test;
//   4. apply those updates to C in place (ingest.hip: mat_apply_sorted_add),
//      which lists the lost entries with their slots;
//   5. recompute the lost entries; entries left without any product are
//      deleted;
//   6. report the rows whose stored content changed (row epochs of C).
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

constexpr uint8_t F_OLD = 1, F_NEW = 2;

struct Log {
  const uint64_t* key;
  const uint64_t* old;
  const uint64_t* nw;
  const uint8_t* code;
  int64_t n;
};

struct Mat {
  const int64_t* off;
  const int32_t* len;
  const int32_t* col;
  const void* val;
};

Mat view(const DMat* m) { return Mat{m->row_off, m->row_len, m->col, m->val}; }

template <class V>
__device__ inline V rawv(uint64_t r) {
  if constexpr (sizeof(V) == 8) return __builtin_bit_cast(V, r);
  else return __builtin_bit_cast(V, (uint32_t)r);
}

template <class V>
__device__ inline V ldv(const void* p, int64_t i) {
  return ((const V*)p)[i];
}

// first log index with key >= k
__device__ inline int64_t log_lower(const uint64_t* key, int64_t n, uint64_t k) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (key[mid] < k) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// index of key k in the sorted log range [lo, hi), or -1
__device__ inline int64_t log_index(const uint64_t* key, int64_t lo, int64_t hi, uint64_t k) {
  const int64_t end = hi;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (key[mid] < k) lo = mid + 1;
    else hi = mid;
  }
  return (lo < end && key[lo] == k) ? lo : -1;
}

// ---- 1. product counts per changed entry ----
__global__ void k_term_counts(Log L, int cbits, const int32_t* a_len, const int32_t* t_len, int64_t* cnt) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= L.n) return;
  int64_t c = 0;
  if (L.code[u] != UPD_NOP && L.code[u] != UPD_LOST) {
    const uint64_t cmask = (1ull << cbits) - 1;
    const int32_t r = (int32_t)(L.key[u] >> cbits), col = (int32_t)(L.key[u] & cmask);
    // left factor: row col of A', plus its deleted entries
    const uint64_t k0 = (uint64_t)col << cbits;
    int64_t e = log_lower(L.key, L.n, k0);
    int64_t ndel = 0;
    for (; e < L.n && (L.key[e] >> cbits) == (uint64_t)col; ++e) ndel += L.code[e] == UPD_DEL;
    c = (int64_t)a_len[col] + ndel + (int64_t)t_len[r];
  }
  cnt[u] = c;
}

// ---- 2. write the products: one wavefront per changed entry ----
template <int SR>
__global__ __launch_bounds__(256) void k_term_write(Log L, int cbits, Mat A, Mat T, const int64_t* base,
                                                    uint64_t* tkey, uint64_t* told, uint64_t* tnew, uint8_t* tfl,
                                                    uint64_t sentinel) {
  using S = Sem<SR>;
  using V = typename S::V;
  const int64_t u = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (u >= L.n) return;
  const uint8_t code = L.code[u];
  if (code == UPD_NOP || code == UPD_LOST) return;
  const uint64_t cmask = (1ull << cbits) - 1;
  const uint64_t dk = L.key[u];
  const int32_t r = (int32_t)(dk >> cbits), c = (int32_t)(dk & cmask);
  const bool op = code != UPD_INS, np = code != UPD_DEL;  // entry present before / after
  const V vo = rawv<V>(L.old[u]), vn = rawv<V>(L.nw[u]);
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  int64_t o = base[u];
  // left factor (i = r, k = c): products a_rc * a_cj
  const int64_t lo = log_lower(L.key, L.n, (uint64_t)c << cbits);
  const int64_t hi = log_lower(L.key, L.n, ((uint64_t)c + 1) << cbits);
  const int64_t ac = A.off[c];
  const int32_t al = A.len[c];
  for (int32_t t = lane; t < al; t += 64) {
    const int32_t j = A.col[ac + t];
    const V bn = ldv<V>(A.val, ac + t);
    bool bop = true;
    V bo = bn;
    if (hi > lo) {
      const int64_t e = log_index(L.key, lo, hi, ((uint64_t)c << cbits) | (uint64_t)(uint32_t)j);
      if (e >= 0) {
        const uint8_t ce = L.code[e];
        if (ce == UPD_INS) bop = false;
        else if (ce == UPD_OVR) bo = rawv<V>(L.old[e]);
      }
    }
    const uint8_t f = (op && bop ? F_OLD : 0) | (np ? F_NEW : 0);
    tkey[o + t] = ((uint64_t)(uint32_t)r << cbits) | (uint64_t)(uint32_t)j;
    told[o + t] = (f & F_OLD) ? (uint64_t)S::mul(vo, bo) : 0ull;
    tnew[o + t] = (f & F_NEW) ? (uint64_t)S::mul(vn, bn) : 0ull;
    tfl[o + t] = f;
  }
  o += al;
  // entries (c, j) this batch deleted: a_rc * a_cj existed only before
  for (int64_t e0 = lo; e0 < hi; e0 += 64) {
    const int64_t e = e0 + lane;
    const bool del = e < hi && L.code[e] == UPD_DEL;
    const uint64_t b = __ballot(del);
    if (del) {
      const int64_t q = o + __popcll(b & lt);
      const int32_t j = (int32_t)(L.key[e] & cmask);
      tkey[q] = ((uint64_t)(uint32_t)r << cbits) | (uint64_t)(uint32_t)j;
      told[q] = op ? (uint64_t)S::mul(vo, rawv<V>(L.old[e])) : 0ull;
      tnew[q] = 0ull;
      tfl[q] = op ? F_OLD : 0;
    }
    o += __popcll(b);
  }
  // right factor (k = r, j = c): products a_ir * a_rc over column r of A'
  const int64_t tc = T.off[r];
  const int32_t tl = T.len[r];
  for (int32_t t = lane; t < tl; t += 64) {
    const int32_t i = T.col[tc + t];
    const V a = ldv<V>(T.val, tc + t);
    const int64_t e = log_index(L.key, 0, L.n, ((uint64_t)(uint32_t)i << cbits) | (uint64_t)(uint32_t)r);
    if (e >= 0 && L.code[e] != UPD_NOP) {
      // (i, r) changed too: that entry's left-factor products include this one
      tkey[o + t] = sentinel;
      tfl[o + t] = 0;
      continue;
    }
    const uint8_t f = (op ? F_OLD : 0) | (np ? F_NEW : 0);
    tkey[o + t] = ((uint64_t)(uint32_t)i << cbits) | (uint64_t)(uint32_t)c;
    told[o + t] = op ? (uint64_t)S::mul(a, vo) : 0ull;
    tnew[o + t] = np ? (uint64_t)S::mul(a, vn) : 0ull;
    tfl[o + t] = f;
  }
}

__global__ void k_iota_u32(uint32_t* p, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = (uint32_t)t;
}

// ---- 3. segments of equal keys ----
__global__ void k_seg_heads(const uint64_t* key, int64_t n, uint64_t sentinel, int cbits, int64_t* head,
                            unsigned long long* nrows) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool newrow = false;
  if (t < n) {
    const uint64_t k = key[t];
    const bool h = k != sentinel && (t == 0 || key[t - 1] != k);
    head[t] = h ? 1 : 0;
    newrow = h && (t == 0 || (key[t - 1] >> cbits) != (k >> cbits));
  }
  const int c = __syncthreads_count(newrow);  // one atomic per workgroup
  if (threadIdx.x == 0 && c) atomicAdd(nrows, (unsigned long long)c);
}

__global__ void k_seg_scatter(const uint64_t* key, int64_t n, uint64_t sentinel, const int64_t* head,
                              const int64_t* segid, const int64_t* d_nseg, int64_t* seg_start) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  if (head[t]) seg_start[segid[t]] = t;
  const bool valid = key[t] != sentinel;
  if (valid && (t + 1 == n || key[t + 1] == sentinel)) seg_start[*d_nseg] = t + 1;
}

// one thread per segment: fold the changed products of one entry of C
template <int SR>
__global__ void k_seg_reduce(const uint64_t* key, const uint32_t* idx, const uint64_t* told,
                             const uint64_t* tnew, const uint8_t* tfl, const int64_t* seg_start,
                             const int64_t* d_nseg, uint64_t* ckey, void* cval, uint64_t* cguard,
                             uint8_t* cflag) {
  using S = Sem<SR>;
  using V = typename S::V;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= *d_nseg) return;
  const int64_t t0 = seg_start[s], t1 = seg_start[s + 1];
  ckey[s] = key[t0];
  if constexpr (SR == 1) {
    // (min,+) over ordered keys
    uint32_t nmin = 0xffffffffu, wmin = 0xffffffffu;
    bool has_new = false, has_w = false;
    for (int64_t t = t0; t < t1; ++t) {
      const uint32_t q = idx[t];
      const uint8_t f = tfl[q];
      const uint32_t o = (uint32_t)told[q], w = (uint32_t)tnew[q];
      if (f & F_NEW) {
        has_new = true;
        nmin = min(nmin, w);
      }
      if ((f & F_OLD) && (!(f & F_NEW) || w > o)) {
        has_w = true;
        wmin = min(wmin, o);
      }
    }
    ((V*)cval)[s] = has_new ? f32_unkey(nmin) : 0.0f;
    cguard[s] = wmin;
    cflag[s] = (has_new ? 1 : 0) | (has_w ? 2 : 0);
  } else {
    // (+,x) int64: the sum of the changes; a vanished product makes the entry lost
    unsigned long long delta = 0;
    bool any = false, lost = false;
    for (int64_t t = t0; t < t1; ++t) {
      const uint32_t q = idx[t];
      const uint8_t f = tfl[q];
      if (f & F_NEW) delta += tnew[q];
      if (f & F_OLD) delta -= told[q];
      any = any || f != 0;
      lost = lost || ((f & F_OLD) && !(f & F_NEW));
    }
    ((V*)cval)[s] = (V)delta;
    cguard[s] = 0;
    cflag[s] = (any ? 1 : 0) | (lost ? 4 : 0);
  }
}

// ---- 5. lost entries ----
__global__ void k_lost_heads(const uint64_t* key, int64_t n, int cbits, int64_t* head) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) head[t] = (t == 0 || (key[t - 1] >> cbits) != (key[t] >> cbits)) ? 1 : 0;
}

// row segments of the sorted lost list, split by the length of A' row i
__global__ void k_lost_rows(const uint64_t* key, int64_t n, int cbits, const int64_t* head, const int64_t* rid,
                            const int64_t* d_nrow, int64_t* row_start, const int32_t* a_len, int32_t small_max,
                            uint8_t* is_small, uint8_t* is_big) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  if (head[t]) {
    const int64_t r = rid[t];
    row_start[r] = t;
    const int32_t d = a_len[(int32_t)(key[t] >> cbits)];
    is_small[r] = d <= small_max ? 1 : 0;
    is_big[r] = d <= small_max ? 0 : 1;
  }
  if (t == n - 1) row_start[*d_nrow] = n;
}

// A lost entry (i, j) is recomputed from the cheaper side: column j of A'
// (probing an LDS hash of A' row i), or A' row i (a binary search of j in the
// column-sorted copy of each row k).  Costs in probes: len(column j) against
// d_i searches of ~8 steps.
__device__ inline bool row_side(int32_t d, int32_t lj) { return (int64_t)d * 8 < (int64_t)lj; }

// work items: each row segment of lost entries in runs of epw entries
__global__ void k_item_counts(const int64_t* row_start, const int64_t* d_nrow, const uint8_t* is_small,
                              int32_t epw_small, int32_t epw_big, int64_t* cs, int64_t* cb) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= *d_nrow) return;
  const int64_t len = row_start[r + 1] - row_start[r];
  cs[r] = is_small[r] ? (len + epw_small - 1) / epw_small : 0;
  cb[r] = is_small[r] ? 0 : (len + epw_big - 1) / epw_big;
}

__global__ void k_item_fill(const int64_t* row_start, const int64_t* d_nrow, const uint8_t* is_small,
                            int32_t epw_small, int32_t epw_big, const int64_t* os, const int64_t* ob,
                            int32_t* srow, int32_t* spart, int32_t* brow, int32_t* bpart) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= *d_nrow) return;
  const int64_t len = row_start[r + 1] - row_start[r];
  const bool sm = is_small[r] != 0;
  const int32_t epw = sm ? epw_small : epw_big;
  const int64_t cnt = (len + epw - 1) / epw;
  const int64_t o = sm ? os[r] : ob[r];
  int32_t* ir = sm ? srow : brow;
  int32_t* ip = sm ? spart : bpart;
  for (int64_t q = 0; q < cnt; ++q) {
    ir[o + q] = (int32_t)r;
    ip[o + q] = (int32_t)q;
  }
}

struct LostArgs {
  const uint64_t* key;
  const int32_t* slot;
  const int64_t* row_start;
  const int32_t* item_row;   // work items of this launch: a row segment ...
  const int32_t* item_part;  // ... and which run of epw of its entries
  int32_t epw;
  int cbits;
  Mat A, T;
  int64_t* c_off;
  void* c_val;
  uint32_t* c_epoch;
  const uint32_t* c_cur_epoch;
  unsigned long long* part_acc;  // big rows: running result per lost entry
  uint32_t* part_hits;
  uint64_t* del_key;
  unsigned long long* ndel;
  int use_rowside;      // 0: every lost entry from the column side
  const int64_t* s_rp;  // column-sorted copy of A' (row side only)
  const int32_t* s_col;
  const void* s_val;
};

template <int SR>
__device__ inline unsigned long long acc_id() {
  return SR == 1 ? 0xffffffffull : 0ull;
}

template <int SR>
__device__ inline unsigned long long acc_comb(unsigned long long a, unsigned long long b) {
  if constexpr (SR == 1) return a < b ? a : b;
  else return a + b;
}

template <int SR>
__device__ inline unsigned long long wave_comb(unsigned long long x) {
  for (int d = 32; d > 0; d >>= 1) x = acc_comb<SR>(x, __shfl_xor(x, d, 64));
  return x;
}

__device__ inline uint32_t wave_sum(uint32_t x) {
  for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// LDS hash of the k's of A' row i (entries [k0, k1)): key k -> position in the row
template <int SLOTS>
__device__ inline void build_hash(int32_t* hk, int32_t* hp, const Mat& A, int64_t aoff, int32_t k0, int32_t k1,
                                  int tid, int nthr) {
  for (int x = tid; x < SLOTS; x += nthr) hk[x] = -1;
  __syncthreads();
  for (int32_t t = k0 + tid; t < k1; t += nthr) {
    const int32_t k = A.col[aoff + t];
    uint32_t h = hash_col(k) & (SLOTS - 1);
    while (atomicCAS(&hk[h], -1, k) != -1) h = (h + 1) & (SLOTS - 1);
    hp[h] = t;
  }
  __syncthreads();
}

template <int SLOTS>
__device__ inline int32_t probe(const int32_t* hk, const int32_t* hp, int32_t k) {
  uint32_t h = hash_col(k) & (SLOTS - 1);
  for (;;) {
    const int32_t x = hk[h];
    if (x == k) return hp[h];
    if (x == -1) return -1;
    h = (h + 1) & (SLOTS - 1);
  }
}

// a wavefront's share of one lost entry over the hashed part of A' row i
template <int SR, int SLOTS>
__device__ inline void column_pass(const LostArgs& L, const int32_t* hk, const int32_t* hp, int64_t aoff, int32_t j,
                                   unsigned long long& acc, uint32_t& hits, int lane) {
  using V = typename Sem<SR>::V;
  const int64_t toff = L.T.off[j];
  const int32_t tl = L.T.len[j];
  for (int32_t t = lane; t < tl; t += 64) {
    const int32_t k = L.T.col[toff + t];
    const int32_t pos = probe<SLOTS>(hk, hp, k);
    if (pos >= 0) {
      const V a = ldv<V>(L.A.val, aoff + pos), b = ldv<V>(L.T.val, toff + t);
      acc = acc_comb<SR>(acc, (unsigned long long)Sem<SR>::mul(a, b));
      ++hits;
    }
  }
}

// write the recomputed entry (lane 0): overwrite at its slot, or list it for deletion
template <int SR>
__device__ inline void finish_entry(const LostArgs& L, int64_t e, unsigned long long acc, uint32_t hits) {
  using S = Sem<SR>;
  using V = typename S::V;
  const uint64_t key = L.key[e];
  const int32_t i = (int32_t)(key >> L.cbits);
  if (hits > 0) {
    const V nv = S::from_acc((typename S::Acc)acc);
    const int64_t p = L.c_off[i] + L.slot[e];
    const V cur = ((V*)L.c_val)[p];
    if (!same_bits(cur, nv)) {
      ((V*)L.c_val)[p] = nv;
      L.c_epoch[i] = *L.c_cur_epoch;
    }
  } else {
    const unsigned long long q = atomicAdd(L.ndel, 1ull);
    L.del_key[q] = key;
  }
}

template <int SR>
__device__ inline unsigned long long group8_comb(unsigned long long x) {
  for (int d = 4; d > 0; d >>= 1) x = acc_comb<SR>(x, __shfl_xor(x, d, 64));
  return x;
}

__device__ inline uint32_t group8_sum(uint32_t x) {
  for (int d = 4; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// rows whose A' row fits one LDS hash: one workgroup per work item; 8 lanes
// per lost entry, so a wavefront works on 8 entries at once
template <int SR, int SLOTS, int WG>
__global__ __launch_bounds__(WG) void k_lost_small(LostArgs L) {
  using V = typename Sem<SR>::V;
  __shared__ int32_t hk[SLOTS];
  __shared__ int32_t hp[SLOTS];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int sub = lane >> 3, l8 = lane & 7;
  const int32_t r = L.item_row[blockIdx.x];
  const int64_t e0 = L.row_start[r] + (int64_t)L.item_part[blockIdx.x] * L.epw;
  const int64_t e1 = min(L.row_start[r + 1], e0 + L.epw);
  const int32_t i = (int32_t)(L.key[e0] >> L.cbits);
  const int64_t aoff = L.A.off[i];
  build_hash<SLOTS>(hk, hp, L.A, aoff, 0, L.A.len[i], tid, WG);
  const uint64_t cmask = (1ull << L.cbits) - 1;
  const int32_t d = L.A.len[i];
  constexpr int PER_ROUND = (WG / 64) * 8;
  for (int64_t eb = e0; eb < e1; eb += PER_ROUND) {
    const int64_t e = eb + wv * 8 + sub;
    bool act = e < e1;
    int32_t j = 0, lj = 0;
    int64_t toff = 0;
    if (act) {
      j = (int32_t)(L.key[e] & cmask);
      lj = L.T.len[j];
      toff = L.T.off[j];
      act = !(L.use_rowside && row_side(d, lj));
    }
    unsigned long long acc = acc_id<SR>();
    uint32_t hits = 0;
    if (act) {
      for (int32_t t = l8; t < lj; t += 8) {
        const int32_t pos = probe<SLOTS>(hk, hp, L.T.col[toff + t]);
        if (pos >= 0) {
          const V a = ldv<V>(L.A.val, aoff + pos), b = ldv<V>(L.T.val, toff + t);
          acc = acc_comb<SR>(acc, (unsigned long long)Sem<SR>::mul(a, b));
          ++hits;
        }
      }
    }
    acc = group8_comb<SR>(acc);
    hits = group8_sum(hits);
    if (act && l8 == 0) finish_entry<SR>(L, e, acc, hits);
  }
}

// rows too long for one hash: A' row i in chunks, partial results per entry
template <int SR, int SLOTS, int WG>
__global__ __launch_bounds__(WG) void k_lost_big(LostArgs L) {
  __shared__ int32_t hk[SLOTS];
  __shared__ int32_t hp[SLOTS];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int32_t r = L.item_row[blockIdx.x];
  const int64_t e0 = L.row_start[r] + (int64_t)L.item_part[blockIdx.x] * L.epw;
  const int64_t e1 = min(L.row_start[r + 1], e0 + L.epw);
  const int32_t i = (int32_t)(L.key[e0] >> L.cbits);
  const int64_t aoff = L.A.off[i];
  const int32_t d = L.A.len[i];
  const uint64_t cmask = (1ull << L.cbits) - 1;
  constexpr int32_t CHUNK = SLOTS / 2;
  for (int32_t k0 = 0; k0 < d; k0 += CHUNK) {
    build_hash<SLOTS>(hk, hp, L.A, aoff, k0, min(d, k0 + CHUNK), tid, WG);
    for (int64_t e = e0 + wv; e < e1; e += WG / 64) {
      const int32_t j = (int32_t)(L.key[e] & cmask);
      if (L.use_rowside && row_side(d, L.T.len[j])) continue;
      unsigned long long acc = acc_id<SR>();
      uint32_t hits = 0;
      column_pass<SR, SLOTS>(L, hk, hp, aoff, j, acc, hits, lane);
      acc = wave_comb<SR>(acc);
      hits = wave_sum(hits);
      if (lane == 0) {
        if (k0 > 0) {
          acc = acc_comb<SR>(acc, L.part_acc[e]);
          hits += L.part_hits[e];
        }
        L.part_acc[e] = acc;
        L.part_hits[e] = hits;
      }
    }
    __syncthreads();
  }
  for (int64_t e = e0 + tid; e < e1; e += WG)
    if (!(L.use_rowside && row_side(d, L.T.len[(int32_t)(L.key[e] & cmask)])))
      finish_entry<SR>(L, e, L.part_acc[e], L.part_hits[e]);
}

// lost entries recomputed from the row side: 8 lanes per entry
template <int SR>
__global__ __launch_bounds__(256) void k_lost_rowside(LostArgs L, int64_t nlost) {
  using V = typename Sem<SR>::V;
  const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const int l8 = threadIdx.x & 7;
  bool act = e < nlost;
  const uint64_t cmask = (1ull << L.cbits) - 1;
  int32_t i = 0, j = 0, d = 0;
  if (act) {
    i = (int32_t)(L.key[e] >> L.cbits);
    j = (int32_t)(L.key[e] & cmask);
    d = L.A.len[i];
    act = L.use_rowside && row_side(d, L.T.len[j]);
  }
  unsigned long long acc = acc_id<SR>();
  uint32_t hits = 0;
  if (act) {
    const int64_t aoff = L.A.off[i];
    for (int32_t t = l8; t < d; t += 8) {
      const int32_t k = L.A.col[aoff + t];
      const int64_t end = L.s_rp[k + 1];
      int64_t lo = L.s_rp[k], hi = end;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (L.s_col[mid] < j) lo = mid + 1;
        else hi = mid;
      }
      if (lo < end && L.s_col[lo] == j) {
        const V a = ldv<V>(L.A.val, aoff + t), b = ldv<V>(L.s_val, lo);
        acc = acc_comb<SR>(acc, (unsigned long long)Sem<SR>::mul(a, b));
        ++hits;
      }
    }
  }
  acc = group8_comb<SR>(acc);
  hits = group8_sum(hits);
  if (act && l8 == 0) finish_entry<SR>(L, e, acc, hits);
}

// row-side entries: their count and the column lengths they would stream
__global__ void k_count_rowside(const uint64_t* key, int64_t n, int cbits, const int32_t* a_len,
                                const int32_t* t_len, unsigned long long* cnt) {
  __shared__ unsigned long long sum;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t cmask = (1ull << cbits) - 1;
  if (threadIdx.x == 0) sum = 0;
  __syncthreads();
  int32_t lj = 0;
  bool rs = false;
  if (e < n) {
    lj = t_len[(int32_t)(key[e] & cmask)];
    rs = row_side(a_len[(int32_t)(key[e] >> cbits)], lj);
  }
  if (rs) atomicAdd(&sum, (unsigned long long)lj);
  const int c = __syncthreads_count(rs);  // one atomic per counter and workgroup
  if (threadIdx.x == 0 && c) {
    atomicAdd(cnt, (unsigned long long)c);
    atomicAdd(cnt + 1, sum);
  }
}

__global__ void k_del_batch(const uint64_t* key, int64_t n, int cbits, int32_t* rows, int32_t* cols, uint8_t* ops) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) {
    rows[t] = (int32_t)(key[t] >> cbits);
    cols[t] = (int32_t)(key[t] & ((1ull << cbits) - 1));
    ops[t] = DSG_OP_DELETE;
  }
}

__global__ void k_copy_u32(const uint32_t* src, uint32_t* dst) { *dst = *src; }

__global__ void k_rows_after(int32_t n, const uint32_t* epoch, const uint32_t* since, uint8_t* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flags[i] = epoch[i] > *since ? 1 : 0;
}

__global__ void k_sync_both(uint32_t* sync, const uint32_t* e) {
  sync[0] = *e;
  sync[1] = *e;
}

__global__ void k_zero_i64(int64_t* p) { *p = 0; }

__global__ void k_zero_n(unsigned long long* p, int n) {
  for (int x = threadIdx.x; x < n; x += blockDim.x) p[x] = 0ull;
}

// phase timing (when the context records kernel times)
struct Phase {
  Ctx* c;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  Phase(Ctx* cc, const char* name) : c(cc) {
    if (c->timing) ctx_timing_begin(c, name, 0.0, &e0, &e1);
  }
  ~Phase() {
    if (c->timing && e1) ctx_timing_end(c, e1);
  }
};

void* ensure_ws(DProd* p, size_t bytes) {
  if (bytes <= p->ews_bytes) return p->ews;
  Ctx* c = p->ctx;
  DSG_HIP(hipStreamSynchronize(c->stream));
  ctx_free(c, p->ews, p->ews_bytes);
  p->ews = nullptr;
  p->ews_bytes = 0;
  const size_t nb = bytes + bytes / 4 + (1 << 20);
  p->ews = ctx_alloc(c, nb);
  p->ews_bytes = nb;
  return p->ews;
}

int64_t read_count(Ctx* c, const int64_t* d) {
  int64_t* h = (int64_t*)((char*)c->pinned + 3072);
  DSG_HIP(hipMemcpyAsync(h, d, 8, hipMemcpyDeviceToHost, c->stream));
  DSG_HIP(hipStreamSynchronize(c->stream));
  return *h;
}

bool eligible(const DProd* p) {
  const DMat* A = p->A;
  if (p->ops || p->B != A || (A->sr != 0 && A->sr != 1)) return false;
  if (p->ctx->tuning.update_path == 1) return false;
  if (!A->tidx || A->tidx->vsz != A->vsz) return false;
  return A->log_seq != 0 && A->log_seq == A->apply_seq && A->apply_seq == p->a_seq + 1;
}

// Step 1, on its own: count the products the last apply changed (the
// offsets stay in the context's second scratch for entry_finish).
const int64_t* count_terms(DProd* p) {
  Ctx* c = p->ctx;
  hipStream_t s = c->stream;
  DMat* A = p->A;
  DMat* T = A->tidx;
  const int cbits = bits_for(A->ncols);
  Log L{A->log_key, A->log_old, A->log_new, A->log_code, A->h_log_n};
  const int64_t nU = L.n;
  const size_t b1 = Carve::need({(size_t)(nU + 1) * 8, (size_t)(nU + 1) * 8, scan_scratch_bytes(nU + 1) + 64, 64});
  Carve cv1(ctx_scratch2(c, b1), b1);
  int64_t* cnt = cv1.take<int64_t>(nU + 1);
  int64_t* off = cv1.take<int64_t>(nU + 1);
  void* scan1 = cv1.take<char>(scan_scratch_bytes(nU + 1) + 64);
  int64_t* d_total = cv1.take<int64_t>(8);
  if (nU > 0) {
    Phase ph(c, "entry_count");
    hipLaunchKernelGGL(k_term_counts, dim3(blocks_for(nU, 256)), dim3(256), 0, s, L, cbits, (const int32_t*)A->row_len,
                       (const int32_t*)T->row_len, cnt);
    exclusive_scan_i64(cnt, off, nU, d_total, scan1, s);
  } else {
    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(1), 0, s, d_total);
  }
  p->entry_nU = nU;
  p->entry_nterm = -1;  // until the caller reads *d_total back
  return d_total;
}

template <int SR>
int32_t entry_update(DProd* p) {
  using V = typename Sem<SR>::V;
  Ctx* c = p->ctx;
  hipStream_t s = c->stream;
  DMat* A = p->A;
  DMat* T = A->tidx;
  DMat* C = p->C;
  const int32_t n = A->nrows;
  const int cbits = bits_for(A->ncols);
  const int kbits = 2 * cbits;
  const uint64_t sentinel = 1ull << kbits;
  dsg_update_stats& st = p->stats;
  st = dsg_update_stats{};
  st.path = 1;

  // the counts of step 1 (count_terms), still in the second scratch
  Log L{A->log_key, A->log_old, A->log_new, A->log_code, p->entry_nU};
  const int64_t nU = L.n;
  const size_t b1 = Carve::need({(size_t)(nU + 1) * 8, (size_t)(nU + 1) * 8, scan_scratch_bytes(nU + 1) + 64, 64});
  Carve cv1(ctx_scratch2(c, b1), b1);
  (void)cv1.take<int64_t>(nU + 1);
  int64_t* off = cv1.take<int64_t>(nU + 1);
  (void)cv1.take<char>(scan_scratch_bytes(nU + 1) + 64);
  int64_t* d_total = cv1.take<int64_t>(8);
  const int64_t nterm = p->entry_nterm;
  // counters: [0] rows of C with changes, [1] lost deletions, [3] lost count,
  // [5..6] work items, [12] reported rows, [14..15] row-side entries and the
  // column lengths they would stream
  st.terms = nterm;

  // ---- workspace for the products, the entry updates and the lost entries ----
  const int64_t NT = std::max<int64_t>(nterm, 1);
  const size_t terms_b = Carve::need({(size_t)NT * 8, (size_t)NT * 4, (size_t)NT * 8, (size_t)NT * 8, (size_t)NT,
                                      radix_scratch_bytes(NT), (size_t)NT * 8, (size_t)NT * 8,
                                      scan_scratch_bytes(NT) + 64, (size_t)(NT + 1) * 8});
  const size_t lost_b = Carve::need({(size_t)NT * 8, (size_t)NT * 4, radix_scratch_bytes(NT), (size_t)NT * 8,
                                     (size_t)NT * 8, scan_scratch_bytes(NT) + 64, (size_t)(NT + 1) * 8,
                                     (size_t)NT, (size_t)NT, (size_t)NT * 4, (size_t)NT * 4, (size_t)NT * 4,
                                     (size_t)NT * 4, (size_t)NT * 8,
                                     (size_t)NT * 4, (size_t)NT * 8, (size_t)NT * 4, (size_t)NT * 4, (size_t)NT});
  const size_t segs_b = Carve::need({(size_t)NT * 8, (size_t)NT * 8, (size_t)NT * 8, (size_t)NT, 256, (size_t)n + 64,
                                     compact_scratch_bytes(std::max<int32_t>(n, 1)) + 64, 256});
  const size_t total_b = std::max(terms_b, lost_b) + segs_b;
  char* region = (char*)ensure_ws(p, total_b);
  Carve cs(region + std::max(terms_b, lost_b), segs_b);
  uint64_t* ckey = cs.take<uint64_t>(NT);
  V* cval = (V*)cs.take<uint64_t>(NT);
  uint64_t* cguard = cs.take<uint64_t>(NT);
  uint8_t* cflag = cs.take<uint8_t>(NT);
  unsigned long long* ctr = cs.take<unsigned long long>(16);
  uint8_t* rflags = cs.take<uint8_t>((size_t)n + 64);
  void* cscr = cs.take<char>(compact_scratch_bytes(std::max<int32_t>(n, 1)) + 64);
  uint32_t* ep_before = (uint32_t*)cs.take<uint64_t>(8);
  hipLaunchKernelGGL(k_zero_n, dim3(1), dim3(64), 0, s, ctr, 16);
  hipLaunchKernelGGL(k_copy_u32, dim3(1), dim3(1), 0, s, (const uint32_t*)C->d_epoch, ep_before);

  int64_t nseg = 0;
  if (nterm > 0) {
    // ---- 2. products ----
    Carve ct(region, terms_b);
    uint64_t* tkey = ct.take<uint64_t>(NT);
    uint32_t* tidx = ct.take<uint32_t>(NT);
    uint64_t* told = ct.take<uint64_t>(NT);
    uint64_t* tnew = ct.take<uint64_t>(NT);
    uint8_t* tfl = ct.take<uint8_t>(NT);
    void* rscr = ct.take<char>(radix_scratch_bytes(NT));
    int64_t* head = ct.take<int64_t>(NT);
    int64_t* segid = ct.take<int64_t>(NT);
    void* scan2 = ct.take<char>(scan_scratch_bytes(NT) + 64);
    int64_t* seg_start = ct.take<int64_t>(NT + 1);
    {
      Phase ph(c, "entry_terms");
      hipLaunchKernelGGL((k_term_write<SR>), dim3(blocks_for(nU * 64, 256)), dim3(256), 0, s, L, cbits, view(A),
                         view(T), (const int64_t*)off, tkey, told, tnew, tfl, sentinel);
      hipLaunchKernelGGL(k_iota_u32, dim3(blocks_for(nterm, 256)), dim3(256), 0, s, tidx, nterm);
    }
    // ---- 3. sort, segments, one update per entry of C ----
    {
      Phase ph(c, "entry_sort");
      radix_sort_pairs(tkey, tidx, nterm, kbits + 1, rscr, s);
    }
    Phase ph(c, "entry_reduce");
    hipLaunchKernelGGL(k_seg_heads, dim3(blocks_for(nterm, 256)), dim3(256), 0, s, tkey, nterm, sentinel, cbits,
                       head, ctr + 0);
    exclusive_scan_i64(head, segid, nterm, d_total, scan2, s);
    hipLaunchKernelGGL(k_seg_scatter, dim3(blocks_for(nterm, 256)), dim3(256), 0, s, tkey, nterm, sentinel,
                       (const int64_t*)head, (const int64_t*)segid, (const int64_t*)d_total, seg_start);
    nseg = read_count(c, d_total);
    if (nseg > 0)
      hipLaunchKernelGGL((k_seg_reduce<SR>), dim3(blocks_for(nseg, 256)), dim3(256), 0, s, tkey, tidx, told, tnew,
                         tfl, (const int64_t*)seg_start, (const int64_t*)d_total, ckey, (void*)cval, cguard, cflag);
  }
  st.entries = nseg;

  // ---- 4. apply to C; the products region now holds the lost entries ----
  Carve cl(region, lost_b);
  uint64_t* lkey = cl.take<uint64_t>(NT);
  int32_t* lslot = cl.take<int32_t>(NT);
  void* lrscr = cl.take<char>(radix_scratch_bytes(NT));
  int64_t* lhead = cl.take<int64_t>(NT);
  int64_t* lrid = cl.take<int64_t>(NT);
  void* lscan = cl.take<char>(scan_scratch_bytes(NT) + 64);
  int64_t* lrow_start = cl.take<int64_t>(NT + 1);
  uint8_t* is_small = cl.take<uint8_t>(NT);
  uint8_t* is_big = cl.take<uint8_t>(NT);
  int32_t* s_item_r = cl.take<int32_t>(NT);
  int32_t* s_item_p = cl.take<int32_t>(NT);
  int32_t* b_item_r = cl.take<int32_t>(NT);
  int32_t* b_item_p = cl.take<int32_t>(NT);
  unsigned long long* part_acc = cl.take<unsigned long long>(NT);
  uint32_t* part_hits = cl.take<uint32_t>(NT);
  uint64_t* dkey = cl.take<uint64_t>(NT);
  int32_t* drows = cl.take<int32_t>(NT);
  int32_t* dcols = cl.take<int32_t>(NT);
  uint8_t* dops = cl.take<uint8_t>(NT);
  int64_t nlost = 0;
  {
    Phase ph(c, "entry_apply_c");
    nlost = mat_apply_sorted_add(C, ckey, cval, cguard, cflag, nseg, lkey, lslot, NT, ctr + 3);
  }
  st.lost = nlost;

  // ---- 5. recompute the lost entries ----
  if (nlost > 0) {
    Phase* ph = new Phase(c, "entry_lost_prep");
    radix_sort_pairs(lkey, (uint32_t*)lslot, nlost, kbits, lrscr, s);
    hipLaunchKernelGGL(k_lost_heads, dim3(blocks_for(nlost, 256)), dim3(256), 0, s, lkey, nlost, cbits, lhead);
    exclusive_scan_i64(lhead, lrid, nlost, d_total, lscan, s);
    constexpr int SMALL_SLOTS = 2048, BIG_SLOTS = 16384;
    hipLaunchKernelGGL(k_lost_rows, dim3(blocks_for(nlost, 256)), dim3(256), 0, s, lkey, nlost, cbits,
                       (const int64_t*)lhead, (const int64_t*)lrid, (const int64_t*)d_total, lrow_start,
                       (const int32_t*)A->row_len, SMALL_SLOTS / 2, is_small, is_big);
    const int64_t nrow = read_count(c, d_total);
    // work items: runs of EPW_S / EPW_B lost entries of one row (a hub row's
    // entries spread over many workgroups); lhead / lrid are free again
    constexpr int32_t EPW_S = 32, EPW_B = 64;
    int64_t* d_ntot = (int64_t*)(ctr + 5);
    hipLaunchKernelGGL(k_item_counts, dim3(blocks_for(nrow, 256)), dim3(256), 0, s, (const int64_t*)lrow_start,
                       (const int64_t*)d_total, (const uint8_t*)is_small, EPW_S, EPW_B, lhead, lrid);
    exclusive_scan_i64(lhead, lhead, nrow, d_ntot, lscan, s);
    exclusive_scan_i64(lrid, lrid, nrow, d_ntot + 1, lscan, s);
    hipLaunchKernelGGL(k_item_fill, dim3(blocks_for(nrow, 256)), dim3(256), 0, s, (const int64_t*)lrow_start,
                       (const int64_t*)d_total, (const uint8_t*)is_small, EPW_S, EPW_B, (const int64_t*)lhead,
                       (const int64_t*)lrid, s_item_r, s_item_p, b_item_r, b_item_p);
    int64_t* hc = (int64_t*)((char*)c->pinned + 3072);
    DSG_HIP(hipMemcpyAsync(hc, d_ntot, 16, hipMemcpyDeviceToHost, s));
    DSG_HIP(hipStreamSynchronize(s));
    const int64_t nsmall = hc[0], nbig = hc[1];
    LostArgs la;
    la.key = lkey;
    la.slot = lslot;
    la.row_start = lrow_start;
    la.cbits = cbits;
    la.A = view(A);
    la.T = view(T);
    la.c_off = C->row_off;
    la.c_val = C->val;
    la.c_epoch = C->row_epoch;
    la.c_cur_epoch = C->d_epoch;
    la.part_acc = part_acc;
    la.part_hits = part_hits;
    la.del_key = dkey;
    la.ndel = ctr + 1;
    la.s_rp = nullptr;
    la.s_col = nullptr;
    la.s_val = nullptr;
    hipLaunchKernelGGL(k_count_rowside, dim3(blocks_for(nlost, 256)), dim3(256), 0, s, lkey, nlost, cbits,
                       (const int32_t*)A->row_len, (const int32_t*)T->row_len, ctr + 14);
    unsigned long long* hrs = (unsigned long long*)((char*)c->pinned + 3072);
    DSG_HIP(hipMemcpyAsync(hrs, ctr + 14, 16, hipMemcpyDeviceToHost, s));
    DSG_HIP(hipStreamSynchronize(s));
    // the sorted copy costs a sort of all of A': only worth it when the
    // row-side entries would otherwise stream a good part of that
    la.use_rowside = hrs[0] > 0 && hrs[1] > (unsigned long long)(A->h_top_ub / 4);
    if (la.use_rowside) {
      // column-sorted copy of A' for the row-side searches
      const int64_t annz = A->h_top_ub;  // bound on nnz(A')
      const size_t sb = Carve::need({(size_t)(n + 1) * 8, (size_t)std::max<int64_t>(annz, 1) * 4,
                                     (size_t)std::max<int64_t>(annz, 1) * A->vsz});
      if (p->srt_bytes < sb) {
        ctx_free(c, p->srt, p->srt_bytes);
        p->srt = nullptr;
        p->srt_bytes = 0;
        p->srt = ctx_alloc(c, sb + sb / 4);
        p->srt_bytes = sb + sb / 4;
      }
      Carve cq(p->srt, sb);
      int64_t* s_rp = cq.take<int64_t>(n + 1);
      int32_t* s_col = cq.take<int32_t>(std::max<int64_t>(annz, 1));
      void* s_val = cq.take<char>((size_t)std::max<int64_t>(annz, 1) * A->vsz);
      mat_export_device(A, s_rp, s_col, s_val, nullptr, s);
      delete ph;
      ph = new Phase(c, "entry_lost_rowside");
      la.s_rp = s_rp;
      la.s_col = s_col;
      la.s_val = s_val;
      hipLaunchKernelGGL((k_lost_rowside<SR>), dim3(blocks_for(nlost * 8, 256)), dim3(256), 0, s, la, nlost);
    }
    delete ph;
    ph = new Phase(c, "entry_lost_column");
    if (nsmall > 0) {
      la.item_row = s_item_r;
      la.item_part = s_item_p;
      la.epw = EPW_S;
      hipLaunchKernelGGL((k_lost_small<SR, SMALL_SLOTS, 128>), dim3((unsigned)nsmall), dim3(128), 0, s, la);
    }
    if (nbig > 0) {
      la.item_row = b_item_r;
      la.item_part = b_item_p;
      la.epw = EPW_B;
      hipLaunchKernelGGL((k_lost_big<SR, BIG_SLOTS, 256>), dim3((unsigned)nbig), dim3(256), 0, s, la);
    }
    DSG_HIP(hipGetLastError());
    delete ph;
    const int64_t ndel = read_count(c, (const int64_t*)(ctr + 1));
    if (ndel > 0) {
      hipLaunchKernelGGL(k_del_batch, dim3(blocks_for(ndel, 256)), dim3(256), 0, s, dkey, ndel, cbits, drows, dcols,
                         dops);
      mat_apply_device(C, drows, dcols, nullptr, dops, ndel);
    }
  }

  // ---- 6. rows whose content changed, and C now reflects A's epoch ----
  if (p->changed_cap < n) {
    ctx_free(c, p->changed_rows, (size_t)p->changed_cap * 4);
    p->changed_rows = nullptr;
    p->changed_cap = 0;
    p->changed_rows = (int32_t*)ctx_alloc(c, (size_t)std::max<int32_t>(n, 1024) * 4);
    p->changed_cap = std::max<int32_t>(n, 1024);
  }
  int32_t* d_nchg = (int32_t*)(ctr + 12);
  Phase ph(c, "entry_tail");
  if (n > 0) {
    hipLaunchKernelGGL(k_rows_after, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, (const uint32_t*)C->row_epoch,
                       (const uint32_t*)ep_before, rflags);
    compact_flags(rflags, n, p->changed_rows, d_nchg, cscr, s);
  }
  hipLaunchKernelGGL(k_sync_both, dim3(1), dim3(1), 0, s, p->d_sync, (const uint32_t*)A->d_epoch);
  struct Tail {
    unsigned long long ctr[4];
    int32_t nchg;
  };
  Tail* ht = (Tail*)((char*)c->pinned + 3072);
  DSG_HIP(hipMemcpyAsync(ht->ctr, ctr, 32, hipMemcpyDeviceToHost, s));
  ht->nchg = 0;
  if (n > 0) DSG_HIP(hipMemcpyAsync(&ht->nchg, d_nchg, 4, hipMemcpyDeviceToHost, s));
  DSG_HIP(hipStreamSynchronize(s));
  st.affected_rows = (int64_t)ht->ctr[0];
  st.flops = nterm;
  st.changed_rows = ht->nchg;
  return ht->nchg;
}

}  // namespace

bool entry_eligible(const DProd* p) { return eligible(p); }

const int64_t* entry_count(DProd* p) { return count_terms(p); }

int32_t entry_finish(DProd* p) { return p->A->sr == 1 ? entry_update<1>(p) : entry_update<0>(p); }
