// Entry-granular dynamic update of C = op(A)*op(B) (B may be A, either may be
// transposed) over (min,+) fp32, (+,x) int64 and (or, and) on 32-bit words.
// Below, A and B name op(A) and op(B): a transposed operand reads its rows
// from the matrix's transpose index, its columns from the matrix, and its
// changes from the transpose index's log.
//
// Section 5 writes the new product as the old one combined with the products
// that involve changed entries (Eq. 1), and observes that C can change only
// where that change pattern is non-zero.  The row path recomputes every row
// the pattern reaches.  This path works one level finer: it lists every
// product a_ik * b_kj the last batches changed, with its value before and
// after, and folds those values into the stored entries of C.
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
//   (or, and)     c' = c | (OR of the changed products' new words), unless a
//                 product vanished or lost bits: then the entry is recomputed.
//
// A recomputed entry takes the minimum (sum, OR) of a'_ik * b'_kj over k, from
// the shorter of row i of A' and column j of B': each k of that list is
// looked up in the per-row column index (rowindex.h) of B' or A', and column
// j comes from B's valued transpose.  C keeps a column index too, so the
// apply of step 4 finds each entry of C in constant time instead of
// streaming its row.
//
// Steps (all on the device, a few host reads of counts in between):
//   1. count the products of each changed entry: (i, k) of A as a left
//      factor, over row k of B' plus the entries the batch deleted from it;
//      (k, j) of B as a right factor, over column k of A' (rows i whose entry
//      (i, k) did not change -- the others are covered as left factors).  For
//      C = A*A every changed entry is both;
//   2. write the products (key i<<bits | j, old value, new value, presence);
//   3. sort them by key, and reduce each key to one ADD update of C
//      (min or sum of the changes), with a guard for the witness test;
//   4. apply those updates to C in place (ingest.hip: mat_apply_sorted_add),
//      which lists the lost entries with their slots;
//   5. recompute the lost entries from the cheaper side; entries left
//      without any product are deleted;
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
// The changed entries are those of A's log, then those of B's log (for
// C = A*A both are A's).  A changed entry (i, k) of A is a left factor: its
// products are the b_kj of row k of B', then the entries (k, j) the batch
// deleted from B (rng[u] keeps that log range of B and its count of
// deletions for the products' writer).  A changed entry (k, j) of B is a
// right factor: its products are the a_ik of column k of A' (rows i whose
// entry (i, k) changed too are covered as left factors).
__global__ void k_term_counts(Log LA, Log LB, int abits, int bbits, const int32_t* b_len, const int32_t* ta_len,
                              int64_t* cnt, int4* rng) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= LA.n + LB.n) return;
  int64_t c = 0;
  int4 g = make_int4(0, 0, 0, 0);
  if (u < LA.n) {
    if (LA.code[u] != UPD_NOP && LA.code[u] != UPD_LOST) {
      const int32_t k = (int32_t)(LA.key[u] & ((1ull << abits) - 1));
      int64_t e = log_lower(LB.key, LB.n, (uint64_t)k << bbits);
      g.x = (int32_t)e;
      int64_t ndel = 0;
      for (; e < LB.n && (LB.key[e] >> bbits) == (uint64_t)k; ++e) ndel += LB.code[e] == UPD_DEL;
      g.y = (int32_t)e;
      g.z = (int32_t)ndel;
      c = (int64_t)b_len[k] + ndel;
    }
  } else {
    const int64_t v = u - LA.n;
    if (LB.code[v] != UPD_NOP && LB.code[v] != UPD_LOST) c = ta_len[(int32_t)(LB.key[v] >> bbits)];
  }
  cnt[u] = c;
  rng[u] = g;
}

// The changed keys of A's log in a hash set (open addressing, all ones when
// empty): the right-factor pass asks for each product whether (i, k)
// changed too.
struct KeySet {
  uint64_t* tab;
  uint32_t mask;
};

__device__ inline uint32_t key_hash(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  return (uint32_t)k;
}

// The step's counters cleared and C's epoch noted, and (clear) the key set
// emptied, in one launch.
__global__ void k_entry_start(unsigned long long* ctr, int nctr, const uint32_t* epoch, uint32_t* ep_before,
                              KeySet H, bool clear) {
  if (blockIdx.x == 0) {
    if (threadIdx.x < nctr) ctr[threadIdx.x] = 0ull;
    if (threadIdx.x == 0) *ep_before = *epoch;
  }
  if (!clear) return;
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x <= H.mask; x += gridDim.x * blockDim.x) H.tab[x] = ~0ull;
}

__global__ void k_keyset_fill(Log L, KeySet H) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= L.n || L.code[u] == UPD_NOP || L.code[u] == UPD_LOST) return;
  const uint64_t k = L.key[u];
  uint32_t h = key_hash(k) & H.mask;
  while (atomicCAS((unsigned long long*)&H.tab[h], ~0ull, (unsigned long long)k) != ~0ull) h = (h + 1) & H.mask;
}

__device__ inline bool keyset_has(const KeySet& H, uint64_t k) {
  uint32_t h = key_hash(k) & H.mask;
  for (;;) {
    const uint64_t e = H.tab[h];
    if (e == k) return true;
    if (e == ~0ull) return false;
    h = (h + 1) & H.mask;
  }
}

// ---- 2. write the products: one thread per product ----
// Product t belongs to the last entry u with off[u] <= t (entries without
// products have none of them).  A wavefront's 64 products mostly share one
// entry, so the wavefront first finds the entries of its first and last
// product (same addresses in every lane) and a lane searches further only
// between those two.  Work is even however long the rows and columns of the
// changed entries are.
__device__ inline int64_t entry_of(const int64_t* off, int64_t lo, int64_t hi, int64_t t) {
  // last u in [lo, hi) with off[u] <= t (off[lo] <= t holds)
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (off[mid] <= t) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <int SR>
__global__ __launch_bounds__(256) void k_term_write(Log LA, Log LB, KeySet H, int abits, int bbits, Mat B, Mat TA,
                                                    const int64_t* off, const int4* rng, int64_t nterm,
                                                    uint64_t* tkey, uint64_t* told, uint64_t* tnew, uint8_t* tfl,
                                                    uint32_t* tidx) {
  using S = Sem<SR>;
  using V = typename S::V;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const int64_t t0 = t - lane;
  if (t0 >= nterm) return;
  const int64_t nu = LA.n + LB.n;
  const int64_t t1 = std::min<int64_t>(t0 + 63, nterm - 1);
  const int64_t u0 = entry_of(off, 0, nu, t0);
  const int64_t u1 = entry_of(off, u0, nu, t1);
  if (t >= nterm) return;
  tidx[t] = (uint32_t)t;  // the sort's values: the products' positions
  const int64_t u = u0 == u1 ? u0 : entry_of(off, u0, u1 + 1, t);
  const int64_t q = t - off[u];
  const uint64_t amask = (1ull << abits) - 1, bmask = (1ull << bbits) - 1;
  if (u < LA.n) {
    // left factor (i, k) of A: a_ik * b_kj
    const uint8_t code = LA.code[u];
    const uint64_t dk = LA.key[u];
    const int32_t i = (int32_t)(dk >> abits), k = (int32_t)(dk & amask);
    const bool op = code != UPD_INS, np = code != UPD_DEL;  // entry present before / after
    const V vo = rawv<V>(LA.old[u]), vn = rawv<V>(LA.nw[u]);
    const int32_t bl = B.len[k];
    const int4 g = rng[u];
    if (q < bl) {
      const int64_t bo = B.off[k] + q;
      const int32_t j = B.col[bo];
      const V bn = ldv<V>(B.val, bo);
      bool bop = true;
      V bold = bn;
      if (g.y > g.x) {  // (k, j) changed in B too: its value before
        const int64_t e = log_index(LB.key, g.x, g.y, ((uint64_t)k << bbits) | (uint64_t)(uint32_t)j);
        if (e >= 0) {
          const uint8_t ce = LB.code[e];
          if (ce == UPD_INS) bop = false;
          else if (ce == UPD_OVR) bold = rawv<V>(LB.old[e]);
        }
      }
      const uint8_t f = (op && bop ? F_OLD : 0) | (np ? F_NEW : 0);
      tkey[t] = ((uint64_t)(uint32_t)i << bbits) | (uint64_t)(uint32_t)j;
      told[t] = (f & F_OLD) ? (uint64_t)S::mul(vo, bold) : 0ull;
      tnew[t] = (f & F_NEW) ? (uint64_t)S::mul(vn, bn) : 0ull;
      tfl[t] = f;
    } else if (q == bl) {
      // entries (k, j) this batch deleted from B: a_ik * b_kj existed only
      // before.  The first of these products writes them all, in log order.
      int64_t w = t;
      for (int64_t e = g.x; e < g.y; ++e) {
        if (LB.code[e] != UPD_DEL) continue;
        const int32_t j = (int32_t)(LB.key[e] & bmask);
        tkey[w] = ((uint64_t)(uint32_t)i << bbits) | (uint64_t)(uint32_t)j;
        told[w] = op ? (uint64_t)S::mul(vo, rawv<V>(LB.old[e])) : 0ull;
        tnew[w] = 0ull;
        tfl[w] = op ? F_OLD : 0;
        ++w;
      }
    }
  } else {
    // right factor (k, j) of B: a_ik * b_kj over column k of A'
    const int64_t v = u - LA.n;
    const uint8_t code = LB.code[v];
    const uint64_t dk = LB.key[v];
    const int32_t k = (int32_t)(dk >> bbits), j = (int32_t)(dk & bmask);
    const bool op = code != UPD_INS, np = code != UPD_DEL;
    const V vo = rawv<V>(LB.old[v]), vn = rawv<V>(LB.nw[v]);
    const int64_t tc = TA.off[k] + q;
    const int32_t i = TA.col[tc];
    const V a = ldv<V>(TA.val, tc);
    // (i, k) changed too: that entry's left-factor products include this
    // one, which stays in the list with no effect (its key (i, j) is among
    // those products' keys, so it adds no entry of C)
    const bool dup = keyset_has(H, ((uint64_t)(uint32_t)i << abits) | (uint64_t)(uint32_t)k);
    const uint8_t f = dup ? 0 : (op ? F_OLD : 0) | (np ? F_NEW : 0);
    tkey[t] = ((uint64_t)(uint32_t)i << bbits) | (uint64_t)(uint32_t)j;
    told[t] = (f & F_OLD) ? (uint64_t)S::mul(a, vo) : 0ull;
    tnew[t] = (f & F_NEW) ? (uint64_t)S::mul(a, vn) : 0ull;
    tfl[t] = f;
  }
}

// ---- 3. segments of equal keys ----
__global__ void k_seg_heads(const uint64_t* key, int64_t n, int64_t* head) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) head[t] = (t == 0 || key[t - 1] != key[t]) ? 1 : 0;
}

__global__ void k_seg_scatter(int64_t n, const int64_t* head, const int64_t* segid, const int64_t* d_nseg,
                              int64_t* seg_start) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  if (head[t]) seg_start[segid[t]] = t;
  if (t + 1 == n) seg_start[*d_nseg] = n;
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
  } else if constexpr (SR == 3) {
    // (or, and) on words: the OR of the new products; a product that vanished
    // or lost bits makes the entry lost (those bits may have come from it
    // alone)
    uint32_t orw = 0;
    bool any = false, lost = false;
    for (int64_t t = t0; t < t1; ++t) {
      const uint32_t q = idx[t];
      const uint8_t f = tfl[q];
      const uint32_t o = (uint32_t)told[q], w = (uint32_t)tnew[q];
      if (f & F_NEW) orw |= w;
      any = any || f != 0;
      lost = lost || ((f & F_OLD) && (!(f & F_NEW) || (o & ~w) != 0u));
    }
    ((V*)cval)[s] = (V)orw;
    cguard[s] = 0;
    cflag[s] = (any ? 1 : 0) | (lost ? 4 : 0);
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
// A lost entry (i, j) takes the minimum (sum, OR) of a'_ik * b'_kj over k from
// the shorter of two lists: row i of A' (each k probed for column j in the
// column index of row k of B') or column j of B' (each k probed for column k
// in the column index of row i of A').  Entries are split into three classes by that length (up
// to LOST_C0_MAX, up to LOST_C1_MAX, longer), taken by groups of 8, 32 and 64
// lanes, so that a group needs about one round of probes.
constexpr int32_t LOST_C0_MAX = 8, LOST_C1_MAX = 32;

struct LostArgs {
  const uint64_t* key;
  const int32_t* slot;
  int cbits;     // column bits of C's keys
  Mat A, B, TB;  // rows of A' and B', columns of B' (B's valued transpose)
  RowIx XA, XB;  // column indexes of A' and B' (every row built)
  int64_t* c_off;
  void* c_val;
  uint32_t* c_epoch;
  const uint32_t* c_cur_epoch;
  uint8_t* del_flag;  // per lost entry: no product left, delete it
};

template <int SR>
__device__ inline unsigned long long acc_id() {
  return SR == 1 ? 0xffffffffull : 0ull;
}

template <int SR>
__device__ inline unsigned long long acc_comb(unsigned long long a, unsigned long long b) {
  if constexpr (SR == 1) return a < b ? a : b;
  else if constexpr (SR == 3) return a | b;
  else return a + b;
}

// position of column c in row r of M (its table in X, or a scan of the row
// when the index pool had no room for it)
__device__ inline int32_t a_find(const RowIx& X, const Mat& M, int32_t r, int32_t c) {
  if (X.tab) {  // M may have no index (refused for room, or switched off)
    // (the table's place is read before its stamp is checked: independent loads)
    const int64_t to = X.off[r];
    const uint32_t tn = (uint32_t)X.sz[r];
    if (X.stamp[r] == X.gen) return ix_find(X.tab + to, tn, c);
  }
  const int64_t o = M.off[r];
  const int32_t n = M.len[r];
  for (int32_t t = 0; t < n; ++t)
    if (M.col[o + t] == c) return t;
  return -1;
}

// write the recomputed entry (one lane): overwrite at its slot, or flag it
// for deletion when no product is left
template <int SR>
__device__ inline void finish_entry(const LostArgs& L, int64_t e, unsigned long long acc, uint32_t hits) {
  using S = Sem<SR>;
  using V = typename S::V;
  const uint64_t key = L.key[e];
  const int32_t i = (int32_t)(key >> L.cbits);
  L.del_flag[e] = hits == 0 ? 1 : 0;
  if (hits > 0) {
    const V nv = S::from_acc((typename S::Acc)acc);
    const int64_t p = L.c_off[i] + L.slot[e];
    const V cur = ((V*)L.c_val)[p];
    if (!same_bits(cur, nv)) {
      ((V*)L.c_val)[p] = nv;
      L.c_epoch[i] = *L.c_cur_epoch;
    }
  }
}

// class of each lost entry by probe count: 0 (at most LOST_C0_MAX), 1 (at
// most LOST_C1_MAX), 2 (more)
__global__ void k_lost_classes(const uint64_t* key, int64_t n, int cbits, const int32_t* a_len, const int32_t* tb_len,
                               uint8_t* cls) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const uint64_t k = key[e];
  const int32_t d = a_len[(int32_t)(k >> cbits)];
  const int32_t lj = tb_len[(int32_t)(k & ((1ull << cbits) - 1))];
  const int32_t cost = d < lj ? d : lj;
  cls[e] = cost <= LOST_C0_MAX ? 0 : cost <= LOST_C1_MAX ? 1 : 2;
}

// G lanes per lost entry; the listed entries taken in turn by the nb blocks
// of this part of the grid (b is the block's index within the part)
template <int SR, int G>
__device__ inline void lost_recompute(const LostArgs& L, const int32_t* list, int64_t n, int64_t b, int64_t nb) {
  using V = typename Sem<SR>::V;
  const int l = threadIdx.x & (G - 1);
  const int64_t ng = (nb * blockDim.x) / G;
  const uint64_t cmask = (1ull << L.cbits) - 1;
  // (the G lanes of a group share q0, so each group runs its rounds together
  // and its shuffles see all of its lanes)
  for (int64_t q0 = (b * blockDim.x + threadIdx.x) / G; q0 < n; q0 += ng) {
    const int64_t e = list[q0];
    const int32_t i = (int32_t)(L.key[e] >> L.cbits);
    const int32_t j = (int32_t)(L.key[e] & cmask);
    const int32_t d = L.A.len[i];
    const int32_t lj = L.TB.len[j];
    unsigned long long acc = acc_id<SR>();
    uint32_t hits = 0;
    const int64_t aoff = L.A.off[i];
    if (d <= lj) {
      // row i of A': is column j in row k of B'?
      for (int32_t t = l; t < d; t += G) {
        const int32_t k = L.A.col[aoff + t];
        const int32_t pos = a_find(L.XB, L.B, k, j);
        if (pos >= 0) {
          const V a = ldv<V>(L.A.val, aoff + t), b = ldv<V>(L.B.val, L.B.off[k] + pos);
          acc = acc_comb<SR>(acc, (unsigned long long)Sem<SR>::mul(a, b));
          ++hits;
        }
      }
    } else {
      // column j of B': is column k in row i of A'?
      const int64_t toff = L.TB.off[j];
      for (int32_t t = l; t < lj; t += G) {
        const int32_t k = L.TB.col[toff + t];
        const int32_t pos = a_find(L.XA, L.A, i, k);
        if (pos >= 0) {
          const V a = ldv<V>(L.A.val, aoff + pos), b = ldv<V>(L.TB.val, toff + t);
          acc = acc_comb<SR>(acc, (unsigned long long)Sem<SR>::mul(a, b));
          ++hits;
        }
      }
    }
#pragma unroll
    for (int x = G / 2; x > 0; x >>= 1) {
      acc = acc_comb<SR>(acc, __shfl_xor(acc, x, 64));
      hits += __shfl_xor(hits, x, 64);
    }
    if (l == 0) finish_entry<SR>(L, e, acc, hits);
  }
}

// the three classes in one launch: blocks [0, nb0) take class 0 by groups of
// 8 lanes, [nb0, nb0 + nb1) class 1 by groups of 32, the rest class 2 by
// groups of 64
template <int SR>
__global__ __launch_bounds__(256) void k_lost_recompute(LostArgs L, const int32_t* l0, const int32_t* l1,
                                                        const int32_t* l2, const int32_t* cnt, int64_t nb0,
                                                        int64_t nb1) {
  const int64_t b = blockIdx.x;
  if (b < nb0) lost_recompute<SR, 8>(L, l0, cnt[0], b, nb0);
  else if (b < nb0 + nb1) lost_recompute<SR, 32>(L, l1, cnt[1], b - nb0, nb1);
  else lost_recompute<SR, 64>(L, l2, cnt[2], b - nb0 - nb1, (int64_t)gridDim.x - nb0 - nb1);
}

__global__ void k_rows_after(int32_t n, const uint32_t* epoch, const uint32_t* since, uint8_t* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flags[i] = epoch[i] > *since ? 1 : 0;
}

__global__ void k_sync_ab(uint32_t* sync, const uint32_t* ea, const uint32_t* eb) {
  sync[0] = *ea;
  sync[1] = *eb;
}

__global__ void k_zero_i64(int64_t* p) { *p = 0; }

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
  const DMat* B = p->B;
  if (p->bloom || (A->sr != 0 && A->sr != 1 && A->sr != 3) || B->sr != A->sr) return false;
  if (p->ctx->tuning.update_path == 1) return false;
  const OpView l = op_view(p, true), r = op_view(p, false);
  if (B == A) return changed_once(l);
  return (changed_once(l) || unchanged(l)) && (changed_once(r) || unchanged(r)) && (changed_once(l) || changed_once(r));
}

// The two logs of the pending update: op(A)'s changed entries (left factors)
// and op(B)'s (right factors); an operand not applied since the last update
// has an empty one.  For C = A*A both are A's log.
struct EntryLogs {
  Log LA, LB;
  int abits, bbits;  // column bits of op(A)'s and op(B)'s keys (op(B)'s are C's too)
};

EntryLogs entry_logs(const DProd* p) {
  const OpView l = op_view(p, true), r = op_view(p, false);
  const bool same = p->B == p->A;
  const bool ca = same || !unchanged(l);
  const bool cb = same || !unchanged(r);
  const DMat* la = l.logm;
  const DMat* lb = r.logm;
  EntryLogs g;
  g.LA = Log{la->log_key, la->log_old, la->log_new, la->log_code, ca ? la->h_log_n : 0};
  g.LB = Log{lb->log_key, lb->log_old, lb->log_new, lb->log_code, cb ? lb->h_log_n : 0};
  g.abits = bits_for(p->A->ncols);
  g.bbits = bits_for(p->B->ncols);
  return g;
}

// Step 1, on its own: count the products the last applies changed (the
// offsets stay in the context's second scratch for entry_finish).
const int64_t* count_terms(DProd* p) {
  Ctx* c = p->ctx;
  hipStream_t s = c->stream;
  DMat* B = p->B;
  DMat* TA = op_view(p, true).cols;  // columns of op(A)'
  const EntryLogs g = entry_logs(p);
  const int64_t nU = g.LA.n + g.LB.n;
  const size_t b1 = Carve::need(
      {(size_t)(nU + 1) * 8, (size_t)(nU + 1) * 8, scan_scratch_bytes(nU + 1) + 64, 64, (size_t)(nU + 1) * 16});
  Carve cv1(ctx_scratch2(c, b1), b1);
  int64_t* cnt = cv1.take<int64_t>(nU + 1);
  int64_t* off = cv1.take<int64_t>(nU + 1);
  void* scan1 = cv1.take<char>(scan_scratch_bytes(nU + 1) + 64);
  int64_t* d_total = cv1.take<int64_t>(8);
  int4* rng = cv1.take<int4>(nU + 1);
  if (nU > 0) {
    Phase ph(c, "entry_count");
    hipLaunchKernelGGL(k_term_counts, dim3(blocks_for(nU, 256)), dim3(256), 0, s, g.LA, g.LB, g.abits, g.bbits,
                       (const int32_t*)B->row_len, (const int32_t*)TA->row_len, cnt, rng);
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
  DMat* A = p->A;  // op(A), op(B): rows
  DMat* B = p->B;
  DMat* TA = op_view(p, true).cols;   // columns of op(A)'
  DMat* TB = op_view(p, false).cols;  // columns of op(B)'
  DMat* C = p->C;
  const int32_t n = A->nrows;
  const EntryLogs g = entry_logs(p);
  const int cbits = g.bbits;  // C's keys: (row << cbits) | column
  const int kbits = bits_for(C->nrows) + cbits;
  dsg_update_stats& st = p->stats;
  st = dsg_update_stats{};
  st.path = 1;
  // column index of C: the apply of its updates looks entries up in it
  // (A' and B' got theirs at eligibility); built on first use
  if (c->tuning.row_index) mat_index_enable(C);

  // the counts of step 1 (count_terms), still in the second scratch
  const int64_t nU = g.LA.n + g.LB.n;
  DSG_REQUIRE(nU == p->entry_nU, DSG_E_STATE, "internal: the logs changed between counting and updating");
  const size_t b1 = Carve::need(
      {(size_t)(nU + 1) * 8, (size_t)(nU + 1) * 8, scan_scratch_bytes(nU + 1) + 64, 64, (size_t)(nU + 1) * 16});
  Carve cv1(ctx_scratch2(c, b1), b1);
  (void)cv1.take<int64_t>(nU + 1);
  int64_t* off = cv1.take<int64_t>(nU + 1);
  (void)cv1.take<char>(scan_scratch_bytes(nU + 1) + 64);
  int64_t* d_total = cv1.take<int64_t>(8);
  const int4* rng = cv1.take<int4>(nU + 1);
  const int64_t nterm = p->entry_nterm;
  // counters: [0] rows of C with changed products, [3] lost entries, [5]
  // the product sort's error flag, [12] reported rows
  st.terms = nterm;

  // ---- workspace for the products, the entry updates and the lost entries ----
  const int64_t NT = std::max<int64_t>(nterm, 1);
  const size_t terms_b = Carve::need({(size_t)NT * 8, (size_t)NT * 4, (size_t)NT * 8, (size_t)NT * 8, (size_t)NT,
                                      radix_scratch_bytes(NT), (size_t)NT * 8, (size_t)NT * 8,
                                      scan_scratch_bytes(NT) + 64, (size_t)(NT + 1) * 8});
  const size_t lost_b = Carve::need({(size_t)NT * 8, (size_t)NT * 4, (size_t)NT, (size_t)NT, (size_t)NT,
                                     (size_t)NT * 4, (size_t)NT * 4, (size_t)NT * 4, (size_t)NT, (size_t)NT * 4,
                                     compact_scratch_bytes(NT) + 64, 64});
  uint32_t hs = 64;  // the key set of A's changed entries
  while (hs < 2 * (uint64_t)std::max<int64_t>(g.LA.n, 1)) hs <<= 1;
  const size_t segs_b = Carve::need({(size_t)NT * 8, (size_t)NT * 8, (size_t)NT * 8, (size_t)NT, 256, (size_t)n + 64,
                                     compact_scratch_bytes(std::max<int32_t>(n, 1)) + 64, 256,
                                     sorted_add_scratch_bytes(NT), (size_t)hs * 8});
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
  void* sa_scr = cs.take<char>(sorted_add_scratch_bytes(NT));
  KeySet H{cs.take<uint64_t>(hs), hs - 1};
  hipLaunchKernelGGL(k_entry_start, dim3(nterm > 0 ? std::min<unsigned>(blocks_for(hs, 256), 1024) : 1u), dim3(256),
                     0, s, ctr, 16, (const uint32_t*)C->d_epoch, ep_before, H, nterm > 0);

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
      if (g.LA.n > 0)
        hipLaunchKernelGGL(k_keyset_fill, dim3(blocks_for(g.LA.n, 256)), dim3(256), 0, s, g.LA, H);
      hipLaunchKernelGGL((k_term_write<SR>), dim3(blocks_for(nterm, 256)), dim3(256), 0, s, g.LA, g.LB, H, g.abits,
                         g.bbits, view(B), view(TA), (const int64_t*)off, rng, nterm, tkey, told, tnew, tfl, tidx);
    }
    // ---- 3. sort, segments, one update per entry of C ----
    {
      Phase ph(c, "entry_sort");
      radix_sort_pairs(tkey, tidx, nterm, kbits, rscr, s, (int*)(ctr + 5));
    }
    Phase ph(c, "entry_reduce");
    hipLaunchKernelGGL(k_seg_heads, dim3(blocks_for(nterm, 256)), dim3(256), 0, s, tkey, nterm, head);
    exclusive_scan_i64(head, segid, nterm, d_total, scan2, s);
    hipLaunchKernelGGL(k_seg_scatter, dim3(blocks_for(nterm, 256)), dim3(256), 0, s, nterm, (const int64_t*)head,
                       (const int64_t*)segid, (const int64_t*)d_total, seg_start);
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
  uint8_t* fcls = cl.take<uint8_t>(NT);
  int32_t* lcls[3] = {cl.take<int32_t>(NT), cl.take<int32_t>(NT), cl.take<int32_t>(NT)};
  uint8_t* fdel = cl.take<uint8_t>(NT);
  int32_t* ldel = cl.take<int32_t>(NT);
  void* lscr = cl.take<char>(compact_scratch_bytes(NT) + 64);
  int32_t* lcnt = cl.take<int32_t>(16);  // [0..2] the classes, [3] deletions
  int64_t nlost = 0;
  {
    Phase ph(c, "entry_apply_c");
    // (ctr[0]: the rows of C with changed products)
    nlost = mat_apply_sorted_add(C, ckey, cval, cguard, cflag, nseg, lkey, lslot, NT, ctr + 3, (int64_t*)ctr,
                                 sa_scr);
  }
  st.lost = nlost;

  // ---- 5. recompute the lost entries ----
  if (nlost > 0) {
    {
      Phase ph(c, "entry_lost");
      // every row of A' and B' needs its column table (the applies dropped
      // the tables of rows they could not keep them for)
      mat_index_build(A, nullptr, nullptr, A->nrows);
      if (B != A) mat_index_build(B, nullptr, nullptr, B->nrows);
      LostArgs la;
      la.key = lkey;
      la.slot = lslot;
      la.cbits = cbits;
      la.A = view(A);
      la.B = view(B);
      la.TB = view(TB);
      la.XA = mat_index_view(A);
      la.XB = mat_index_view(B);
      la.c_off = C->row_off;
      la.c_val = C->val;
      la.c_epoch = C->row_epoch;
      la.c_cur_epoch = C->d_epoch;
      la.del_flag = fdel;
      hipLaunchKernelGGL(k_lost_classes, dim3(blocks_for(nlost, 256)), dim3(256), 0, s, (const uint64_t*)lkey, nlost,
                         cbits, (const int32_t*)A->row_len, (const int32_t*)TB->row_len, fcls);
      compact_classes3(fcls, nlost, lcls[0], lcls[1], lcls[2], lcnt, lscr, s);
      // bounded grids over the device counts
      auto grid = [&](int g) {
        return std::max<int64_t>(1, std::min<int64_t>(blocks_for(nlost * g, 256), 32 * (int64_t)c->num_cus));
      };
      const int64_t nb0 = grid(8), nb1 = grid(32), nb2 = grid(64);
      hipLaunchKernelGGL((k_lost_recompute<SR>), dim3((unsigned)(nb0 + nb1 + nb2)), dim3(256), 0, s, la,
                         (const int32_t*)lcls[0], (const int32_t*)lcls[1], (const int32_t*)lcls[2],
                         (const int32_t*)lcnt, nb0, nb1);
      compact_flags(fdel, nlost, ldel, lcnt + 3, lscr, s);
      DSG_HIP(hipGetLastError());
    }
    int32_t* hd = (int32_t*)((char*)c->pinned + 3072);
    DSG_HIP(hipMemcpyAsync(hd, lcnt + 3, 4, hipMemcpyDeviceToHost, s));
    DSG_HIP(hipStreamSynchronize(s));
    const int64_t ndel = hd[0];
    if (ndel > 0) {
      Phase ph(c, "entry_delete");
      mat_apply_sorted_delete(C, lkey, lslot, ldel, ndel);
    }
  }

  // ---- 6. rows whose content changed, and C now reflects A's and B's epochs ----
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
  hipLaunchKernelGGL(k_sync_ab, dim3(1), dim3(1), 0, s, p->d_sync, (const uint32_t*)A->d_epoch,
                     (const uint32_t*)B->d_epoch);
  struct Tail {
    unsigned long long ctr[6];
    unsigned long long ix_top[3];  // index pool tops of C, A and B
    int32_t nchg;
  };
  Tail* ht = (Tail*)((char*)c->pinned + 3072);
  FetchList F;
  F.add(ctr, 48, 3072 + (int32_t)offsetof(Tail, ctr));
  F.add(C->ix_top, 8, 3072 + (int32_t)offsetof(Tail, ix_top));
  F.add(A->ix_top, 8, 3072 + (int32_t)offsetof(Tail, ix_top) + 8);
  F.add(B != A ? (const void*)B->ix_top : nullptr, 8, 3072 + (int32_t)offsetof(Tail, ix_top) + 16);
  F.add(n > 0 ? (const void*)d_nchg : nullptr, 4, 3072 + (int32_t)offsetof(Tail, nchg));
  fetch_to_pinned(c, F, s);
  DSG_HIP(hipStreamSynchronize(s));
  mat_index_note_top(C, ht->ix_top[0]);
  mat_index_note_top(A, ht->ix_top[1]);
  if (B != A) mat_index_note_top(B, ht->ix_top[2]);
  DSG_REQUIRE(ht->ctr[5] == 0, DSG_E_DEVICE, "internal: the product sort could not complete");
  st.affected_rows = (int64_t)ht->ctr[0];
  st.flops = nterm;
  st.changed_rows = ht->nchg;
  return ht->nchg;
}

}  // namespace

bool entry_eligible(DProd* p) {
  // the products of op(B)'s changed entries run over columns of op(A)', and
  // the lost entries over columns of op(B)': both need that operand's columns
  // as rows, with values -- the matrix itself for a transposed operand, else
  // its valued transpose index (A's exists for the discovery; B's is built
  // here on first use, and every later apply of B keeps it, with its log)
  for (DMat* m : {p->src_a, p->src_b}) {
    if (!m->tidx) {
      if (!eligible(p)) return false;
      try {
        mat_build_transpose(m);
      } catch (const DsgError& e) {
        if (e.code != DSG_E_OOM) throw;
        return false;
      }
    }
    if (!m->tidx || m->tidx->vsz != m->vsz) return false;
  }
  if (!eligible(p)) return false;
  // the lost entries probe rows of A' and B' through their column indexes:
  // without them (no room) the row path runs instead; with the index
  // switched off the probes scan the rows
  if (!p->ctx->tuning.row_index) return true;
  return mat_index_enable(p->A) && (p->B == p->A || mat_index_enable(p->B));
}

const int64_t* entry_count(DProd* p) { return count_terms(p); }

int32_t entry_finish(DProd* p) {
  switch (p->A->sr) {
    case 1: return entry_update<1>(p);
    case 3: return entry_update<3>(p);
    default: return entry_update<0>(p);
  }
}
