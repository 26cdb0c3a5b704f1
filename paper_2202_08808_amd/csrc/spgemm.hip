// Dynamic and static products: affected-row discovery, row analysis and
// binning, binned row-wise Gustavson recompute, merge into the dynamic C.
//
// What is computed (Section 5): C' = A' B' over the semiring.  C' can differ
// from C only in entries where C* = A* B' + A B* (Eq. 1) is non-zero, where
// A*, B* mark the changed entries (for general updates only their structure
// matters, and deletions count as changed entries).  Rows of C* are the
// changed rows of A plus every row i with A[i,k] present for a changed row
// k of B; since rows of A outside the changed set are equal in A and A',
// the post-update transpose index finds them.  Each such row is recomputed
// in full with Gustavson's row-wise algorithm (Section 6.1), then compared
// with the stored row and written back only if it differs.
//
// Accumulators, by an upper bound ub_i = min(flops_i, ncols) of the output
// row length:
//   bins 0-7  a lane group of G = 8<<b lanes per row with an LDS hash table of
//             8G slots (load <= 1/2);
//   bin 8     one 1024-lane workgroup per row with a dense LDS accumulator
//             over column chunks (one pass per chunk);
//   bin 9     one workgroup per row with a hash table in device memory.
// Semiring additions that are exactly associative (int64 wrap-around, fp32
// min) combine with LDS/global atomics in any order.  fp64 sums take the
// A-row entries one k at a time in ascending k (lanes cover the columns of
// B[k,:], which are distinct), so every c_ij is summed in ascending k.
#include "internal.h"
#include "kernel_common.h"

namespace {

unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

constexpr int NBINS = 10;
constexpr int BIN_DENSE = 8;
constexpr int BIN_GLOBAL = 9;
constexpr int NSTAT = 7;  // rows, a_entries, flops, nnz_new, nnz_old, old_read, written
// Workgroups of the one-row-per-workgroup bins.  The dense bin holds one
// workgroup per CU (its accumulator fills the LDS), so its size sets how many
// wavefronts hide the latency of each row's gathers.
// (512: at 1024 lanes the kernel spills registers and runs slower.)
constexpr int DENSE_WG = 512;
constexpr int GLOBAL_WG = 512;
constexpr int DENSE_ACHUNK = 512;

template <int VSZ>
constexpr int dense_cols() {
  return VSZ == 8 ? 16384 : 32768;
}

struct RowArgs {
  // A (left operand), B (right operand), C (result)
  const int64_t* a_off;
  const int32_t* a_len;
  const int32_t* a_col;
  const void* a_val;
  const int64_t* b_off;
  const int32_t* b_len;
  const int32_t* b_col;
  const void* b_val;
  int64_t* c_off;
  int32_t* c_len;
  int32_t* c_cap;
  int32_t* c_col;
  void* c_val;
  int64_t* c_top;
  int64_t c_pool_cap;
  int32_t ncols;
  const int32_t* aff;   // affected rows, indexed by q
  int32_t* ub;          // per q
  uint8_t* chg;         // per q: row reported
  unsigned long long* stats;  // [NBINS][NSTAT]
  char* arena;
  unsigned long long* arena_top;
  int64_t arena_cap;
  int force_write;      // 1: write every recomputed row, no comparison
  int* err;
  struct RowStat* rstat;  // per q
  uint8_t* binof;         // per q
  int32_t* flq;           // per q: flops (clamped to int32)
  unsigned int* dense_next;  // row counter of the persistent dense kernel
  const int* defer;          // non-null and set: skip this product
  uint8_t* retry;            // per q: row could not be placed, recompute it
  unsigned long long* c_short;      // C slots the flagged rows need
  unsigned long long* arena_short;  // arena bytes the flagged rows need
  // B split by dense column chunk (bs_parts > 0): part p of row k spans
  // [bs_ps[k*(bs_parts+1) + p], bs_ps[k*(bs_parts+1) + p + 1]) of bs_col /
  // bs_val (positions inside the row's slots of B's pool)
  int32_t bs_parts;
  const int64_t* bs_ps;
  const int32_t* bs_col;
  const void* bs_val;
};

// Per-row work record, summed per bin by k_reduce_stats.
struct RowStat {
  int32_t d, flops, nnew, olen, old_read, written;
};

__device__ inline void row_stat(const RowArgs& R, int32_t q, int32_t d, int64_t flops, int32_t nnew,
                                int32_t olen, int64_t old_read, int32_t written) {
  RowStat s;
  s.d = d;
  s.flops = (int32_t)flops;
  s.nnew = nnew;
  s.olen = olen;
  s.old_read = (int32_t)old_read;
  s.written = written;
  R.rstat[q] = s;
}

// ---------------------------------------------------------------------------
// lane-group primitives: G <= 64 lanes inside one wavefront, or G == blockDim
// ---------------------------------------------------------------------------

template <int G>
struct Grp {
  static constexpr bool sub = G <= 64;
  int lane;   // lane in group
  int goff;   // offset of the group inside its wavefront (sub-wave groups)
  __device__ Grp() {
    lane = threadIdx.x % G;
    goff = (threadIdx.x & 63) & ~(G < 64 ? G - 1 : 63);
  }
  __device__ void sync() const {
    if constexpr (sub) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      __syncthreads();
    }
  }
  __device__ uint64_t gmask(uint64_t ballot) const {
    if constexpr (G >= 64) return ballot;
    else return (ballot >> goff) & ((1ull << G) - 1);
  }
  // exclusive rank of pred among group lanes, and the group's total
  __device__ int rank(bool pred, int& total, int* wscr) const {
    uint64_t b = __ballot(pred);
    if constexpr (sub) {
      uint64_t m = gmask(b);
      total = __popcll(m);
      return __popcll(m & ((1ull << lane) - 1));
    } else {
      const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = G / 64;
      if (l == 0) wscr[w] = __popcll(b);
      __syncthreads();
      int before = 0, tot = 0;
      for (int x = 0; x < nw; ++x) {
        int c = wscr[x];
        if (x < w) before += c;
        tot += c;
      }
      __syncthreads();
      total = tot;
      uint64_t lt = l ? (~0ull >> (64 - l)) : 0ull;
      return before + __popcll(b & lt);
    }
  }
  __device__ bool any(bool pred, int* wscr) const {
    int t;
    rank(pred, t, wscr);
    return t > 0;
  }
  // inclusive scan of int32 over the group
  __device__ int32_t scan(int32_t x, int32_t& total, int* wscr) const {
    if constexpr (sub) {
#pragma unroll
      for (int d = 1; d < G; d <<= 1) {
        int32_t y = __shfl_up(x, d, G);
        if (lane >= d) x += y;
      }
      total = __shfl(x, G - 1, G);
      return x;
    } else {
      const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = G / 64;
      x = wave_inclusive_scan(x);
      if (l == 63) wscr[w] = x;
      __syncthreads();
      int32_t before = 0, tot = 0;
      for (int q = 0; q < nw; ++q) {
        int32_t c = wscr[q];
        if (q < w) before += c;
        tot += c;
      }
      __syncthreads();
      total = tot;
      return x + before;
    }
  }
  __device__ int64_t bcast64(int64_t v, int src, int64_t* slot) const {
    if constexpr (sub) {
      return __shfl(v, src, G);
    } else {
      if (lane == src) *slot = v;
      __syncthreads();
      int64_t r = *slot;
      __syncthreads();
      return r;
    }
  }
};

// largest t in [0, cnt) with pre[t] <= f  (pre non-decreasing, pre[0] = 0)
__device__ inline int find_seg(const int32_t* pre, int cnt, int32_t f) {
  int lo = 0, hi = cnt - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= f) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <class V>
__device__ inline V ldv(const void* p, int64_t i) {
  return ((const V*)p)[i];
}

// ---------------------------------------------------------------------------
// LDS open-addressing hash (linear probing), keys -1 = empty
// ---------------------------------------------------------------------------

template <int SLOTS>
__device__ inline int hash_insert(int32_t* keys, int32_t c, bool& fresh) {
  uint32_t h = hash_col(c) >> (32 - __builtin_ctz(SLOTS));
  for (int p = 0; p < SLOTS; ++p) {
    int32_t k = keys[h];
    if (k == c) {
      fresh = false;
      return (int)h;
    }
    if (k == -1) {
      int32_t old = atomicCAS(&keys[h], -1, c);
      if (old == -1) {
        fresh = true;
        return (int)h;
      }
      if (old == c) {
        fresh = false;
        return (int)h;
      }
    }
    h = (h + 1) & (SLOTS - 1);
  }
  fresh = false;
  return -1;
}

template <int SLOTS>
__device__ inline int hash_find(const int32_t* keys, int32_t c) {
  uint32_t h = hash_col(c) >> (32 - __builtin_ctz(SLOTS));
  for (int p = 0; p < SLOTS; ++p) {
    int32_t k = keys[h];
    if (k == c) return (int)h;
    if (k == -1) return -1;
    h = (h + 1) & (SLOTS - 1);
  }
  return -1;
}

// Take `ncap` slots of C's pool (lane `0` of the group asks, all get it).
template <int G>
__device__ inline int64_t take_pool(const RowArgs& R, int32_t ncap, const Grp<G>& grp, int64_t* slot) {
  int64_t no = 0;
  if (grp.lane == 0) no = (int64_t)atomicAdd((unsigned long long*)R.c_top, (unsigned long long)ncap);
  no = grp.bcast64(no, 0, slot);
  return no + ncap > R.c_pool_cap ? -1 : no;
}

// Row q could not be placed (C pool or staging arena full): nothing of it was
// written.  Record the exact room it needs; the host grows the space and
// recomputes the flagged rows.
__device__ inline void mark_retry(const RowArgs& R, int32_t q, unsigned long long* counter,
                                  unsigned long long need) {
  R.retry[q] = 1;
  R.chg[q] = 0;
  atomicAdd(counter, need);
}

// ---------------------------------------------------------------------------
// bins 0-7: lane group per row, LDS hash
// ---------------------------------------------------------------------------

template <int SR, int G, int WG>
__global__ __launch_bounds__(WG) void k_rows_group(RowArgs R, const int32_t* list, const unsigned long long* d_cnt,
                                                   int bin) {
  using S = Sem<SR>;
  using V = typename S::V;
  using Acc = typename S::Acc;
  constexpr int SLOTS = 8 * G;
  constexpr int GPB = WG / G;
  __shared__ int32_t hk[GPB][SLOTS];
  __shared__ Acc hv[GPB][SLOTS];
  __shared__ int32_t ck[GPB][G];
  __shared__ V ca[GPB][G];
  __shared__ int64_t cb[GPB][G];
  __shared__ int32_t cp[GPB][G + 1];
  __shared__ int32_t so[GPB][S::order_free ? 1 : G];
  __shared__ int wscr[16];
  __shared__ int64_t bslot;

  const Grp<G> grp;
  const int g = threadIdx.x / G;
  const int lane = grp.lane;
  if (R.defer && *R.defer) return;
  const int64_t count = (int64_t)*d_cnt;
  int32_t* keys = hk[g];
  Acc* vals = hv[g];
  // rows qi = group, group + all groups of the grid, ... (one pass when the
  // grid covers the bin; persistent when it does not)
  for (int64_t qi = (int64_t)blockIdx.x * GPB + g; qi < count; qi += (int64_t)gridDim.x * GPB) {
  grp.sync();  // the previous row's readers are done with the table
  const int32_t q = list[qi];
  const int32_t i = R.aff[q];

  for (int s = lane; s < SLOTS; s += G) {
    keys[s] = -1;
    if constexpr (S::order_free) vals[s] = S::identity();
  }
  grp.sync();

  const int64_t aoff = R.a_off[i];
  const int32_t d = R.a_len[i];
  int64_t flops = 0;
  bool overflow = false;
  int32_t fresh_n = 0;  // keys this lane inserted first: the new row length sums them
  for (int32_t cbase = 0; cbase < d; cbase += G) {
    const int32_t t = cbase + lane;
    const int cnt = min(G, d - cbase);
    int32_t k = 0, len = 0;
    V a = V(0);
    int64_t boff = 0;
    if (t < d) {
      k = R.a_col[aoff + t];
      a = ldv<V>(R.a_val, aoff + t);
      len = R.b_len[k];
      boff = R.b_off[k];
    }
    int32_t tot;
    int32_t incl = grp.scan(len, tot, wscr);
    ck[g][lane] = k;
    ca[g][lane] = a;
    cb[g][lane] = boff;
    cp[g][lane + 1] = incl;
    if (lane == 0) cp[g][0] = 0;
    flops += tot;
    grp.sync();
    if constexpr (S::order_free) {
      for (int32_t fb = 0; fb < tot; fb += G) {
        int32_t f = fb + lane;
        if (f < tot) {
          int ts = find_seg(cp[g], cnt, f);
          int64_t pos = cb[g][ts] + (f - cp[g][ts]);
          int32_t j = R.b_col[pos];
          Acc p = S::mul(ca[g][ts], ldv<V>(R.b_val, pos));
          bool fresh;
          int h = hash_insert<SLOTS>(keys, j, fresh);
          if (h >= 0) S::atomic_combine(&vals[h], p);
          else overflow = true;
          fresh_n += fresh;
        }
      }
    } else {
      // ascending k inside the chunk (the whole row when d <= G)
      if (t < d) {
        int r = 0;
        for (int x = 0; x < cnt; ++x) r += ck[g][x] < k;
        so[g][r] = lane;
      }
      grp.sync();
      for (int x = 0; x < cnt; ++x) {
        const int ts = so[g][x];
        const int32_t blen = cp[g][ts + 1] - cp[g][ts];
        const int64_t bo = cb[g][ts];
        const V av = ca[g][ts];
        for (int32_t e = lane; e < blen; e += G) {
          int32_t j = R.b_col[bo + e];
          Acc p = S::mul(av, ldv<V>(R.b_val, bo + e));
          bool fresh;
          int h = hash_insert<SLOTS>(keys, j, fresh);
          if (h >= 0) vals[h] = fresh ? p : __dadd_rn(vals[h], p);
          else overflow = true;
          fresh_n += fresh;
        }
        grp.sync();
      }
    }
    grp.sync();
  }
  if (grp.any(overflow, wscr)) {
    if (lane == 0) atomicOr(R.err, 2);
    continue;
  }

  // new row length
  int32_t nnew = 0;
  grp.scan(fresh_n, nnew, wscr);
  const int64_t ooff = R.c_off[i];
  const int32_t olen = R.c_len[i];
  bool changed = R.force_write || nnew != olen;
  int64_t old_read = 0;
  if (!changed) {
    old_read = olen;
    for (int32_t ob = 0; ob < olen; ob += G) {
      int32_t e = ob + lane;
      bool bad = false;
      if (e < olen) {
        int h = hash_find<SLOTS>(keys, R.c_col[ooff + e]);
        bad = h < 0 || !same_bits(vals[h], S::to_acc(ldv<V>(R.c_val, ooff + e)));
      }
      if (grp.any(bad, wscr)) {
        changed = true;
        break;
      }
    }
  }
  if (changed) {
    int64_t dest = ooff;
    int32_t ncap = 0;
    if (nnew > R.c_cap[i]) {
      ncap = slack_cap(nnew);
      dest = take_pool<G>(R, ncap, grp, &bslot);
      if (dest < 0) {
        if (lane == 0) mark_retry(R, q, R.c_short, (unsigned long long)ncap);
        continue;
      }
    }
    // lane l writes its slots l, l + G, ... in a run of its own (one scan)
    constexpr int SPL = SLOTS / G;
    int32_t mine = 0;
#pragma unroll
    for (int u = 0; u < SPL; ++u) mine += keys[u * G + lane] != -1;
    int32_t ntot;
    int32_t w = grp.scan(mine, ntot, wscr) - mine;
#pragma unroll
    for (int u = 0; u < SPL; ++u) {
      const int s = u * G + lane;
      const int32_t key = keys[s];
      if (key != -1) {
        R.c_col[dest + w] = key;
        ((V*)R.c_val)[dest + w] = S::from_acc(vals[s]);
        ++w;
      }
    }
    if (lane == 0) {
      R.c_len[i] = nnew;
      if (ncap) {
        R.c_off[i] = dest;
        R.c_cap[i] = ncap;
      }
    }
  }
  if (lane == 0) {
    R.chg[q] = changed ? 1 : 0;
    row_stat(R, q, d, flops, nnew, olen, old_read, changed ? nnew : 0);
  }
  }  // rows
}

// ---------------------------------------------------------------------------
// A-row chunk staging shared by the workgroup-per-row kernels (bins 8, 9)
// ---------------------------------------------------------------------------

template <class V>
struct AChunk {
  int32_t k[DENSE_ACHUNK];
  V a[DENSE_ACHUNK];
  int64_t b[DENSE_ACHUNK];
  int32_t pre[DENSE_ACHUNK + 1];
  int32_t so[DENSE_ACHUNK];
};

// Entries of a staged chunk split by B-row length.  Long rows are cut into
// 64-entry tiles that the wavefronts share (each tile is one coalesced
// wavefront load, and one hub row cannot stall a single wavefront); short
// rows are flattened over the workgroup with a binary search in their own
// prefix sums.
constexpr int LONG_ROW = 64;
struct ChunkSplit {
  int32_t lidx[DENSE_ACHUNK];
  int32_t tpre[DENSE_ACHUNK + 1];  // tile prefix over long entries
  int32_t sidx[DENSE_ACHUNK];
  int32_t spre[DENSE_ACHUNK + 1];  // flop prefix over short entries
  int32_t nlong, nshort;
};

template <class V, int WG>
__device__ inline void split_chunk(const AChunk<V>& ch, int cnt, ChunkSplit& sp, const Grp<WG>& grp,
                                   int* wscr) {
  const int lane = grp.lane;
  const bool act = lane < cnt;
  const int32_t len = act ? ch.pre[lane + 1] - ch.pre[lane] : 0;
  const bool lng = act && len >= LONG_ROW;
  const bool sht = act && len > 0 && len < LONG_ROW;
  int nl, ns;
  const int rl = grp.rank(lng, nl, wscr);
  const int rs = grp.rank(sht, ns, wscr);
  int32_t stot, ttot;
  const int32_t sincl = grp.scan(sht ? len : 0, stot, wscr);
  const int32_t tincl = grp.scan(lng ? (len + 63) >> 6 : 0, ttot, wscr);
  if (lng) {
    sp.lidx[rl] = lane;
    sp.tpre[rl + 1] = tincl;
  }
  if (sht) {
    sp.sidx[rs] = lane;
    sp.spre[rs + 1] = sincl;
  }
  if (lane == 0) {
    sp.spre[0] = 0;
    sp.tpre[0] = 0;
    sp.nlong = nl;
    sp.nshort = ns;
  }
  grp.sync();
}

// Stage A entries [cbase, cbase+cnt) and prefix sums of their B-row lengths.
// Returns the chunk's flop count.  Whole-workgroup call.
// part >= 0: B rows are the entries of column chunk `part` in the split copy.
template <class V, int WG>
__device__ inline int32_t stage_chunk(const RowArgs& R, int64_t aoff, int32_t d, int32_t cbase, AChunk<V>& ch,
                                      const Grp<WG>& grp, int* wscr, bool sort_k, int part = -1) {
  const int lane = grp.lane;
  const int32_t t = cbase + lane;
  const bool act = lane < DENSE_ACHUNK && t < d;
  int32_t k = 0, len = 0;
  V a = V(0);
  int64_t boff = 0;
  if (act) {
    k = R.a_col[aoff + t];
    a = ldv<V>(R.a_val, aoff + t);
    if (part >= 0) {
      const int64_t* ps = R.bs_ps + (int64_t)k * (R.bs_parts + 1) + part;
      boff = ps[0];
      len = (int32_t)(ps[1] - boff);
    } else {
      len = R.b_len[k];
      boff = R.b_off[k];
    }
  }
  int32_t tot;
  int32_t incl = grp.scan(len, tot, wscr);
  if (lane < DENSE_ACHUNK) {
    ch.k[lane] = k;
    ch.a[lane] = a;
    ch.b[lane] = boff;
    ch.pre[lane + 1] = incl;
  }
  if (lane == 0) ch.pre[0] = 0;
  grp.sync();
  if (sort_k) {
    const int cnt = min(DENSE_ACHUNK, d - cbase);
    if (act) {
      int r = 0;
      for (int x = 0; x < cnt; ++x) r += ch.k[x] < k;
      ch.so[r] = lane;
    }
    grp.sync();
  }
  return tot;
}

// ---------------------------------------------------------------------------
// bin 8: dense LDS accumulator over column chunks, one workgroup per row
// ---------------------------------------------------------------------------

// Slot of key c in an LDS open-addressing table (linear probing from slot h,
// whose key k was already read), inserting c where it was absent; -1 when
// `probes` slots are taken by other keys.
template <int SLOTS, int PROBES>
__device__ inline int hash_place(int32_t* keys, int32_t c, uint32_t h, int32_t k) {
  for (int p = 0; p < PROBES; ++p) {
    if (k == c) return (int)h;
    if (k == -1) {
      const int32_t old = atomicCAS(&keys[h], -1, c);
      if (old == -1 || old == c) return (int)h;
    }
    h = (h + 1) & (SLOTS - 1);
    k = keys[h];
  }
  return -1;
}

// Orders the LDS accesses of the lanes of one wavefront.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Value of lane src of a VGPR (src uniform), 64-bit and value-typed forms.
__device__ inline int64_t lane64(int64_t v, int src) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), src);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <class V>
__device__ inline V lanev(V v, int src) {
  if constexpr (sizeof(V) == 4) {
    return __builtin_bit_cast(V, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
  } else {
    return __builtin_bit_cast(V, lane64(__builtin_bit_cast(int64_t, v), src));
  }
}

template <int SR>
__global__ __launch_bounds__(DENSE_WG) void k_rows_dense(RowArgs R, const int32_t* list,
                                                         const unsigned long long* d_cnt) {
  using S = Sem<SR>;
  using V = typename S::V;
  using Acc = typename S::Acc;
  constexpr int CH = dense_cols<sizeof(V)>();
  constexpr int NWV = DENSE_WG / 64;
  constexpr int NW32 = CH / 32;       // bitmap words per column chunk
  constexpr int SEGW = NW32 / NWV;    // words of the segment each wavefront drains
  constexpr int SEG = SEGW * 32;      // columns of that segment
  static_assert(SEGW >= 2 && SEGW % 2 == 0, "segments are walked 64 columns at a time");
  // The accumulator and its touched-column bitmap are all identity / zero
  // between chunks and rows: the drain that reads a chunk out clears it.
  __shared__ Acc acc[CH];
  __shared__ uint32_t bits[NW32];
  __shared__ AChunk<V> ch;
  __shared__ ChunkSplit sp;
  __shared__ int wscr[16];
  __shared__ uint64_t wscr64[NWV];
  __shared__ int64_t bslot;
  __shared__ int32_t next_row;
  const Grp<DENSE_WG> grp;
  const int tid = threadIdx.x;
  const int wv = tid >> 6, ln = tid & 63;
  const uint64_t lt = ln ? (~0ull >> (64 - ln)) : 0ull;
  if (R.defer && *R.defer) return;
  const int64_t count = (int64_t)*d_cnt;
  for (int x = tid; x < CH; x += DENSE_WG) acc[x] = S::identity();
  for (int x = tid; x < NW32; x += DENSE_WG) bits[x] = 0u;
  // persistent: rows are taken in list order (longest first) from a counter;
  // each workgroup claims its next row while it works on the current one
  unsigned int pending = 0;
  if (tid == 0) pending = atomicAdd(R.dense_next, 1u);
  for (;;) {
  if (tid == 0) {
    next_row = (int32_t)pending;
    pending = atomicAdd(R.dense_next, 1u);
  }
  grp.sync();
  const int32_t qi = next_row;
  grp.sync();
  if (qi >= count) break;
  const int32_t q = list[qi];
  const int32_t i = R.aff[q];
  const int64_t aoff = R.a_off[i];
  const int32_t d = R.a_len[i];
  const int32_t ub = R.ub[q];
  const int64_t ooff = R.c_off[i];
  const int32_t olen = R.c_len[i];
  const int32_t stage_n = min(ub, R.ncols);
  const int passes = (R.ncols + CH - 1) / CH;
  // MLP rounds of UNR independent flops per lane: all loads first, then the
  // LDS updates, so each lane keeps UNR gathers in flight
  constexpr int UNR = DENSE_WG >= 1024 ? 4 : 16;  // 16: 3% faster than 8; 32 spills
  // Stage A entries [cbase, cbase + 512) (column k, value, B row offset and
  // length: the whole B row, or its column chunk `part` of the split copy)
  // and split them by B-row length with one 64-bit workgroup scan.  Packed
  // fields: bits 0-23 quads (256 entries) of long rows, 24-39 entries of
  // short rows, 40-49 short rows, 50-59 long rows (none overflows: at most
  // 512 rows of at most 2^15 quads, or of fewer than 64 entries).
  auto stage_split = [&](int32_t cbase, bool use_split, int part) {
    const int32_t t = cbase + tid;
    const bool act = tid < DENSE_ACHUNK && t < d;
    int32_t k = 0, len = 0;
    V a = V(0);
    int64_t boff = 0;
    if (act) {
      k = R.a_col[aoff + t];
      a = ldv<V>(R.a_val, aoff + t);
      if (use_split) {
        const int64_t* ps = R.bs_ps + (int64_t)k * (R.bs_parts + 1) + part;
        boff = ps[0];
        len = (int32_t)(ps[1] - boff);
      } else {
        len = R.b_len[k];
        boff = R.b_off[k];
      }
    }
    const bool lng = act && len >= LONG_ROW;
    const bool sht = act && len > 0 && len < LONG_ROW;
    const uint64_t v = (lng ? (uint64_t)((len + 255) >> 8) : 0ull) | (sht ? (uint64_t)len << 24 : 0ull) |
                       ((uint64_t)sht << 40) | ((uint64_t)lng << 50);
    uint64_t inc = wave_inclusive_scan(v);
    if (ln == 63) wscr64[wv] = inc;
    grp.sync();
    uint64_t before = 0, tot = 0;
    for (int x = 0; x < NWV; ++x) {
      const uint64_t c = wscr64[x];
      if (x < wv) before += c;
      tot += c;
    }
    inc += before;
    const uint64_t exc = inc - v;
    if (tid < DENSE_ACHUNK) {
      ch.k[tid] = k;
      ch.a[tid] = a;
      ch.b[tid] = boff;
      ch.so[tid] = len;  // (lengths: the order-free path sorts nothing)
    }
    if (lng) {
      const int rl = (int)((exc >> 50) & 0x3ff);
      sp.lidx[rl] = tid;
      sp.tpre[rl + 1] = (int32_t)(inc & 0xffffff);
    }
    if (sht) {
      const int rs = (int)((exc >> 40) & 0x3ff);
      sp.sidx[rs] = tid;
      sp.spre[rs + 1] = (int32_t)((inc >> 24) & 0xffff);
    }
    if (tid == 0) {
      sp.spre[0] = 0;
      sp.tpre[0] = 0;
      sp.nlong = (int32_t)((tot >> 50) & 0x3ff);
      sp.nshort = (int32_t)((tot >> 40) & 0x3ff);
    }
    grp.sync();
  };
  // Every product of the staged chunk through round(jp, vp, av, ok), UNR per
  // lane at a time: jp/vp point at the lane's B column index and value (in
  // bcol/bval), av is the A value, ok whether the product exists.  Every
  // pointer is readable, so the rounds load without branches.
  auto for_rounds = [&](auto&& round, const int32_t* bcol, const void* bval) {
    // Long B rows as quads: four 64-entry tiles, 256 entries of one row.
    // Wavefront w takes QPR quads per round, rounds QSTRIDE quads apart.
    // Lane l describes the (l % QPR)-th quad of the (l / QPR)-th of the next
    // RPD rounds (one segment search per lane), and each round reads its
    // quads' position, remaining length and A value from those lanes.  The
    // four loads of a quad share one wave-uniform base address; lanes past
    // the row's end read the next entries of the pool (or its padding) and
    // are masked.
    constexpr int QPR = UNR / 4;
    constexpr int RPD = 64 / QPR;  // rounds per description
    constexpr int QSTRIDE = NWV * QPR;
    static_assert(UNR % 4 == 0 && 4 * 64 <= POOL_PAD, "quads of four tiles within the pool padding");
    const int nl = sp.nlong;
    const int nquads = sp.tpre[nl];
    const uint32_t lane_c = (uint32_t)ln * 4u;
    const uint32_t lane_v = (uint32_t)ln * (uint32_t)sizeof(V);
    for (int qb0 = wv * QPR; qb0 < nquads; qb0 += QSTRIDE * RPD) {
      const int my = qb0 + (ln / QPR) * QSTRIDE + (ln % QPR);
      int64_t mpos = 0;
      V ma = V(0);
      int32_t mrem = 0;
      if (my < nquads) {
        const int e = find_seg(sp.tpre, nl, my);
        const int t = sp.lidx[e];
        const int32_t x0 = (my - sp.tpre[e]) << 8;
        mrem = ch.so[t] - x0;
        mpos = ch.b[t] + x0;
        ma = ch.a[t];
      }
      for (int r = 0; r < RPD && qb0 + r * QSTRIDE < nquads; ++r) {
        const int32_t* jp[UNR];
        const V* vp[UNR];
        V av[UNR];
        bool ok[UNR];
#pragma unroll
        for (int g = 0; g < QPR; ++g) {
          const int src = r * QPR + g;
          const int32_t rem = __builtin_amdgcn_readlane(mrem, src);
          const int64_t q0 = lane64(mpos, src);
          const V a = lanev<V>(ma, src);
          const char* cb = (const char*)(bcol + q0);
          const char* vb = (const char*)((const V*)bval + q0);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int u = g * 4 + t;
            jp[u] = (const int32_t*)(cb + lane_c + t * 256);
            vp[u] = (const V*)(vb + lane_v + t * 64 * (int)sizeof(V));
            av[u] = a;
            ok[u] = t * 64 + ln < rem;
          }
        }
        round(jp, vp, av, ok);
      }
    }
    // short B rows: 8-lane sub-groups, each streaming 4 rows at once (no
    // search; lanes past a row's end re-read its last entry)
    const int ns = sp.nshort;
    constexpr int NSG = DENSE_WG / 8;
    const int sg = tid >> 3, l8 = tid & 7;
    for (int eb = sg; eb < ns; eb += 4 * NSG) {
      int64_t bo[4];
      int32_t bl[4];
      V ba[4];
      int32_t mx = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = eb + u * NSG;
        bl[u] = 0;
        bo[u] = 0;
        ba[u] = V(0);
        if (e < ns) {
          const int t = sp.sidx[e];
          bo[u] = ch.b[t];
          bl[u] = ch.so[t];
          ba[u] = ch.a[t];
          mx = max(mx, bl[u]);
        }
      }
      for (int32_t x = l8; x < mx; x += 2 * UNR) {
        const int32_t* jp[UNR];
        const V* vp[UNR];
        V av[UNR];
        bool ok[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const int r = u & 3;
          const int32_t xx = x + (u >> 2) * 8;
          ok[u] = xx < bl[r];
          const int64_t pp = bo[r] + min(xx, max(bl[r] - 1, 0));
          jp[u] = bcol + pp;
          vp[u] = (const V*)bval + pp;
          av[u] = ba[r];
        }
        round(jp, vp, av, ok);
      }
    }
  };
  // (min,+) rows expected to hold at most HFILL entries take one pass over
  // all columns with an open-addressing hash in the accumulator's space
  // (HSLOTS keys, then HSLOTS values; empty keys and values are both all
  // ones, the accumulator's identity, so the cleared table is the cleared
  // accumulator).  The expectation is the old row's length plus slack (the
  // flop bound when the row is new); a row that outgrows it overflows a probe
  // chain and is redone with the column passes below.
  if constexpr (SR == 1) {
    constexpr int HSLOTS = CH / 2;
    constexpr int HBITS = __builtin_ctz(HSLOTS);
    constexpr int HFILL = HSLOTS * 3 / 5;  // measured: 1/3 2/5 1/2 3/5 2/3 3/4 4/5, 3/5 fastest
    constexpr int HPROBES = 128;
    static_assert(sizeof(Acc) == 4, "(min,+) keys: the identity 0xffffffff doubles as the empty key -1");
    int32_t* hk = (int32_t*)acc;
    Acc* hv = acc + HSLOTS;
    const int32_t expect = olen > 0 ? olen + (olen >> 3) + 64 : stage_n;
    if (expect <= HFILL) {
      bool over = false;
      auto hash_round = [&](const int32_t* const* jp, const V* const* vp, const V* av, const bool* ok) {
        int32_t j[UNR];
        V bv[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          j[u] = *jp[u];
          bv[u] = *vp[u];
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u)
          if (!ok[u]) j[u] = -1;
        uint32_t h[UNR];
        int32_t k[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {  // first probes read together
          h[u] = hash_col(j[u]) >> (32 - HBITS);
          k[u] = ok[u] ? hk[h[u]] : 0;
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          if (ok[u]) {
            const int hh = hash_place<HSLOTS, HPROBES>(hk, j[u], h[u], k[u]);
            if (hh >= 0) atomicMin(&hv[hh], S::mul(av[u], bv[u]));
            else over = true;
          }
        }
      };
      for (int32_t cbase = 0; cbase < d; cbase += DENSE_ACHUNK) {
        stage_split(cbase, false, 0);
        for_rounds(hash_round, R.b_col, R.b_val);
        grp.sync();
      }
      if (grp.any(over, wscr)) {
        for (int x = tid; x < CH; x += DENSE_WG) acc[x] = S::identity();
        grp.sync();
      } else {
        // entries per wavefront segment of HSLOTS / NWV slots
        constexpr int HSEG = HSLOTS / NWV;
        int32_t mine = 0;
        for (int r = 0; r < HSEG; r += 64) mine += __popcll(__ballot(hk[wv * HSEG + r + ln] != -1));
        if (ln == 0) wscr[wv] = mine;
        grp.sync();
        int32_t before = 0, nnew = 0;
        for (int x = 0; x < NWV; ++x) {
          const int32_t c = wscr[x];
          if (x < wv) before += c;
          nnew += c;
        }
        grp.sync();
        bool changed = R.force_write || nnew != olen;
        int64_t old_read = 0;
        if (!changed) {  // every old entry present with the same value
          bool bad = false;
          for (int32_t e0 = tid; e0 < olen; e0 += 8 * DENSE_WG) {
            int32_t oc[8];
            V ov[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int32_t e = e0 + u * DENSE_WG;
              oc[u] = e < olen ? R.c_col[ooff + e] : -1;
              ov[u] = e < olen ? ldv<V>(R.c_val, ooff + e) : V(0);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              if (oc[u] < 0) continue;
              uint32_t hh = hash_col(oc[u]) >> (32 - HBITS);
              bool found = false;
              for (int p = 0; p < HSLOTS; ++p) {
                const int32_t kk = hk[hh];
                if (kk == oc[u]) {
                  found = true;
                  break;
                }
                if (kk == -1) break;
                hh = (hh + 1) & (HSLOTS - 1);
              }
              bad |= !found || !same_bits(hv[hh], S::to_acc(ov[u]));
            }
          }
          if (grp.any(bad, wscr)) changed = true;
          old_read = olen;
        }
        int64_t dest = ooff;
        int32_t ncap = 0;
        bool parked = false;
        if (changed && nnew > R.c_cap[i]) {
          ncap = slack_cap(nnew);
          dest = take_pool<DENSE_WG>(R, ncap, grp, &bslot);
          if (dest < 0) {
            if (tid == 0) mark_retry(R, q, R.c_short, (unsigned long long)ncap);
            parked = true;
          }
        }
        // read the table out (slot order) and clear it
        const bool write = changed && !parked;
        int32_t o = before;
        constexpr int HU = 4;  // slot blocks of 64 read together per step
        static_assert(HSEG % (64 * HU) == 0, "readout steps");
        for (int r = 0; r < HSEG; r += 64 * HU) {
          int32_t kk[HU];
          Acc vv[HU];
#pragma unroll
          for (int u = 0; u < HU; ++u) {
            const int sl = wv * HSEG + r + u * 64 + ln;
            kk[u] = hk[sl];
            vv[u] = hv[sl];
          }
#pragma unroll
          for (int u = 0; u < HU; ++u) {
            const int sl = wv * HSEG + r + u * 64 + ln;
            const uint64_t b = __ballot(kk[u] != -1);
            if (write && kk[u] != -1) {
              const int64_t pos = dest + o + __popcll(b & lt);
              R.c_col[pos] = kk[u];
              ((V*)R.c_val)[pos] = S::from_acc(vv[u]);
            }
            hk[sl] = -1;
            hv[sl] = S::identity();
            o += __popcll(b);
          }
        }
        if (write && tid == 0) {
          R.c_len[i] = nnew;
          if (ncap) {
            R.c_off[i] = dest;
            R.c_cap[i] = ncap;
          }
        }
        grp.sync();
        if (!parked && tid == 0) {
          R.chg[q] = changed ? 1 : 0;
          row_stat(R, q, d, R.flq[q], nnew, olen, old_read, changed ? nnew : 0);
        }
        continue;
      }
    }
  }
  // staging space holds the chunks before the last one (none for a one-pass row)
  int32_t* scol = nullptr;
  V* sval = nullptr;
  if (passes > 1) {
    const size_t stage_bytes = (((size_t)stage_n * (4 + sizeof(V))) + 255) & ~size_t(255);
    int64_t sbase = 0;
    if (tid == 0) sbase = (int64_t)atomicAdd(R.arena_top, (unsigned long long)stage_bytes);
    sbase = grp.bcast64(sbase, 0, &bslot);
    if (sbase + (int64_t)stage_bytes > R.arena_cap) {
      if (tid == 0) mark_retry(R, q, R.arena_short, (unsigned long long)stage_bytes);
      continue;
    }
    scol = (int32_t*)(R.arena + sbase);
    sval = (V*)(R.arena + sbase + (size_t)stage_n * 4);
  }

  bool changed = R.force_write;
  bool direct = false;  // the chunks drained so far sit in the row's own place in C
  bool fault = false, parked = false;
  int32_t nnew = 0;
  const int64_t flops = R.flq[q];  // the row's products, from the analysis
  int64_t old_read = 0;
  // with the split copy of B each pass streams only its own column chunk
  const bool split = R.bs_parts == passes && passes > 1;
  const int32_t* bcol = split ? R.bs_col : R.b_col;
  const void* bval = split ? R.bs_val : R.b_val;
  for (int pc = 0; pc < passes; ++pc) {
    const int32_t c0 = pc * CH;
    const int32_t c1 = min(c0 + CH, R.ncols);
    auto accumulate_round = [&](const int32_t* const* jp, const V* const* vp, const V* av, const bool* ok) {
      int32_t j[UNR];
      V bv[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        j[u] = *jp[u];
        bv[u] = *vp[u];
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u)
        if (!ok[u]) j[u] = -1;
      if constexpr (S::order_free) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          if (j[u] >= c0 && j[u] < c1) {
            const int x = j[u] - c0;
            S::atomic_combine(&acc[x], S::mul(av[u], bv[u]));
            atomicOr(&bits[x >> 5], 1u << (x & 31));
          }
        }
      }
    };
    for (int32_t cbase = 0; cbase < d; cbase += DENSE_ACHUNK) {
      const int cnt = min(DENSE_ACHUNK, d - cbase);
      if constexpr (S::order_free) {
        stage_split(cbase, split, pc);
        for_rounds(accumulate_round, bcol, bval);
      } else {
        stage_chunk<V>(R, aoff, d, cbase, ch, grp, wscr, true, split ? pc : -1);
        for (int y = 0; y < cnt; ++y) {
          const int ts = ch.so[y];
          const int32_t blen = ch.pre[ts + 1] - ch.pre[ts];
          const int64_t bo = ch.b[ts];
          const V av = ch.a[ts];
          for (int32_t e = tid; e < blen; e += DENSE_WG) {
            int32_t j = bcol[bo + e];
            if (j >= c0 && j < c1) {
              int x = j - c0;
              Acc p = S::mul(av, ldv<V>(bval, bo + e));
              uint32_t m = 1u << (x & 31);
              uint32_t was = atomicOr(&bits[x >> 5], m);
              acc[x] = (was & m) ? __dadd_rn(acc[x], p) : p;
            }
          }
          grp.sync();
        }
      }
      grp.sync();
    }
    // entries of this chunk from the bitmap: wavefront w owns columns
    // [w*SEG, (w+1)*SEG)
    int32_t mine = 0;
    for (int w = ln; w < SEGW; w += 64) mine += __popc(bits[wv * SEGW + w]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mine += __shfl_xor(mine, o, 64);
    if (ln == 0) wscr[wv] = mine;
    grp.sync();
    int32_t before = 0, ctot = 0;
    for (int x = 0; x < NWV; ++x) {
      const int32_t c = wscr[x];
      if (x < wv) before += c;
      ctot += c;
    }
    grp.sync();
    // compare the old entries that fall into this chunk (8 loads in flight per
    // lane).  (min,+): an untouched slot holds the identity key, which no
    // stored value maps to, so the key comparison alone decides.
    if (!changed) {
      int32_t in_chunk = 0;
      bool bad = false;
      for (int32_t e0 = tid; e0 < olen; e0 += 8 * DENSE_WG) {
        int32_t oc[8];
        V ov[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int32_t e = e0 + u * DENSE_WG;
          oc[u] = e < olen ? R.c_col[ooff + e] : -1;
          ov[u] = e < olen ? ldv<V>(R.c_val, ooff + e) : V(0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (oc[u] >= c0 && oc[u] < c1) {
            ++in_chunk;
            const int x = oc[u] - c0;
            const bool hit = SR == 1 || ((bits[x >> 5] >> (x & 31)) & 1u);
            bad |= !hit || !same_bits(acc[x], S::to_acc(ov[u]));
          }
        }
      }
      int32_t itot;
      grp.scan(in_chunk, itot, wscr);
      if (grp.any(bad, wscr) || itot != ctot) changed = true;
      old_read = olen;
    }
    // Read the chunk out in ascending column order and clear it: each step
    // reads the bitmap words and accumulator slots of DU blocks of 64 columns
    // together, and the touched columns of a block are stored straight to
    // out[base + ...] at consecutive positions (one coalesced run per block;
    // the cache merges the runs of consecutive blocks).
    auto drain = [&](int32_t* ocol, V* oval, int64_t base, int32_t limit, bool write) {
      int32_t o = before;  // row position of the wavefront's next entry
      constexpr int DU = 4;
      static_assert(SEG % (64 * DU) == 0, "drain steps");
      for (int r = 0; r < SEG; r += 64 * DU) {
        uint64_t b[DU];
        Acc a[DU];
#pragma unroll
        for (int u = 0; u < DU; ++u) {
          const int w0 = (wv * SEG + r + u * 64) >> 5;
          b[u] = (uint64_t)bits[w0] | ((uint64_t)bits[w0 + 1] << 32);
          a[u] = acc[wv * SEG + r + u * 64 + ln];
        }
#pragma unroll
        for (int u = 0; u < DU; ++u) {
          const int x = wv * SEG + r + u * 64 + ln;
          if (write && ((b[u] >> ln) & 1ull)) {
            const int64_t pos = base + o + __popcll(b[u] & lt);
            if (pos < limit) {
              ocol[pos] = c0 + x;
              oval[pos] = S::from_acc(a[u]);
            }
          }
          acc[x] = S::identity();
          o += __popcll(b[u]);
        }
      }
      for (int w = ln; w < SEGW; w += 64) bits[wv * SEGW + w] = 0u;
    };
    // cnt entries from (sc, sv) to (dc, dv), 8 loads in flight per lane
    auto copy_entries = [&](const int32_t* sc, const V* sv, int32_t* dc, V* dv, int32_t cnt) {
      for (int32_t e0 = tid; e0 < cnt; e0 += 8 * DENSE_WG) {
        int32_t cc[8];
        V vv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int32_t e = e0 + u * DENSE_WG;
          cc[u] = e < cnt ? sc[e] : 0;
          vv[u] = e < cnt ? sv[e] : V(0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int32_t e = e0 + u * DENSE_WG;
          if (e < cnt) {
            dc[e] = cc[u];
            dv[e] = vv[u];
          }
        }
      }
    };
    int32_t* const ccol = R.c_col + ooff;
    V* const cval = (V*)R.c_val + ooff;
    const int32_t ccap = R.c_cap[i];
    if (pc + 1 < passes) {
      // Not the last chunk.  A row already known to change whose chunks so
      // far fit its place in C goes straight there; otherwise the chunk is
      // parked in the staging space.
      if (direct && nnew + ctot > ccap) {
        // (rows of three chunks or more) it outgrew its place: what is in C
        // moves to the staging space, and staging goes on from there
        copy_entries(ccol, cval, scol, sval, min(nnew, stage_n));
        direct = false;
      } else if (pc == 0 && changed && ctot <= ccap) {
        direct = true;
      }
      if (direct) drain(ccol, cval, nnew, ccap, true);
      else drain(scol, sval, nnew, stage_n, true);
      nnew += ctot;
      grp.sync();
      continue;
    }
    // last chunk: the row length is known, so the row goes straight to C
    nnew += ctot;
    if (nnew > stage_n) {
      if (tid == 0) atomicOr(R.err, 8);
      fault = true;
      break;
    }
    if (changed) {
      const int32_t prev = nnew - ctot;  // entries of the earlier chunks
      int64_t dest = ooff;
      int32_t ncap = 0;
      if (nnew > ccap) {
        ncap = slack_cap(nnew);
        dest = take_pool<DENSE_WG>(R, ncap, grp, &bslot);
        if (dest < 0) {
          if (tid == 0) {
            // its place may already hold new entries: as an empty row it is
            // seen (and reported) as changed when it is recomputed
            if (direct) R.c_len[i] = 0;
            mark_retry(R, q, R.c_short, (unsigned long long)ncap);
          }
          drain(nullptr, nullptr, 0, 0, false);
          parked = true;
          break;
        }
      }
      // earlier chunks: from the staging space, or from the row's old place
      // when it moves
      if (!direct) copy_entries(scol, sval, R.c_col + dest, (V*)R.c_val + dest, prev);
      else if (dest != ooff) copy_entries(ccol, cval, R.c_col + dest, (V*)R.c_val + dest, prev);
      drain(R.c_col + dest, (V*)R.c_val + dest, prev, nnew, true);
      if (tid == 0) {
        R.c_len[i] = nnew;
        if (ncap) {
          R.c_off[i] = dest;
          R.c_cap[i] = ncap;
        }
      }
    } else {
      drain(nullptr, nullptr, 0, 0, false);
    }
    grp.sync();
  }
  if (fault) break;
  if (parked) continue;
  if (tid == 0) {
    R.chg[q] = changed ? 1 : 0;
    row_stat(R, q, d, flops, nnew, olen, old_read, changed ? nnew : 0);
  }
  }  // rows
}

// ---------------------------------------------------------------------------
// bin 9: hash table in device memory, one workgroup per row
// ---------------------------------------------------------------------------

template <class T>
__device__ inline T aload(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int64_t global_slots(int32_t ub) {
  int64_t s = 2048;
  while (s < 2 * (int64_t)ub) s <<= 1;
  return s;
}

__device__ inline int64_t ghash_insert(int32_t* keys, int64_t slots, int32_t c, bool& fresh) {
  int64_t h = (int64_t)(hash_col(c) & (uint32_t)(slots - 1));
  for (int64_t p = 0; p < slots; ++p) {
    int32_t k = aload(&keys[h]);
    if (k == c) {
      fresh = false;
      return h;
    }
    if (k == -1) {
      int32_t old = atomicCAS(&keys[h], -1, c);
      if (old == -1) {
        fresh = true;
        return h;
      }
      if (old == c) {
        fresh = false;
        return h;
      }
    }
    h = (h + 1) & (slots - 1);
  }
  fresh = false;
  return -1;
}

__device__ inline int64_t ghash_find(const int32_t* keys, int64_t slots, int32_t c) {
  int64_t h = (int64_t)(hash_col(c) & (uint32_t)(slots - 1));
  for (int64_t p = 0; p < slots; ++p) {
    int32_t k = aload(&keys[h]);
    if (k == c) return h;
    if (k == -1) return -1;
    h = (h + 1) & (slots - 1);
  }
  return -1;
}

template <int SR>
__global__ __launch_bounds__(GLOBAL_WG) void k_rows_global(RowArgs R, const int32_t* list,
                                                          const unsigned long long* d_cnt) {
  using S = Sem<SR>;
  using V = typename S::V;
  using Acc = typename S::Acc;
  __shared__ AChunk<V> ch;
  __shared__ int wscr[16];
  __shared__ int64_t bslot;
  const Grp<GLOBAL_WG> grp;
  const int tid = threadIdx.x;
  if (R.defer && *R.defer) return;
  const int64_t count = (int64_t)*d_cnt;
  for (int64_t qi = blockIdx.x; qi < count; qi += gridDim.x) {
  grp.sync();
  const int32_t q = list[qi];
  const int32_t i = R.aff[q];
  const int64_t aoff = R.a_off[i];
  const int32_t d = R.a_len[i];
  const int64_t slots = global_slots(R.ub[q]);
  const size_t tbytes = ((size_t)slots * (4 + sizeof(Acc)) + 255) & ~size_t(255);
  int64_t tb = 0;
  if (tid == 0) tb = (int64_t)atomicAdd(R.arena_top, (unsigned long long)tbytes);
  tb = grp.bcast64(tb, 0, &bslot);
  if (tb + (int64_t)tbytes > R.arena_cap) {
    if (tid == 0) mark_retry(R, q, R.arena_short, (unsigned long long)tbytes);
    continue;
  }
  int32_t* keys = (int32_t*)(R.arena + tb);
  Acc* vals = (Acc*)(R.arena + tb + (size_t)slots * 4);
  for (int64_t s = tid; s < slots; s += GLOBAL_WG) {
    __hip_atomic_store(&keys[s], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&vals[s], S::identity(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __threadfence();
  grp.sync();
  int64_t flops = 0;
  bool overflow = false;
  for (int32_t cbase = 0; cbase < d; cbase += DENSE_ACHUNK) {
    const int cnt = min(DENSE_ACHUNK, d - cbase);
    int32_t tot = stage_chunk<V>(R, aoff, d, cbase, ch, grp, wscr, !S::order_free);
    flops += tot;
    if constexpr (S::order_free) {
      for (int32_t fb = 0; fb < tot; fb += GLOBAL_WG) {
        int32_t f = fb + tid;
        if (f < tot) {
          int ts = find_seg(ch.pre, cnt, f);
          int64_t pos = ch.b[ts] + (f - ch.pre[ts]);
          bool fresh;
          int64_t h = ghash_insert(keys, slots, R.b_col[pos], fresh);
          if (h >= 0) S::atomic_combine(&vals[h], S::mul(ch.a[ts], ldv<V>(R.b_val, pos)));
          else overflow = true;
        }
      }
    } else {
      for (int y = 0; y < cnt; ++y) {
        const int ts = ch.so[y];
        const int32_t blen = ch.pre[ts + 1] - ch.pre[ts];
        const int64_t bo = ch.b[ts];
        const V av = ch.a[ts];
        for (int32_t e = tid; e < blen; e += GLOBAL_WG) {
          Acc p = S::mul(av, ldv<V>(R.b_val, bo + e));
          bool fresh;
          int64_t h = ghash_insert(keys, slots, R.b_col[bo + e], fresh);
          if (h < 0) {
            overflow = true;
          } else if (fresh) {
            __hip_atomic_store(&vals[h], p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          } else {
            Acc cur = aload(&vals[h]);
            __hip_atomic_store(&vals[h], __dadd_rn(cur, p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
        __threadfence();
        grp.sync();
      }
    }
    __threadfence();
    grp.sync();
  }
  if (grp.any(overflow, wscr)) {
    if (tid == 0) atomicOr(R.err, 2);
    continue;
  }
  int32_t nnew = 0;
  for (int64_t sb = 0; sb < slots; sb += GLOBAL_WG) {
    int tot;
    grp.rank(aload(&keys[sb + tid]) != -1, tot, wscr);
    nnew += tot;
  }
  const int64_t ooff = R.c_off[i];
  const int32_t olen = R.c_len[i];
  bool changed = R.force_write || nnew != olen;
  int64_t old_read = 0;
  if (!changed) {
    old_read = olen;
    for (int32_t ob = 0; ob < olen; ob += GLOBAL_WG) {
      int32_t e = ob + tid;
      bool bad = false;
      if (e < olen) {
        int64_t h = ghash_find(keys, slots, R.c_col[ooff + e]);
        bad = h < 0 || !same_bits(aload(&vals[h]), S::to_acc(ldv<V>(R.c_val, ooff + e)));
      }
      if (grp.any(bad, wscr)) {
        changed = true;
        break;
      }
    }
  }
  if (changed) {
    int64_t dest = ooff;
    int32_t ncap = 0;
    if (nnew > R.c_cap[i]) {
      ncap = slack_cap(nnew);
      dest = take_pool<GLOBAL_WG>(R, ncap, grp, &bslot);
      if (dest < 0) {
        if (tid == 0) mark_retry(R, q, R.c_short, (unsigned long long)ncap);
        continue;
      }
    }
    int32_t w = 0;
    for (int64_t sb = 0; sb < slots; sb += GLOBAL_WG) {
      const int64_t s = sb + tid;
      const int32_t key = aload(&keys[s]);
      int tot;
      int r = grp.rank(key != -1, tot, wscr);
      if (key != -1) {
        R.c_col[dest + w + r] = key;
        ((V*)R.c_val)[dest + w + r] = S::from_acc(aload(&vals[s]));
      }
      w += tot;
    }
    if (tid == 0) {
      R.c_len[i] = nnew;
      if (ncap) {
        R.c_off[i] = dest;
        R.c_cap[i] = ncap;
      }
    }
  }
  if (tid == 0) {
    R.chg[q] = changed ? 1 : 0;
    row_stat(R, q, d, flops, nnew, olen, old_read, changed ? nnew : 0);
  }
  }  // rows
}

// ---------------------------------------------------------------------------
// discovery and analysis
// ---------------------------------------------------------------------------

__global__ void k_mark_changed(int32_t n, const uint32_t* epoch, const uint32_t* since, uint8_t* flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flags[i] = epoch[i] > *since ? 1 : 0;
}

// one wavefront per changed row k of B: flag every row i with A'[i,k] present
__global__ __launch_bounds__(256) void k_scatter_dB(const int32_t* dB, const int32_t* d_nB,
                                                    const int64_t* t_off, const int32_t* t_len,
                                                    const int32_t* t_col, uint8_t* aff) {
  const int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int lane = threadIdx.x & 63;
  const int32_t nB = *d_nB;
  for (int64_t x = wv; x < nB; x += nw) {
    const int32_t k = dB[x];
    const int64_t o = t_off[k];
    const int32_t l = t_len[k];
    for (int32_t e0 = lane; e0 < l; e0 += 64 * 8) {  // 8 loads in flight per lane (hub columns)
      int32_t c[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) c[u] = e0 + u * 64 < l ? t_col[o + e0 + u * 64] : -1;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (c[u] >= 0) aff[c[u]] = 1;
    }
  }
}

struct Tun {
  int32_t group_ub[8];
  int32_t dense_passes;  // passes the dense bin needs for this product
  int32_t dense_max_passes;
  int32_t force_bin;
  int32_t fp64;
};

struct Plan {
  int32_t count;         // affected rows
  int32_t pad;
  unsigned long long bin_count[NBINS];
  unsigned long long c_demand;      // upper bound of C slots moved rows may take
  unsigned long long arena_demand;  // upper bound of staging bytes
  unsigned int dense_next;
  unsigned int pad2;
  unsigned long long c_short;       // exact C slots that rows flagged for retry need
  unsigned long long arena_short;   // exact arena bytes they need
  unsigned long long flops;         // products the affected rows take
};

// longest rows first, to within 1/8: the key is 255 minus a log-scale bucket
// of the row's products (the exponent and the next three bits), so that one
// 8-bit radix pass orders the dense rows
constexpr int FLOP_KEY_BITS = 8;
__device__ inline uint32_t flop_bucket(int32_t f) {
  if (f < 8) return (uint32_t)max(f, 0);
  const int e = 31 - __clz(f);  // 3..30
  return (uint32_t)((e - 2) * 8 + ((f >> (e - 3)) & 7));  // 8..231, monotone in f
}
__global__ void k_flop_keys(const int32_t* list, int32_t n, const int32_t* flq, uint64_t* keys, uint32_t* vals) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) {
    const int32_t q = list[t];
    keys[t] = (uint64_t)(255u - flop_bucket(flq[q]));
    vals[t] = (uint32_t)q;
  }
}

__device__ inline int pick_bin(int32_t ub, int32_t d, const Tun& T) {
  if (T.force_bin >= BIN_DENSE) return T.force_bin;
  int first = 0;
  if (T.fp64) {  // the lane group must hold the whole A row to sum in ascending k
    while (first < 8 && (8 << first) < d) ++first;
  }
  if (T.force_bin >= 0) first = max(first, T.force_bin);
  for (int b = first; b < 8; ++b)
    if (T.group_ub[b] > 0 && ub <= T.group_ub[b] && ub <= (32 << b)) return b;
  return T.dense_passes <= T.dense_max_passes ? BIN_DENSE : BIN_GLOBAL;
}

// One wavefront per affected row (8 column loads in flight per lane, so a hub
// row is no long chain of dependent loads): flops, ub, bin
constexpr int ANALYZE_UNR = 16;
__global__ __launch_bounds__(256) void k_analyze(RowArgs R, const int32_t* d_count, Tun T) {
  const int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int l = threadIdx.x & 63;
  if (q >= *d_count) return;
  const int32_t i = R.aff[q];
  const int64_t aoff = R.a_off[i];
  const int32_t d = R.a_len[i];
  int64_t f = 0;
  for (int32_t t0 = l; t0 < d; t0 += 64 * ANALYZE_UNR) {
    int32_t k[ANALYZE_UNR];
#pragma unroll
    for (int u = 0; u < ANALYZE_UNR; ++u) k[u] = t0 + u * 64 < d ? R.a_col[aoff + t0 + u * 64] : -1;
#pragma unroll
    for (int u = 0; u < ANALYZE_UNR; ++u) f += k[u] >= 0 ? R.b_len[k[u]] : 0;
  }
  for (int s = 32; s > 0; s >>= 1) f += __shfl_xor(f, s, 64);
  if (l != 0) return;
  const int32_t ub = (int32_t)min(f, (int64_t)R.ncols);
  R.ub[q] = ub;
  R.flq[q] = (int32_t)min(f, (int64_t)0x7fffffff);
  // (rows with an empty new row go to the smallest bin like any other: nothing
  // is written before the row kernels run)
  R.binof[q] = (uint8_t)pick_bin(ub, d, T);
}

// Bin lists and space needs, aggregated per workgroup: one global atomic per
// bin and per counter and workgroup, not one per row.
constexpr int SCATTER_NT = 1024;
__global__ __launch_bounds__(SCATTER_NT) void k_bin_scatter(RowArgs R, const int32_t* d_count, Plan* plan,
                                                            int32_t* bins, int32_t bin_stride,
                                                            const uint8_t* filter) {
  __shared__ int32_t cnt[NBINS];
  __shared__ unsigned long long base[NBINS];
  __shared__ unsigned long long dem[3];
  const int tid = threadIdx.x;
  if (tid < NBINS) cnt[tid] = 0;
  if (tid < 3) dem[tid] = 0;
  __syncthreads();
  const int64_t q = (int64_t)blockIdx.x * SCATTER_NT + tid;
  int b = -1, local = 0;
  if (q < *d_count && (!filter || filter[q])) {
    const int32_t ub = R.ub[q];
    b = R.binof[q];
    local = atomicAdd(&cnt[b], 1);
    const int32_t i = R.aff[q];
    if (!filter) atomicAdd(&dem[2], (unsigned long long)R.flq[q]);
    if (ub > R.c_cap[i]) atomicAdd(&dem[0], (unsigned long long)slack_cap(ub));
    if (b == BIN_DENSE) {
      atomicAdd(&dem[1], (unsigned long long)(((size_t)min(ub, R.ncols) * 12 + 255) & ~size_t(255)));
    } else if (b == BIN_GLOBAL) {
      atomicAdd(&dem[1], (unsigned long long)(((size_t)global_slots(ub) * 12 + 255) & ~size_t(255)));
    }
  }
  __syncthreads();
  if (tid < NBINS) base[tid] = cnt[tid] ? atomicAdd(&plan->bin_count[tid], (unsigned long long)cnt[tid]) : 0;
  if (tid == NBINS && dem[0]) atomicAdd(&plan->c_demand, dem[0]);
  if (tid == NBINS + 1 && dem[1]) atomicAdd(&plan->arena_demand, dem[1]);
  if (tid == NBINS + 2 && dem[2]) atomicAdd(&plan->flops, dem[2]);
  __syncthreads();
  if (b >= 0) bins[(int64_t)b * bin_stride + (int64_t)(base[b] + local)] = (int32_t)q;
}

// Sum the per-row records into per-bin totals.
__global__ __launch_bounds__(256) void k_reduce_stats(const RowStat* rs, const uint8_t* binof,
                                                      const int32_t* d_count, unsigned long long* stats) {
  __shared__ unsigned long long acc[NBINS * NSTAT];
  for (int x = threadIdx.x; x < NBINS * NSTAT; x += blockDim.x) acc[x] = 0;
  __syncthreads();
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < *d_count) {
    const RowStat s = rs[q];
    unsigned long long* a = acc + binof[q] * NSTAT;
    atomicAdd(&a[0], 1ull);
    if (s.d) atomicAdd(&a[1], (unsigned long long)s.d);
    if (s.flops) atomicAdd(&a[2], (unsigned long long)s.flops);
    if (s.nnew) atomicAdd(&a[3], (unsigned long long)s.nnew);
    if (s.olen) atomicAdd(&a[4], (unsigned long long)s.olen);
    if (s.old_read) atomicAdd(&a[5], (unsigned long long)s.old_read);
    if (s.written) atomicAdd(&a[6], (unsigned long long)s.written);
  }
  __syncthreads();
  for (int x = threadIdx.x; x < NBINS * NSTAT; x += blockDim.x)
    if (acc[x]) atomicAdd(&stats[x], acc[x]);
}

__global__ void k_set_count(int32_t* d, int32_t v) { *d = v; }

// zero fills that a captured graph may hold (graphs here carry no memset nodes)
__global__ void k_zero_words(unsigned long long* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0ull;
}

__global__ void k_zero_bytes(uint8_t* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// rows flagged for retry become the filter of the next pass; flags reset
__global__ void k_take_retry(uint8_t* retry, uint8_t* filter, const int32_t* d_count) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < *d_count) {
    filter[q] = retry[q];
    retry[q] = 0;
  }
}

// a retry pass starts with empty bins and shortfalls
__global__ void k_reset_bins(Plan* plan) {
  const int t = threadIdx.x;
  if (t < NBINS) plan->bin_count[t] = 0;
  if (t == 0) {
    plan->c_short = 0;
    plan->arena_short = 0;
    plan->dense_next = 0;
  }
}

// C now reflects the operands' current epochs -- unless rows still wait for
// room or a row kernel failed (then the rows it skipped stay affected, and the
// next update recomputes them)
__global__ void k_set_sync(uint32_t* sync, const uint32_t* ea, const uint32_t* eb, const Plan* plan,
                           const int* err) {
  if (plan->c_short || plan->arena_short || *err != 0) return;
  sync[0] = *ea;
  sync[1] = *eb;
}

__global__ void k_publish(const int32_t* nchg, const int32_t* naff, const int* err, const Plan* plan,
                          int64_t* out) {
  out[0] = *nchg;
  out[1] = *naff;
  out[2] = *err;
  out[3] = (plan->c_short || plan->arena_short) ? 1 : 0;
  out[4] = (int64_t)plan->c_short;
  out[5] = (int64_t)plan->arena_short;
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

namespace {

int dense_passes_for(int vsz, int32_t ncols) {
  int ch = vsz == 8 ? dense_cols<8>() : dense_cols<4>();
  return (ncols + ch - 1) / ch;
}

const char* kBinNames[NBINS] = {"rows_g8",   "rows_g16",  "rows_g32",   "rows_g64",   "rows_g128",
                                "rows_g256", "rows_g512", "rows_g1024", "rows_dense", "rows_global"};

// Launch the non-empty bins in [lo, hi) on stream s.  plan == nullptr (graph
// mode): bin sizes are only on the device, so every bin is launched with a
// persistent grid that reads its count from d_counts.
template <int SR>
void launch_bins(Ctx* c, const RowArgs& R, const int32_t* bins, int32_t stride, const unsigned long long* d_counts,
                 const Plan* plan, int64_t nrows, std::vector<std::pair<int, size_t>>& timed, int lo, int hi,
                 hipStream_t s) {
  const int64_t cus = c->num_cus;
  for (int b = lo; b < hi; ++b) {
    const int64_t cnt = plan ? (int64_t)plan->bin_count[b] : nrows;
    if (cnt == 0) continue;
    const int32_t* list = bins + (int64_t)b * stride;
    const unsigned long long* dc = d_counts + b;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing && plan && ctx_timing_begin(c, kBinNames[b], 0.0, &e0, &e1, s))
      timed.push_back({b, c->timings.size() - 1});
    switch (b) {
#define GROUP_CASE(B, G, WG)                                                                              \
  case B: {                                                                                               \
    const int64_t blocks = plan ? (int64_t)blocks_for(cnt, WG / G)                                        \
                                : std::min<int64_t>(blocks_for(cnt, WG / G), cus * (2048 / WG));          \
    hipLaunchKernelGGL((k_rows_group<SR, G, WG>), dim3((unsigned)blocks), dim3(WG), 0, s, R, list, dc, B); \
    break;                                                                                                \
  }
      GROUP_CASE(0, 8, 256)
      GROUP_CASE(1, 16, 256)
      GROUP_CASE(2, 32, 256)
      GROUP_CASE(3, 64, 256)
      GROUP_CASE(4, 128, 128)
      GROUP_CASE(5, 256, 256)
      GROUP_CASE(6, 512, 512)
      GROUP_CASE(7, 1024, 1024)
#undef GROUP_CASE
      case BIN_DENSE: {
        // persistent workgroups, one per CU (each holds ~150 KB of LDS)
        const unsigned grid = (unsigned)std::min<int64_t>(cnt, cus);
        hipLaunchKernelGGL((k_rows_dense<SR>), dim3(grid), dim3(DENSE_WG), 0, s, R, list, dc);
        break;
      }
      case BIN_GLOBAL: {
        const unsigned grid = (unsigned)(plan ? cnt : std::min<int64_t>(cnt, cus * 2));
        hipLaunchKernelGGL((k_rows_global<SR>), dim3(grid), dim3(GLOBAL_WG), 0, s, R, list, dc);
        break;
      }
    }
    if (c->timing && plan) ctx_timing_end(c, e1, s);
  }
  DSG_HIP(hipGetLastError());
}

constexpr int32_t ENTRY_INSTEAD = -2;  // prod_sequence: the entry-granular path is cheaper

struct ProdWork {
  uint8_t* aff_flags;
  uint8_t* b_flags;
  int32_t* aff;
  int32_t* d_count;
  int32_t* dB;
  int32_t* d_nB;
  int32_t* ub;
  uint8_t* chg;
  int32_t* bins;
  Plan* plan;
  unsigned long long* stats;
  RowStat* rstat;
  uint8_t* binof;
  int32_t* flq;
  uint8_t* retry;
  uint8_t* filter;
  int* err;
  int32_t* d_nchg;
  void* cscr;
};

size_t work_bytes_for(int64_t N, int64_t nB) {
  return Carve::need({(size_t)N, (size_t)nB, (size_t)N * 4, 64, (size_t)nB * 4, 64, (size_t)N * 4, (size_t)N,
                      (size_t)N * 4 * NBINS, sizeof(Plan) + 64, NBINS * NSTAT * 8 + 64, (size_t)N * sizeof(RowStat),
                      (size_t)N, (size_t)N * 4, (size_t)N, (size_t)N, 64, 64,
                      compact_scratch_bytes(std::max(N, nB)) + 64});
}

ProdWork carve_prod(void* base, int64_t N, int64_t nB) {
  Carve cv(base, work_bytes_for(N, nB));
  ProdWork w;
  w.aff_flags = cv.take<uint8_t>(N);
  w.b_flags = cv.take<uint8_t>(nB);
  w.aff = cv.take<int32_t>(N);
  w.d_count = cv.take<int32_t>(16);
  w.dB = cv.take<int32_t>(nB);
  w.d_nB = cv.take<int32_t>(16);
  w.ub = cv.take<int32_t>(N);
  w.chg = cv.take<uint8_t>(N);
  w.bins = cv.take<int32_t>(N * NBINS);
  w.plan = cv.take<Plan>(1);
  w.stats = cv.take<unsigned long long>(NBINS * NSTAT);
  w.rstat = cv.take<RowStat>(N);
  w.binof = cv.take<uint8_t>(N);
  w.flq = cv.take<int32_t>(N);
  w.retry = cv.take<uint8_t>(N);
  w.filter = cv.take<uint8_t>(N);
  w.err = cv.take<int>(16);
  w.d_nchg = cv.take<int32_t>(16);
  w.cscr = cv.take<char>(compact_scratch_bytes(std::max(N, nB)) + 64);
  return w;
}

void ensure_changed_cap(DProd* p, int64_t need) {
  if (need <= p->changed_cap) return;
  Ctx* c = p->ctx;
  if (p->changed_rows) ctx_free(c, p->changed_rows, (size_t)p->changed_cap * 4);
  p->changed_rows = nullptr;
  p->changed_cap = 0;
  const int64_t cap = std::max<int64_t>(need, 1024);
  p->changed_rows = (int32_t*)ctx_alloc(c, (size_t)cap * 4);
  p->changed_cap = cap;
}

void ensure_arena(DProd* p, size_t bytes) {
  Ctx* c = p->ctx;
  if (!p->arena_top) p->arena_top = (unsigned long long*)ctx_alloc(c, 64);
  if (bytes <= p->arena_bytes) return;
  if (p->arena) ctx_free(c, p->arena, p->arena_bytes);
  p->arena = nullptr;
  p->arena_bytes = 0;
  const size_t nb = bytes + bytes / 4 + 4096;
  p->arena = ctx_alloc(c, nb);
  p->arena_bytes = nb;
}

// ---------------------------------------------------------------------------
// B split by dense column chunk: the dense bin's passes each stream only the
// entries of their own chunk instead of every entry of every B row
// ---------------------------------------------------------------------------

constexpr int BSPLIT_MAXP = 8;
constexpr int BSPLIT_UNR = 8;     // loads in flight per lane (hub rows)
constexpr int BSPLIT_LONG = 2048; // longer rows are split by a workgroup each (k_bsplit_long)
constexpr int BSPLIT_WG = 512;

// One wavefront per row of B: the row's entries, grouped by column chunk,
// into the copy at the row's own pool offset (tombstones left out), and the
// P + 1 chunk boundaries of the row into bs[k*(P+1) ...].  The row is read
// twice, to count and to place, and no scan over rows is needed.  Entries
// keep their order inside a chunk.
template <int VSZ>
__global__ __launch_bounds__(256) void k_bsplit(const int64_t* b_off, const int32_t* b_len, const int32_t* b_col,
                                                const void* b_val, int32_t n, int P, int chbits, int64_t* bs,
                                                int32_t* out_col, void* out_val) {
  using W = typename std::conditional<VSZ == 8, uint64_t, uint32_t>::type;
  const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int ln = threadIdx.x & 63;
  if (k >= n) return;
  const int64_t off = b_off[k];
  const int32_t len = b_len[k];
  if (len > BSPLIT_LONG) return;  // k_bsplit_long
  const uint64_t lt = ln ? (~0ull >> (64 - ln)) : 0ull;
  int64_t o[BSPLIT_MAXP];
#pragma unroll
  for (int q = 0; q < BSPLIT_MAXP; ++q) o[q] = 0;
  for (int32_t e0 = 0; e0 < len; e0 += 64 * BSPLIT_UNR) {  // count; BSPLIT_UNR loads in flight per lane
    int part[BSPLIT_UNR];
#pragma unroll
    for (int v = 0; v < BSPLIT_UNR; ++v) {
      const int32_t e = e0 + v * 64 + ln;
      part[v] = e < len ? (b_col[off + e] >> chbits) : -1;
    }
#pragma unroll
    for (int v = 0; v < BSPLIT_UNR; ++v)
#pragma unroll
      for (int q = 0; q < BSPLIT_MAXP; ++q)
        if (q < P) o[q] += __popcll(__ballot(part[v] == q));
  }
  // chunk starts inside the row's slots
  int64_t run = off;
#pragma unroll
  for (int q = 0; q < BSPLIT_MAXP; ++q) {
    if (q < P) {
      const int64_t c = o[q];
      o[q] = run;
      run += c;
    }
  }
  if (ln == 0) {
#pragma unroll
    for (int q = 0; q < BSPLIT_MAXP; ++q)
      if (q < P) bs[k * (P + 1) + q] = o[q];
    bs[k * (P + 1) + P] = run;
  }
  for (int32_t e0 = 0; e0 < len; e0 += 64 * BSPLIT_UNR) {  // place
    int32_t col[BSPLIT_UNR];
    W val[BSPLIT_UNR];
#pragma unroll
    for (int v = 0; v < BSPLIT_UNR; ++v) {
      const int32_t e = e0 + v * 64 + ln;
      col[v] = e < len ? b_col[off + e] : -1;
      val[v] = e < len ? ((const W*)b_val)[off + e] : W(0);
    }
#pragma unroll
    for (int v = 0; v < BSPLIT_UNR; ++v) {
      const int part = col[v] >= 0 ? (col[v] >> chbits) : -1;
      int64_t dst = -1;
#pragma unroll
      for (int q = 0; q < BSPLIT_MAXP; ++q) {
        if (q < P) {
          const uint64_t m = __ballot(part == q);
          if (part == q) dst = o[q] + __popcll(m & lt);
          o[q] += __popcll(m);
        }
      }
      if (dst >= 0) {
        out_col[dst] = col[v];
        ((W*)out_val)[dst] = val[v];
      }
    }
  }
}

// Rows longer than BSPLIT_LONG (hub rows, which one wavefront walks in
// many dependent rounds): one workgroup per row, taken in turn by a
// persistent grid.  Each wavefront counts and places one contiguous segment
// of the row; a chunk holds the segments' entries in segment order, so the
// order inside a chunk is the row's order, as in k_bsplit.
template <int VSZ>
__global__ __launch_bounds__(BSPLIT_WG) void k_bsplit_long(const int64_t* b_off, const int32_t* b_len,
                                                           const int32_t* b_col, const void* b_val, int32_t n, int P,
                                                           int chbits, int64_t* bs, int32_t* out_col,
                                                           void* out_val) {
  using W = typename std::conditional<VSZ == 8, uint64_t, uint32_t>::type;
  constexpr int NW = BSPLIT_WG / 64;
  __shared__ int64_t wcnt[NW][BSPLIT_MAXP];
  const int tid = threadIdx.x, ln = tid & 63, wv = tid >> 6;
  const uint64_t lt = ln ? (~0ull >> (64 - ln)) : 0ull;
  for (int64_t k = blockIdx.x; k < n; k += gridDim.x) {
    const int32_t len = b_len[k];
    if (len <= BSPLIT_LONG) continue;  // the same for the whole workgroup
    const int64_t off = b_off[k];
    const int32_t seg = (len + NW - 1) / NW;
    const int32_t s0 = min(len, wv * seg), s1 = min(len, s0 + seg);
    int64_t o[BSPLIT_MAXP];
#pragma unroll
    for (int q = 0; q < BSPLIT_MAXP; ++q) o[q] = 0;
    for (int32_t e0 = s0; e0 < s1; e0 += 64 * BSPLIT_UNR) {  // count this wavefront's segment
      int part[BSPLIT_UNR];
#pragma unroll
      for (int v = 0; v < BSPLIT_UNR; ++v) {
        const int32_t e = e0 + v * 64 + ln;
        part[v] = e < s1 ? (b_col[off + e] >> chbits) : -1;
      }
#pragma unroll
      for (int v = 0; v < BSPLIT_UNR; ++v)
#pragma unroll
        for (int q = 0; q < BSPLIT_MAXP; ++q)
          if (q < P) o[q] += __popcll(__ballot(part[v] == q));
    }
    if (ln == 0) {
#pragma unroll
      for (int q = 0; q < BSPLIT_MAXP; ++q) wcnt[wv][q] = o[q];
    }
    __syncthreads();
    // chunk q starts after chunks 0..q-1; this segment's part of chunk q
    // after the earlier segments' parts
    int64_t run = off;
#pragma unroll
    for (int q = 0; q < BSPLIT_MAXP; ++q) {
      if (q < P) {
        int64_t tot = 0, before = 0;
        for (int w = 0; w < NW; ++w) {
          const int64_t c = wcnt[w][q];
          tot += c;
          if (w < wv) before += c;
        }
        if (tid == 0) bs[k * (P + 1) + q] = run;
        o[q] = run + before;
        run += tot;
      }
    }
    if (tid == 0) bs[k * (P + 1) + P] = run;
    for (int32_t e0 = s0; e0 < s1; e0 += 64 * BSPLIT_UNR) {  // place
      int32_t col[BSPLIT_UNR];
      W val[BSPLIT_UNR];
#pragma unroll
      for (int v = 0; v < BSPLIT_UNR; ++v) {
        const int32_t e = e0 + v * 64 + ln;
        col[v] = e < s1 ? b_col[off + e] : -1;
        val[v] = e < s1 ? ((const W*)b_val)[off + e] : W(0);
      }
#pragma unroll
      for (int v = 0; v < BSPLIT_UNR; ++v) {
        const int part = col[v] >= 0 ? (col[v] >> chbits) : -1;
        int64_t dst = -1;
#pragma unroll
        for (int q = 0; q < BSPLIT_MAXP; ++q) {
          if (q < P) {
            const uint64_t m = __ballot(part == q);
            if (part == q) dst = o[q] + __popcll(m & lt);
            o[q] += __popcll(m);
          }
        }
        if (dst >= 0) {
          out_col[dst] = col[v];
          ((W*)out_val)[dst] = val[v];
        }
      }
    }
    __syncthreads();  // wcnt is reused by the next row
  }
}

size_t round256(size_t x) { return (x + 255) & ~size_t(255); }

// Build the split copy of B for this update (when the dense bin needs more
// than one pass); leaves p->bsp_live set.
void build_bsplit(DProd* p) {
  Ctx* c = p->ctx;
  hipStream_t s = c->stream;
  DMat* B = p->B;
  const int vsz = p->C->vsz;
  const int P = dense_passes_for(vsz, B->ncols);
  p->bsp_live = false;
  if (P < 2 || P > BSPLIT_MAXP || B->nrows == 0) return;
  const int chbits = vsz == 8 ? 14 : 15;
  static_assert(dense_cols<8>() == (1 << 14) && dense_cols<4>() == (1 << 15), "chunk widths");
  const int64_t nps = (int64_t)B->nrows * (P + 1);
  const int64_t cap = std::max<int64_t>(B->h_top_ub, 1);  // every row's slots lie below the pool top
  const size_t col_off = round256((size_t)nps * 8);
  const size_t val_off = col_off + round256((size_t)cap * 4);
  // (padded like the entry pools: windows of POOL_PAD entries may be read
  // from any position inside a row)
  const size_t bytes = val_off + round256((size_t)cap * vsz) + (size_t)POOL_PAD * 8;
  if (bytes > p->bsp_bytes) {
    if (p->bsp) ctx_free(c, p->bsp, p->bsp_bytes);
    p->bsp = nullptr;
    p->bsp_bytes = 0;
    const size_t nb = bytes + bytes / 4;
    p->bsp = ctx_alloc(c, nb);
    p->bsp_bytes = nb;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->timing) ctx_timing_begin(c, "b_split", (double)cap * (4 + vsz) * 2, &e0, &e1);
  int64_t* bs = (int64_t*)p->bsp;
  int32_t* ocol = (int32_t*)((char*)p->bsp + col_off);
  void* oval = (char*)p->bsp + val_off;
  const unsigned nb = (unsigned)blocks_for((int64_t)B->nrows * 64, 256);
  // long rows first, a workgroup each (four per CU), then the rest
  const unsigned nl = (unsigned)std::min<int64_t>(B->nrows, (int64_t)c->num_cus * 4);
  if (vsz == 8) {
    hipLaunchKernelGGL(k_bsplit_long<8>, dim3(nl), dim3(BSPLIT_WG), 0, s, B->row_off, B->row_len, B->col, B->val,
                       B->nrows, P, chbits, bs, ocol, oval);
    hipLaunchKernelGGL(k_bsplit<8>, dim3(nb), dim3(256), 0, s, B->row_off, B->row_len, B->col, B->val, B->nrows,
                       P, chbits, bs, ocol, oval);
  } else {
    hipLaunchKernelGGL(k_bsplit_long<4>, dim3(nl), dim3(BSPLIT_WG), 0, s, B->row_off, B->row_len, B->col, B->val,
                       B->nrows, P, chbits, bs, ocol, oval);
    hipLaunchKernelGGL(k_bsplit<4>, dim3(nb), dim3(256), 0, s, B->row_off, B->row_len, B->col, B->val, B->nrows,
                       P, chbits, bs, ocol, oval);
  }
  DSG_HIP(hipGetLastError());
  if (c->timing) ctx_timing_end(c, e1);
  p->bsp_col_off = col_off;
  p->bsp_val_off = val_off;
  p->bsp_parts = P;
  p->bsp_live = true;
}

RowArgs row_args(DProd* p, ProdWork& w, int mode, bool report_affected) {
  DMat* A = p->A;
  DMat* B = p->B;
  DMat* C = p->C;
  RowArgs R;
  R.a_off = A->row_off; R.a_len = A->row_len; R.a_col = A->col; R.a_val = A->val;
  R.b_off = B->row_off; R.b_len = B->row_len; R.b_col = B->col; R.b_val = B->val;
  R.c_off = C->row_off; R.c_len = C->row_len; R.c_cap = C->row_cap; R.c_col = C->col; R.c_val = C->val;
  R.c_top = C->d_top; R.c_pool_cap = C->pool_cap;
  R.ncols = B->ncols;
  R.aff = w.aff; R.ub = w.ub; R.chg = w.chg; R.stats = w.stats;
  R.arena = (char*)p->arena; R.arena_top = p->arena_top; R.arena_cap = (int64_t)p->arena_bytes;
  R.force_write = (mode == 1 || report_affected) ? 1 : 0;
  R.err = w.err;
  R.rstat = w.rstat;
  R.binof = w.binof;
  R.flq = w.flq;
  R.dense_next = &w.plan->dense_next;
  R.defer = nullptr;
  R.retry = w.retry;
  R.c_short = &w.plan->c_short;
  R.arena_short = &w.plan->arena_short;
  R.bs_parts = 0;
  R.bs_ps = nullptr;
  R.bs_col = nullptr;
  R.bs_val = nullptr;
  if (p->bsp_live) {
    R.bs_parts = p->bsp_parts;
    R.bs_ps = (const int64_t*)p->bsp;
    R.bs_col = (const int32_t*)((char*)p->bsp + p->bsp_col_off);
    R.bs_val = (const char*)p->bsp + p->bsp_val_off;
  }
  return R;
}

// Discovery, analysis and binning (no host round trip).
void launch_front(DProd* p, int mode, ProdWork& w, const RowArgs& R) {
  Ctx* c = p->ctx;
  hipStream_t s = c->stream;
  DMat* A = p->A;
  DMat* B = p->B;
  const int32_t n = A->nrows;
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, s, (unsigned long long*)w.plan, (int)(sizeof(Plan) / 8));
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, s, w.stats, NBINS * NSTAT);
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, (unsigned long long*)w.err, 1);
  if (n > 0) hipLaunchKernelGGL(k_zero_bytes, dim3(blocks_for(n, 256)), dim3(256), 0, s, w.retry, (int64_t)n);
  if (mode == 1) {
    iota_i32(w.aff, n, s);
    hipLaunchKernelGGL(k_set_count, dim3(1), dim3(1), 0, s, w.d_count, n);
  } else if (n > 0) {
    hipLaunchKernelGGL(k_mark_changed, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, A->row_epoch,
                       (const uint32_t*)p->d_sync, w.aff_flags);
    if (B->nrows > 0) {
      hipLaunchKernelGGL(k_mark_changed, dim3(blocks_for(B->nrows, 256)), dim3(256), 0, s, B->nrows, B->row_epoch,
                         (const uint32_t*)p->d_sync + 1, w.b_flags);
      compact_flags(w.b_flags, B->nrows, w.dB, w.d_nB, w.cscr, s);
      DMat* T = p->lt;
      unsigned nbk = (unsigned)std::min<int64_t>(blocks_for((int64_t)B->nrows * 64, 256), 8192);
      hipLaunchKernelGGL(k_scatter_dB, dim3(nbk), dim3(256), 0, s, w.dB, w.d_nB, T->row_off, T->row_len, T->col,
                         w.aff_flags);
    }
    compact_flags(w.aff_flags, n, w.aff, w.d_count, w.cscr, s);
  } else {
    hipLaunchKernelGGL(k_set_count, dim3(1), dim3(1), 0, s, w.d_count, 0);
  }
  Tun T;
  const dsg_tuning& tu = c->tuning;
  for (int b = 0; b < 8; ++b) T.group_ub[b] = tu.group_ub[b];
  T.dense_passes = dense_passes_for(p->C->vsz, B->ncols);
  T.dense_max_passes = tu.dense_max_passes;
  T.force_bin = tu.force_bin;
  T.fp64 = A->sr == 2 ? 1 : 0;
  if (n > 0) {
    hipLaunchKernelGGL(k_analyze, dim3(blocks_for((int64_t)n * 64, 256)), dim3(256), 0, s, R, w.d_count, T);
    hipLaunchKernelGGL(k_bin_scatter, dim3(blocks_for(n, SCATTER_NT)), dim3(SCATTER_NT), 0, s, R, w.d_count, w.plan,
                       w.bins, n, (const uint8_t*)nullptr);
  }
}

void launch_bin_range(DProd* p, const RowArgs& R, ProdWork& w, const Plan* hplan,
                      std::vector<std::pair<int, size_t>>& timed, int lo, int hi, hipStream_t s) {
  Ctx* c = p->ctx;
  const int32_t n = p->A->nrows;
  switch (p->A->sr) {
    case 0: launch_bins<0>(c, R, w.bins, n, w.plan->bin_count, hplan, n, timed, lo, hi, s); break;
    case 1: launch_bins<1>(c, R, w.bins, n, w.plan->bin_count, hplan, n, timed, lo, hi, s); break;
    case 2: launch_bins<2>(c, R, w.bins, n, w.plan->bin_count, hplan, n, timed, lo, hi, s); break;
    default: launch_bins<3>(c, R, w.bins, n, w.plan->bin_count, hplan, n, timed, lo, hi, s); break;
  }
}

// With the bin sizes known, bins [0, hi) may run on a second stream beside
// bins [hi, NBINS): the short lane-group launches are mostly latency.  The
// bins touch disjoint rows and share only atomically claimed pools and
// counters.  Not under graph capture.
bool side_split(Ctx* c, const Plan* plan, int hi) {
  if (!plan) return false;
  int64_t lo_rows = 0, hi_rows = 0;
  for (int b = 0; b < NBINS; ++b) (b < hi ? lo_rows : hi_rows) += (int64_t)plan->bin_count[b];
  if (lo_rows == 0 || hi_rows == 0) return false;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  DSG_HIP(hipStreamIsCapturing(c->stream, &cap));
  return cap == hipStreamCaptureStatusNone;
}

void zero_arena_top(DProd* p) {
  if (p->arena_top) hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, p->ctx->stream, p->arena_top, 1);
}

// bins [0, hi) on the side stream, after everything queued so far on the
// context's stream; join_side makes the context's stream wait for them
void fork_side(DProd* p, const RowArgs& R, ProdWork& w, const Plan* hplan,
               std::vector<std::pair<int, size_t>>& timed, int hi) {
  Ctx* c = p->ctx;
  hipStream_t side = ctx_side_stream(c);
  DSG_HIP(hipEventRecord(c->fork_ev, c->stream));
  DSG_HIP(hipStreamWaitEvent(side, c->fork_ev, 0));
  try {
    launch_bin_range(p, R, w, hplan, timed, 0, hi, side);
  } catch (...) {
    (void)hipEventRecord(c->join_ev, side);
    (void)hipStreamWaitEvent(c->stream, c->join_ev, 0);
    throw;
  }
  DSG_HIP(hipEventRecord(c->join_ev, side));
}

void join_side(Ctx* c) { DSG_HIP(hipStreamWaitEvent(c->stream, c->join_ev, 0)); }

// Bins 0-5 (lane groups of up to 256 lanes) finish beside the 512- and
// 1024-lane groups, before the persistent dense workgroups take every CU.
constexpr int SIDE_BINS = 6;

void launch_rows(DProd* p, const RowArgs& R, ProdWork& w, const Plan* hplan,
                 std::vector<std::pair<int, size_t>>& timed) {
  Ctx* c = p->ctx;
  mat_index_invalidate(p->C);  // recomputed rows are written in a new order
  zero_arena_top(p);
  if (side_split(c, hplan, SIDE_BINS)) {
    fork_side(p, R, w, hplan, timed, SIDE_BINS);
    try {
      launch_bin_range(p, R, w, hplan, timed, SIDE_BINS, NBINS, c->stream);
    } catch (...) {
      join_side(c);  // later work on the context's stream still waits for the side bins
      throw;
    }
    join_side(c);
  } else {
    launch_bin_range(p, R, w, hplan, timed, 0, NBINS, c->stream);
  }
}

void launch_set_sync(DProd* p, ProdWork& w) {
  hipLaunchKernelGGL(k_set_sync, dim3(1), dim3(1), 0, p->ctx->stream, p->d_sync, (const uint32_t*)p->A->d_epoch,
                     (const uint32_t*)p->B->d_epoch, (const Plan*)w.plan, (const int*)w.err);
}

// reported rows, statistics and (when the rows are complete) the epochs C
// now reflects (no host round trip)
void launch_tail(DProd* p, ProdWork& w, int64_t nmax, bool set_sync = true) {
  hipStream_t s = p->ctx->stream;
  compact_list_by_flags(w.aff, w.chg, w.d_count, nmax, p->changed_rows, w.d_nchg, w.cscr, s);
  hipLaunchKernelGGL(k_reduce_stats, dim3(blocks_for(nmax, 256)), dim3(256), 0, s, w.rstat, w.binof, w.d_count,
                     w.stats);
  if (set_sync) launch_set_sync(p, w);
}

// Read the plan back; also refresh the host's view of C's pool top, which the
// row kernels advance on the device (and, when given, one more device count
// in the same wait).
Plan read_plan(Ctx* c, ProdWork& w, DMat* C, const int64_t* d_extra = nullptr, int64_t* h_extra = nullptr) {
  static_assert(sizeof(Plan) % 4 == 0 && sizeof(Plan) <= 2048, "pinned staging");
  Plan* hp = (Plan*)c->pinned;
  int64_t* htop = (int64_t*)((char*)c->pinned + 2048);
  FetchList F;
  F.add(w.plan, (int32_t)sizeof(Plan), 0);
  F.add(C->d_top, 8, 2048);
  F.add(d_extra, 8, 2048 + 8);
  F.add(w.d_count, 4, 2048 + 16);
  fetch_to_pinned(c, F, c->stream);
  DSG_HIP(hipStreamSynchronize(c->stream));
  C->h_top_ub = *htop;
  if (h_extra) *h_extra = htop[1];
  Plan plan = *hp;
  plan.count = *(const int32_t*)(htop + 2);
  return plan;
}

// Recompute the rows flagged for retry after growing C and the arena by
// exactly what they asked for.  Returns the plan of the last pass.
Plan retry_rows(DProd* p, ProdWork& w, int mode, bool report_affected, Plan plan,
                std::vector<std::pair<int, size_t>>& timed) {
  Ctx* c = p->ctx;
  hipStream_t s = c->stream;
  const int32_t n = p->A->nrows;
  for (int pass = 0; (plan.c_short || plan.arena_short) && pass < 8; ++pass) {
    if (plan.c_short) {
      mat_reserve(p->C, (int64_t)(plan.c_short + plan.c_short / 4));
      p->C->h_top_ub += (int64_t)plan.c_short;
    }
    if (plan.arena_short) ensure_arena(p, plan.arena_short);
    RowArgs R = row_args(p, w, mode, report_affected);
    hipLaunchKernelGGL(k_take_retry, dim3(blocks_for(std::max<int32_t>(n, 1), 256)), dim3(256), 0, s, w.retry,
                       w.filter, (const int32_t*)w.d_count);
    hipLaunchKernelGGL(k_reset_bins, dim3(1), dim3(64), 0, s, w.plan);
    hipLaunchKernelGGL(k_bin_scatter, dim3(blocks_for(std::max<int32_t>(n, 1), SCATTER_NT)), dim3(SCATTER_NT), 0, s,
                       R, w.d_count, w.plan, w.bins, n, (const uint8_t*)w.filter);
    Plan bins = read_plan(c, w, p->C);
    launch_rows(p, R, w, &bins, timed);
    plan = read_plan(c, w, p->C);
  }
  DSG_REQUIRE(!plan.c_short && !plan.arena_short, DSG_E_OOM, "rows still without room after growing C");
  return plan;
}

// Plain mode: one product update (mode 0) or full recompute (mode 1), with
// host round trips after the analysis (bin sizes) and at the end (results).
// The entry-granular path wins while its changed products stay few next to
// the products the affected rows would take: the rule's two constants come
// from the tuning (their defaults separate every measured R-MAT and
// Erdos-Renyi case of 1e2..3e4 updates on MI355X).
bool entry_cheaper(const dsg_tuning& t, int64_t nterm, unsigned long long row_flops) {
  return (double)row_flops > t.entry_fixed + t.entry_per_term * (double)nterm;
}

int32_t prod_sequence(DProd* p, int mode, bool report_affected, ProdWork& w, const int64_t* d_entry_terms) {
  Ctx* c = p->ctx;
  hipStream_t s = c->stream;
  DMat* C = p->C;
  const int32_t n = p->A->nrows;
  RowArgs R = row_args(p, w, mode, report_affected);
  launch_front(p, mode, w, R);
  int64_t entry_terms = -1;
  Plan plan = read_plan(c, w, p->C, d_entry_terms, &entry_terms);
  // nothing of C was touched so far: hand over to the entry-granular path
  if (d_entry_terms) {
    p->entry_nterm = entry_terms;
    if (entry_cheaper(c->tuning, entry_terms, plan.flops)) return ENTRY_INSTEAD;
  }
  // room: C grows only by what rows that do not fit ask for (retry below);
  // the arena keeps the largest size used so far, up to the analysis bound
  if (plan.arena_demand > p->arena_bytes) ensure_arena(p, std::min<size_t>(plan.arena_demand, std::max<size_t>(p->arena_bytes * 2, (size_t)64 << 20)));
  ensure_changed_cap(p, plan.count);
  // the dense bin runs persistent workgroups: hand them the longest rows first
  const int64_t ndense = (int64_t)plan.bin_count[BIN_DENSE];
  struct SplitLive {  // the split copy of B serves this update only
    DProd* p;
    ~SplitLive() { p->bsp_live = false; }
  } split_live{p};
  if (ndense > 0) build_bsplit(p);
  R = row_args(p, w, mode, report_affected);
  if (ndense > 1) {
    int32_t* dl = w.bins + (int64_t)BIN_DENSE * n;
    const size_t nb = Carve::need({(size_t)ndense * 8, (size_t)ndense * 4, radix_scratch_bytes(ndense)});
    Carve dc(ctx_scratch2(c, nb), nb);
    uint64_t* keys = dc.take<uint64_t>(ndense);
    uint32_t* vals = dc.take<uint32_t>(ndense);
    void* rs = dc.take<char>(radix_scratch_bytes(ndense));
    hipLaunchKernelGGL(k_flop_keys, dim3(blocks_for(ndense, 256)), dim3(256), 0, s, dl, (int32_t)ndense, w.flq, keys,
                       vals);
    radix_sort_pairs(keys, vals, ndense, FLOP_KEY_BITS, rs, s, w.err);
    DSG_HIP(hipMemcpyAsync(dl, vals, (size_t)ndense * 4, hipMemcpyDeviceToDevice, s));
  }
  std::vector<std::pair<int, size_t>> timed;
  launch_rows(p, R, w, &plan, timed);
  // ---- results, statistics, errors; with them, whether rows wait for room ----
  struct Tail {
    int32_t nchg;
    int32_t err;
    unsigned long long c_short, arena_short;
    int64_t c_top;
    unsigned long long stats[NBINS * NSTAT];
  };
  Tail* ht = (Tail*)((char*)c->pinned + 1024);
  static_assert(1024 + sizeof(Tail) <= 4096, "pinned staging");
  auto read_tail = [&]() {
    launch_tail(p, w, std::max<int32_t>(plan.count, 1), false);
    FetchList F;
    F.add(w.d_nchg, 4, 1024 + (int32_t)offsetof(Tail, nchg));
    F.add(w.err, 4, 1024 + (int32_t)offsetof(Tail, err));
    F.add(&w.plan->c_short, 16, 1024 + (int32_t)offsetof(Tail, c_short));
    F.add(C->d_top, 8, 1024 + (int32_t)offsetof(Tail, c_top));
    F.add(w.stats, (int32_t)sizeof(ht->stats), 1024 + (int32_t)offsetof(Tail, stats));
    fetch_to_pinned(c, F, s);
    DSG_HIP(hipStreamSynchronize(s));
    C->h_top_ub = ht->c_top;
    return *ht;
  };
  Tail tail = read_tail();
  if (tail.c_short || tail.arena_short) {
    // some rows found no room: grow it, recompute them, and take the tail again
    Plan after = plan;
    after.c_short = tail.c_short;
    after.arena_short = tail.arena_short;
    retry_rows(p, w, mode, report_affected, after, timed);
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, s, w.stats, NBINS * NSTAT);
    tail = read_tail();
  }
  launch_set_sync(p, w);
  DSG_REQUIRE(tail.err == 0, DSG_E_DEVICE, "internal: row kernel reported error code " + std::to_string(tail.err));
  dsg_update_stats& st = p->stats;
  st = dsg_update_stats{};
  st.affected_rows = plan.count;
  st.changed_rows = tail.nchg;
  const double sz = 4.0 + (double)C->vsz;
  for (int b = 0; b < NBINS; ++b) {
    const unsigned long long* x = tail.stats + b * NSTAT;
    st.bin_rows[b] = (int64_t)x[0];
    st.bin_flops[b] = (int64_t)x[2];
    st.a_entries += (int64_t)x[1];
    st.flops += (int64_t)x[2];
    st.nnz_new += (int64_t)x[3];
    st.nnz_old += (int64_t)x[4];
  }
  p->last_c_demand = (int64_t)plan.c_demand;
  p->last_arena_demand = (int64_t)plan.arena_demand;
  for (auto& tb : timed) {
    const unsigned long long* x = tail.stats + tb.first * NSTAT;
    // A row, B row lookups (offset + length), B entries, old C row when compared, new C row when written
    c->timings[tb.second].bytes =
        sz * (double)x[1] + 12.0 * (double)x[1] + sz * (double)x[2] + sz * (double)x[5] + sz * (double)x[6];
  }
  return tail.nchg;
}

}  // namespace

DProd* prod_create(Ctx* c, DMat* A, DMat* B, uint32_t ops) {
  DProd* p = new DProd();
  p->ctx = c;
  p->src_a = A;
  p->src_b = B;
  p->ops = ops & (DSG_TRANS_A | DSG_TRANS_B);
  p->bloom = (ops & DSG_GENERAL_BLOOM) != 0;
  try {
    // A's transpose serves either as the left operand (A^T) or as the
    // column index of the left operand (A); every apply of A keeps it current
    mat_build_transpose(A);
    if (ops & DSG_TRANS_B) mat_build_transpose(B);
    p->A = (ops & DSG_TRANS_A) ? A->tidx : A;
    p->lt = (ops & DSG_TRANS_A) ? A : A->tidx;
    p->B = (ops & DSG_TRANS_B) ? B->tidx : B;
    p->C = mat_create(c, p->A->nrows, p->B->ncols, A->sr, nullptr, nullptr, nullptr);
    p->d_sync = (uint32_t*)ctx_alloc(c, 16);
  } catch (...) {
    if (p->C) mat_destroy(p->C);
    delete p;
    throw;
  }
  A->refs++;
  B->refs++;
  p->a_seq = A->apply_seq;
  p->b_seq = B->apply_seq;
  try {
    prod_run(p, 1, true);
  } catch (...) {
    prod_destroy(p);
    throw;
  }
  return p;
}

void prod_destroy(DProd* p) {
  if (!p) return;
  Ctx* c = p->ctx;
  if (p->changed_rows) ctx_free(c, p->changed_rows, (size_t)p->changed_cap * 4);
  if (p->query_rows) ctx_free(c, p->query_rows, (size_t)p->query_cap * 4);
  if (p->arena) ctx_free(c, p->arena, p->arena_bytes);
  if (p->arena_top) ctx_free(c, p->arena_top, 64);
  if (p->d_sync) ctx_free(c, p->d_sync, 16);
  if (p->ews) ctx_free(c, p->ews, p->ews_bytes);
  if (p->bsp) ctx_free(c, p->bsp, p->bsp_bytes);
  if (p->gws) ctx_free(c, p->gws, p->gws_bytes);
  if (p->F) mat_destroy(p->F);
  if (p->C) mat_destroy(p->C);
  if (p->src_a) p->src_a->refs--;
  if (p->src_b) p->src_b->refs--;
  delete p;
}

int32_t prod_run(DProd* p, int mode, bool report_affected) {
  int32_t nchg = 0;
  if (p->bloom) {
    // Algorithm 2 keeps C and F current together; where it cannot run (no F
    // yet, a static recompute, several applies since the last update, every
    // recomputed row asked for), the row path brings C up to date and F is
    // built again from it
    if (mode == 0 && !report_affected && general_eligible(p)) {
      nchg = general_update(p);
    } else {
      const bool b = p->bloom;
      p->bloom = false;
      try {
        nchg = prod_run(p, mode, report_affected);
      } catch (...) {
        p->bloom = b;
        throw;
      }
      p->bloom = b;
      bloom_build(p);
    }
    p->a_seq = p->src_a->apply_seq;
    p->b_seq = p->src_b->apply_seq;
    return nchg;
  }
  // entry-granular candidate: count its changed products first (cheap)
  const int64_t* d_nterm = nullptr;
  if (mode == 0 && !report_affected && entry_eligible(p)) {
    d_nterm = entry_count(p);
    if (p->ctx->tuning.update_path == 2) {
      int64_t* h = (int64_t*)((char*)p->ctx->pinned + 3072);
      DSG_HIP(hipMemcpyAsync(h, d_nterm, 8, hipMemcpyDeviceToHost, p->ctx->stream));
      DSG_HIP(hipStreamSynchronize(p->ctx->stream));
      p->entry_nterm = *h;
      nchg = entry_finish(p);
      p->a_seq = p->src_a->apply_seq;
      p->b_seq = p->src_b->apply_seq;
      return nchg;
    }
  }
  const int64_t N = std::max<int32_t>(p->A->nrows, 1);
  const int64_t nB = std::max<int32_t>(p->B->nrows, 1);
  ensure_changed_cap(p, 0);
  const size_t need = work_bytes_for(N, nB);
  ProdWork w = carve_prod(ctx_scratch(p->ctx, need), N, nB);
  nchg = prod_sequence(p, mode, report_affected, w, d_nterm);
  if (nchg == ENTRY_INSTEAD) nchg = entry_finish(p);
  p->a_seq = p->src_a->apply_seq;
  p->b_seq = p->src_b->apply_seq;
  return nchg;
}

size_t prod_graph_work_bytes(const DProd* p) {
  return work_bytes_for(std::max<int32_t>(p->A->nrows, 1), std::max<int32_t>(p->B->nrows, 1));
}

void prod_prepare_graph(DProd* p, int64_t c_headroom, size_t arena_bytes, int64_t c_want) {
  ensure_changed_cap(p, std::max<int32_t>(p->A->nrows, 1));
  ensure_arena(p, arena_bytes);
  mat_reserve(p->C, c_headroom, std::max(c_headroom, c_want));
}

void prod_update_graph(DProd* p, void* work, int64_t* d_out) {
  const int64_t N = std::max<int32_t>(p->A->nrows, 1);
  const int64_t nB = std::max<int32_t>(p->B->nrows, 1);
  ProdWork w = carve_prod(work, N, nB);
  RowArgs R = row_args(p, w, 0, false);
  launch_front(p, 0, w, R);
  std::vector<std::pair<int, size_t>> none;
  launch_rows(p, R, w, nullptr, none);
  launch_tail(p, w, N);
  hipLaunchKernelGGL(k_publish, dim3(1), dim3(1), 0, p->ctx->stream, (const int32_t*)w.d_nchg,
                     (const int32_t*)w.d_count, (const int*)w.err, (const Plan*)w.plan, d_out);
  DSG_HIP(hipGetLastError());
}

int32_t prod_finish_graph(DProd* p, void* work) {
  Ctx* c = p->ctx;
  const int64_t N = std::max<int32_t>(p->A->nrows, 1);
  const int64_t nB = std::max<int32_t>(p->B->nrows, 1);
  ProdWork w = carve_prod(work, N, nB);
  Plan plan = read_plan(c, w, p->C);
  // the next replay should find room for every row: grow the arena by what
  // this one lacked (C's room follows its measured growth)
  if (plan.arena_short) ensure_arena(p, p->arena_bytes + plan.arena_short);
  std::vector<std::pair<int, size_t>> none;
  retry_rows(p, w, 0, false, plan, none);
  launch_tail(p, w, N);
  int32_t* h = (int32_t*)c->pinned;
  DSG_HIP(hipMemcpyAsync(h, w.d_nchg, 4, hipMemcpyDeviceToHost, c->stream));
  DSG_HIP(hipStreamSynchronize(c->stream));
  return h[0];
}
