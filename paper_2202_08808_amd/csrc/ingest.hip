// Batch ingest: apply (i, j, x) updates to a device dynamic matrix.
//
// Semantics (Section 4.1): SET replaces or inserts ("merge"), DELETE removes a
// present entry ("mask"), ADD folds x in with the semiring addition or
// inserts it.  A batch means its updates applied one after the other in batch
// order.
//
// Pipeline, all on the device:
//   1. key = (row << colbits) | col, stable LSD radix sort of (key, index);
//   2. segment heads -> unique keys and unique rows (the doubly compressed,
//      hypersparse shape the paper gives update matrices, Section 4);
//   3. fold each key's run in batch order: the last SET/DELETE is the base,
//      the ADDs after it are folded on top when the row is visited;
//   4. plan: one wavefront per touched row streams the row once, matches its
//      slots against the row's sorted unique updates by binary search, and
//      decides each update's outcome (insert / delete / overwrite / no-op);
//      rows that outgrow their slack request new space;
//   5. the host reserves pool space for the requested moves (one small
//      device-to-host read), then
//   6. commit: in place (holes left by deletions are filled by insertions
//      first, then by entries moved down from the row's tail) or into fresh
//      space; changed rows get the matrix's new epoch, and every structural
//      change is emitted for the transpose index, which is updated by the
//      same pipeline.
#include <algorithm>

#include "internal.h"
#include "kernel_common.h"

namespace {

constexpr uint8_t K_KEEP = 0, K_SET = 1, K_DEL = 2;
constexpr uint8_t OP_GUARD_ONLY = 3;  // internal op of mat_apply_sorted_add: no value
constexpr int PLAN_LDS = 1024;        // update columns of a row held in LDS by the plan
constexpr uint8_t PL_DEL = 1;         // plan flags of a touched row
constexpr uint8_t PL_HEAVY = 2;
constexpr uint8_t PL_FLAT = 4;        // heavy row planned update by update through its column index
constexpr uint8_t PL_PURE_DEL = 8;    // ... whose updates all delete: committed update by update too
constexpr int HEAVY_LEN = 2048;       // rows longer than this are planned by a whole workgroup
constexpr uint8_t C_NOP = UPD_NOP, C_INS = UPD_INS, C_DEL = UPD_DEL, C_OVR = UPD_OVR, C_LOST = UPD_LOST;
// the outcomes that change the operand, so the transpose index too
__device__ inline bool emits_delta(uint8_t code) { return code == C_INS || code == C_DEL || code == C_OVR; }

int bits_for(int64_t n) {
  int b = 0;
  while ((int64_t(1) << b) < n) ++b;
  return b;
}

unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// structure-only matrices (transpose index) carry no values
struct SemNone {
  using V = uint32_t;
  __device__ static V add(V a, V) { return a; }
};
template <int SR>
struct SemOf {
  using S = Sem<SR>;
};
template <>
struct SemOf<-1> {
  using S = SemNone;
};

__global__ void k_batch_keys(const int32_t* rows, const int32_t* cols, int64_t n, int cbits, uint64_t* keys,
                             uint32_t* idx) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) {
    keys[t] = ((uint64_t)(uint32_t)rows[t] << cbits) | (uint64_t)(uint32_t)cols[t];
    idx[t] = (uint32_t)t;
  }
}

__global__ void k_heads(const uint64_t* keys, int64_t n, int cbits, uint64_t sentinel, int64_t* kh,
                        int64_t* rh) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  uint64_t k = keys[t];
  bool valid = k != sentinel;
  bool newk = valid && (t == 0 || keys[t - 1] != k);
  bool newr = valid && (t == 0 || (keys[t - 1] >> cbits) != (k >> cbits));
  kh[t] = newk ? 1 : 0;
  rh[t] = newr ? 1 : 0;
}

struct Uniq {
  uint64_t* key;
  uint8_t* kind;
  uint64_t* val;  // raw value bits of the base (SET) value
  int32_t* add_start;
  int32_t* add_cnt;
  int32_t* slot;
  uint8_t* code;
  uint64_t* fin;  // raw bits of the final value
  uint64_t* old;  // raw bits of the value before (0 when absent)
  int32_t* urow;
  int32_t* row_first;
  int32_t* plen;
  int32_t* pcap;
  uint8_t* pchg;
  uint8_t* pdel;  // plan flags: PL_DEL the row loses entries, PL_HEAVY planned by the workgroup kernel
  int32_t* holes;
  int32_t* mv_src;
  int32_t* ur;      // per unique update: its row's index r
  int32_t* pcnt;    // per row r: deletions, inserts, overwrites, insert cursor (rows planned flat)
  uint8_t* pix;     // per row r planned flat: 1 when its column index takes the inserts
};

template <int VSZ>
__device__ inline uint64_t load_raw(const void* p, int64_t i) {
  if constexpr (VSZ == 8) return ((const uint64_t*)p)[i];
  if constexpr (VSZ == 4) return ((const uint32_t*)p)[i];
  return 0;
}
template <int VSZ>
__device__ inline void store_raw(void* p, int64_t i, uint64_t v) {
  if constexpr (VSZ == 8) ((uint64_t*)p)[i] = v;
  if constexpr (VSZ == 4) ((uint32_t*)p)[i] = (uint32_t)v;
}

template <class V>
__device__ inline V from_raw(uint64_t r) {
  if constexpr (sizeof(V) == 8) return __builtin_bit_cast(V, r);
  else return __builtin_bit_cast(V, (uint32_t)r);
}
template <class V>
__device__ inline uint64_t to_raw(V v) {
  if constexpr (sizeof(V) == 8) return __builtin_bit_cast(uint64_t, v);
  else return (uint64_t)__builtin_bit_cast(uint32_t, v);
}

// fold each unique key's run (in batch order, since the sort is stable)
template <int VSZ>
__global__ void k_fold(const uint64_t* keys, const uint32_t* idx, int64_t n, int cbits, const uint8_t* ops,
                       const void* vals, const int64_t* kh, const int64_t* ukpos, const int64_t* rh,
                       const int64_t* urpos, const int64_t* d_nU, const int64_t* d_nR, Uniq U) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) U.row_first[*d_nR] = (int32_t)*d_nU;
  // the flat plan's per-row counts start at zero (at most n rows)
  if (t < n) reinterpret_cast<int4*>(U.pcnt)[t] = make_int4(0, 0, 0, 0);
  if (t >= n || !kh[t]) return;
  uint64_t k = keys[t];
  int64_t u = ukpos[t];
  int64_t last = -1, e = t;
  while (e < n && keys[e] == k) {
    if (ops[idx[e]] != DSG_OP_ADD) last = e;
    ++e;
  }
  U.key[u] = k;
  if (ops[idx[t]] == OP_GUARD_ONLY) {
    // a key that only carries a guard (unique keys of a sorted ADD input)
    U.kind[u] = K_KEEP;
    U.val[u] = 0;
    U.add_start[u] = (int32_t)t;
    U.add_cnt[u] = 0;
  } else if (last < 0) {
    U.kind[u] = K_KEEP;
    U.val[u] = 0;
    U.add_start[u] = (int32_t)t;
    U.add_cnt[u] = (int32_t)(e - t);
  } else {
    bool del = ops[idx[last]] == DSG_OP_DELETE;
    U.kind[u] = del ? K_DEL : K_SET;
    U.val[u] = del ? 0 : load_raw<VSZ>(vals, idx[last]);
    U.add_start[u] = (int32_t)(last + 1);
    U.add_cnt[u] = (int32_t)(e - last - 1);
  }
  if (rh[t]) {
    int64_t r = urpos[t];
    U.urow[r] = (int32_t)(k >> cbits);
    U.row_first[r] = (int32_t)u;
  }
  U.ur[u] = (int32_t)(urpos[t] + rh[t] - 1);
}

// position of column c among the unique updates [u0, u1) of a row, or -1
__device__ inline int32_t find_update(const uint64_t* ukey, int32_t u0, int32_t u1, uint64_t cmask, int32_t c) {
  int32_t lo = u0, hi = u1;
  while (lo < hi) {
    int32_t mid = (lo + hi) >> 1;
    int32_t mc = (int32_t)(ukey[mid] & cmask);
    if (mc < c) lo = mid + 1;
    else hi = mid;
  }
  return (lo < u1 && (int32_t)(ukey[lo] & cmask) == c) ? lo : -1;
}

// Optional guard of an update (sorted ADD updates of a product, see
// mat_apply_sorted_add): entries it marks are left unchanged and get the
// outcome UPD_LOST (listed afterwards).
struct Guard {
  const uint64_t* key = nullptr;  // ordered key of the guarded value, per unique update
  const uint8_t* flag = nullptr;  // 2: guarded by key; 4: always lost when present
  // deletions of present entries whose slots are known (unique update u
  // deletes the entry at row-relative slot known_slot[known_list[u]]): no
  // plan, no row streamed (mat_apply_sorted_delete)
  const int32_t* known_slot = nullptr;
  const int32_t* known_list = nullptr;
};

// The outcome of unique update u of a row whose slot (or -1) the plan found:
// fold its chain onto the stored value, record code / final / previous
// value, and apply the guard (outcome UPD_LOST, the slot kept in U.slot).
template <int SR, int VSZ>
__device__ inline uint8_t plan_update(const DMat& m, int64_t off, const uint32_t* idx, const void* vals,
                                      const Uniq& U, const Guard& G, int32_t u) {
  using S = typename SemOf<SR>::S;
  using V = typename S::V;
  const int32_t s = U.slot[u];
  const bool present = s >= 0;
  const uint64_t old = present ? load_raw<VSZ>(m.val, off + s) : 0;
  uint64_t v = old;
  bool ex = present;
  const uint8_t kind = U.kind[u];
  if (kind == K_SET) {
    ex = true;
    v = U.val[u];
  } else if (kind == K_DEL) {
    ex = false;
  }
  const int32_t a0 = U.add_start[u], a1 = a0 + U.add_cnt[u];
  for (int32_t q = a0; q < a1; ++q) {
    const uint64_t x = load_raw<VSZ>(vals, idx[q]);
    if (ex) v = to_raw<V>(S::add(from_raw<V>(v), from_raw<V>(x)));
    else v = x;
    ex = true;
  }
  uint8_t code;
  if (present) code = ex ? ((VSZ && v != old) ? C_OVR : C_NOP) : C_DEL;
  else code = ex ? C_INS : C_NOP;
  if constexpr (VSZ > 0) {
    if (G.flag && present) {
      const uint8_t gf = G.flag[u];
      bool lost = (gf & 4) != 0;
      if (gf & 2) {
        // (min,+): the stored value came from a term that got worse and
        // nothing new beats or ties it
        const uint32_t kc = f32_key(__uint_as_float((uint32_t)old));
        const bool beats = a1 > a0 && f32_key(__uint_as_float((uint32_t)load_raw<VSZ>(vals, idx[a0]))) <= kc;
        lost = lost || ((uint64_t)kc == G.key[u] && !beats);
      }
      if (lost) {
        code = C_LOST;
        v = old;
      }
    }
  }
  U.code[u] = code;
  U.fin[u] = v;
  U.old[u] = present ? old : 0;
  return code;
}

template <int SR, int VSZ>
__global__ __launch_bounds__(256) void k_plan(DMat m, const int64_t* d_nR, uint64_t cmask, const uint32_t* idx,
                                              const void* vals, Uniq U, unsigned long long* demand, Guard G,
                                              RowIx X) {
  // the row's update columns (sorted) in LDS, per wavefront, when they fit
  __shared__ int32_t lcol[4][PLAN_LDS];
  const int lane = threadIdx.x & 63;
  int32_t* lk = lcol[(threadIdx.x >> 6) & 3];
  // one wavefront per touched row, rows taken in turn
  const int64_t nR = *d_nR;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < nR; r += nw) {
    const int32_t i = U.urow[r];
    const int32_t u0 = U.row_first[r], u1 = U.row_first[r + 1];
    const int32_t nu = u1 - u0;
    const int64_t off = m.row_off[i];
    const int32_t len = m.row_len[i], cap = m.row_cap[i];
    if (nu > PLAN_LDS || len > HEAVY_LEN) continue;  // k_plan_heavy takes this row
    if (ix_valid(X, i)) {
      // the row's column index gives each update's slot
      const uint64_t* t = X.tab + X.off[i];
      const uint32_t tn = (uint32_t)X.sz[i];
      for (int32_t u = u0 + lane; u < u1; u += 64) U.slot[u] = ix_find(t, tn, (int32_t)(U.key[u] & cmask));
    } else {
      const bool in_lds = true;
      for (int32_t u = u0 + lane; u < u1; u += 64) {
        U.slot[u] = -1;
        if (in_lds) lk[u - u0] = (int32_t)(U.key[u] & cmask);
      }
      __threadfence_block();
      __builtin_amdgcn_wave_barrier();
      // stream the row once (PU loads in flight per lane) and find each slot's update
      constexpr int PU = 8;
      for (int32_t s0 = lane; s0 < len; s0 += 64 * PU) {
        int32_t cc[PU];
#pragma unroll
        for (int v = 0; v < PU; ++v) cc[v] = s0 + v * 64 < len ? m.col[off + s0 + v * 64] : -1;
#pragma unroll
        for (int v = 0; v < PU; ++v) {
          if (cc[v] < 0) continue;
          int32_t u;
          if (in_lds) {
            int32_t lo = 0, hi = nu;
            while (lo < hi) {
              const int32_t mid = (lo + hi) >> 1;
              if (lk[mid] < cc[v]) lo = mid + 1;
              else hi = mid;
            }
            u = (lo < nu && lk[lo] == cc[v]) ? u0 + lo : -1;
          } else {
            u = find_update(U.key, u0, u1, cmask, cc[v]);
          }
          if (u >= 0) U.slot[u] = s0 + v * 64;
        }
      }
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    int32_t n_del = 0, n_ins = 0, n_ovr = 0;
    for (int32_t base = u0; base < u1; base += 64) {
      const int32_t u = base + lane;
      const uint8_t code = u < u1 ? plan_update<SR, VSZ>(m, off, idx, vals, U, G, u) : C_NOP;
      n_del += __popcll(__ballot(code == C_DEL));
      n_ins += __popcll(__ballot(code == C_INS));
      n_ovr += __popcll(__ballot(code == C_OVR));
    }
    if (lane == 0) {
      int32_t nl = len - n_del + n_ins;
      bool chg = (n_del + n_ins + n_ovr) > 0;
      bool reloc = nl > cap;
      U.plen[r] = nl;
      U.pchg[r] = chg ? 1 : 0;
      U.pdel[r] = n_del > 0 ? PL_DEL : 0;
      U.pcap[r] = reloc ? slack_cap(nl) : 0;
      if (reloc) atomicAdd(demand, (unsigned long long)slack_cap(nl));
    }
  }
}

template <int SR, int VSZ>
__global__ __launch_bounds__(256) void k_commit(DMat m, const int64_t* d_nR, uint64_t cmask, int cbits,
                                                Uniq U, const uint32_t* d_epoch, int tbits, uint64_t* dkey,
                                                uint8_t* dop, void* dval,
                                                int64_t dcap, int* err, RowIx X) {
  const int lane = threadIdx.x & 63;
  // one wavefront per touched row, rows taken in turn
  const int64_t nR = *d_nR;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < nR; r += nw) {
    if (!U.pchg[r]) continue;
    const int32_t i = U.urow[r];
    const int32_t u0 = U.row_first[r], u1 = U.row_first[r + 1];
    const int64_t off = m.row_off[i];
    const int32_t len = m.row_len[i];
    const int32_t nl = U.plen[r];
    const int32_t ncap = U.pcap[r];
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    // heavy rows (as the plan recorded them: many updates or a long row)
    // belong to k_commit_heavy, which runs after this kernel.  (The split goes
    // by the plan's flags: a row's length changes here.)
    if (U.pdel[r] & PL_HEAVY) continue;
    const bool nodel = !(U.pdel[r] & PL_DEL);
    if (nodel) {
      // ---- nothing deleted: the entries keep their order (moved as a block
      // when the row outgrows its space), overwrites go to the planned slots,
      // inserts after the row's entries ----
      int64_t dest = off;
      if (ncap) {
        unsigned long long no = 0;
        if (lane == 0) no = atomicAdd((unsigned long long*)m.d_top, (unsigned long long)ncap);
        no = __shfl(no, 0, 64);
        if ((int64_t)no + ncap > m.pool_cap) {
          if (lane == 0) atomicOr(err, 1);
          continue;
        }
        dest = (int64_t)no;
        for (int32_t s0 = lane; s0 < len; s0 += 256) {
          int32_t cc[4];
          uint64_t vv[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int32_t t = s0 + v * 64;
            cc[v] = t < len ? m.col[off + t] : 0;
            vv[v] = t < len ? load_raw<VSZ>(m.val, off + t) : 0;
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int32_t t = s0 + v * 64;
            if (t < len) {
              m.col[dest + t] = cc[v];
              store_raw<VSZ>(m.val, dest + t, vv[v]);
            }
          }
        }
      }
      // the row's column index keeps its positions; the inserts join it
      // unless they would fill it past 3/4 (then it is dropped)
      const bool ixv = ix_valid(X, i);
      const bool ixk = ixv && ix_fits(X, i, nl - len);
      uint64_t* ixt = ixk ? X.tab + X.off[i] : nullptr;
      const uint32_t ixn = ixk ? (uint32_t)X.sz[i] : 0u;
      int32_t k = 0;
      for (int32_t base = u0; base < u1; base += 64) {
        const int32_t u = base + lane;
        const uint8_t code = u < u1 ? U.code[u] : C_NOP;
        if (code == C_OVR) store_raw<VSZ>(m.val, dest + U.slot[u], U.fin[u]);
        const bool ins = code == C_INS;
        const uint64_t ib = __ballot(ins);
        if (ins) {
          const int32_t pos = len + k + __popcll(ib & lt);
          const int64_t dst = dest + pos;
          m.col[dst] = (int32_t)(U.key[u] & cmask);
          store_raw<VSZ>(m.val, dst, U.fin[u]);
          if (ixk) ix_put(ixt, ixn, (int32_t)(U.key[u] & cmask), pos);
        }
        k += __popcll(ib);
      }
      if (ncap && lane == 0) {
        m.row_off[i] = dest;
        m.row_cap[i] = ncap;
      }
      if (ixv && lane == 0) {
        if (ixk) X.used[i] += nl - len;
        else X.stamp[i] = 0;
      }
    } else {
      // ---- the row loses entries: mark the deleted slots (column -1) and
      // apply the overwrites where they stand ----
      const bool ixv = ix_valid(X, i);
      int32_t n_del = 0;
      for (int32_t base = u0; base < u1; base += 64) {
        const int32_t u = base + lane;
        const uint8_t code = u < u1 ? U.code[u] : C_NOP;
        if (code == C_DEL) m.col[off + U.slot[u]] = -1;
        else if (code == C_OVR) store_raw<VSZ>(m.val, off + U.slot[u], U.fin[u]);
        n_del += __popcll(__ballot(code == C_DEL));
      }
      // in place, the column index follows the entries (deleted ones leave
      // tombstones, moved ones get their new slot, inserts are recorded) while
      // it has room; a row moved to new space, or a full table, drops it
      const bool ixk = ixv && ncap == 0 && ix_fits(X, i, nl - len + n_del);
      uint64_t* ixt = ixk ? X.tab + X.off[i] : nullptr;
      const uint32_t ixn = ixk ? (uint32_t)X.sz[i] : 0u;
      if (ixk) {
        for (int32_t u = u0 + lane; u < u1; u += 64)
          if (U.code[u] == C_DEL) {
            const int32_t h = ix_slot(ixt, ixn, (int32_t)(U.key[u] & cmask));
            if (h >= 0) ixt[h] = IX_TOMB;
          }
      }
      if (ixv && lane == 0) {
        if (ixk) X.used[i] += nl - len + n_del;
        else X.stamp[i] = 0;
      }
      __threadfence_block();
      __builtin_amdgcn_wave_barrier();
      if (ncap == 0) {
        // in place: holes are the deleted slots below the new length, movers
        // the entries left at or above it; inserts fill the remaining holes,
        // then the space after the old length
        int32_t H = 0;
        for (int32_t base = u0; base < u1; base += 64) {
          const int32_t u = base + lane;
          const bool hole = u < u1 && U.code[u] == C_DEL && U.slot[u] < nl;
          const uint64_t hb = __ballot(hole);
          if (hole) U.holes[u0 + H + __popcll(hb & lt)] = U.slot[u];
          H += __popcll(hb);
        }
        int32_t Mc = 0;
        for (int32_t s0 = nl; s0 < len; s0 += 256) {  // 4 loads in flight per lane
          int32_t cc[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int32_t sl = s0 + v * 64 + lane;
            cc[v] = sl < len ? m.col[off + sl] : -1;
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const bool mover = cc[v] != -1;
            const uint64_t mb = __ballot(mover);
            if (mover) U.mv_src[u0 + Mc + __popcll(mb & lt)] = s0 + v * 64 + lane;
            Mc += __popcll(mb);
          }
        }
        __threadfence_block();
        __builtin_amdgcn_wave_barrier();
        for (int32_t q = lane; q < Mc; q += 64) {
          const int32_t src = U.mv_src[u0 + q], dst = U.holes[u0 + q];
          const int32_t cm = m.col[off + src];
          m.col[off + dst] = cm;
          store_raw<VSZ>(m.val, off + dst, load_raw<VSZ>(m.val, off + src));
          if (ixk) {
            const int32_t h = ix_slot(ixt, ixn, cm);
            if (h >= 0) ixt[h] = ((uint64_t)(uint32_t)dst << 32) | (uint64_t)(uint32_t)cm;
          }
        }
        int32_t k = 0;
        for (int32_t base = u0; base < u1; base += 64) {
          const int32_t u = base + lane;
          const bool ins = u < u1 && U.code[u] == C_INS;
          const uint64_t ib = __ballot(ins);
          if (ins) {
            const int32_t mm = Mc + k + __popcll(ib & lt);
            const int32_t dst = mm < H ? U.holes[u0 + mm] : len + (mm - H);
            m.col[off + dst] = (int32_t)(U.key[u] & cmask);
            store_raw<VSZ>(m.val, off + dst, U.fin[u]);
            if (ixk) ix_put(ixt, ixn, (int32_t)(U.key[u] & cmask), dst);
          }
          k += __popcll(ib);
        }
      } else {
        // move the row to fresh space, dropping the marked slots
        unsigned long long no = 0;
        if (lane == 0) no = atomicAdd((unsigned long long*)m.d_top, (unsigned long long)ncap);
        no = __shfl(no, 0, 64);
        if ((int64_t)no + ncap > m.pool_cap) {
          if (lane == 0) atomicOr(err, 1);
          continue;
        }
        int32_t kept = 0;
        for (int32_t base = 0; base < len; base += 256) {  // 4 loads in flight per lane
          int32_t cc[4];
          uint64_t vv[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int32_t sl = base + v * 64 + lane;
            cc[v] = sl < len ? m.col[off + sl] : -1;
            vv[v] = sl < len ? load_raw<VSZ>(m.val, off + sl) : 0;
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const bool keep = cc[v] != -1;
            const uint64_t kb = __ballot(keep);
            if (keep) {
              const int64_t dst = (int64_t)no + kept + __popcll(kb & lt);
              m.col[dst] = cc[v];
              store_raw<VSZ>(m.val, dst, vv[v]);
            }
            kept += __popcll(kb);
          }
        }
        for (int32_t base = u0; base < u1; base += 64) {
          const int32_t u = base + lane;
          const bool ins = u < u1 && U.code[u] == C_INS;
          const uint64_t ib = __ballot(ins);
          if (ins) {
            const int64_t dst = (int64_t)no + kept + __popcll(ib & lt);
            m.col[dst] = (int32_t)(U.key[u] & cmask);
            store_raw<VSZ>(m.val, dst, U.fin[u]);
          }
          kept += __popcll(ib);
        }
        if (lane == 0) {
          m.row_off[i] = (int64_t)no;
          m.row_cap[i] = ncap;
        }
      }
    }
    if (lane == 0) {
      m.row_len[i] = nl;
      m.row_epoch[i] = *d_epoch;
    }
    // changes for the transpose index at the update's own index: key
    // (col << tbits) | row, with the value (k_delta_keys reads the codes)
    if (dkey) {
      for (int32_t u = u0 + lane; u < u1; u += 64) {
        const uint8_t code = U.code[u];
        if (!emits_delta(code)) continue;
        if (u >= dcap) {  // an internal error, never written past the list
          atomicOr(err, 4);
          continue;
        }
        const uint64_t j = U.key[u] & cmask;
        dkey[u] = (j << tbits) | (uint64_t)(uint32_t)i;
        dop[u] = code == C_DEL ? DSG_OP_DELETE : DSG_OP_SET;
        store_raw<VSZ>(dval, u, U.fin[u]);
      }
    }
  }
}

// The plan of deletions at known slots: one wavefront per touched row
// records each update's slot and outcome and the row's new length; a heavy
// row with a usable column index is committed update by update
// (k_delete_flat), the others by k_commit / k_commit_heavy.
__global__ __launch_bounds__(256) void k_plan_known(DMat m, const int64_t* d_nR, Uniq U, Guard G, RowIx X) {
  const int lane = threadIdx.x & 63;
  const int64_t nR = *d_nR;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < nR; r += nw) {
    const int32_t i = U.urow[r];
    const int32_t u0 = U.row_first[r], u1 = U.row_first[r + 1];
    for (int32_t u = u0 + lane; u < u1; u += 64) {
      U.slot[u] = G.known_slot[G.known_list ? G.known_list[u] : u];
      U.code[u] = C_DEL;
      U.fin[u] = 0;
      U.old[u] = 0;
    }
    if (lane == 0) {
      const int32_t len = m.row_len[i], nd = u1 - u0;
      const bool heavy = nd > PLAN_LDS || len > HEAVY_LEN;
      U.plen[r] = len - nd;
      U.pchg[r] = 1;
      U.pcap[r] = 0;
      U.pdel[r] = PL_DEL | (heavy ? PL_HEAVY | (ix_valid(X, i) ? PL_FLAT | PL_PURE_DEL : 0) : 0);
      for (int x = 0; x < 4; ++x) U.pcnt[4 * r + x] = 0;
    }
  }
}

// per-row counts of the rows planned flat, cleared before each plan
__global__ void k_zero_pcnt(int32_t* pcnt, const int64_t* d_nR) {
  const int64_t n = 4 * *d_nR;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
    pcnt[x] = 0;
}

// Heavy rows (more than PLAN_LDS updates or longer than HEAVY_LEN) whose
// column index is usable, planned update by update: each thread looks its
// update's entry up and decides the outcome; the counts of deletions,
// inserts and overwrites go to the row (one atomic per counter and
// wavefront for the lanes of the wavefront's first row, one per lane for
// the few others).  A hub row's updates thus spread over the whole grid.
template <int SR, int VSZ>
__global__ __launch_bounds__(256) void k_plan_flat(DMat m, const int64_t* d_nU, uint64_t cmask, const uint32_t* idx,
                                                   const void* vals, Uniq U, Guard G, RowIx X) {
  const int lane = threadIdx.x & 63;
  const int64_t nU = *d_nU;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // (every lane of a wavefront runs the same number of rounds)
  for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); b0 < nU; b0 += stride) {
    const int64_t u = b0 + lane;
    int32_t r = -1;
    uint8_t code = C_NOP;
    if (u < nU) {
      r = U.ur[u];
      const int32_t i = U.urow[r];
      const int32_t u0 = U.row_first[r], u1 = U.row_first[r + 1];
      const int32_t len = m.row_len[i];
      if ((u1 - u0 > PLAN_LDS || len > HEAVY_LEN) && ix_valid(X, i)) {
        U.slot[u] = ix_lookup(X, i, (int32_t)(U.key[u] & cmask));
        code = plan_update<SR, VSZ>(m, m.row_off[i], idx, vals, U, G, (int32_t)u);
      } else {
        r = -1;  // planned by k_plan / k_plan_heavy
      }
    }
    const int32_t r0 = __shfl(r, 0, 64);
    const bool mine = r >= 0 && r == r0;
    const int32_t cd = __popcll(__ballot(mine && code == C_DEL));
    const int32_t ci = __popcll(__ballot(mine && code == C_INS));
    const int32_t co = __popcll(__ballot(mine && code == C_OVR));
    if (lane == 0 && r0 >= 0) {
      if (cd) atomicAdd(&U.pcnt[4 * r0], cd);
      if (ci) atomicAdd(&U.pcnt[4 * r0 + 1], ci);
      if (co) atomicAdd(&U.pcnt[4 * r0 + 2], co);
    }
    if (r >= 0 && !mine) {
      if (code == C_DEL) atomicAdd(&U.pcnt[4 * r], 1);
      else if (code == C_INS) atomicAdd(&U.pcnt[4 * r + 1], 1);
      else if (code == C_OVR) atomicAdd(&U.pcnt[4 * r + 2], 1);
    }
  }
}

// Heavy rows (more than PLAN_LDS updates): one 512-lane workgroup per row,
// rows taken in turn by a persistent grid.  The row's update columns go into
// an LDS hash (in runs of HEAVY_SLOTS/2 updates when there are more), the row
// is streamed once per run, and the outcomes are decided by all 8 waves.
// The two 4096-slot tables (32 KB) leave room for HEAVY_PLAN_PER_CU
// workgroups per CU: streaming a long row is latency-bound, and most heavy
// rows are long rows with few updates (an apply of sums to a product's rows).
constexpr int HEAVY_WG = 512;
constexpr int HEAVY_SLOTS = 4096;
constexpr int HEAVY_PLAN_PER_CU = 4;

template <int SR, int VSZ>
__global__ __launch_bounds__(HEAVY_WG) void k_plan_heavy(DMat m, const int64_t* d_nR, uint64_t cmask,
                                                         const uint32_t* idx, const void* vals, Uniq U,
                                                         unsigned long long* demand, Guard G, RowIx X) {
  __shared__ int32_t hk[HEAVY_SLOTS];
  __shared__ int32_t hu[HEAVY_SLOTS];
  __shared__ int32_t cnt[3];
  __shared__ int32_t wc[HEAVY_WG / 64];
  __shared__ int32_t picked[HEAVY_WG];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t nR = *d_nR;
  // this workgroup's share of the touched rows, scanned HEAVY_WG at a time by
  // every thread at once; the heavy ones are then taken in turn
  const int64_t per = (nR + gridDim.x - 1) / gridDim.x;
  const int64_t rb = (int64_t)blockIdx.x * per, re = min(nR, rb + per);
  for (int64_t c0 = rb; c0 < re; c0 += HEAVY_WG) {
    int32_t npick;
    {
      const int64_t rr = c0 + tid;
      bool f = false;
      if (rr < re) {
        const int32_t nu = U.row_first[rr + 1] - U.row_first[rr];
        f = nu > PLAN_LDS || m.row_len[U.urow[rr]] > HEAVY_LEN;
      }
      const int32_t q = block_flag_prefix<HEAVY_WG>(f, wc, npick);
      if (f) picked[q] = (int32_t)rr;
      __syncthreads();
    }
    for (int32_t pq = 0; pq < npick; ++pq) {
      const int64_t r = picked[pq];
      const int32_t u0 = U.row_first[r], u1 = U.row_first[r + 1];
      const int32_t i = U.urow[r];
      const int64_t off = m.row_off[i];
      const int32_t len = m.row_len[i], cap = m.row_cap[i];
      if (u1 - u0 <= PLAN_LDS && len <= HEAVY_LEN) continue;
      if (ix_valid(X, i)) {
        // (the same for every thread: no stamp changes during the plan)
        // k_plan_flat planned its updates; the row's outcome from its counts
        if (tid == 0) {
          const int32_t nd = U.pcnt[4 * r], ni = U.pcnt[4 * r + 1], no = U.pcnt[4 * r + 2];
          const int32_t nl = len - nd + ni;
          const bool reloc = nl > cap;
          U.plen[r] = nl;
          U.pchg[r] = (nd + ni + no) > 0 ? 1 : 0;
          U.pdel[r] = (nd > 0 ? PL_DEL : 0) | PL_HEAVY | PL_FLAT | (nd == u1 - u0 ? PL_PURE_DEL : 0);
          U.pcap[r] = reloc ? slack_cap(nl) : 0;
          if (reloc) atomicAdd(demand, (unsigned long long)slack_cap(nl));
        }
        continue;
      }
      if (tid < 3) cnt[tid] = 0;
      for (int32_t u = u0 + tid; u < u1; u += HEAVY_WG) U.slot[u] = -1;
      for (int32_t c0 = u0; c0 < u1; c0 += HEAVY_SLOTS / 2) {
        const int32_t c1 = min(u1, c0 + HEAVY_SLOTS / 2);
        // a table of twice this pass's updates (load <= 1/2): a long row with
        // few updates clears a few hundred slots, not all of them
        int32_t S = 256;
        while (S < 2 * (c1 - c0)) S <<= 1;
        const uint32_t hm = (uint32_t)S - 1;
        for (int x = tid; x < S; x += HEAVY_WG) hk[x] = -1;
        __syncthreads();
        for (int32_t u = c0 + tid; u < c1; u += HEAVY_WG) {
          const int32_t col = (int32_t)(U.key[u] & cmask);
          uint32_t h = hash_col(col) & hm;
          while (atomicCAS(&hk[h], -1, col) != -1) h = (h + 1) & hm;
          hu[h] = u;
        }
        __syncthreads();
        constexpr int SU = 8;  // row loads in flight per lane
        for (int32_t s0 = tid; s0 < len; s0 += SU * HEAVY_WG) {
          int32_t cc[SU];
#pragma unroll
          for (int v = 0; v < SU; ++v) cc[v] = s0 + v * HEAVY_WG < len ? m.col[off + s0 + v * HEAVY_WG] : -1;
#pragma unroll
          for (int v = 0; v < SU; ++v) {
            if (cc[v] < 0) continue;
            uint32_t h = hash_col(cc[v]) & hm;
            for (;;) {
              const int32_t x = hk[h];
              if (x == cc[v]) {
                U.slot[hu[h]] = s0 + v * HEAVY_WG;
                break;
              }
              if (x == -1) break;
              h = (h + 1) & hm;
            }
          }
        }
        __syncthreads();
      }
      int32_t nd = 0, ni = 0, no = 0;
      for (int32_t base = u0 + wv * 64; base < u1; base += HEAVY_WG) {
        const int32_t u = base + lane;
        const uint8_t code = u < u1 ? plan_update<SR, VSZ>(m, off, idx, vals, U, G, u) : C_NOP;
        nd += __popcll(__ballot(code == C_DEL));
        ni += __popcll(__ballot(code == C_INS));
        no += __popcll(__ballot(code == C_OVR));
      }
      if (lane == 0) {
        atomicAdd(&cnt[0], nd);
        atomicAdd(&cnt[1], ni);
        atomicAdd(&cnt[2], no);
      }
      __syncthreads();
      if (tid == 0) {
        const int32_t nl = len - cnt[0] + cnt[1];
        const bool chg = (cnt[0] + cnt[1] + cnt[2]) > 0;
        const bool reloc = nl > cap;
        U.plen[r] = nl;
        U.pchg[r] = chg ? 1 : 0;
        U.pdel[r] = (cnt[0] > 0 ? PL_DEL : 0) | PL_HEAVY;
        U.pcap[r] = reloc ? slack_cap(nl) : 0;
        if (reloc) atomicAdd(demand, (unsigned long long)slack_cap(nl));
      }
      __syncthreads();
    }
    __syncthreads();  // before the next share overwrites the picked rows
  }
}

// Commit of heavy rows (more than PLAN_LDS updates or longer than HEAVY_LEN),
// one workgroup per row, rows taken in turn:
//   - planned flat, no deletions: only the move to fresh space (when the row
//     outgrows it) and the row's bookkeeping; k_commit_flat then writes the
//     overwrites and inserts update by update;
//   - no deletions: move as a block if needed (4 loads in flight per lane),
//     overwrite at the planned slots, append the inserts;
//   - with deletions: overwrite and mark the deleted slots, then in place
//     fill the holes below the new length with the entries above it and the
//     inserts (the column index follows), or compact into fresh space when
//     the row outgrows its space (the column index is dropped).
// The transpose changes of every row but the flat ones are emitted here.
template <int SR, int VSZ>
__global__ __launch_bounds__(HEAVY_WG) void k_commit_heavy(DMat m, const int64_t* d_nR, uint64_t cmask, Uniq U,
                                                           const uint32_t* d_epoch, int tbits, uint64_t* dkey,
                                                           uint8_t* dop, void* dval,
                                                           int64_t dcap, int* err, RowIx X) {
  __shared__ int32_t wc[HEAVY_WG / 64];
  __shared__ int32_t picked[HEAVY_WG];
  __shared__ unsigned long long dest_s;
  const int tid = threadIdx.x;
  const int64_t nR = *d_nR;
  // this workgroup's share of the touched rows, scanned HEAVY_WG at a time by
  // every thread at once; the changed heavy ones are then taken in turn
  const int64_t per = (nR + gridDim.x - 1) / gridDim.x;
  const int64_t rb = (int64_t)blockIdx.x * per, re = min(nR, rb + per);
  for (int64_t c0 = rb; c0 < re; c0 += HEAVY_WG) {
    int32_t npick;
    {
      const int64_t rr = c0 + tid;
      const bool f = rr < re && U.pchg[rr] && (U.pdel[rr] & PL_HEAVY);
      const int32_t q = block_flag_prefix<HEAVY_WG>(f, wc, npick);
      if (f) picked[q] = (int32_t)rr;
      __syncthreads();
    }
    for (int32_t pq = 0; pq < npick; ++pq) {
      const int64_t r = picked[pq];
      const int32_t u0 = U.row_first[r], u1 = U.row_first[r + 1];
      const uint8_t pf = U.pdel[r];
      // unchanged or light: k_commit did it
      if (!U.pchg[r] || !(pf & PL_HEAVY)) continue;
      const bool nodel = !(pf & PL_DEL);
      const bool flat = (pf & PL_FLAT) != 0;
      const int32_t i = U.urow[r];
      if (pf & PL_PURE_DEL) {
        // k_delete_flat moves the entries; the row keeps its space and index
        if (tid == 0) {
          m.row_len[i] = U.plen[r];
          m.row_epoch[i] = *d_epoch;
        }
        continue;
      }
      const int64_t off = m.row_off[i];
      const int32_t len = m.row_len[i];
      const int32_t nl = U.plen[r];
      const int32_t ncap = U.pcap[r];
      const bool ixv = ix_valid(X, i);  // read by every thread before anyone changes it
      int64_t dest = off;
      if (ncap) {
        if (tid == 0) dest_s = atomicAdd((unsigned long long*)m.d_top, (unsigned long long)ncap);
        __syncthreads();
        dest = (int64_t)dest_s;
        __syncthreads();
        if (dest + ncap > m.pool_cap) {
          if (tid == 0) atomicOr(err, 1);
          continue;
        }
      }
      bool ixk = false;  // the column index stays usable
      if (nodel) {
        if (ncap) {
          for (int32_t t0 = tid; t0 < len; t0 += 4 * HEAVY_WG) {
            int32_t cc[4];
            uint64_t vv[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int32_t t = t0 + v * HEAVY_WG;
              cc[v] = t < len ? m.col[off + t] : 0;
              vv[v] = t < len ? load_raw<VSZ>(m.val, off + t) : 0;
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int32_t t = t0 + v * HEAVY_WG;
              if (t < len) {
                m.col[dest + t] = cc[v];
                store_raw<VSZ>(m.val, dest + t, vv[v]);
              }
            }
          }
        }
        // the inserts join the column index unless it would be past 3/4 full
        ixk = ixv && ix_fits(X, i, nl - len);
        if (!flat) {
          uint64_t* ixt = ixk ? X.tab + X.off[i] : nullptr;
          const uint32_t ixn = ixk ? (uint32_t)X.sz[i] : 0u;
          for (int32_t u = u0 + tid; u < u1; u += HEAVY_WG)
            if (U.code[u] == C_OVR) store_raw<VSZ>(m.val, dest + U.slot[u], U.fin[u]);
          // inserts after the row's entries, in update order
          int32_t k = 0;
          for (int32_t base = u0; base < u1; base += HEAVY_WG) {
            const int32_t u = base + tid;
            const bool ins = u < u1 && U.code[u] == C_INS;
            int32_t tot;
            const int32_t q = block_flag_prefix<HEAVY_WG>(ins, wc, tot);
            if (ins) {
              const int32_t pos = len + k + q;
              m.col[dest + pos] = (int32_t)(U.key[u] & cmask);
              store_raw<VSZ>(m.val, dest + pos, U.fin[u]);
              if (ixk) ix_put(ixt, ixn, (int32_t)(U.key[u] & cmask), pos);
            }
            k += tot;
          }
        } else if (tid == 0) {
          U.pix[r] = ixk ? 1 : 0;
        }
      } else {
        // overwrites and deletion marks at the planned slots
        int32_t nd = 0;
        for (int32_t base = u0; base < u1; base += HEAVY_WG) {
          const int32_t u = base + tid;
          const uint8_t code = u < u1 ? U.code[u] : C_NOP;
          if (code == C_DEL) m.col[off + U.slot[u]] = -1;
          else if (code == C_OVR) store_raw<VSZ>(m.val, off + U.slot[u], U.fin[u]);
          int32_t tot;
          (void)block_flag_prefix<HEAVY_WG>(code == C_DEL, wc, tot);
          nd += tot;
        }
        const int32_t ni = nl - len + nd;
        __threadfence_block();
        __syncthreads();
        if (ncap == 0) {
          ixk = ixv && ix_fits(X, i, ni);
          uint64_t* ixt = ixk ? X.tab + X.off[i] : nullptr;
          const uint32_t ixn = ixk ? (uint32_t)X.sz[i] : 0u;
          // holes: deleted slots below the new length (their columns leave
          // tombstones in the index)
          int32_t H = 0;
          for (int32_t base = u0; base < u1; base += HEAVY_WG) {
            const int32_t u = base + tid;
            const bool del = u < u1 && U.code[u] == C_DEL;
            if (del && ixk) {
              const int32_t h = ix_slot(ixt, ixn, (int32_t)(U.key[u] & cmask));
              if (h >= 0) ixt[h] = IX_TOMB;
            }
            const bool hole = del && U.slot[u] < nl;
            int32_t tot;
            const int32_t q = block_flag_prefix<HEAVY_WG>(hole, wc, tot);
            if (hole) U.holes[u0 + H + q] = U.slot[u];
            H += tot;
          }
          // movers: entries left at or above the new length
          int32_t Mc = 0;
          for (int32_t s0 = nl; s0 < len; s0 += HEAVY_WG) {
            const int32_t sl = s0 + tid;
            const bool mover = sl < len && m.col[off + sl] != -1;
            int32_t tot;
            const int32_t q = block_flag_prefix<HEAVY_WG>(mover, wc, tot);
            if (mover) U.mv_src[u0 + Mc + q] = sl;
            Mc += tot;
          }
          __threadfence_block();
          __syncthreads();
          for (int32_t q = tid; q < Mc; q += HEAVY_WG) {
            const int32_t src = U.mv_src[u0 + q], dst = U.holes[u0 + q];
            const int32_t cm = m.col[off + src];
            m.col[off + dst] = cm;
            store_raw<VSZ>(m.val, off + dst, load_raw<VSZ>(m.val, off + src));
            if (ixk) {
              const int32_t h = ix_slot(ixt, ixn, cm);
              if (h >= 0) ixt[h] = ((uint64_t)(uint32_t)dst << 32) | (uint64_t)(uint32_t)cm;
            }
          }
          // inserts: the remaining holes, then the space after the old length
          int32_t k = 0;
          for (int32_t base = u0; base < u1; base += HEAVY_WG) {
            const int32_t u = base + tid;
            const bool ins = u < u1 && U.code[u] == C_INS;
            int32_t tot;
            const int32_t q = block_flag_prefix<HEAVY_WG>(ins, wc, tot);
            if (ins) {
              const int32_t mm = Mc + k + q;
              const int32_t dst = mm < H ? U.holes[u0 + mm] : len + (mm - H);
              m.col[off + dst] = (int32_t)(U.key[u] & cmask);
              store_raw<VSZ>(m.val, off + dst, U.fin[u]);
              if (ixk) ix_put(ixt, ixn, (int32_t)(U.key[u] & cmask), dst);
            }
            k += tot;
          }
        } else {
          // compact into fresh space, then append the inserts
          int32_t kept = 0;
          for (int32_t s0 = 0; s0 < len; s0 += HEAVY_WG) {
            const int32_t sl = s0 + tid;
            const int32_t cc = sl < len ? m.col[off + sl] : -1;
            const uint64_t vv = sl < len ? load_raw<VSZ>(m.val, off + sl) : 0;
            int32_t tot;
            const int32_t q = block_flag_prefix<HEAVY_WG>(cc != -1, wc, tot);
            if (cc != -1) {
              m.col[dest + kept + q] = cc;
              store_raw<VSZ>(m.val, dest + kept + q, vv);
            }
            kept += tot;
          }
          for (int32_t base = u0; base < u1; base += HEAVY_WG) {
            const int32_t u = base + tid;
            const bool ins = u < u1 && U.code[u] == C_INS;
            int32_t tot;
            const int32_t q = block_flag_prefix<HEAVY_WG>(ins, wc, tot);
            if (ins) {
              m.col[dest + kept + q] = (int32_t)(U.key[u] & cmask);
              store_raw<VSZ>(m.val, dest + kept + q, U.fin[u]);
            }
            kept += tot;
          }
        }
        if (ixk && tid == 0) X.used[i] += ni;
      }
      __syncthreads();  // every thread has used the row's old bookkeeping
      if (tid == 0) {
        if (ixv) {
          if (!ixk) X.stamp[i] = 0;
          else if (nodel) X.used[i] += nl - len;
        }
        m.row_len[i] = nl;
        m.row_epoch[i] = *d_epoch;
        if (ncap) {
          m.row_off[i] = dest;
          m.row_cap[i] = ncap;
        }
      }
      if (dkey && !(flat && nodel)) {  // at the update's own index, as in k_commit
        for (int32_t u = u0 + tid; u < u1; u += HEAVY_WG) {
          const uint8_t code = U.code[u];
          if (!emits_delta(code)) continue;
          if (u >= dcap) {
            atomicOr(err, 4);
            continue;
          }
          const uint64_t j = U.key[u] & cmask;
          dkey[u] = (j << tbits) | (uint64_t)(uint32_t)i;
          dop[u] = code == C_DEL ? DSG_OP_DELETE : DSG_OP_SET;
          store_raw<VSZ>(dval, u, U.fin[u]);
        }
      }
      __syncthreads();
    }
    __syncthreads();  // before the next share overwrites the picked rows
  }
}

// Heavy rows planned flat whose updates all delete (nd of them, new length
// nl = len - nd, always in place), update by update in three launches:
//   1. mark each deleted slot, leave a tombstone in the column index, emit
//      the transpose change; a deleted slot below nl is a hole (ticket from
//      the row's hole counter);
//   2. update q of the row looks at slot nl + q of the old tail: a live
//      entry there is a mover (ticket from the row's mover counter);
//   3. mover t goes to hole t (its index slot follows).
// Holes and movers are equally many; which hole a mover fills does not
// matter.  Counters are taken once per wavefront for the lanes of its first
// row.
__device__ inline int32_t row_ticket(int32_t* ctr, int32_t r, bool take, int lane) {
  const int32_t r0 = __shfl(r, 0, 64);
  const bool mine = take && r == r0;
  const uint64_t bm = __ballot(mine);
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  int32_t base = 0;
  if (lane == 0 && bm) base = atomicAdd(&ctr[4 * r0], (int32_t)__popcll(bm));
  base = __shfl(base, 0, 64);
  if (!take) return -1;
  return mine ? base + __popcll(bm & lt) : atomicAdd(&ctr[4 * r], 1);
}

template <int VSZ>
__global__ __launch_bounds__(256) void k_delete_flat(DMat m, const int64_t* d_nU, uint64_t cmask, Uniq U,
                                                     int stage, int tbits, uint64_t* dkey, uint8_t* dop,
                                                     void* dval, int64_t dcap, int* err, RowIx X) {
  const int lane = threadIdx.x & 63;
  const int64_t nU = *d_nU;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); b0 < nU; b0 += stride) {
    const int64_t u = b0 + lane;
    int32_t r = -1;
    if (u < nU) {
      r = U.ur[u];
      if (!(U.pdel[r] & PL_PURE_DEL)) r = -1;
    }
    const int32_t i = r >= 0 ? U.urow[r] : 0;
    const int64_t off = r >= 0 ? m.row_off[i] : 0;
    const int32_t nl = r >= 0 ? U.plen[r] : 0;
    const bool ixk = r >= 0 && ix_valid(X, i);
    if (stage == 1) {
      bool hole = false;
      int32_t sl = 0;
      if (r >= 0) {
        sl = U.slot[u];
        const int32_t c = (int32_t)(U.key[u] & cmask);
        m.col[off + sl] = -1;
        if (ixk) {
          const int32_t h = ix_slot(X.tab + X.off[i], (uint32_t)X.sz[i], c);
          if (h >= 0) X.tab[X.off[i] + h] = IX_TOMB;
        }
        hole = sl < nl;
        if (dkey) {
          if (u >= dcap) {
            atomicOr(err, 4);
          } else {
            dkey[u] = ((uint64_t)(uint32_t)c << tbits) | (uint64_t)(uint32_t)i;
            dop[u] = DSG_OP_DELETE;
            store_raw<VSZ>(dval, u, U.fin[u]);
          }
        }
      }
      const int32_t t = row_ticket(U.pcnt + 1, r, hole, lane);
      if (hole) U.holes[U.row_first[r] + t] = sl;
    } else if (stage == 2) {
      bool mover = false;
      int32_t p = 0;
      if (r >= 0) {
        p = nl + (int32_t)(u - U.row_first[r]);
        mover = m.col[off + p] != -1;
      }
      const int32_t t = row_ticket(U.pcnt + 2, r, mover, lane);
      if (mover) U.mv_src[U.row_first[r] + t] = p;
    } else if (r >= 0) {
      const int32_t t = (int32_t)(u - U.row_first[r]);
      if (t < U.pcnt[4 * r + 2]) {
        const int32_t src = U.mv_src[U.row_first[r] + t], dst = U.holes[U.row_first[r] + t];
        const int32_t cm = m.col[off + src];
        m.col[off + dst] = cm;
        store_raw<VSZ>(m.val, off + dst, load_raw<VSZ>(m.val, off + src));
        if (ixk) {
          const int32_t h = ix_slot(X.tab + X.off[i], (uint32_t)X.sz[i], cm);
          if (h >= 0) X.tab[X.off[i] + h] = ((uint64_t)(uint32_t)dst << 32) | (uint64_t)(uint32_t)cm;
        }
      }
    }
  }
}

// The overwrites and inserts of heavy rows planned flat without deletions,
// update by update (after k_commit_heavy moved such rows and decided on
// their column index): inserts take places after the row's old entries
// from the row's cursor (one atomic per wavefront for the lanes of its
// first row), in no particular order.
template <int SR, int VSZ>
__global__ __launch_bounds__(256) void k_commit_flat(DMat m, const int64_t* d_nU, uint64_t cmask, Uniq U, int tbits,
                                                     uint64_t* dkey, uint8_t* dop, void* dval, int64_t dcap,
                                                     int* err, RowIx X) {
  const int lane = threadIdx.x & 63;
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int64_t nU = *d_nU;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); b0 < nU; b0 += stride) {
    const int64_t u = b0 + lane;
    int32_t r = -1;
    uint8_t code = C_NOP;
    if (u < nU) {
      r = U.ur[u];
      // (a row that had to move but found no room is left alone: the
      // commit reported the error)
      if (U.pdel[r] == (PL_HEAVY | PL_FLAT) && U.pchg[r] &&
          !(U.pcap[r] && m.row_cap[U.urow[r]] != U.pcap[r]))
        code = U.code[u];
      else
        r = -1;
    }
    const bool ins = code == C_INS;
    const int32_t r0 = __shfl(r, 0, 64);
    const bool mine = ins && r == r0;
    const uint64_t bm = __ballot(mine);
    int32_t base = 0;
    if (lane == 0 && bm) base = atomicAdd(&U.pcnt[4 * r0 + 3], (int32_t)__popcll(bm));
    base = __shfl(base, 0, 64);
    if (r < 0) continue;
    const int32_t i = U.urow[r];
    const int64_t off = m.row_off[i];
    if (code == C_OVR) {
      store_raw<VSZ>(m.val, off + U.slot[u], U.fin[u]);
    } else if (ins) {
      const int32_t k = mine ? base + __popcll(bm & lt) : atomicAdd(&U.pcnt[4 * r + 3], 1);
      const int32_t pos = U.plen[r] - U.pcnt[4 * r + 1] + k;  // after the old entries
      const int32_t c = (int32_t)(U.key[u] & cmask);
      m.col[off + pos] = c;
      store_raw<VSZ>(m.val, off + pos, U.fin[u]);
      if (U.pix[r]) ix_put(X.tab + X.off[i], (uint32_t)X.sz[i], c, pos);
    }
    if (dkey && emits_delta(code)) {
      if (u >= dcap) {
        atomicOr(err, 4);
      } else {
        const uint64_t j = U.key[u] & cmask;
        dkey[u] = (j << tbits) | (uint64_t)(uint32_t)i;
        dop[u] = DSG_OP_SET;
        store_raw<VSZ>(dval, u, U.fin[u]);
      }
    }
  }
}

// Sort input of the transpose's apply: the delta of unique update t where it
// changed the operand, the sentinel elsewhere (and past the unique updates).
__global__ void k_delta_keys(const uint64_t* dkey, const uint8_t* code, const int64_t* d_nU, uint64_t sentinel,
                             uint64_t* keys, uint32_t* idx, int64_t n) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) {
    keys[t] = t < *d_nU && emits_delta(code[t]) ? dkey[t] : sentinel;
    idx[t] = (uint32_t)t;
  }
}

__global__ void k_validate(const int32_t* rows, const int32_t* cols, const uint8_t* ops, int64_t n,
                           int32_t nrows, int32_t ncols, int* flags) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  if (rows[t] < 0 || rows[t] >= nrows || cols[t] < 0 || cols[t] >= ncols) atomicOr(flags, 1);
  if (ops[t] > DSG_OP_ADD) atomicOr(flags, 2);
}

struct Work {
  uint64_t* keys;
  uint32_t* idx;
  void* radix;
  int64_t* kh;
  int64_t* rh;
  int64_t* ukpos;
  int64_t* urpos;
  int64_t* nU;
  int64_t* nR;
  void* scan;
  Uniq U;
  unsigned long long* demand;
  unsigned long long* ndelta;
  int* err;
  uint64_t* dkey;
  uint8_t* dop;
  void* dval;
  uint8_t* allops;  // presorted ADD input: one ADD op per entry
};

size_t work_bytes(int64_t n, bool deltas) {
  size_t N = (size_t)(n > 0 ? n : 1);
  return Carve::need({N * 8, N * 4, radix_scratch_bytes(n), N * 8, N * 8, N * 8, N * 8, 64, 64,
                      scan_scratch_bytes(n), N * 8, N, N * 8, N * 4, N * 4, N * 4, N, N * 8, N * 4,
                      (N + 1) * 4, N * 4, N * 4, N, N * 4, N * 4, N * 4, 64, 64, 64,
                      deltas ? N * 8 : 0, deltas ? N : 0, deltas ? N * 8 : 0, N * 8, N, N, N * 16, N});
}

Work carve_work(void* base, int64_t n, bool deltas) {
  size_t N = (size_t)(n > 0 ? n : 1);
  Carve cv(base, work_bytes(n, deltas));
  Work w;
  w.keys = cv.take<uint64_t>(N);
  w.idx = cv.take<uint32_t>(N);
  w.radix = cv.take<char>(radix_scratch_bytes(n));
  w.kh = cv.take<int64_t>(N);
  w.rh = cv.take<int64_t>(N);
  w.ukpos = cv.take<int64_t>(N);
  w.urpos = cv.take<int64_t>(N);
  w.nU = cv.take<int64_t>(8);
  w.nR = cv.take<int64_t>(8);
  w.scan = cv.take<char>(scan_scratch_bytes(n));
  w.U.key = cv.take<uint64_t>(N);
  w.U.kind = cv.take<uint8_t>(N);
  w.U.val = cv.take<uint64_t>(N);
  w.U.add_start = cv.take<int32_t>(N);
  w.U.add_cnt = cv.take<int32_t>(N);
  w.U.slot = cv.take<int32_t>(N);
  w.U.code = cv.take<uint8_t>(N);
  w.U.fin = cv.take<uint64_t>(N);
  w.U.urow = cv.take<int32_t>(N);
  w.U.row_first = cv.take<int32_t>(N + 1);
  w.U.plen = cv.take<int32_t>(N);
  w.U.pcap = cv.take<int32_t>(N);
  w.U.pchg = cv.take<uint8_t>(N);
  w.U.holes = cv.take<int32_t>(N);
  w.U.mv_src = cv.take<int32_t>(N);
  w.U.ur = cv.take<int32_t>(N);
  w.demand = cv.take<unsigned long long>(8);
  w.ndelta = cv.take<unsigned long long>(8);
  w.err = cv.take<int>(16);
  w.dkey = deltas ? cv.take<uint64_t>(N) : nullptr;
  w.dop = deltas ? cv.take<uint8_t>(N) : nullptr;
  w.dval = deltas ? (void*)cv.take<uint64_t>(N) : nullptr;
  w.U.old = cv.take<uint64_t>(N);
  w.allops = cv.take<uint8_t>(N);
  w.U.pdel = cv.take<uint8_t>(N);
  w.U.pcnt = cv.take<int32_t>(N * 4);
  w.U.pix = cv.take<uint8_t>(N);
  return w;
}

// Entries of the rows an apply touches, before it changes them (the rows its
// plan streams): one atomic per workgroup.
__global__ __launch_bounds__(256) void k_touched_len(const int32_t* urow, const int64_t* d_nR, const int32_t* row_len,
                                                     unsigned long long* acc) {
  __shared__ unsigned long long sum;
  if (threadIdx.x == 0) sum = 0;
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < *d_nR) atomicAdd(&sum, (unsigned long long)row_len[urow[r]]);
  __syncthreads();
  if (threadIdx.x == 0 && sum) atomicAdd(acc, sum);
}
__global__ void k_zero_u64(unsigned long long* a) { *a = 0; }
// The apply's counters cleared and the matrix's epoch advanced, in one launch.
__global__ void k_zero_counters(unsigned long long* a, unsigned long long* b, int* c, uint32_t* epoch) {
  *a = 0;
  *b = 0;
  *c = 0;
  *epoch += 1;
}

// The transpose deltas of a planned apply (what k_commit / k_commit_heavy
// write while committing), taken from the plan's outcomes before anything is
// committed, so that the transpose index can be planned -- and its room
// reserved -- before either matrix changes.
template <int VSZ>
__global__ void k_plan_deltas(Uniq U, const int64_t* d_nU, uint64_t cmask, int cbits, int tbits, uint64_t* dkey,
                              uint8_t* dop, void* dval) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= *d_nU) return;
  const uint8_t code = U.code[u];
  if (!emits_delta(code)) return;
  const uint64_t i = U.key[u] >> cbits, j = U.key[u] & cmask;
  dkey[u] = (j << tbits) | i;
  dop[u] = code == C_DEL ? DSG_OP_DELETE : DSG_OP_SET;
  store_raw<VSZ>(dval, u, U.fin[u]);
}

// Phases of one matrix's apply: PH_PLAN plans the unique updates; PH_ROOM
// (outside graphs) reserves the room moved rows need, re-planning after a
// compaction -- from the demand the caller already read back (demand0 >= 0)
// or after reading it; PH_COMMIT commits them, writing the transpose deltas
// too unless they were taken from the plan already (deltas_done).
constexpr int PH_PLAN = 1, PH_COMMIT = 2, PH_ROOM = 4;

template <int SR, int VSZ>
void launch_plan_commit(DMat* m, Work& w, int64_t n, uint64_t cmask, int cbits, const void* vals, int tbits,
                        bool graph, const Guard& G, int phases = PH_PLAN | PH_ROOM | PH_COMMIT,
                        bool deltas_done = false, int64_t demand0 = -1) {
  Ctx* c = m->ctx;
  hipStream_t s = c->stream;
  // plan and commit take the touched rows in turn: a grid of at most 32
  // workgroups per CU, not one wavefront per update
  unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks_for(n * 64, 256), 32 * (int64_t)c->num_cus));
  const unsigned nh = (unsigned)std::max(1, c->num_cus);
  const unsigned nph = nh * HEAVY_PLAN_PER_CU;  // the heavy commit takes the same grid
  // the column index is used outside graphs only (a captured launch would
  // keep the index generation of its capture); whoever replays a graph
  // apply drops the matrix's index
  const RowIx X = graph ? RowIx() : mat_index_view(m);
  // the flat kernels: one thread per unique update, bounded grid
  const unsigned nf = (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks_for(n, 256), 32 * (int64_t)c->num_cus));
  if ((phases & PH_PLAN) && G.known_slot) {
    // deletions at known slots: nothing to look up, no row moves
    hipLaunchKernelGGL(k_plan_known, dim3(nb), dim3(256), 0, s, *m, w.nR, w.U, G, X);
  } else if (phases & PH_PLAN) {
  // tables for the touched rows that have none, before the plan looks them up
  if (X.tab) {
    // (the fold cleared the per-row counts)
    mat_index_build(m, w.U.urow, w.nR, n);
    hipLaunchKernelGGL((k_plan_flat<SR, VSZ>), dim3(nf), dim3(256), 0, s, *m, (const int64_t*)w.nU, cmask, w.idx,
                       vals, w.U, G, X);
  }
  hipLaunchKernelGGL((k_plan<SR, VSZ>), dim3(nb), dim3(256), 0, s, *m, w.nR, cmask, w.idx, vals, w.U,
                     w.demand, G, X);
  hipLaunchKernelGGL((k_plan_heavy<SR, VSZ>), dim3(nph), dim3(HEAVY_WG), 0, s, *m, w.nR, cmask, w.idx, vals, w.U,
                     w.demand, G, X);
  }
  if ((phases & PH_ROOM) && !graph && !G.known_slot) {
    // the one host round trip: how much pool space moved rows need
    unsigned long long* h = (unsigned long long*)c->pinned;
    for (;;) {
      if (demand0 >= 0) {
        h[0] = (unsigned long long)demand0;
        demand0 = -1;
      } else {
        DSG_HIP(hipMemcpyAsync(h, w.demand, 8, hipMemcpyDeviceToHost, s));
        DSG_HIP(hipStreamSynchronize(s));
      }
      const int64_t demand = (int64_t)h[0];
      if (demand == 0) break;
      const uint64_t version = m->version;
      mat_reserve(m, demand);
      if (m->version == version) {
        m->h_top_ub += demand;
        break;
      }
      // the pool was compacted, which reset every row's capacity to the slack
      // of its length: a row planned to grow in place may no longer fit, so
      // plan again against the new capacities
      hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, w.demand);
      if (X.tab) {
        hipLaunchKernelGGL(k_zero_pcnt, dim3(nf), dim3(256), 0, s, w.U.pcnt, (const int64_t*)w.nR);
        hipLaunchKernelGGL((k_plan_flat<SR, VSZ>), dim3(nf), dim3(256), 0, s, *m, (const int64_t*)w.nU, cmask,
                           w.idx, vals, w.U, G, X);
      }
      hipLaunchKernelGGL((k_plan<SR, VSZ>), dim3(nb), dim3(256), 0, s, *m, w.nR, cmask, w.idx, vals, w.U,
                         w.demand, G, X);
      hipLaunchKernelGGL((k_plan_heavy<SR, VSZ>), dim3(nph), dim3(HEAVY_WG), 0, s, *m, w.nR, cmask, w.idx, vals,
                         w.U, w.demand, G, X);
    }
  }
  if (!(phases & PH_COMMIT)) return;
  // (graph mode: the caller reserved the worst case, see apply_headroom)
  uint64_t* dk = deltas_done ? nullptr : w.dkey;
  hipLaunchKernelGGL((k_commit<SR, VSZ>), dim3(nb), dim3(256), 0, s, *m, w.nR, cmask, cbits, w.U,
                     (const uint32_t*)m->d_epoch, tbits, dk, w.dop, w.dval, n, w.err, X);
  hipLaunchKernelGGL((k_commit_heavy<SR, VSZ>), dim3(nph), dim3(HEAVY_WG), 0, s, *m, w.nR, cmask, w.U,
                     (const uint32_t*)m->d_epoch, tbits, dk, w.dop, w.dval, n, w.err, X);
  if (X.tab) {
    hipLaunchKernelGGL((k_commit_flat<SR, VSZ>), dim3(nf), dim3(256), 0, s, *m, (const int64_t*)w.nU, cmask, w.U,
                       tbits, dk, w.dop, w.dval, n, w.err, X);
    for (int stage = 1; stage <= 3; ++stage)
      hipLaunchKernelGGL((k_delete_flat<VSZ>), dim3(nf), dim3(256), 0, s, *m, (const int64_t*)w.nU, cmask, w.U,
                         stage, tbits, dk, w.dop, w.dval, n, w.err, X);
  }
}

// Steps 2-6 on keys/idx already filled (n entries, sentinel-padded allowed);
// phases as launch_plan_commit (sorting, folding and the epoch bump belong to
// the plan).
void run_core(DMat* m, Work& w, int64_t n, int key_bits, bool padded, const uint8_t* ops, const void* vals,
              bool graph, bool presorted = false, const Guard& G = Guard(),
              int phases = PH_PLAN | PH_ROOM | PH_COMMIT, bool deltas_done = false, int64_t demand0 = -1,
              int key_lo = 0) {
  Ctx* c = m->ctx;
  hipStream_t s = c->stream;
  int cbits = bits_for(m->ncols);
  uint64_t sentinel = 1ull << key_bits;
  uint64_t cmask = (1ull << cbits) - 1;
  int tbits = bits_for(m->nrows);
  if (!(phases & PH_PLAN)) {
    const int ph = phases;
    const bool dd = deltas_done;
    const int64_t d0 = demand0;
    switch (m->sr) {
      case 0: launch_plan_commit<0, 8>(m, w, n, cmask, cbits, vals, tbits, graph, G, ph, dd, d0); break;
      case 1: launch_plan_commit<1, 4>(m, w, n, cmask, cbits, vals, tbits, graph, G, ph, dd, d0); break;
      case 2: launch_plan_commit<2, 8>(m, w, n, cmask, cbits, vals, tbits, graph, G, ph, dd, d0); break;
      case 3: launch_plan_commit<3, 4>(m, w, n, cmask, cbits, vals, tbits, graph, G, ph, dd, d0); break;
      default: launch_plan_commit<-1, 0>(m, w, n, cmask, cbits, vals, tbits, graph, G, ph, dd, d0); break;
    }
    DSG_HIP(hipGetLastError());
    return;
  }
  hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(1), 0, s, w.demand, w.ndelta, w.err, m->d_epoch);
  if (!presorted) radix_sort_pairs(w.keys, w.idx, n, key_bits + (padded ? 1 : 0), w.radix, s, w.err, key_lo);
  unsigned nb = blocks_for(n, 256);
  hipLaunchKernelGGL(k_heads, dim3(nb), dim3(256), 0, s, w.keys, n, cbits, sentinel, w.kh, w.rh);
  exclusive_scan_i64_pair(w.kh, w.ukpos, w.nU, w.rh, w.urpos, w.nR, n, w.scan, s);
  int vsz = m->vsz;
  if (vsz == 8)
    hipLaunchKernelGGL(k_fold<8>, dim3(nb), dim3(256), 0, s, w.keys, w.idx, n, cbits, ops, vals, w.kh,
                       w.ukpos, w.rh, w.urpos, w.nU, w.nR, w.U);
  else if (vsz == 4)
    hipLaunchKernelGGL(k_fold<4>, dim3(nb), dim3(256), 0, s, w.keys, w.idx, n, cbits, ops, vals, w.kh,
                       w.ukpos, w.rh, w.urpos, w.nU, w.nR, w.U);
  else
    hipLaunchKernelGGL(k_fold<0>, dim3(nb), dim3(256), 0, s, w.keys, w.idx, n, cbits, ops, vals, w.kh,
                       w.ukpos, w.rh, w.urpos, w.nU, w.nR, w.U);
  switch (m->sr) {
    case 0: launch_plan_commit<0, 8>(m, w, n, cmask, cbits, vals, tbits, graph, G, phases, deltas_done); break;
    case 1: launch_plan_commit<1, 4>(m, w, n, cmask, cbits, vals, tbits, graph, G, phases, deltas_done); break;
    case 2: launch_plan_commit<2, 8>(m, w, n, cmask, cbits, vals, tbits, graph, G, phases, deltas_done); break;
    case 3: launch_plan_commit<3, 4>(m, w, n, cmask, cbits, vals, tbits, graph, G, phases, deltas_done); break;
    default: launch_plan_commit<-1, 0>(m, w, n, cmask, cbits, vals, tbits, graph, G, phases, deltas_done); break;
  }
  DSG_HIP(hipGetLastError());
}

// The transpose's deltas come in the order of the matrix's unique updates,
// by (row, column): for each column of the matrix -- a row of the transpose
// -- already by row.  Sorting them by the transpose's row bits alone (a
// stable sort) therefore gives their full order: the passes skip the low
// bits(t->ncols) bits.
int delta_key_lo(const DMat* t) { return bits_for(t->ncols); }

// Everything of mat_apply_device.  In a graph (no host round trips, on
// caller-owned workspaces, error flags left on the device) the matrix is
// planned and committed, then its transpose index.  Outside graphs both are
// planned first -- the transpose's deltas come from the matrix's plan -- and
// room is reserved for both before either is committed, so that a failed
// reservation (DSG_E_OOM) leaves both unchanged.
void apply_pipeline(DMat* m, const int32_t* d_rows, const int32_t* d_cols, const void* d_vals,
                    const uint8_t* d_ops, int64_t n, Work& w, Work* wt, bool graph, bool count_touched = false) {
  hipStream_t s = m->ctx->stream;
  int cbits = bits_for(m->ncols);
  int kbits = cbits + bits_for(m->nrows);
  unsigned nb = blocks_for(n, 256);
  hipLaunchKernelGGL(k_batch_keys, dim3(nb), dim3(256), 0, s, d_rows, d_cols, n, cbits, w.keys, w.idx);
  DMat* t = m->tidx;
  if (graph || !t) {
    run_core(m, w, n, kbits, false, d_ops, d_vals, graph);
    if (t) {
      int tk = bits_for(t->ncols) + bits_for(t->nrows);
      hipLaunchKernelGGL(k_delta_keys, dim3(nb), dim3(256), 0, s, w.dkey, (const uint8_t*)w.U.code,
                         (const int64_t*)w.nU, 1ull << tk, wt->keys, wt->idx, n);
      run_core(t, *wt, n, tk, true, w.dop, t->vsz ? w.dval : nullptr, graph, false, Guard(),
               PH_PLAN | PH_ROOM | PH_COMMIT, false, -1, delta_key_lo(t));
    }
    return;
  }
  run_core(m, w, n, kbits, false, d_ops, d_vals, false, false, Guard(), PH_PLAN);
  if (count_touched)
    hipLaunchKernelGGL(k_touched_len, dim3(nb), dim3(256), 0, s, (const int32_t*)w.U.urow, (const int64_t*)w.nR,
                       (const int32_t*)m->row_len, w.demand + 2);
  const int tbits = bits_for(m->nrows);
  const uint64_t cmask = (1ull << cbits) - 1;
  if (m->vsz == 8)
    hipLaunchKernelGGL(k_plan_deltas<8>, dim3(nb), dim3(256), 0, s, w.U, (const int64_t*)w.nU, cmask, cbits, tbits,
                       w.dkey, w.dop, w.dval);
  else if (m->vsz == 4)
    hipLaunchKernelGGL(k_plan_deltas<4>, dim3(nb), dim3(256), 0, s, w.U, (const int64_t*)w.nU, cmask, cbits, tbits,
                       w.dkey, w.dop, w.dval);
  else
    hipLaunchKernelGGL(k_plan_deltas<0>, dim3(nb), dim3(256), 0, s, w.U, (const int64_t*)w.nU, cmask, cbits, tbits,
                       w.dkey, w.dop, w.dval);
  int tk = bits_for(t->ncols) + bits_for(t->nrows);
  hipLaunchKernelGGL(k_delta_keys, dim3(nb), dim3(256), 0, s, w.dkey, (const uint8_t*)w.U.code,
                     (const int64_t*)w.nU, 1ull << tk, wt->keys, wt->idx, n);
  const void* tvals = t->vsz ? (const void*)w.dval : nullptr;
  run_core(t, *wt, n, tk, true, w.dop, tvals, false, false, Guard(), PH_PLAN, false, -1, delta_key_lo(t));
  if (count_touched)
    hipLaunchKernelGGL(k_touched_len, dim3(nb), dim3(256), 0, s, (const int32_t*)wt->U.urow, (const int64_t*)wt->nR,
                       (const int32_t*)t->row_len, wt->demand + 2);
  // one round trip for the room both plans need; then a compaction of either
  // pool re-plans that matrix alone (the transpose's deltas do not depend on
  // where the matrix's rows sit)
  int64_t* hd = (int64_t*)((char*)m->ctx->pinned + 512);
  DSG_HIP(hipMemcpyAsync(hd, w.demand, 8, hipMemcpyDeviceToHost, s));
  DSG_HIP(hipMemcpyAsync(hd + 1, wt->demand, 8, hipMemcpyDeviceToHost, s));
  DSG_HIP(hipStreamSynchronize(s));
  const int64_t dm = hd[0], dt = hd[1];
  run_core(m, w, n, kbits, false, d_ops, d_vals, false, false, Guard(), PH_ROOM, false, dm);
  run_core(t, *wt, n, tk, true, w.dop, tvals, false, false, Guard(), PH_ROOM, false, dt);
  run_core(m, w, n, kbits, false, d_ops, d_vals, false, false, Guard(), PH_COMMIT, true);
  run_core(t, *wt, n, tk, true, w.dop, tvals, false, false, Guard(), PH_COMMIT);
}

// Room for the log of an apply of n updates (taken before the apply changes
// anything, so that a failed allocation leaves the matrix as it was).
void reserve_log(DMat* m, int64_t n) {
  Ctx* c = m->ctx;
  if (m->log_cap < n) {
    m->log_seq = 0;  // the held log goes with its buffers
    ctx_free(c, m->log_key, (size_t)m->log_cap * 8);
    ctx_free(c, m->log_old, (size_t)m->log_cap * 8);
    ctx_free(c, m->log_new, (size_t)m->log_cap * 8);
    ctx_free(c, m->log_code, (size_t)m->log_cap);
    m->log_key = m->log_old = m->log_new = nullptr;
    m->log_code = nullptr;
    m->log_cap = 0;
    const int64_t cap = std::max<int64_t>(n + n / 2, 1024);
    m->log_key = (uint64_t*)ctx_alloc(c, (size_t)cap * 8);
    m->log_old = (uint64_t*)ctx_alloc(c, (size_t)cap * 8);
    m->log_new = (uint64_t*)ctx_alloc(c, (size_t)cap * 8);
    m->log_code = (uint8_t*)ctx_alloc(c, (size_t)cap);
    m->log_cap = cap;
  }
  if (!m->d_log_n) m->d_log_n = (int64_t*)ctx_alloc(c, 64);
}

// the log of an apply in one launch: its unique keys, values before and
// after and outcomes, and their count
__global__ void k_keep_log(const Uniq U, const int64_t* d_nU, uint64_t* key, uint64_t* old, uint64_t* nw,
                           uint8_t* code, int64_t* d_n) {
  const int64_t n = *d_nU;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t0 == 0) *d_n = n;
  for (int64_t u = t0; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    key[u] = U.key[u];
    old[u] = U.old[u];
    nw[u] = U.fin[u];
    code[u] = U.code[u];
  }
}

// Keep the unique keys of this apply with their values before and after and
// their outcomes: the entry-granular and general-update product paths read
// them.  reserve_log(m, n) must have run.
void keep_log(DMat* m, Work& w, int64_t n) {
  hipStream_t s = m->ctx->stream;
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks_for(n, 256), 4096));
  hipLaunchKernelGGL(k_keep_log, dim3(nb), dim3(256), 0, s, (const Uniq)w.U, (const int64_t*)w.nU, m->log_key,
                     m->log_old, m->log_new, m->log_code, m->d_log_n);
}

__global__ void k_lost_flags(const uint8_t* code, const int64_t* d_nU, int64_t n, uint8_t* flag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) flag[t] = (t < *d_nU && code[t] == C_LOST) ? 1 : 0;
}

__global__ void k_lost_gather(const int32_t* li, const int32_t* d_cnt, int64_t n, const uint64_t* key,
                              const int32_t* slot, uint64_t* lost_key, int32_t* lost_slot,
                              unsigned long long* d_nlost, const int64_t* d_nR, int64_t* d_nrows) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q == 0) {
    *d_nlost = (unsigned long long)*d_cnt;
    if (d_nrows) *d_nrows = *d_nR;
  }
  if (q < n && q < *d_cnt) {
    const int32_t u = li[q];
    lost_key[q] = key[u];
    lost_slot[q] = slot[u];
  }
}

// sorted unique keys keys[list[t]] as DELETE updates
__global__ void k_delete_keys(const uint64_t* keys, const int32_t* list, int64_t n, uint64_t* wkeys, uint32_t* idx,
                              uint8_t* ops) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) {
    wkeys[t] = keys[list ? list[t] : t];
    idx[t] = (uint32_t)t;
    ops[t] = DSG_OP_DELETE;
  }
}

__global__ void k_ops_from_flags(const uint8_t* flag, int64_t n, uint8_t* ops, const uint64_t* keys,
                                 uint64_t* wkeys, uint32_t* idx) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) {
    ops[t] = (flag[t] & 1) ? DSG_OP_ADD : OP_GUARD_ONLY;
    wkeys[t] = keys[t];
    idx[t] = (uint32_t)t;
  }
}

}  // namespace

size_t sorted_add_scratch_bytes(int64_t n) {
  const size_t N = (size_t)std::max<int64_t>(n, 1);
  return Carve::need({N, N * 4, compact_scratch_bytes(N), 64});
}

int64_t mat_apply_sorted_add(DMat* m, const uint64_t* keys, const void* vals, const uint64_t* guard,
                             const uint8_t* flag, int64_t n, uint64_t* lost_key, int32_t* lost_slot,
                             int64_t lost_cap, unsigned long long* d_nlost, int64_t* d_nrows, void* scratch) {
  DSG_REQUIRE(!m->tidx, DSG_E_STATE, "internal: sorted ADD apply on a matrix with a transpose");
  DSG_REQUIRE(lost_cap >= n, DSG_E_STATE, "internal: lost-entry list shorter than the updates");
  Ctx* c = m->ctx;
  hipStream_t s = c->stream;
  if (n == 0) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, d_nlost);
    if (d_nrows) hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, (unsigned long long*)d_nrows);
    return 0;
  }
  // (k_lost_gather sets *d_nlost and *d_nrows below)
  Work w = carve_work(ctx_scratch(c, work_bytes(n, false)), n, false);
  hipLaunchKernelGGL(k_ops_from_flags, dim3(blocks_for(n, 256)), dim3(256), 0, s, flag, n, w.allops, keys, w.keys,
                     w.idx);
  Guard G;
  G.key = guard;
  G.flag = flag;
  const int kbits = bits_for(m->ncols) + bits_for(m->nrows);
  run_core(m, w, n, kbits, false, w.allops, vals, false, true, G);
  // the lost entries, in key order: a compaction of the outcomes (no
  // contended counter)
  Carve cv(scratch, sorted_add_scratch_bytes(n));
  uint8_t* lf = cv.take<uint8_t>((size_t)n);
  int32_t* li = cv.take<int32_t>((size_t)n);
  void* cscr = cv.take<char>(compact_scratch_bytes(n));
  int32_t* d_cnt = cv.take<int32_t>(16);
  hipLaunchKernelGGL(k_lost_flags, dim3(blocks_for(n, 256)), dim3(256), 0, s, (const uint8_t*)w.U.code,
                     (const int64_t*)w.nU, n, lf);
  compact_flags(lf, n, li, d_cnt, cscr, s);
  hipLaunchKernelGGL(k_lost_gather, dim3(blocks_for(n, 256)), dim3(256), 0, s, (const int32_t*)li,
                     (const int32_t*)d_cnt, n, (const uint64_t*)w.U.key, (const int32_t*)w.U.slot, lost_key, lost_slot,
                     d_nlost, (const int64_t*)w.nR, d_nrows);
  unsigned long long* h = (unsigned long long*)c->pinned;
  int* he = (int*)((char*)c->pinned + 64);
  FetchList F;
  F.add(d_nlost, 8, 0);
  F.add(w.err, 4, 64);
  fetch_to_pinned(c, F, s);
  DSG_HIP(hipStreamSynchronize(s));
  DSG_REQUIRE(he[0] == 0, DSG_E_DEVICE, "internal: pool overflow while applying product updates");
  return (int64_t)h[0];
}

void mat_apply_sorted_delete(DMat* m, const uint64_t* keys, const int32_t* slots, const int32_t* list, int64_t n) {
  DSG_REQUIRE(!m->tidx, DSG_E_STATE, "internal: sorted delete on a matrix with a transpose");
  if (n == 0) return;
  Ctx* c = m->ctx;
  hipStream_t s = c->stream;
  Work w = carve_work(ctx_scratch(c, work_bytes(n, false)), n, false);
  hipLaunchKernelGGL(k_delete_keys, dim3(blocks_for(n, 256)), dim3(256), 0, s, keys, list, n, w.keys, w.idx,
                     w.allops);
  const int kbits = bits_for(m->ncols) + bits_for(m->nrows);
  Guard G;
  G.known_slot = slots;
  G.known_list = list;
  run_core(m, w, n, kbits, false, w.allops, nullptr, false, true, G);
  int* he = (int*)((char*)c->pinned + 64);
  DSG_HIP(hipMemcpyAsync(he, w.err, 4, hipMemcpyDeviceToHost, s));
  DSG_HIP(hipStreamSynchronize(s));
  DSG_REQUIRE(he[0] == 0, DSG_E_DEVICE, "internal: pool overflow while deleting product entries");
}

size_t apply_work_bytes(int64_t n, bool deltas) { return work_bytes(n, deltas); }

int* apply_err_ptr(void* work, int64_t n, bool deltas) { return carve_work(work, n, deltas).err; }

int64_t apply_headroom(const DMat* m, int64_t n) {
  // moved rows take at most slack_cap(len + inserts) each: <= 9/8 (nnz + n) + 4 per row
  return m->h_top_ub + m->h_top_ub / 8 + 6 * n + 64;
}

void mat_apply_graph(DMat* m, const int32_t* d_rows, const int32_t* d_cols, const void* d_vals,
                     const uint8_t* d_ops, int64_t n, void* work_main, void* work_tidx) {
  if (n == 0) return;
  Work w = carve_work(work_main, n, m->tidx != nullptr);
  Work wt;
  if (m->tidx) wt = carve_work(work_tidx, n, false);
  apply_pipeline(m, d_rows, d_cols, d_vals, d_ops, n, w, m->tidx ? &wt : nullptr, true);
}

void validate_batch_async(DMat* m, const int32_t* d_rows, const int32_t* d_cols, const uint8_t* d_ops, int64_t n,
                          int* d_flag) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_validate, dim3(blocks_for(n, 256)), dim3(256), 0, m->ctx->stream, d_rows, d_cols, d_ops, n,
                     m->nrows, m->ncols, d_flag);
}

dsg_status validate_batch_device(DMat* m, const int32_t* d_rows, const int32_t* d_cols, const uint8_t* d_ops,
                                 int64_t n) {
  if (n == 0) return DSG_OK;
  Ctx* c = m->ctx;
  if (validate_to_pinned(d_rows, d_cols, d_ops, n, m->nrows, m->ncols, c, 0)) {
    DSG_HIP(hipStreamSynchronize(c->stream));
    const int v = *(volatile int*)c->pinned;
    if (v & 1) return DSG_E_RANGE;
    if (v & 2) return DSG_E_ARG;
    return DSG_OK;
  }
  int* flags = (int*)ctx_scratch(c, 64);
  DSG_HIP(hipMemsetAsync(flags, 0, 4, c->stream));
  hipLaunchKernelGGL(k_validate, dim3(blocks_for(n, 256)), dim3(256), 0, c->stream, d_rows, d_cols, d_ops, n,
                     m->nrows, m->ncols, flags);
  int* h = (int*)c->pinned;
  DSG_HIP(hipMemcpyAsync(h, flags, 4, hipMemcpyDeviceToHost, c->stream));
  DSG_HIP(hipStreamSynchronize(c->stream));
  if (h[0] & 1) return DSG_E_RANGE;
  if (h[0] & 2) return DSG_E_ARG;
  return DSG_OK;
}

void mat_apply_device(DMat* m, const int32_t* d_rows, const int32_t* d_cols, const void* d_vals,
                      const uint8_t* d_ops, int64_t n) {
  if (n == 0) return;
  Ctx* c = m->ctx;
  hipStream_t s = c->stream;
  bool deltas = m->tidx != nullptr;
  Work w = carve_work(ctx_scratch(c, work_bytes(n, deltas)), n, deltas);
  Work wt;
  if (deltas) wt = carve_work(ctx_scratch2(c, work_bytes(n, false)), n, false);
  reserve_log(m, n);
  if (deltas) reserve_log(m->tidx, n);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool timed = c->timing && ctx_timing_begin(c, "apply", 0.0, &e0, &e1);
  const size_t tslot = c->timings.size() - (timed ? 1 : 0);
  // (timed: the entries of the touched rows, counted before the commits change them)
  unsigned long long* touched = (unsigned long long*)((char*)c->pinned + 256);
  if (timed) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, w.demand + 2);
    if (deltas) hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, wt.demand + 2);
  }
  apply_pipeline(m, d_rows, d_cols, d_vals, d_ops, n, w, deltas ? &wt : nullptr, false, timed);
  keep_log(m, w, n);
  // (and the transpose index's own: the same changes keyed by column, for a
  // product that uses the matrix transposed)
  if (deltas) keep_log(m->tidx, wt, n);
  if (c->timing) ctx_timing_end(c, e1);
  if (timed) {
    DSG_HIP(hipMemcpyAsync(touched, w.demand + 2, 8, hipMemcpyDeviceToHost, s));
    touched[1] = 0;
    if (deltas) DSG_HIP(hipMemcpyAsync(touched + 1, wt.demand + 2, 8, hipMemcpyDeviceToHost, s));
  }
  int* h = (int*)c->pinned;
  int64_t* hn = (int64_t*)((char*)c->pinned + 64);
  // a failed move (pool exhausted) would leave the batch half applied: report
  // it loudly; the log's length comes in the same wait
  FetchList F;
  F.add(w.err, 4, 0);
  F.add(deltas ? (const void*)wt.err : nullptr, 4, 4);
  F.add(w.nU, 8, 64);
  F.add(deltas ? (const void*)wt.nU : nullptr, 8, 72);
  fetch_to_pinned(c, F, s);
  DSG_HIP(hipStreamSynchronize(s));
  DSG_REQUIRE(h[0] == 0 && h[1] == 0, DSG_E_DEVICE, "internal: pool overflow while applying a batch");
  m->h_log_n = hn[0];
  if (deltas) m->tidx->h_log_n = hn[1];
  if (timed && tslot < c->timings.size()) {
    // algorithmic bytes: the batch read (row, column, value, op), the touched
    // rows streamed by the plan, the unique updates written; for the
    // transpose index its deltas, its touched rows and its writes
    const double v = (double)m->vsz, nu = (double)*hn;
    double bytes = (double)n * (9.0 + v) + (double)touched[0] * (4.0 + v) + nu * (4.0 + v);
    if (deltas) {
      const double vt = (double)m->tidx->vsz;
      bytes += nu * (9.0 + vt) + (double)touched[1] * (4.0 + vt) + nu * (4.0 + vt);
    }
    c->timings[tslot].bytes = bytes;
  }
  m->apply_seq++;
  m->log_seq = m->apply_seq;
  if (deltas) m->tidx->log_seq = m->apply_seq;  // (its own apply count is not kept: the matrix's stands for it)
}
