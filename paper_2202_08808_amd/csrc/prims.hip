// Device primitives: scans, flag compaction, stable LSD radix sort.
//
// Block-level scans use 64-wide wavefront shuffles plus one LDS slot per
// wave.  Radix sort ranks keys inside a tile with a wavefront multi-split
// (8 ballots build the set of lanes holding the same digit), which keeps the
// sort stable without per-digit loops.  The digit histograms of every pass
// are counted in one launch up front; each pass is then one launch whose
// tiles find the keys of their digit in the tiles before them by a
// decoupled look-back (each tile publishes its count, then its inclusive
// prefix, per digit, in one status word), so a sort of p passes takes p + 2
// launches instead of three per pass.
#include "internal.h"
#include "kernel_common.h"

namespace {

constexpr int SCAN_NT = 1024;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_NT * SCAN_ITEMS;

template <class T>
__device__ T block_exclusive_scan(T v, T* lds, T& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  T x = wave_inclusive_scan(v);
  if (lane == 63) lds[w] = x;
  __syncthreads();
  if (w == 0) {
    T s = lane < nw ? lds[lane] : T(0);
    s = wave_inclusive_scan(s);
    if (lane < nw) lds[lane] = s;
  }
  __syncthreads();
  T base = w > 0 ? lds[w - 1] : T(0);
  total = lds[nw - 1];
  __syncthreads();
  return base + x - v;
}

template <class In>
__global__ __launch_bounds__(SCAN_NT) void k_tile_sums(const In* in, int64_t n, int64_t* sums) {
  __shared__ int64_t lds[SCAN_NT / 64];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  int64_t s = 0;
  for (int t = 0; t < SCAN_ITEMS; ++t) {
    int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + t;
    if (i < n) s += (int64_t)in[i];
  }
  int64_t total;
  block_exclusive_scan<int64_t>(s, lds, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// single block: exclusive scan of sums[0..m) in place, grand total to *total
__global__ __launch_bounds__(SCAN_NT) void k_scan_sums(int64_t* sums, int64_t m, int64_t* total) {
  __shared__ int64_t lds[SCAN_NT / 64];
  int64_t carry = 0;
  for (int64_t base = 0; base < m; base += SCAN_NT) {
    int64_t i = base + threadIdx.x;
    int64_t v = i < m ? sums[i] : 0;
    int64_t t;
    int64_t ex = block_exclusive_scan<int64_t>(v, lds, t);
    if (i < m) sums[i] = carry + ex;
    carry += t;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

template <class In>
__global__ __launch_bounds__(SCAN_NT) void k_scan_apply(const In* in, int64_t* out, int64_t n,
                                                        const int64_t* sums) {
  __shared__ int64_t lds[SCAN_NT / 64];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  int64_t v[SCAN_ITEMS];
  int64_t s = 0;
  for (int t = 0; t < SCAN_ITEMS; ++t) {
    int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + t;
    v[t] = i < n ? (int64_t)in[i] : 0;
    s += v[t];
  }
  int64_t total;
  int64_t run = sums[blockIdx.x] + block_exclusive_scan<int64_t>(s, lds, total);
  for (int t = 0; t < SCAN_ITEMS; ++t) {
    int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + t;
    if (i < n) out[i] = run;
    run += v[t];
  }
}

// one tile: the whole exclusive scan (and its total) in a single launch
template <class In>
__global__ __launch_bounds__(SCAN_NT) void k_scan_single(const In* in, int64_t* out, int64_t n, int64_t* total) {
  __shared__ int64_t lds[SCAN_NT / 64];
  int64_t v[SCAN_ITEMS];
  int64_t s = 0;
  for (int t = 0; t < SCAN_ITEMS; ++t) {
    const int64_t i = (int64_t)threadIdx.x * SCAN_ITEMS + t;
    v[t] = i < n ? (int64_t)in[i] : 0;
    s += v[t];
  }
  int64_t tot;
  int64_t run = block_exclusive_scan<int64_t>(s, lds, tot);
  for (int t = 0; t < SCAN_ITEMS; ++t) {
    const int64_t i = (int64_t)threadIdx.x * SCAN_ITEMS + t;
    if (i < n) out[i] = run;
    run += v[t];
  }
  if (threadIdx.x == 0 && total) *total = tot;
}

// up to SCAN_WG_MAX entries: one workgroup walks the tiles in order,
// carrying the running sum (one launch instead of three)
constexpr int64_t SCAN_WG_MAX = 4 * SCAN_TILE;

template <class In>
__global__ __launch_bounds__(SCAN_NT) void k_scan_wg(const In* in, int64_t* out, int64_t n, int64_t* total) {
  __shared__ int64_t lds[SCAN_NT / 64];
  int64_t carry = 0;
  for (int64_t base = 0; base < n; base += SCAN_TILE) {
    int64_t v[SCAN_ITEMS];
    int64_t s = 0;
    for (int t = 0; t < SCAN_ITEMS; ++t) {
      const int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + t;
      v[t] = i < n ? (int64_t)in[i] : 0;
      s += v[t];
    }
    int64_t tot;
    int64_t run = carry + block_exclusive_scan<int64_t>(s, lds, tot);
    for (int t = 0; t < SCAN_ITEMS; ++t) {
      const int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + t;
      if (i < n) out[i] = run;
      run += v[t];
    }
    carry += tot;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

// two scans of the same length, one per workgroup, in one launch
__global__ __launch_bounds__(SCAN_NT) void k_scan_wg_pair(const int64_t* in0, int64_t* out0, int64_t* tot0,
                                                          const int64_t* in1, int64_t* out1, int64_t* tot1,
                                                          int64_t n) {
  __shared__ int64_t lds[SCAN_NT / 64];
  const int64_t* in = blockIdx.x ? in1 : in0;
  int64_t* out = blockIdx.x ? out1 : out0;
  int64_t carry = 0;
  for (int64_t base = 0; base < n; base += SCAN_TILE) {
    int64_t v[SCAN_ITEMS];
    int64_t s = 0;
    for (int t = 0; t < SCAN_ITEMS; ++t) {
      const int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + t;
      v[t] = i < n ? in[i] : 0;
      s += v[t];
    }
    int64_t tot;
    int64_t run = carry + block_exclusive_scan<int64_t>(s, lds, tot);
    for (int t = 0; t < SCAN_ITEMS; ++t) {
      const int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + t;
      if (i < n) out[i] = run;
      run += v[t];
    }
    carry += tot;
  }
  int64_t* total = blockIdx.x ? tot1 : tot0;
  if (threadIdx.x == 0 && total) *total = carry;
}

template <class In>
void scan_impl(const In* in, int64_t* out, int64_t n, int64_t* d_total, void* scratch, hipStream_t s) {
  if (n <= SCAN_TILE) {
    hipLaunchKernelGGL(k_scan_single<In>, dim3(1), dim3(SCAN_NT), 0, s, in, out, n, d_total);
    return;
  }
  if (n <= SCAN_WG_MAX) {
    hipLaunchKernelGGL(k_scan_wg<In>, dim3(1), dim3(SCAN_NT), 0, s, in, out, n, d_total);
    return;
  }
  int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (tiles == 0) tiles = 1;
  int64_t* sums = (int64_t*)scratch;
  hipLaunchKernelGGL(k_tile_sums<In>, dim3((unsigned)tiles), dim3(SCAN_NT), 0, s, in, n, sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_NT), 0, s, sums, tiles, d_total);
  hipLaunchKernelGGL(k_scan_apply<In>, dim3((unsigned)tiles), dim3(SCAN_NT), 0, s, in, out, n, sums);
}

// ---- flag compaction ----

__global__ __launch_bounds__(SCAN_NT) void k_flag_counts(const uint8_t* flags, int64_t n, int64_t* sums,
                                                         const int32_t* d_n) {
  __shared__ int64_t lds[SCAN_NT / 64];
  if (d_n) n = *d_n;
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  int64_t c = 0;
  for (int t = 0; t < SCAN_ITEMS; ++t) {
    int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + t;
    if (i < n && flags[i]) ++c;
  }
  int64_t total;
  block_exclusive_scan<int64_t>(c, lds, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(SCAN_NT) void k_flag_write(const uint8_t* flags, const int32_t* list,
                                                        int64_t n, const int64_t* sums, int32_t* out,
                                                        const int32_t* d_n) {
  __shared__ int64_t lds[SCAN_NT / 64];
  if (d_n) n = *d_n;
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  uint8_t f[SCAN_ITEMS];
  int64_t c = 0;
  for (int t = 0; t < SCAN_ITEMS; ++t) {
    int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + t;
    f[t] = (i < n && flags[i]) ? 1 : 0;
    c += f[t];
  }
  int64_t total;
  int64_t pos = sums[blockIdx.x] + block_exclusive_scan<int64_t>(c, lds, total);
  for (int t = 0; t < SCAN_ITEMS; ++t) {
    int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + t;
    if (f[t]) out[pos++] = list ? list[i] : (int32_t)i;
  }
}

__global__ void k_store_count(const int64_t* total, int32_t* d_count) { *d_count = (int32_t)*total; }

// up to SCAN_WG_MAX flags: the whole compaction in one workgroup (one
// launch instead of four)
__global__ __launch_bounds__(SCAN_NT) void k_compact_wg(const uint8_t* flags, const int32_t* list, int64_t n,
                                                        int32_t* out, const int32_t* d_n, int32_t* d_count) {
  __shared__ int64_t lds[SCAN_NT / 64];
  if (d_n) n = *d_n;
  int64_t carry = 0;
  for (int64_t base = 0; base < n; base += SCAN_TILE) {
    uint8_t f[SCAN_ITEMS];
    int64_t c = 0;
    for (int t = 0; t < SCAN_ITEMS; ++t) {
      const int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + t;
      f[t] = (i < n && flags[i]) ? 1 : 0;
      c += f[t];
    }
    int64_t tot;
    int64_t pos = carry + block_exclusive_scan<int64_t>(c, lds, tot);
    for (int t = 0; t < SCAN_ITEMS; ++t) {
      const int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + t;
      if (f[t]) out[pos++] = list ? list[i] : (int32_t)i;
    }
    carry += tot;
  }
  if (threadIdx.x == 0) *d_count = (int32_t)carry;
}

// ---- radix sort ----

constexpr int RS_NT = 256;
constexpr int RS_WAVES = RS_NT / 64;
constexpr int RS_ITEMS = 8;
constexpr int RS_TILE = RS_NT * RS_ITEMS;

__global__ __launch_bounds__(RS_NT) void k_rs_hist(const uint64_t* keys, int64_t n, int shift,
                                                    int64_t* counts, int64_t ntiles) {
  __shared__ int32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int t = 0; t < RS_ITEMS; ++t) {
    int64_t i = base + t * RS_NT + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255], 1);
  }
  __syncthreads();
  counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(RS_NT) void k_rs_scatter(const uint64_t* kin, const uint32_t* vin,
                                                       uint64_t* kout, uint32_t* vout, int64_t n,
                                                       int shift, const int64_t* offs, int64_t ntiles) {
  __shared__ int32_t wcount[RS_WAVES][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int d = threadIdx.x; d < RS_WAVES * 256; d += RS_NT) (&wcount[0][0])[d] = 0;
  __syncthreads();
  const int64_t seg = (int64_t)blockIdx.x * RS_TILE + (int64_t)w * (64 * RS_ITEMS);
  uint64_t k[RS_ITEMS];
  uint32_t v[RS_ITEMS];
  int32_t rank[RS_ITEMS];
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < RS_ITEMS; ++r) {
    int64_t i = seg + r * 64 + lane;
    bool act = i < n;
    k[r] = act ? kin[i] : 0;
    v[r] = act ? vin[i] : 0;
    uint32_t d = (uint32_t)(k[r] >> shift) & 255u;
    uint64_t peers = __ballot(act);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      bool bit = (d >> b) & 1u;
      uint64_t m = __ballot(act && bit);
      peers &= bit ? m : ~m;
    }
    int before = __popcll(peers & lt);
    int32_t base = act ? wcount[w][d] : 0;
    __builtin_amdgcn_wave_barrier();
    if (act && before == 0) wcount[w][d] = base + __popcll(peers);
    __builtin_amdgcn_wave_barrier();
    rank[r] = base + before;
  }
  __syncthreads();
  {
    int d = threadIdx.x;  // RS_NT == 256 digits
    int32_t run = 0;
    for (int ww = 0; ww < RS_WAVES; ++ww) {
      int32_t c = wcount[ww][d];
      wcount[ww][d] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int r = 0; r < RS_ITEMS; ++r) {
    int64_t i = seg + r * 64 + lane;
    if (i < n) {
      uint32_t d = (uint32_t)(k[r] >> shift) & 255u;
      int64_t pos = offs[(int64_t)d * ntiles + blockIdx.x] + wcount[w][d] + rank[r];
      kout[pos] = k[r];
      vout[pos] = v[r];
    }
  }
}

// ---- single-sweep passes ----
// Status word of (tile, digit): 0 while unknown, LB_AGG | the tile's own count
// of the digit, then LB_PRE | the count over this tile and all before it.
constexpr uint32_t LB_AGG = 1u << 30, LB_PRE = 2u << 30, LB_CNT = LB_AGG - 1;
constexpr int RS_MAX_PASSES = 8;
constexpr int64_t RS_SWEEP_MAX = (int64_t)LB_CNT;  // counts fit the status word's 30 bits
// polls of a predecessor's status before the sort gives up (tiles start in
// ticket order, so a predecessor is running and publishes within microseconds)
constexpr uint32_t RS_SPIN_MAX = 1u << 24;

__global__ void k_rs_zero(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// digit histograms of every pass (pass p: bits lo + 8p and up), summed over
// the whole input into g[pass][256]
__global__ __launch_bounds__(RS_NT) void k_rs_hist_all(const uint64_t* keys, int64_t n, int lo, int passes,
                                                       uint32_t* g) {
  __shared__ uint32_t h[RS_MAX_PASSES][256];
  for (int p = 0; p < passes; ++p) h[p][threadIdx.x] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int t = 0; t < RS_ITEMS; ++t) {
    const int64_t i = base + t * RS_NT + threadIdx.x;
    if (i < n) {
      const uint64_t k = keys[i];
      for (int p = 0; p < passes; ++p) atomicAdd(&h[p][(k >> (lo + 8 * p)) & 255], 1u);
    }
  }
  __syncthreads();
  for (int p = 0; p < passes; ++p)
    if (h[p][threadIdx.x]) atomicAdd(&g[p * 256 + threadIdx.x], h[p][threadIdx.x]);
}

// One pass: tile t (taken from a ticket, so tiles start in input order)
// ranks its keys by digit, publishes its per-digit counts, adds those of the
// tiles before it, and scatters.  It also clears the status words of the
// pass before it (`clr`, n_clr words) for the pass after it.
__global__ __launch_bounds__(RS_NT) void k_rs_sweep(const uint64_t* kin, const uint32_t* vin, uint64_t* kout,
                                                     uint32_t* vout, int64_t n, int shift, const uint32_t* ghist,
                                                     uint32_t* ticket, uint32_t* st, uint32_t* clr, int64_t n_clr,
                                                     int64_t ntiles, int* err) {
  __shared__ int32_t wcount[RS_WAVES][256];
  __shared__ uint32_t base_of[256];
  __shared__ uint32_t lds_scan[RS_WAVES];
  __shared__ uint32_t tile_s;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int d0 = threadIdx.x;  // RS_NT == 256 digits
  if (threadIdx.x == 0) tile_s = atomicAdd(ticket, 1u);
  for (int d = threadIdx.x; d < RS_WAVES * 256; d += RS_NT) (&wcount[0][0])[d] = 0;
  __syncthreads();
  const int64_t t = tile_s;
  for (int64_t x = t * RS_NT + threadIdx.x; x < n_clr; x += ntiles * RS_NT) clr[x] = 0u;
  const int64_t seg = t * RS_TILE + (int64_t)w * (64 * RS_ITEMS);
  uint64_t k[RS_ITEMS];
  uint32_t v[RS_ITEMS];
  int32_t rank[RS_ITEMS];
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < RS_ITEMS; ++r) {
    const int64_t i = seg + r * 64 + lane;
    const bool act = i < n;
    k[r] = act ? kin[i] : 0;
    v[r] = act ? vin[i] : 0;
    const uint32_t d = (uint32_t)(k[r] >> shift) & 255u;
    uint64_t peers = __ballot(act);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(act && bit);
      peers &= bit ? m : ~m;
    }
    const int before = __popcll(peers & lt);
    const int32_t base = act ? wcount[w][d] : 0;
    __builtin_amdgcn_wave_barrier();
    if (act && before == 0) wcount[w][d] = base + __popcll(peers);
    __builtin_amdgcn_wave_barrier();
    rank[r] = base + before;
  }
  __syncthreads();
  // this tile's count of digit d0, and the waves' offsets inside the tile
  uint32_t mine = 0;
  for (int ww = 0; ww < RS_WAVES; ++ww) {
    const int32_t c = wcount[ww][d0];
    wcount[ww][d0] = (int32_t)mine;
    mine += (uint32_t)c;
  }
  // keys of digit d0 in the tiles before this one (decoupled look-back)
  uint32_t* my = st + t * 256 + d0;
  uint32_t excl = 0;
  if (t == 0) {
    __hip_atomic_store(my, LB_PRE | mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    __hip_atomic_store(my, LB_AGG | mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int64_t j = t - 1; j >= 0; --j) {
      const uint32_t* q = st + j * 256 + d0;
      uint32_t sv = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      uint32_t spins = 0;
      while (sv == 0u && ++spins < RS_SPIN_MAX) {
        __builtin_amdgcn_s_sleep(1);
        sv = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (sv == 0u) {  // never published: report it, and end the walk
        if (err) atomicOr(err, 16);
        break;
      }
      excl += sv & LB_CNT;
      if (sv & LB_PRE) break;
    }
    __hip_atomic_store(my, LB_PRE | (excl + mine), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // first output position of digit d0 over the whole input
  const uint32_t gc = ghist[d0];
  uint32_t x = gc;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds_scan[w] = x;
  __syncthreads();
  uint32_t wbase = 0;
  for (int ww = 0; ww < w; ++ww) wbase += lds_scan[ww];
  base_of[d0] = wbase + x - gc + excl;
  __syncthreads();
  for (int r = 0; r < RS_ITEMS; ++r) {
    const int64_t i = seg + r * 64 + lane;
    if (i < n) {
      const uint32_t d = (uint32_t)(k[r] >> shift) & 255u;
      const int64_t pos = (int64_t)base_of[d] + wcount[w][d] + rank[r];
      kout[pos] = k[r];
      vout[pos] = v[r];
    }
  }
}

__global__ void k_copy_pairs(const uint64_t* ks, const uint32_t* vs, uint64_t* kd, uint32_t* vd, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    kd[i] = ks[i];
    vd[i] = vs[i];
  }
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_iota_i32(int32_t* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

}  // namespace

size_t scan_scratch_bytes(int64_t n) {
  int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE + 1;
  return (size_t)tiles * sizeof(int64_t) + 256;
}

void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* d_total, void* scratch,
                        hipStream_t s) {
  scan_impl<int64_t>(in, out, n, d_total, scratch, s);
}

void exclusive_scan_i64_pair(const int64_t* in0, int64_t* out0, int64_t* tot0, const int64_t* in1, int64_t* out1,
                             int64_t* tot1, int64_t n, void* scratch, hipStream_t s) {
  if (n <= SCAN_WG_MAX) {
    hipLaunchKernelGGL(k_scan_wg_pair, dim3(2), dim3(SCAN_NT), 0, s, in0, out0, tot0, in1, out1, tot1, n);
    return;
  }
  scan_impl<int64_t>(in0, out0, n, tot0, scratch, s);
  scan_impl<int64_t>(in1, out1, n, tot1, scratch, s);
}

__global__ void k_fetch(FetchList F, char* dst) {
  const int i = threadIdx.x;
  if (i >= F.n) return;
  uint32_t* d = (uint32_t*)(dst + F.off[i]);
  const uint32_t* p = (const uint32_t*)F.src[i];
  for (int w = 0; w < F.bytes[i] / 4; ++w) d[w] = p ? p[w] : 0u;
}

void fetch_to_pinned(Ctx* c, const FetchList& F, hipStream_t s) {
  if (F.n == 0) return;
  hipLaunchKernelGGL(k_fetch, dim3(1), dim3(64), 0, s, F, (char*)c->pinned_dev);
}

constexpr int64_t VALIDATE_ONE_MAX = 1 << 16;

// one workgroup checks the whole batch and writes the result itself
__global__ __launch_bounds__(1024) void k_validate_one(const int32_t* rows, const int32_t* cols, const uint8_t* ops,
                                                       int64_t n, int32_t nrows, int32_t ncols, int* out) {
  __shared__ int bits;
  if (threadIdx.x == 0) bits = 0;
  __syncthreads();
  int b = 0;
  for (int64_t t = threadIdx.x; t < n; t += 1024) {
    if (rows[t] < 0 || rows[t] >= nrows || cols[t] < 0 || cols[t] >= ncols) b |= 1;
    if (ops[t] > DSG_OP_ADD) b |= 2;
  }
  if (b) atomicOr(&bits, b);
  __syncthreads();
  if (threadIdx.x == 0) *out = bits;
}

bool validate_to_pinned(const int32_t* rows, const int32_t* cols, const uint8_t* ops, int64_t n, int32_t nrows,
                        int32_t ncols, Ctx* c, int32_t off) {
  if (n > VALIDATE_ONE_MAX) return false;
  hipLaunchKernelGGL(k_validate_one, dim3(1), dim3(1024), 0, c->stream, rows, cols, ops, n, nrows, ncols,
                     (int*)((char*)c->pinned_dev + off));
  return true;
}

void exclusive_scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, int64_t* d_total,
                               void* scratch, hipStream_t s) {
  scan_impl<int32_t>(in, out, n, d_total, scratch, s);
}

size_t compact_scratch_bytes(int64_t n) { return scan_scratch_bytes(n) + 256; }

// ---- three-class compaction ----
// A position's class as packed counts: class 0 in the low 32 bits, class 1
// in the high 32; class 2's count before a position is the position minus
// the other two.

__device__ inline int64_t cls_pack(uint8_t c) { return c == 0 ? 1ll : c == 1 ? (1ll << 32) : 0ll; }

__device__ inline void cls_place(uint8_t c, int64_t i, int64_t pre, int32_t* o0, int32_t* o1, int32_t* o2) {
  const int64_t p0 = pre & 0xffffffffll, p1 = (int64_t)((uint64_t)pre >> 32);
  if (c == 0) o0[p0] = (int32_t)i;
  else if (c == 1) o1[p1] = (int32_t)i;
  else o2[i - p0 - p1] = (int32_t)i;
}

__global__ __launch_bounds__(SCAN_NT) void k_cls_counts(const uint8_t* cls, int64_t n, int64_t* sums) {
  __shared__ int64_t lds[SCAN_NT / 64];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  int64_t c = 0;
  for (int t = 0; t < SCAN_ITEMS; ++t) {
    const int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + t;
    if (i < n) c += cls_pack(cls[i]);
  }
  int64_t total;
  block_exclusive_scan<int64_t>(c, lds, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(SCAN_NT) void k_cls_write(const uint8_t* cls, int64_t n, const int64_t* sums,
                                                       int32_t* o0, int32_t* o1, int32_t* o2) {
  __shared__ int64_t lds[SCAN_NT / 64];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  uint8_t f[SCAN_ITEMS];
  int64_t c = 0;
  for (int t = 0; t < SCAN_ITEMS; ++t) {
    const int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + t;
    f[t] = i < n ? cls[i] : 3;
    if (i < n) c += cls_pack(f[t]);
  }
  int64_t total;
  int64_t pre = sums[blockIdx.x] + block_exclusive_scan<int64_t>(c, lds, total);
  for (int t = 0; t < SCAN_ITEMS; ++t) {
    const int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + t;
    if (i < n) {
      cls_place(f[t], i, pre, o0, o1, o2);
      pre += cls_pack(f[t]);
    }
  }
}

__global__ void k_cls_store(const int64_t* total, int64_t n, int32_t* d_count) {
  const int64_t t = *total;
  const int64_t c0 = t & 0xffffffffll, c1 = (int64_t)((uint64_t)t >> 32);
  d_count[0] = (int32_t)c0;
  d_count[1] = (int32_t)c1;
  d_count[2] = (int32_t)(n - c0 - c1);
}

// up to SCAN_WG_MAX entries in one workgroup
__global__ __launch_bounds__(SCAN_NT) void k_cls_wg(const uint8_t* cls, int64_t n, int32_t* o0, int32_t* o1,
                                                    int32_t* o2, int32_t* d_count) {
  __shared__ int64_t lds[SCAN_NT / 64];
  int64_t carry = 0;
  for (int64_t base = 0; base < n; base += SCAN_TILE) {
    uint8_t f[SCAN_ITEMS];
    int64_t c = 0;
    for (int t = 0; t < SCAN_ITEMS; ++t) {
      const int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + t;
      f[t] = i < n ? cls[i] : 3;
      if (i < n) c += cls_pack(f[t]);
    }
    int64_t tot;
    int64_t pre = carry + block_exclusive_scan<int64_t>(c, lds, tot);
    for (int t = 0; t < SCAN_ITEMS; ++t) {
      const int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + t;
      if (i < n) {
        cls_place(f[t], i, pre, o0, o1, o2);
        pre += cls_pack(f[t]);
      }
    }
    carry += tot;
  }
  if (threadIdx.x == 0) {
    const int64_t c0 = carry & 0xffffffffll, c1 = (int64_t)((uint64_t)carry >> 32);
    d_count[0] = (int32_t)c0;
    d_count[1] = (int32_t)c1;
    d_count[2] = (int32_t)(n - c0 - c1);
  }
}

void compact_flags(const uint8_t* flags, int64_t n, int32_t* out, int32_t* d_count, void* scratch,
                   hipStream_t s) {
  if (n <= SCAN_WG_MAX) {
    hipLaunchKernelGGL(k_compact_wg, dim3(1), dim3(SCAN_NT), 0, s, flags, (const int32_t*)nullptr, n, out,
                       (const int32_t*)nullptr, d_count);
    return;
  }
  int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (tiles == 0) tiles = 1;
  int64_t* sums = (int64_t*)scratch;
  int64_t* total = sums + tiles + 1;
  hipLaunchKernelGGL(k_flag_counts, dim3((unsigned)tiles), dim3(SCAN_NT), 0, s, flags, n, sums,
                     (const int32_t*)nullptr);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_NT), 0, s, sums, tiles, total);
  hipLaunchKernelGGL(k_flag_write, dim3((unsigned)tiles), dim3(SCAN_NT), 0, s, flags,
                     (const int32_t*)nullptr, n, sums, out, (const int32_t*)nullptr);
  hipLaunchKernelGGL(k_store_count, dim3(1), dim3(1), 0, s, total, d_count);
}

void compact_classes3(const uint8_t* cls, int64_t n, int32_t* out0, int32_t* out1, int32_t* out2, int32_t* d_count,
                      void* scratch, hipStream_t s) {
  if (n <= SCAN_WG_MAX) {
    hipLaunchKernelGGL(k_cls_wg, dim3(1), dim3(SCAN_NT), 0, s, cls, n, out0, out1, out2, d_count);
    return;
  }
  const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  int64_t* sums = (int64_t*)scratch;
  int64_t* total = sums + tiles + 1;
  hipLaunchKernelGGL(k_cls_counts, dim3((unsigned)tiles), dim3(SCAN_NT), 0, s, cls, n, sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_NT), 0, s, sums, tiles, total);
  hipLaunchKernelGGL(k_cls_write, dim3((unsigned)tiles), dim3(SCAN_NT), 0, s, cls, n, (const int64_t*)sums, out0,
                     out1, out2);
  hipLaunchKernelGGL(k_cls_store, dim3(1), dim3(1), 0, s, (const int64_t*)total, n, d_count);
}

void compact_list_by_flags(const int32_t* list, const uint8_t* flags, const int32_t* d_n, int64_t n_max,
                           int32_t* out, int32_t* d_count, void* scratch, hipStream_t s) {
  if (n_max <= SCAN_WG_MAX) {
    hipLaunchKernelGGL(k_compact_wg, dim3(1), dim3(SCAN_NT), 0, s, flags, list, n_max, out, d_n, d_count);
    return;
  }
  int64_t tiles = (n_max + SCAN_TILE - 1) / SCAN_TILE;
  if (tiles == 0) tiles = 1;
  int64_t* sums = (int64_t*)scratch;
  int64_t* total = sums + tiles + 1;
  hipLaunchKernelGGL(k_flag_counts, dim3((unsigned)tiles), dim3(SCAN_NT), 0, s, flags, n_max, sums, d_n);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_NT), 0, s, sums, tiles, total);
  hipLaunchKernelGGL(k_flag_write, dim3((unsigned)tiles), dim3(SCAN_NT), 0, s, flags, list, n_max, sums,
                     out, d_n);
  hipLaunchKernelGGL(k_store_count, dim3(1), dim3(1), 0, s, total, d_count);
}

namespace {

// Bitonic sort of up to SMALL_SORT (key, value) pairs in LDS by (key, value),
// padded with (max, max).
constexpr int SMALL_SORT = 4096;

__global__ __launch_bounds__(1024) void k_small_sort(uint64_t* keys, uint32_t* vals, int n) {
  __shared__ uint64_t sk[SMALL_SORT];
  __shared__ uint32_t sv[SMALL_SORT];
  int m = 1;
  while (m < n) m <<= 1;
  for (int i = threadIdx.x; i < m; i += 1024) {
    sk[i] = i < n ? keys[i] : ~0ull;
    sv[i] = i < n ? vals[i] : ~0u;
  }
  __syncthreads();
  for (int k = 2; k <= m; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < m; i += 1024) {
        const int p = i ^ j;
        if (p > i) {
          const bool up = (i & k) == 0;
          const uint64_t a = sk[i], b = sk[p];
          const uint32_t va = sv[i], vb = sv[p];
          const bool gt = a > b || (a == b && va > vb);
          if (gt == up) {
            sk[i] = b;
            sk[p] = a;
            sv[i] = vb;
            sv[p] = va;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < n; i += 1024) {
    keys[i] = sk[i];
    vals[i] = sv[i];
  }
}

// Bitonic sort of up to MID_SORT keys of at most MID_KEY_BITS bits in one
// workgroup: each key is packed with its input position into one 64-bit word,
// so the words sort by (key, position), which is exactly the stable order,
// and the values follow through their positions.  64 KB of LDS holds the
// words and then the values.  Each of the log2(m)(log2(m)+1)/2 stages moves
// 32 bytes of LDS per pair, so beyond 8192 keys the multi-pass radix sort is
// faster (16384 keys: ~90 us here against ~65 us).
constexpr int MID_SORT = 8192;
constexpr int MID_POS_BITS = 13;
constexpr int MID_KEY_BITS = 64 - MID_POS_BITS;
constexpr int MID_NT = 1024;
constexpr int MID_PER = MID_SORT / MID_NT;
static_assert((1 << MID_POS_BITS) == MID_SORT, "positions fill the low bits");

__global__ __launch_bounds__(MID_NT) void k_mid_sort(uint64_t* keys, uint32_t* vals, int n) {
  __shared__ uint64_t sw[MID_SORT];
  int m = 1;
  while (m < n) m <<= 1;
  for (int i = threadIdx.x; i < m; i += MID_NT)
    sw[i] = i < n ? ((keys[i] << MID_POS_BITS) | (uint64_t)i) : ~0ull;  // padding sorts last
  __syncthreads();
  const int half = m >> 1;
  for (int k = 2; k <= m; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      // pair q: i has a 0 at bit log2(j), its partner i + j a 1
      for (int q = threadIdx.x; q < half; q += MID_NT) {
        const int i = ((q & ~(j - 1)) << 1) | (q & (j - 1));
        const int p = i | j;
        const uint64_t a = sw[i], b = sw[p];
        if ((a > b) == ((i & k) == 0)) {
          sw[i] = b;
          sw[p] = a;
        }
      }
      __syncthreads();
    }
  }
  uint32_t pos[MID_PER];
#pragma unroll
  for (int r = 0; r < MID_PER; ++r) {
    const int j = threadIdx.x + r * MID_NT;
    pos[r] = 0;
    if (j < n) {
      const uint64_t w = sw[j];
      pos[r] = (uint32_t)(w & (MID_SORT - 1));
      keys[j] = w >> MID_POS_BITS;
    }
  }
  __syncthreads();
  uint32_t* sv = (uint32_t*)sw;
  for (int i = threadIdx.x; i < n; i += MID_NT) sv[i] = vals[i];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < MID_PER; ++r) {
    const int j = threadIdx.x + r * MID_NT;
    if (j < n) vals[j] = sv[pos[r]];
  }
}

}  // namespace

size_t radix_scratch_bytes(int64_t n) {
  int64_t ntiles = (n + RS_TILE - 1) / RS_TILE + 1;
  // ping-pong pairs; the multi-launch passes' tile counts and their scan, or
  // the single-sweep histograms, tickets and two status regions
  return Carve::need({(size_t)n * 8, (size_t)n * 4,
                      std::max((size_t)(256 * ntiles) * 8 + scan_scratch_bytes(256 * ntiles) + 256,
                               (size_t)(RS_MAX_PASSES * 256 + 64 + 2 * 256 * ntiles) * 4 + 256)});
}

void radix_sort_pairs(uint64_t* keys, uint32_t* vals, int64_t n, int key_bits, void* scratch,
                      hipStream_t s, int* err, int key_lo) {
  if (n <= 1 || key_bits <= 0) return;
  if (n <= MID_SORT && key_bits <= MID_KEY_BITS) {
    hipLaunchKernelGGL(k_mid_sort, dim3(1), dim3(MID_NT), 0, s, keys, vals, (int)n);
    return;
  }
  if (n <= SMALL_SORT) {
    // one workgroup: the same order as the stable radix sort when equal keys
    // carry ascending values (their original positions)
    hipLaunchKernelGGL(k_small_sort, dim3(1), dim3(1024), 0, s, keys, vals, (int)n);
    return;
  }
  int64_t ntiles = (n + RS_TILE - 1) / RS_TILE;
  Carve cv(scratch, radix_scratch_bytes(n));
  uint64_t* k2 = cv.take<uint64_t>(n);
  uint32_t* v2 = cv.take<uint32_t>(n);
  uint64_t* ka = keys;
  uint32_t* va = vals;
  uint64_t* kb = k2;
  uint32_t* vb = v2;
  // (bits below key_lo already ordered: the passes start there)
  if (key_lo < 0 || key_lo >= key_bits) key_lo = 0;
  int passes = (key_bits - key_lo + 7) / 8;
  if (n <= RS_SWEEP_MAX && passes <= RS_MAX_PASSES) {
    uint32_t* ghist = cv.take<uint32_t>(RS_MAX_PASSES * 256);
    uint32_t* tickets = cv.take<uint32_t>(64);
    uint32_t* st[2] = {cv.take<uint32_t>(256 * ntiles), cv.take<uint32_t>(256 * ntiles)};
    // the four takes are whole multiples of 256 bytes, so they lie end to end
    const int64_t nz = (int64_t)(RS_MAX_PASSES * 256 + 64) + 2 * 256 * ntiles;
    DSG_REQUIRE((char*)(st[1] + 256 * ntiles) == (char*)(ghist + nz), DSG_E_DEVICE, "internal: sort scratch layout");
    hipLaunchKernelGGL(k_rs_zero, dim3((unsigned)std::min<int64_t>((nz + 255) / 256, 1024)), dim3(256), 0, s,
                       ghist, nz);
    hipLaunchKernelGGL(k_rs_hist_all, dim3((unsigned)ntiles), dim3(RS_NT), 0, s, ka, n, key_lo, passes, ghist);
    for (int p = 0; p < passes; ++p) {
      // pass p uses region p % 2 and clears the other one, which pass p - 1
      // used, for pass p + 1 (both start cleared)
      uint32_t* clr = p >= 1 ? st[(p + 1) & 1] : nullptr;
      hipLaunchKernelGGL(k_rs_sweep, dim3((unsigned)ntiles), dim3(RS_NT), 0, s, ka, va, kb, vb, n, key_lo + 8 * p,
                         ghist + 256 * p, tickets + p, st[p & 1], clr, clr ? 256 * ntiles : (int64_t)0, ntiles,
                         err);
      uint64_t* tk = ka; ka = kb; kb = tk;
      uint32_t* tv = va; va = vb; vb = tv;
    }
    if (ka != keys)
      hipLaunchKernelGGL(k_copy_pairs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ka, va, keys, vals, n);
    return;
  }
  int64_t* counts = cv.take<int64_t>(256 * ntiles + 1);
  void* sscr = cv.take<char>(scan_scratch_bytes(256 * ntiles));
  for (int p = 0; p < passes; ++p) {
    int shift = key_lo + 8 * p;
    hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)ntiles), dim3(RS_NT), 0, s, ka, n, shift, counts, ntiles);
    exclusive_scan_i64(counts, counts, 256 * ntiles, nullptr, sscr, s);
    hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)ntiles), dim3(RS_NT), 0, s, ka, va, kb, vb, n, shift,
                       counts, ntiles);
    uint64_t* tk = ka; ka = kb; kb = tk;
    uint32_t* tv = va; va = vb; vb = tv;
  }
  if (ka != keys)  // a kernel rather than a copy, so the sort stays capturable
    hipLaunchKernelGGL(k_copy_pairs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ka, va, keys, vals, n);
}

void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
}

void iota_i32(int32_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_iota_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
}
