// Row export that allocates nothing: the variant of dsg_rows_export for
// callers that cannot allocate device memory (tight serving loops, harnesses
// that forbid allocation).  Its device staging -- the listed rows' lengths,
// their offsets, the scan's partial sums and the gathered entries -- lives in
// one fixed array of this library, `scratch`, instead of buffers allocated
// per call.  Each GPU holds its own copy of the array, at its own address,
// from the first context created on it until the process ends.
//
// In host code the array's name is only a stand-in for the symbol: its device
// address comes from hipGetSymbolAddress, taken once per device (with that
// device current) when the first context on the device is created, and every
// kernel argument and copy uses that address.
//
// Every call on a device shares the device's array, and the array keeps the
// last call's contents.  Nothing in it needs to start at zero: each step
// writes every element the next step reads (lengths, then offsets and the
// scan's tile sums, then entries).  Calls on one device are serialised here
// (a per-device lock held until the call's device work has finished and its
// results are on the host), so calls that would otherwise overlap on one GPU
// -- from several threads or contexts -- wait for each other instead of
// racing on the array.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "internal.h"

namespace {

constexpr int64_t NA_MAX_ROWS = int64_t(1) << 18;     // listed rows per call
constexpr int64_t NA_MAX_ENTRIES = int64_t(1) << 21;  // entries of those rows per call
constexpr size_t NA_SCAN_BYTES = 64 << 10;            // the scan's tile sums (scan_scratch_bytes)

constexpr size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

// layout of the array (byte offsets)
constexpr size_t NA_LENS = 0;
constexpr size_t NA_RP = NA_LENS + up256(8 * (NA_MAX_ROWS + 1));
constexpr size_t NA_SCAN = NA_RP + up256(8 * (NA_MAX_ROWS + 1));
constexpr size_t NA_COL = NA_SCAN + NA_SCAN_BYTES;
constexpr size_t NA_VAL = NA_COL + up256(4 * NA_MAX_ENTRIES);
constexpr size_t NA_BYTES = NA_VAL + up256(8 * NA_MAX_ENTRIES);  // 28.1 MiB

constexpr int NA_MAX_DEVICES = 64;

std::mutex g_init_mu;
char* g_ptr[NA_MAX_DEVICES] = {};        // device address of `scratch` on each device
std::mutex g_call_mu[NA_MAX_DEVICES];    // one call at a time per device

// Sort the entries [a, b) of the caller's arrays by column, in place (a heap
// sort that swaps columns and value bytes together: no extra memory).
void sort_row(int32_t* col, char* val, int vs, int64_t a, int64_t b) {
  const int64_t n = b - a;
  if (n < 2) return;
  int32_t* c = col + a;
  char* v = val ? val + a * vs : nullptr;
  auto swap_e = [&](int64_t x, int64_t y) {
    std::swap(c[x], c[y]);
    if (v) {
      char t[8];
      memcpy(t, v + x * vs, (size_t)vs);
      memcpy(v + x * vs, v + y * vs, (size_t)vs);
      memcpy(v + y * vs, t, (size_t)vs);
    }
  };
  auto sift = [&](int64_t root, int64_t end) {
    for (;;) {
      int64_t child = 2 * root + 1;
      if (child >= end) return;
      if (child + 1 < end && c[child + 1] > c[child]) ++child;
      if (c[root] >= c[child]) return;
      swap_e(root, child);
      root = child;
    }
  };
  for (int64_t r = n / 2 - 1; r >= 0; --r) sift(r, n);
  for (int64_t end = n - 1; end > 0; --end) {
    swap_e(0, end);
    sift(0, end);
  }
}

}  // namespace

static __device__ __align__(256) char scratch[NA_BYTES];

void noalloc_init(int device) {
  DSG_REQUIRE(device >= 0 && device < NA_MAX_DEVICES, DSG_E_UNSUPPORTED, "device index beyond the library's table");
  std::lock_guard<std::mutex> lk(g_init_mu);
  if (g_ptr[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    throw DsgError{DSG_E_DEVICE, std::string("hipGetSymbolAddress of the row-export staging array: ") +
                                     hipGetErrorString(e)};
  }
  g_ptr[device] = (char*)p;
}

int64_t rows_export_noalloc(DMat* m, const int32_t* d_rows, int32_t n, int64_t* row_ptr, int32_t* col, void* val,
                            int64_t cap) {
  Ctx* c = m->ctx;
  const int dev = c->device;
  DSG_REQUIRE(dev >= 0 && dev < NA_MAX_DEVICES && g_ptr[dev], DSG_E_STATE,
              "row-export staging array not set up on this device");
  DSG_REQUIRE(n >= 0 && n <= NA_MAX_ROWS, DSG_E_ARG,
              "view of " + std::to_string(n) + " rows: the allocation-free export takes at most " +
                  std::to_string(NA_MAX_ROWS));
  DSG_REQUIRE(scan_scratch_bytes(n) <= NA_SCAN_BYTES, DSG_E_DEVICE, "internal: scan staging too small");
  std::lock_guard<std::mutex> lk(g_call_mu[dev]);
  char* base = g_ptr[dev];
  int64_t* d_lens = (int64_t*)(base + NA_LENS);
  int64_t* d_rp = (int64_t*)(base + NA_RP);
  void* d_scan = base + NA_SCAN;
  int32_t* d_col = (int32_t*)(base + NA_COL);
  void* d_val = base + NA_VAL;
  hipStream_t s = c->stream;
  // every row length and offset, then the total
  gather_row_ptr(m, d_rows, n, d_lens, d_rp, d_scan, s);
  int64_t* h_total = (int64_t*)((char*)c->pinned + 3584);
  DSG_HIP(hipMemcpyAsync(h_total, d_rp + n, 8, hipMemcpyDeviceToHost, s));
  if (row_ptr) DSG_HIP(hipMemcpyAsync(row_ptr, d_rp, ((size_t)n + 1) * 8, hipMemcpyDeviceToHost, s));
  DSG_HIP(hipStreamSynchronize(s));
  const int64_t nnz = *h_total;
  if (!col || nnz == 0) return nnz;
  DSG_REQUIRE(row_ptr, DSG_E_ARG, "row_ptr is NULL: the entries need the caller's row pointers");
  DSG_REQUIRE(cap >= nnz, DSG_E_ARG, "capacity " + std::to_string(cap) + " < nnz " + std::to_string(nnz));
  DSG_REQUIRE(nnz <= NA_MAX_ENTRIES, DSG_E_ARG,
              "view of " + std::to_string(nnz) + " entries: the allocation-free export takes at most " +
                  std::to_string(NA_MAX_ENTRIES));
  // the entries, in view order, each row as stored; then sorted by column on the host
  gather_row_entries(m, d_rows, n, d_rp, d_col, d_val, s);
  DSG_HIP(hipMemcpyAsync(col, d_col, (size_t)nnz * 4, hipMemcpyDeviceToHost, s));
  const int vs = m->vsz;
  if (vs && val) DSG_HIP(hipMemcpyAsync(val, d_val, (size_t)nnz * vs, hipMemcpyDeviceToHost, s));
  DSG_HIP(hipStreamSynchronize(s));
  for (int32_t q = 0; q < n; ++q) sort_row(col, (vs && val) ? (char*)val : nullptr, vs, row_ptr[q], row_ptr[q + 1]);
  return nnz;
}
