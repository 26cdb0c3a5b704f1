// Internal declarations of the dsg library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/dsg.h"
#include "rowindex.h"

// ---------------------------------------------------------------------------
// host-side error plumbing
// ---------------------------------------------------------------------------

struct DsgError {
  dsg_status code;
  std::string msg;
};

#define DSG_HIP(call)                                                                 \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      throw DsgError{DSG_E_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)};  \
  } while (0)

#define DSG_REQUIRE(cond, code, text)                     \
  do {                                                    \
    if (!(cond)) throw DsgError{(code), std::string(text)}; \
  } while (0)

// ---------------------------------------------------------------------------
// storage
// ---------------------------------------------------------------------------

// Slack row capacity for a row of `len` entries: room to grow without moving.
__host__ __device__ inline int32_t slack_cap(int32_t len) {
  int32_t extra = len >> 3;
  return len + (extra < 4 ? 4 : extra);
}

struct Ctx;

// Outcome of one unique update key when it is applied to a row.
enum : uint8_t { UPD_NOP = 0, UPD_INS = 1, UPD_DEL = 2, UPD_OVR = 3, UPD_LOST = 4 };

// Entry pools (col and val) are allocated POOL_PAD entries beyond their
// capacity.  A kernel may then read a window of up to POOL_PAD entries from
// any position inside a row without a per-lane bounds check: the entries
// past the row are read and discarded, never used as content.
constexpr int64_t POOL_PAD = 256;
inline size_t pool_bytes(int64_t cap, int entry_size) { return (size_t)(cap + POOL_PAD) * (size_t)entry_size; }


// Device-resident dynamic matrix: every row owns a slot range
// [row_off[i], row_off[i] + row_cap[i]) of the column/value pools and uses its
// first row_len[i] slots, in no particular column order.  Rows that outgrow
// their capacity move to fresh space taken from the pool top.
struct DMat {
  Ctx* ctx = nullptr;
  int32_t nrows = 0, ncols = 0;
  int sr = 0;          // semiring id; -1 for a structure-only matrix
  int vsz = 0;         // bytes per value (0: structure only)
  int64_t* row_off = nullptr;
  int32_t* row_len = nullptr;
  int32_t* row_cap = nullptr;
  uint32_t* row_epoch = nullptr;  // epoch of the last change of each row
  int32_t* col = nullptr;
  void* val = nullptr;
  int64_t pool_cap = 0;           // slots in col/val
  int64_t* d_top = nullptr;       // device: first free slot (16-byte block: top, epoch)
  uint32_t* d_epoch = nullptr;    // device: bumped by every apply (lives in the d_top block)
  int64_t h_top_ub = 0;           // host: upper bound of *d_top
  uint64_t version = 0;           // bumped whenever the pools are reallocated
  DMat* tidx = nullptr;           // transpose (rows = columns of this), same values
  int refs = 0;                   // products using this matrix
  bool counted = false;           // registered in ctx->objects
  // log of the last plain apply: every unique key it touched, in key order,
  // with the stored value before and after and the outcome (UPD_*)
  uint64_t* log_key = nullptr;
  uint64_t* log_old = nullptr;
  uint64_t* log_new = nullptr;
  uint8_t* log_code = nullptr;
  int64_t* d_log_n = nullptr;     // device: entries in the log
  int64_t h_log_n = 0;            // host copy of *d_log_n
  int64_t log_cap = 0;
  uint64_t apply_seq = 0;         // applies so far
  uint64_t log_seq = 0;           // the apply whose log is held (0: none)
  // per-row column index (rowindex.h); ix_tab == nullptr: none
  uint64_t* ix_tab = nullptr;
  int64_t* ix_off = nullptr;
  int32_t* ix_sz = nullptr;
  int32_t* ix_used = nullptr;
  uint32_t* ix_stamp = nullptr;
  unsigned long long* ix_top = nullptr;  // device: first free slot of ix_tab
  int64_t ix_cap = 0;
  uint32_t ix_gen = 1;            // a row's table is usable while its stamp equals this
  bool ix_refused = false;        // no room for an index: the matrix runs without one
};

// Per-kernel timing record.
struct KernelTiming {
  std::string name;
  hipEvent_t start, stop;
  double bytes;
};

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t budget = 0;
  size_t held = 0;
  size_t ix_held = 0;  // bytes of the per-row column index pools of all matrices
  dsg_allocator allocator{};   // the caller's allocator (alloc == nullptr: hipMalloc / hipFree)
  std::mutex alloc_mu;  // ctx_alloc / ctx_free may run on a server's threads
  std::string last_error = "";
  bool served = false;  // owned by a server thread: the ABI refuses other calls
  int objects = 0;
  int num_cus = 256;  // compute units of the device
  dsg_tuning tuning;
  bool timing = false;
  std::string timing_phase;  // when not empty, only phases of this name are timed
  std::vector<KernelTiming> timings;
  std::vector<hipEvent_t> event_pool;
  // pinned host staging block for small device->host reads (4 KB), and its
  // device address, which kernels write to directly
  void* pinned = nullptr;
  void* pinned_dev = nullptr;
  // reusable device scratch, grown on demand
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  void* scratch2 = nullptr;
  size_t scratch2_bytes = 0;
  // second stream (default priority) for the short row bins, which run beside
  // the long ones; created on first use, joined back through the two events
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
};

void* ctx_alloc(Ctx* c, size_t bytes);
void ctx_free(Ctx* c, void* p, size_t bytes);
void* ctx_scratch(Ctx* c, size_t bytes);   // contents undefined; valid until the next call
void* ctx_scratch2(Ctx* c, size_t bytes);
void ctx_sync(Ctx* c);
// Records a phase's start unless a phase filter excludes it (then both
// events are null and false is returned); ctx_timing_end ignores a null event.
// Both record on stream `on` (nullptr: the context's stream).
bool ctx_timing_begin(Ctx* c, const char* name, double bytes, hipEvent_t* start, hipEvent_t* stop,
                      hipStream_t on = nullptr);
void ctx_timing_end(Ctx* c, hipEvent_t stop, hipStream_t on = nullptr);
// The side stream and its fork/join events, created on first use.
hipStream_t ctx_side_stream(Ctx* c);

// Bump allocator for device scratch carved out of one allocation.
struct Carve {
  char* base;
  size_t off = 0, cap;
  Carve(void* b, size_t c) : base((char*)b), cap(c) {}
  template <class T>
  T* take(size_t n) {
    size_t a = (off + 255) & ~size_t(255);
    T* p = (T*)(base + a);
    off = a + n * sizeof(T);
    if (off > cap) throw DsgError{DSG_E_OOM, "internal scratch overflow"};
    return p;
  }
  static size_t need(std::initializer_list<size_t> bytes) {
    size_t s = 0;
    for (size_t b : bytes) s += (b + 255) & ~size_t(255);
    return s + 256;
  }
};

// ---------------------------------------------------------------------------
// primitives (prims.hip)
// ---------------------------------------------------------------------------

// Exclusive scan of n int64 values (in place allowed); total written to
// *d_total (device) if not null.  Scratch: scan_scratch_bytes(n).
size_t scan_scratch_bytes(int64_t n);
// Small device values copied into the context's pinned block by one kernel
// (in place of one copy each): up to 8 sources of 4-byte multiples, each to
// its byte offset in the block; a null source writes zeros.  Read them after
// the stream is synchronized.
struct FetchList {
  const void* src[8] = {};
  int32_t bytes[8] = {};
  int32_t off[8] = {};
  int32_t n = 0;
  void add(const void* p, int32_t nbytes, int32_t offset) {
    src[n] = p;
    bytes[n] = nbytes;
    off[n] = offset;
    ++n;
  }
};
void fetch_to_pinned(Ctx* c, const FetchList& F, hipStream_t s);
// Validity of a batch on the device (bit 0: an index out of range, bit 1: an
// unknown op) written into the pinned block at byte offset `off` (n small:
// one launch), or -1 when n is too large for that (the caller checks the
// usual way).
bool validate_to_pinned(const int32_t* rows, const int32_t* cols, const uint8_t* ops, int64_t n, int32_t nrows,
                        int32_t ncols, Ctx* c, int32_t off);

// Two such scans of n values each (one launch when n is small; one scratch,
// used by each in turn).
void exclusive_scan_i64_pair(const int64_t* in0, int64_t* out0, int64_t* tot0, const int64_t* in1, int64_t* out1,
                             int64_t* tot1, int64_t n, void* scratch, hipStream_t s);
void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* d_total, void* scratch,
                        hipStream_t s);
// Exclusive scan of int32 counts into int64 offsets.
void exclusive_scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, int64_t* d_total,
                               void* scratch, hipStream_t s);

// Indices i < n with flags[i] != 0, ascending, into out; count into *d_count.
size_t compact_scratch_bytes(int64_t n);
// Positions of the entries of each class 0, 1, 2 of cls[0..n) (every value
// one of those), in order, into out0/out1/out2; their counts to
// d_count[0..2].
// Scratch: compact_scratch_bytes(n).
void compact_classes3(const uint8_t* cls, int64_t n, int32_t* out0, int32_t* out1, int32_t* out2, int32_t* d_count,
                      void* scratch, hipStream_t s);
void compact_flags(const uint8_t* flags, int64_t n, int32_t* out, int32_t* d_count, void* scratch,
                   hipStream_t s);
// Entries list[q], q < *d_n, with flags[q] != 0, in order, into out; count into *d_count.
void compact_list_by_flags(const int32_t* list, const uint8_t* flags, const int32_t* d_n, int64_t n_max,
                           int32_t* out, int32_t* d_count, void* scratch, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on the low key_bits bits.
size_t radix_scratch_bytes(int64_t n);
// Sorts keys/vals in place (using the scratch as ping-pong buffers).  err,
// when given, gets bit 16 if a pass could not complete its look-back.  When
// the input is already in order on the bits below key_lo among keys equal
// above it, key_lo > 0 lets the radix passes start there (the order is the
// same, with fewer passes).
void radix_sort_pairs(uint64_t* keys, uint32_t* vals, int64_t n, int key_bits, void* scratch,
                      hipStream_t s, int* err = nullptr, int key_lo = 0);

void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
void iota_i32(int32_t* p, int64_t n, hipStream_t s);

// ---------------------------------------------------------------------------
// matrices (matrix.hip) and updates (ingest.hip)
// ---------------------------------------------------------------------------

DMat* mat_create(Ctx* c, int32_t nrows, int32_t ncols, int sr, const int64_t* d_row_ptr,
                 const int32_t* d_col, const void* d_val);  // device CSR or null
void mat_destroy(DMat* m);
// Make sure `extra` more slots can be taken from the pool top; may compact.
void mat_reserve(DMat* m, int64_t extra);
// Same, but a compaction (only when fewer than `extra` slots are free) makes
// room for `want` >= extra: fewer compactions for pools that grow fast.
void mat_reserve(DMat* m, int64_t extra, int64_t want);
void mat_compact(DMat* m, int64_t extra);
int64_t mat_nnz(DMat* m);
// Canonical (column-sorted) CSR copy on the device: row_ptr[nrows+1], col, val.
void mat_export_device(DMat* m, int64_t* d_row_ptr, int32_t* d_col, void* d_val, void* scratch,
                       hipStream_t s);
// Build the valued transpose index of m (its columns as rows, with their
// values); every later apply of m keeps it current.
void mat_build_transpose(DMat* m);

// Per-row column index (rowindex.hip).  mat_index_enable allocates it (false
// when there is no room: the matrix then goes on without one); every table
// starts invalid.  mat_index_invalidate drops every table at once (any
// writer that may reorder rows of m without maintaining the tables calls
// it).  mat_index_build makes the tables of the listed rows (*d_n of them,
// at most n_max; all rows when d_rows is null, then d_n may be null too)
// usable, as far as the pool has room.  mat_index_note_top takes a host
// copy of the pool top and resets the pool when most of it is taken.
RowIx mat_index_view(const DMat* m);
bool mat_index_enable(DMat* m);
void mat_index_free(DMat* m);
void mat_index_invalidate(DMat* m);
void mat_index_build(DMat* m, const int32_t* d_rows, const int64_t* d_n, int64_t n_max);
void mat_index_note_top(DMat* m, uint64_t top);

// Listed rows of a matrix, copied to the host with each row sorted by column.
struct RowsHost {
  std::vector<int64_t> row_ptr;  // n + 1
  std::vector<int32_t> col;
  std::vector<char> val;         // vsz bytes per entry
};
// Reusable device buffers of mat_gather_rows (grown on demand).
struct GatherBufs {
  void* lens = nullptr;
  size_t lens_bytes = 0;
  void* rp = nullptr;
  size_t rp_bytes = 0;
  void* scan = nullptr;
  size_t scan_bytes = 0;
  void* col = nullptr;
  size_t col_bytes = 0;
  void* val = nullptr;
  size_t val_bytes = 0;
};
// d_rows: n valid row ids on the device.  Synchronizes stream s.  With
// entries false only the row pointers are filled.
void mat_gather_rows(DMat* m, const int32_t* d_rows, int32_t n, GatherBufs& g, RowsHost& out, hipStream_t s,
                     bool entries = true);
void gather_bufs_free(Ctx* c, GatherBufs& g);
// The device steps of mat_gather_rows on caller-owned buffers (nothing
// allocated): the n listed rows' lengths into d_lens[n] and their offsets
// into d_rp[n + 1] (total in d_rp[n]; d_scan: scan_scratch_bytes(n) bytes),
// then their entries, in list order and in each row's stored order, into
// d_col / d_val at those offsets.  Queued on stream s.
void gather_row_ptr(DMat* m, const int32_t* d_rows, int32_t n, int64_t* d_lens, int64_t* d_rp, void* d_scan,
                    hipStream_t s);
void gather_row_entries(DMat* m, const int32_t* d_rows, int32_t n, const int64_t* d_rp, int32_t* d_col,
                        void* d_val, hipStream_t s);

// Row export that allocates no device memory (noalloc.hip): the listed rows
// of m, each sorted by column, into the caller's host arrays, staged through
// a fixed device array of the library.  noalloc_init looks that array up on
// the current device (once per device; the context creation calls it).
void noalloc_init(int device);
int64_t rows_export_noalloc(DMat* m, const int32_t* d_rows, int32_t n, int64_t* row_ptr, int32_t* col, void* val,
                            int64_t cap);

// Apply a device-resident batch (validated).  Returns nothing; updates epochs.
void mat_apply_device(DMat* m, const int32_t* d_rows, const int32_t* d_cols, const void* d_vals,
                      const uint8_t* d_ops, int64_t n);
// Graph-capturable apply (no host round trips) on caller-owned workspaces of
// apply_work_bytes(n, ...) bytes (work_tidx only when m->tidx).  The caller
// must have reserved apply_headroom(m, n) free pool slots in m and in
// m->tidx; error flags stay on the device (apply_err_ptr).
size_t apply_work_bytes(int64_t n, bool deltas);
int* apply_err_ptr(void* work, int64_t n, bool deltas);
int64_t apply_headroom(const DMat* m, int64_t n);
void mat_apply_graph(DMat* m, const int32_t* d_rows, const int32_t* d_cols, const void* d_vals,
                     const uint8_t* d_ops, int64_t n, void* work_main, void* work_tidx);
// Apply n unique keys (row << colbits | col), sorted ascending, to m as ADD
// updates: vals[u] is folded in with the semiring addition when flag[u] & 1
// (else the key only carries a guard).  An entry present in m is left
// unchanged and listed as lost -- (key, row-relative slot) in key order, at
// most lost_cap >= n, count in *d_nlost -- when flag[u] & 4, or when
// flag[u] & 2 and its stored value has the ordered key guard[u] while
// vals[u] (if any) is strictly larger.  *d_nrows (when not null) receives
// the number of distinct rows among the keys.  scratch holds
// sorted_add_scratch_bytes(n) bytes.  Returns the number of lost entries.
// m must have no transpose.
size_t sorted_add_scratch_bytes(int64_t n);
int64_t mat_apply_sorted_add(DMat* m, const uint64_t* keys, const void* vals, const uint64_t* guard,
                             const uint8_t* flag, int64_t n, uint64_t* lost_key, int32_t* lost_slot,
                             int64_t lost_cap, unsigned long long* d_nlost, int64_t* d_nrows, void* scratch);
// Delete the n present entries whose keys (row << colbits | col) are
// keys[list[t]] (list null: keys[t]), sorted ascending and unique, and
// which sit at the row-relative slots slots[list[t]] (nothing is looked up
// or streamed).  m must have no transpose.
void mat_apply_sorted_delete(DMat* m, const uint64_t* keys, const int32_t* slots, const int32_t* list, int64_t n);
// Device validation of a batch: returns dsg_status.
dsg_status validate_batch_device(DMat* m, const int32_t* d_rows, const int32_t* d_cols,
                                 const uint8_t* d_ops, int64_t n);

// ---------------------------------------------------------------------------
// products (spgemm.hip)
// ---------------------------------------------------------------------------

struct DProd {
  Ctx* ctx = nullptr;
  // The operands as the kernels read them: the caller's matrices, or their
  // valued transposes when the product takes an operand transposed.
  DMat* A = nullptr;
  DMat* B = nullptr;
  DMat* C = nullptr;
  DMat* src_a = nullptr;  // the caller's matrices: referenced, and the ones updates are applied to
  DMat* src_b = nullptr;
  DMat* lt = nullptr;     // transpose of the left operand (rows of A per column), for discovery
  uint32_t ops = 0;       // DSG_TRANS_A / DSG_TRANS_B
  uint32_t* d_sync = nullptr;      // device [2]: epochs of A and B that C reflects
  int32_t* changed_rows = nullptr;  // device list of the last update's reported rows
  int64_t changed_cap = 0;
  int32_t* query_rows = nullptr;
  int64_t query_cap = 0;
  void* arena = nullptr;                     // per-row staging / global hash tables
  size_t arena_bytes = 0;
  unsigned long long* arena_top = nullptr;   // device bump pointer into the arena
  dsg_update_stats stats{};
  int64_t last_c_demand = 0;      // C pool and arena needs of the last plain-path run
  int64_t last_arena_demand = 0;
  int64_t last_c_growth = 0;      // C pool slots the last batched run took
  uint64_t a_seq = 0, b_seq = 0;  // applies of A and B that C reflects
  void* ews = nullptr;            // workspace of the entry-granular path
  size_t ews_bytes = 0;
  void* bsp = nullptr;            // B with each row's entries grouped by dense column chunk
  size_t bsp_bytes = 0;
  size_t bsp_col_off = 0, bsp_val_off = 0;
  int bsp_parts = 0;
  bool bsp_live = false;          // bsp holds the current B for the running update
  int64_t entry_nU = 0;           // entry-granular path: log entries and changed
  int64_t entry_nterm = 0;        // products counted for the pending update
  int refs = 0;                   // batched executors and servers using this product
  // general updates filtered by a Bloom matrix (DSG_GENERAL_BLOOM): F has C's
  // structure, bit (k mod 64) of f_ij set when a_ik b_kj is a term of c_ij
  bool bloom = false;
  DMat* F = nullptr;
  void* gws = nullptr;            // workspace of the general-update path
  size_t gws_bytes = 0;
};

// C = op(A) op(B), op(X) = X^T under DSG_TRANS_A / DSG_TRANS_B in ops.
DProd* prod_create(Ctx* c, DMat* A, DMat* B, uint32_t ops = 0);
// A new matrix (alpha (x) C) (+) (beta (x) X) from the product's current C;
// X may be null (then beta is not read).  alpha, beta: host values.
DMat* prod_scale_add(DProd* p, const void* alpha, DMat* X, const void* beta);
void prod_destroy(DProd* p);
// mode 0: dynamic update; 1: recompute every row (static); with report_affected.
int32_t prod_run(DProd* p, int mode, bool report_affected);

// One operand of a product as the dynamic paths see it: the matrix whose
// rows they read (op(X): X, or X's transpose index), the matrix holding its
// columns as rows (X's transpose index, or X itself), the matrix whose log
// lists its changes in its own coordinates (the transpose index keeps the
// transposed log of every apply), the source matrix that counts applies, and
// the apply count the product last reflected.
struct OpView {
  DMat* rows;
  DMat* cols;
  const DMat* logm;
  const DMat* src;
  uint64_t seq;
};

inline OpView op_view(const DProd* p, bool left) {
  const bool trans = (p->ops & (left ? DSG_TRANS_A : DSG_TRANS_B)) != 0;
  DMat* src = left ? p->src_a : p->src_b;
  OpView v;
  v.rows = left ? p->A : p->B;
  v.cols = trans ? src : src->tidx;
  v.logm = trans ? src->tidx : src;
  v.src = src;
  v.seq = left ? p->a_seq : p->b_seq;
  return v;
}

// An operand applied once since the last update, with the log of that apply
// (in its own coordinates); or not applied since.
inline bool changed_once(const OpView& v) {
  return v.logm && v.src->log_seq != 0 && v.src->log_seq == v.src->apply_seq && v.logm->log_seq == v.src->apply_seq &&
         v.src->apply_seq == v.seq + 1;
}
inline bool unchanged(const OpView& v) { return v.src->apply_seq == v.seq; }

// Entry-granular dynamic update (entry.hip): for C = op(A) op(B) over
// (min,+), int64 (+,x) or (or, and) when C reflects every apply but the last
// and the operands hold that apply's logs (entry_eligible).  entry_count
// lists how many products the last applies changed (kept in the context's
// second scratch); entry_finish, called next with nothing else on that
// scratch in between, updates C and returns the reported-row count.
bool entry_eligible(DProd* p);
// Queues the count; its total lands in *entry_count's result (device) and is
// read back by the caller's next synchronisation into p->entry_nterm.
const int64_t* entry_count(DProd* p);
int32_t entry_finish(DProd* p);

// General updates with the Bloom matrix (general.hip, Section 5.2,
// Algorithm 2), for C = op(A) op(B).  bloom_build computes F from the
// current C, op(A) and op(B); general_eligible tells whether the logs of the
// operands cover every apply since the product last saw them (then general_update brings C and F up to
// date and returns the reported-row count).
void bloom_build(DProd* p);
bool general_eligible(const DProd* p);
int32_t general_update(DProd* p);

// Graph-capturable dynamic update (no host round trips) on a caller-owned
// workspace of prod_graph_work_bytes(p) bytes, after prod_prepare_graph set
// room aside.  Rows that find no room in C or the staging arena write
// nothing and are flagged; d_out[0..5] receives: reported rows, affected
// rows, error flags, rows waiting for room (0/1), C slots and arena bytes
// they need.  When d_out[3] is set, prod_finish_graph (plain, with host
// round trips) grows the room, recomputes those rows and returns the final
// reported-row count.
size_t prod_graph_work_bytes(const DProd* p);
void prod_prepare_graph(DProd* p, int64_t c_headroom, size_t arena_bytes, int64_t c_want = 0);
void prod_update_graph(DProd* p, void* work, int64_t* d_out);
int32_t prod_finish_graph(DProd* p, void* work);

// asynchronous validation of a device batch: ORs 1 (range) / 2 (op) into *d_flag
void validate_batch_async(DMat* m, const int32_t* d_rows, const int32_t* d_cols, const uint8_t* d_ops, int64_t n,
                          int* d_flag);

// ---------------------------------------------------------------------------
// batched form (batch.hip)
// ---------------------------------------------------------------------------

struct DBatchSet {
  DMat* m;
  const int32_t* rows;
  const int32_t* cols;
  const void* vals;
  const uint8_t* ops;
  int64_t n;
};
struct DBatch;
DBatch* batch_create(Ctx* c, const std::vector<DProd*>& prods);
void batch_destroy(DBatch* b);
// returns DSG_OK, or DSG_E_RANGE / DSG_E_ARG for a bad set (nothing applied)
dsg_status batch_run(DBatch* b, const std::vector<DBatchSet>& sets, std::vector<int32_t>& counts);
DProd* batch_prod(DBatch* b, int i);

// ---------------------------------------------------------------------------
// served form (server.hip)
// ---------------------------------------------------------------------------

struct DServer;
DServer* server_create(Ctx* c, DProd* p, const dsg_server_cfg* cfg);
void server_destroy(DServer* s);  // drains first
uint64_t server_submit_update(DServer* s, DMat* m, const int32_t* rows, const int32_t* cols, const void* vals,
                              const uint8_t* ops, int64_t n);
uint64_t server_submit_query(DServer* s, const int32_t* rows, int32_t nq);
void server_poll(DServer* s, uint64_t ticket, bool wait, dsg_server_result* out);
void server_query_result(DServer* s, uint64_t ticket, int64_t* row_ptr, int32_t* col, void* val, int64_t cap,
                         int64_t* nnz_out);
void server_release(DServer* s, uint64_t ticket);
void server_drain(DServer* s);
void server_stats(DServer* s, dsg_server_stats* out);
void batch_info(const DBatch* b, dsg_batch_stats* out);
