/* dsg -- batch-dynamic sparse matrix-matrix multiplication on AMD MI355X (gfx950).
 *
 * The library keeps the product C = A B of sparse matrices current while
 * batches of entry insertions, deletions and value changes are applied to A
 * and B, recomputing only the rows of C that the changes can reach.  It
 * follows the problem statement of "Fast Dynamic Updates and Dynamic SpGEMM
 * on MPI-Distributed Graphs" (van der Grinten et al., arXiv 2202.08808):
 *   - Section 3:   matrices over a semiring; an absent entry equals the
 *                  semiring's additive neutral element; a present entry is a
 *                  structural non-zero whatever its value;
 *   - Section 4.1: updates are (i, j, x) tuples applied by "merge"
 *                  (insert/overwrite), "mask" (delete) or algebraic addition;
 *   - Section 5:   given C = A B and the updated operands A', B', compute
 *                  C' = A' B'; C' can differ from C only in rows holding a
 *                  non-zero of C* = A* B' + A B* (Eq. 1 and the discussion of
 *                  general updates), where A*, B* mark the changed entries.
 *
 * All numeric work runs in HIP kernels on one GPU.  Objects live in device
 * memory (HBM).  Every call is ordered on the context's HIP stream.
 *
 * Conventions
 *   Status:     every function returns a dsg_status; no exceptions cross the
 *               boundary.  On failure no object is modified (arguments are
 *               validated before any mutation) and dsg_last_error() holds a
 *               message.
 *   Ownership:  input arrays are borrowed for the duration of the call.  The
 *               library owns matrices and products until *_destroy.  Views
 *               (dsg_rows) point into library memory and stay valid until the
 *               next call that mutates that product.
 *   Host/device pointers: input arrays are host pointers unless the call's
 *               flags contain DSG_INPUT_DEVICE, in which case they are device
 *               pointers readable on the context's device.
 *   Threading:  a context and its objects may be used by one host thread at a
 *               time.
 *   Indices:    int32 row and column indices, 0-based; int64 offsets.
 */
#ifndef DSG_H
#define DSG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DSG_OK = 0,
  DSG_E_ARG = 1,         /* null pointer, bad size, bad op code or flag */
  DSG_E_RANGE = 2,       /* an index outside [0, nrows) x [0, ncols) */
  DSG_E_OOM = 3,         /* device allocation failed or the memory budget is exceeded */
  DSG_E_DEVICE = 4,      /* a HIP call failed */
  DSG_E_STATE = 5,       /* semiring/shape mismatch, or object still referenced */
  DSG_E_UNSUPPORTED = 6
} dsg_status;

/* Semirings (Section 3).  The semiring fixes the value type:
 *   DSG_PLUS_TIMES_I64: (+, x) over int64, two's-complement wrap-around;
 *   DSG_MIN_PLUS_F32:   (min, +) over fp32, +inf neutral, -0 ordered below +0;
 *   DSG_PLUS_TIMES_F64: (+, x) over fp64, each product and sum rounded once
 *                       (no fused multiply-add);
 *   DSG_OR_AND_U32:     the Boolean (or, and) semiring applied bitwise to
 *                       uint32 words: 32 Boolean semirings side by side, 0
 *                       neutral; values 0 and 1 give the plain Boolean
 *                       product. */
typedef enum {
  DSG_PLUS_TIMES_I64 = 0,
  DSG_MIN_PLUS_F32 = 1,
  DSG_PLUS_TIMES_F64 = 2,
  DSG_OR_AND_U32 = 3
} dsg_semiring;

/* Update operations (Section 4.1). */
typedef enum {
  DSG_OP_SET = 0,     /* "merge": overwrite if present, else insert */
  DSG_OP_DELETE = 1,  /* "mask": remove if present, else no-op */
  DSG_OP_ADD = 2      /* algebraic: a <- a (+) x if present, else insert x */
} dsg_op;

/* flags */
#define DSG_INPUT_DEVICE 0x1u     /* input arrays are device pointers */
#define DSG_SYNC 0x2u             /* return only after the device work has finished */
#define DSG_REPORT_AFFECTED 0x4u  /* dsg_prod_update: report every recomputed row, skip the comparison with the old row */

typedef struct dsg_ctx dsg_ctx;
typedef struct dsg_mat dsg_mat;
typedef struct dsg_prod dsg_prod;

/* A set of rows of a product, as device views into the product's storage.
 * Row rows[q] has row_len[rows[q]] entries at positions
 * row_off[rows[q]] .. +row_len[rows[q]]-1 of col[] and val[] (val holds the
 * semiring's value type).  Entries inside a row are in no particular order.
 * rows[] is ascending.  All pointers are device pointers. */
typedef struct {
  int32_t n;
  const int32_t* rows;
  const int64_t* row_off;
  const int32_t* row_len;
  const int32_t* col;
  const void* val;
} dsg_rows;

/* ---- context ---- */

/* Create a context on HIP device `device`.  hip_stream is a hipStream_t to
 * order all work on (NULL: the library creates its own).  mem_budget caps the
 * device bytes the context may hold (0: no cap); exceeding it gives
 * DSG_E_OOM. */
dsg_status dsg_ctx_create(int device, void* hip_stream, size_t mem_budget, dsg_ctx** out);
/* Device memory from the caller's allocator instead of hipMalloc / hipFree
 * (a framework's caching allocator, a pool): once set, every device
 * allocation of the context -- matrix pools, products, workspaces, scratch --
 * is alloc(bytes, stream, user) and is returned through free(ptr, bytes,
 * stream, user), with the context's HIP stream; the library uses a block
 * only in that stream's order (other streams it forks join it before the
 * block is freed).  alloc returns NULL when it cannot allocate (DSG_E_OOM);
 * both may be called from the served form's threads.  The memory budget
 * still applies.  Set before the context allocates anything (DSG_E_STATE
 * afterwards); a = NULL keeps hipMalloc.  This is the allocator callback the
 * problem's boundary leaves to the caller: the library holds no device
 * memory of its own beyond what it asks for here (and the fixed staging
 * array of dsg_rows_export_noalloc). */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* ptr, size_t bytes, void* stream, void* user);
  void* user;
} dsg_allocator;
dsg_status dsg_ctx_set_allocator(dsg_ctx* ctx, const dsg_allocator* a);

/* Destroy a context.  DSG_E_STATE while it still owns matrices or products. */
dsg_status dsg_ctx_destroy(dsg_ctx* ctx);
/* Message describing the last failure on this context (never NULL). */
const char* dsg_last_error(const dsg_ctx* ctx);
/* Block until all work queued on the context's stream has finished. */
dsg_status dsg_ctx_synchronize(dsg_ctx* ctx);
/* Device bytes currently held by the context. */
dsg_status dsg_ctx_memory(const dsg_ctx* ctx, size_t* bytes);
/* Turn per-kernel timing with HIP events on (1) or off (0); turning it on
 * clears the record.  dsg_ctx_timing_report writes a JSON object
 * {"kernels": {name: {"launches": n, "ms": total, "bytes": algorithmic
 * bytes}}} into buf (NUL-terminated, truncated to cap) after synchronising. */
dsg_status dsg_ctx_set_timing(dsg_ctx* ctx, int on);
/* Time only the phases named `phase` (as in the report; NULL or "": every
 * phase), so that a timed run pays two event records per launch of the one
 * kernel of interest and none elsewhere. */
dsg_status dsg_ctx_set_timing_phase(dsg_ctx* ctx, const char* phase);
dsg_status dsg_ctx_timing_report(dsg_ctx* ctx, char* buf, size_t cap);

/* Row-kernel tuning: output-row-size thresholds of the accumulator bins.
 * Results never depend on these settings. */
typedef struct {
  int32_t group_ub[8];     /* bin b (lane-group hash in LDS) takes rows with ub <= group_ub[b];
                              ascending, each at most the bin's capacity (32<<b); 0 disables bin b */
  int32_t dense_max_passes;/* rows above the group bins use the chunked dense LDS accumulator when
                              it needs at most this many column passes, else a global-memory hash */
  int32_t force_bin;       /* -1: automatic; 0..7 group bin; 8 dense; 9 global hash (for tests;
                              a group bin is only used for rows that fit it) */
  int32_t update_path;     /* dynamic updates of C = op(A)*op(B) (no Bloom matrix) over (min,+),
                              int64 (+,x) or (or, and), each operand applied at most once since the last
                              update: 0 automatic (see below); 1 always whole rows; 2
                              entry-granular whenever it applies.  Same results every way. */
  int32_t batch_direct_log2; /* batched form: products whose C holds at least 2^this slots take the
                              plain path beside the graph replay (default 24; 0..62) */
  /* Automatic choice: the entry-granular path runs when the products of the
   * affected rows exceed entry_fixed + entry_per_term * (the changed
   * products).  Defaults 1e8 and 70 (fitted on MI355X); both finite, >= 0. */
  double entry_fixed;
  double entry_per_term;
  int32_t row_index;       /* 1 (default): the entry-granular path gives C, A and B a per-row column
                              index (Section 4's per-row hash; about 20 bytes per entry of C), and
                              the general path with the Bloom matrix, where C's rows average at
                              least 128 slots, gives one to B (its masked product probes B' rows),
                              C and F.  The index pools of a context take at most 1/8 of
                              the device, and only memory that stays free beyond a reserve (and at
                              most half of what a budget leaves); without room for the operands'
                              indexes the row path runs.  0: never (applies stream the touched
                              rows; the entry path's lost entries scan rows of A' and B'; the
                              general path walks rows of B' and streams rows of F) */
} dsg_tuning;
dsg_status dsg_ctx_get_tuning(const dsg_ctx* ctx, dsg_tuning* t);
/* t == NULL restores the defaults.  DSG_E_ARG for thresholds outside the
 * bins' capacities, a descending order, or force_bin outside [-1, 9]. */
dsg_status dsg_ctx_set_tuning(dsg_ctx* ctx, const dsg_tuning* t);

/* ---- dynamic matrices (Section 4: dynamic storage with O(1) updates) ---- */

/* Create an nrows x ncols dynamic matrix from CSR arrays (row_ptr[nrows+1],
 * col[nnz], val[nnz] of the semiring's value type), each row free of
 * duplicate columns, in any column order.  row_ptr == NULL creates an empty
 * matrix.  flags: DSG_INPUT_DEVICE.  Errors: DSG_E_ARG (sizes, duplicates,
 * non-monotone row_ptr), DSG_E_RANGE (column index), DSG_E_OOM. */
dsg_status dsg_mat_create(dsg_ctx* ctx, int32_t nrows, int32_t ncols, dsg_semiring sr,
                          const int64_t* row_ptr, const int32_t* col, const void* val,
                          uint32_t flags, dsg_mat** out);

/* Apply a batch of n updates (Section 4.1) with the semantics of applying
 * them one after the other in batch order: for repeated (i, j) the last
 * SET/DELETE wins and later ADDs fold on top.  rows/cols/vals/ops are arrays
 * of n entries (vals of the value type; ignored for DELETE).  Rows whose
 * stored content changes are logged for the next dsg_prod_update of every
 * product using the matrix.  flags: DSG_INPUT_DEVICE, DSG_SYNC.
 * Errors (nothing applied): DSG_E_ARG (bad op), DSG_E_RANGE (index),
 * DSG_E_OOM. */
dsg_status dsg_mat_apply(dsg_mat* m, const int32_t* rows, const int32_t* cols, const void* vals,
                         const uint8_t* ops, int64_t n, uint32_t flags);

/* Number of stored entries of the matrix, nnz(A) in the notation of
 * Section 3 (a dynamic matrix of Section 4: slots that hold a tombstone are
 * not counted).  Synchronises with the device.  Errors: DSG_E_ARG (null). */
dsg_status dsg_mat_nnz(dsg_mat* m, int64_t* nnz);
/* Shape and semiring the matrix was created with (any pointer may be NULL).
 * DSG_E_ARG for a NULL or destroyed matrix. */
dsg_status dsg_mat_shape(const dsg_mat* m, int32_t* nrows, int32_t* ncols, dsg_semiring* sr);

/* Copy the matrix to host CSR arrays in canonical form (rows sorted by
 * column).  row_ptr has nrows+1 entries; col/val have room for cap entries.
 * *nnz_out receives nnz; with col == NULL only *nnz_out (and row_ptr if not
 * NULL) is written.  DSG_E_ARG if cap < nnz. */
dsg_status dsg_mat_export(dsg_mat* m, int64_t* row_ptr, int32_t* col, void* val, int64_t cap,
                          int64_t* nnz_out);

/* Destroy a matrix.  DSG_E_STATE while a product uses it. */
dsg_status dsg_mat_destroy(dsg_mat* m);

/* ---- products (Section 5) ---- */

/* Create the product C = A B (B may be A) and compute it from scratch with
 * the row kernels.  DSG_E_STATE on semiring mismatch or ncols(A) != nrows(B).
 * The matrix keeps a transpose index (valued) of A current: every apply of A
 * updates it, and updates use it to find the rows of A that reach a changed
 * row of B.  Same as dsg_prod_create with ops = 0. */
dsg_status dsg_prod_create_static(dsg_ctx* ctx, dsg_mat* A, dsg_mat* B, dsg_prod** out);

/* Operand forms (Section 3: either operand of SpGEMM may be transposed;
 * Section 5, "Handling Transposition"). */
#define DSG_TRANS_A 0x1u  /* the product reads A^T in place of A */
#define DSG_TRANS_B 0x2u  /* the product reads B^T in place of B */
/* General updates filtered by a Bloom matrix (Section 5.2, Algorithm 2): the
 * product keeps, beside C, the matrix F of C's structure whose entry f_ij has
 * bit (k mod 64) set when a_ik b_kj is a term of c_ij.  Each dynamic multiply
 * then finds the pattern C* = A* B + A' B* of the changed terms with their
 * bits F*, ors F and F* over each row of C* into a filter R, recomputes only
 * the entries of C* from the columns k of A' that R lets through, and merges
 * the new entries and bits into C and F.  When an operand took more than one
 * apply since the last update (the change logs hold one apply), or an fp64
 * row of A' keeps more than 4096 columns after the filter, the row path runs
 * and F is rebuilt.  Combines with DSG_TRANS_A / DSG_TRANS_B (then A
 * and B above are op(A) and op(B)); in the batched form such a product takes
 * the plain path beside the graph replay.  Results equal those of the other
 * paths. */
#define DSG_GENERAL_BLOOM 0x4u

/* Create C = op(A) op(B), op(X) = X^T when ops holds X's flag, and compute
 * it from scratch.  A transposed operand is read from its transpose index,
 * which every apply of the matrix keeps current (the index is built here if
 * the matrix has none), so updates are applied to A and B as usual and
 * dsg_prod_update brings C up to date from op(A)'s and op(B)'s changes by
 * any of the update paths (dsg_tuning.update_path).  Errors: DSG_E_ARG
 * (unknown flag), DSG_E_STATE (semiring mismatch, inner dimensions of op(A)
 * and op(B) differ). */
dsg_status dsg_prod_create(dsg_ctx* ctx, dsg_mat* A, dsg_mat* B, uint32_t ops, dsg_prod** out);

/* Canonical host CSR of a DSG_GENERAL_BLOOM product's Bloom matrix F (same
 * structure as C; val holds one uint64 bit field per entry), as
 * dsg_prod_export.  DSG_E_STATE for a product without F. */
dsg_status dsg_prod_export_bloom(dsg_prod* p, int64_t* row_ptr, int32_t* col, uint64_t* val, int64_t cap,
                                 int64_t* nnz_out);

/* A new matrix D = (alpha (x) C) (+) (beta (x) X), the general SpGEMM result
 * alpha op(A) op(B) + beta X of Section 3, from the product's C as of its
 * last update or recompute.  D holds an entry wherever C or X holds one:
 * alpha (x) c where only C has it, beta (x) x where only X has it, and
 * (alpha (x) c) (+) (beta (x) x) where both do (each operation rounded
 * once).  alpha and beta are host pointers to one value of the semiring's
 * type; X is a matrix of C's shape and semiring, or NULL (then D =
 * alpha (x) C and beta may be NULL).  D is a plain matrix owned by the caller
 * (dsg_mat_destroy): later updates of the product do not change it.  Errors:
 * DSG_E_ARG (NULL product, alpha or out; destroyed X), DSG_E_STATE (X of
 * another context, semiring or shape). */
dsg_status dsg_prod_scale_add(dsg_prod* p, const void* alpha, dsg_mat* X, const void* beta, dsg_mat** out);

/* Recompute every row of C from the current A and B (the static baseline),
 * consuming the pending changes.  flags: DSG_SYNC. */
dsg_status dsg_prod_recompute_static(dsg_prod* p, uint32_t flags);

/* Dynamic multiply: bring C up to date with all changes applied to A and B
 * since the previous update, recomputing only the affected rows: the changed
 * rows of A and every row i with A'[i,k] present for a changed row k of B.
 * *changed receives the rows whose stored content differs from before the
 * call (with DSG_REPORT_AFFECTED: every recomputed row).  Synchronises with
 * the device to learn the row count. */
dsg_status dsg_prod_update(dsg_prod* p, uint32_t flags, dsg_rows* changed);

/* Views of nq rows of C (rows: host int32 array, or device with
 * DSG_INPUT_DEVICE; any order, repeats allowed; out->rows lists them as
 * given).  C is kept as a dynamic matrix (Section 4; Section 6.1 keeps C' in
 * that form), so a row is read in place by its offset and length, without a
 * search.  The view points into C's storage: it holds until the next call
 * that changes C (an update, a static recompute) or the next dsg_prod_rows
 * on this product.  DSG_E_RANGE for a bad row. */
dsg_status dsg_prod_rows(dsg_prod* p, const int32_t* rows, int32_t nq, uint32_t flags,
                         dsg_rows* out);

/* Copy the rows of a view (from dsg_prod_update or dsg_prod_rows on this
 * product, still valid) to host CSR arrays in view order, each row sorted by
 * column: row_ptr[v->n + 1], col/val with room for cap entries.  With col ==
 * NULL only *nnz_out and row_ptr are written.  The rows are those of the
 * dynamic matrix C' (Sections 4 and 6.1); the host arrays are the plain CSR
 * of Section 4's static matrices.  DSG_E_ARG if cap < nnz; a view that no
 * longer holds is not detected. */
dsg_status dsg_rows_export(dsg_prod* p, const dsg_rows* v, int64_t* row_ptr, int32_t* col, void* val,
                           int64_t cap, int64_t* nnz_out);

/* The same export for callers that cannot allocate device memory (tight
 * serving loops, harnesses that forbid allocation): no hipMalloc, hipFree or
 * allocating library routine is called.  The device staging (row lengths,
 * offsets, gathered entries) lives in a fixed array of the library, one per
 * GPU, held from the first context on that GPU until the process ends.
 * Limits: at most 262,144 rows and 2,097,152 entries per call (DSG_E_ARG
 * beyond them; when the entry limit is what fails, *nnz_out and row_ptr are
 * still written); row_ptr and val are required whenever col is given.  Calls
 * on one GPU share its array and run one at a time (each returns after its
 * device work has finished). */
dsg_status dsg_rows_export_noalloc(dsg_prod* p, const dsg_rows* v, int64_t* row_ptr, int32_t* col, void* val,
                                   int64_t cap, int64_t* nnz_out);

/* nnz(C) (Section 3), as dsg_mat_nnz.  Synchronises with the device. */
dsg_status dsg_prod_nnz(dsg_prod* p, int64_t* nnz);
/* Canonical host CSR of C = op(A)·op(B) over the product's semiring
 * (Section 3), as dsg_mat_export: rows sorted by column, tombstones dropped.
 * row_ptr[nrows + 1]; col/val with room for cap entries; col == NULL writes
 * only row_ptr and *nnz_out.  DSG_E_ARG if cap < nnz. */
dsg_status dsg_prod_export(dsg_prod* p, int64_t* row_ptr, int32_t* col, void* val, int64_t cap,
                           int64_t* nnz_out);

/* Statistics of the last dsg_prod_update / recompute. */
typedef struct {
  int64_t affected_rows;
  int64_t changed_rows;
  int64_t a_entries;    /* sum over recomputed rows of nnz(A'[i,:]) */
  int64_t flops;        /* sum of semiring multiplications */
  int64_t nnz_new;      /* entries of the recomputed rows after the update */
  int64_t nnz_old;      /* entries of those rows before it */
  int64_t bin_rows[10]; /* rows per accumulator bin (8 group bins, dense, global hash) */
  int64_t bin_flops[10];
  int32_t path;         /* 0: affected rows recomputed; 1: entry-granular; 2: general updates with the
                           Bloom filter (affected_rows: rows of C*, entries: entries of C*, terms: terms
                           of the pattern, a_entries: columns of A' kept by the filter, flops: products
                           of the masked multiply tried or, in rows that probe, lookups of b'_kj;
                           bin_rows[0] / [1]: parts of rows of C* (a row's kept k in up to 32 parts;
                           fp64 rows whole) that walked rows of B' / probed them through B's column
                           index) */
  int32_t pad;
  int64_t terms;        /* entry-granular: changed products a_ik * b_kj enumerated */
  int64_t entries;      /* entry-granular: entries of C with changed products */
  int64_t lost;         /* entry-granular: entries recomputed because their best term got worse
                           (min-plus) or lost a contributor (plus-times) */
} dsg_update_stats;
dsg_status dsg_prod_stats(const dsg_prod* p, dsg_update_stats* s);

/* Autotuner: time `reps` full recomputes of C (same kernels as updates, all
 * rows) under each of a fixed set of candidate tunings (accumulator-bin
 * thresholds and the dense-versus-global-hash switch), keep the fastest as
 * the context's tuning and return it in *best with its median time in
 * *best_ms.  report (may be NULL) receives a JSON array of every candidate
 * and its time.  C is recomputed by every trial and ends equal to A·B;
 * pending changes of A and B are consumed as by dsg_prod_recompute_static. */
dsg_status dsg_prod_autotune(dsg_prod* p, int32_t reps, dsg_tuning* best, double* best_ms, char* report,
                             size_t cap);

/* DSG_E_STATE while a batched executor uses the product. */
dsg_status dsg_prod_destroy(dsg_prod* p);

/* ---- batched form: many independent products in one hipGraph replay ---- */

typedef struct dsg_batch dsg_batch;

/* The updates of one matrix inside a batched run: device arrays laid out as
 * for dsg_mat_apply with DSG_INPUT_DEVICE. */
typedef struct {
  dsg_mat* mat;
  const int32_t* rows;
  const int32_t* cols;
  const void* vals;
  const uint8_t* ops;
  int64_t n;
} dsg_update_set;

/* Create a batched executor over nprod products of ctx.  The products must
 * not share operands (each instance is independent): a product may name one
 * matrix as both operands (C = A A), but no matrix may belong to two entries
 * of the list, so neither two products over one matrix nor one product
 * listed twice are accepted (DSG_E_STATE).  The products and their operands
 * stay alive until dsg_batch_destroy. */
dsg_status dsg_batch_create(dsg_ctx* ctx, dsg_prod* const* prods, int32_t nprod, dsg_batch** out);

/* Apply nsets update sets (each to a distinct operand of one of the batch's
 * products) and bring every product up to date: the same C, row contents and
 * reported rows as dsg_mat_apply on each set followed by dsg_prod_update on
 * each product.  The chains (ingest, discovery, row recompute, merge) of
 * products whose C holds fewer than 2^batch_direct_log2 slots (tuning) are one hipGraph replay, with
 * one host round trip before it (validation of every set) and one after it
 * (results); the replay runs on a stream of its own while the products with a
 * larger C, and those with the Bloom matrix (DSG_GENERAL_BLOOM), take the
 * plain path (apply and update, with their round trips) on the context's
 * stream.  The graph is captured on the first run and replayed
 * while the set arrays, their sizes and the storage of every object it
 * touches stay the same (a run with other arrays or after storage grew
 * captures again).  Rows of C that find no room in C's pool or in the staging
 * space set aside write nothing during the replay; after it, the room grows
 * by exactly what they asked for and only those rows are recomputed, with the
 * same result.  changed_counts (host, nprod entries)
 * receives each product's reported row count; dsg_batch_rows gives the rows.
 * Errors: DSG_E_RANGE / DSG_E_ARG for a bad set (nothing is applied). */
dsg_status dsg_batch_run(dsg_batch* b, const dsg_update_set* sets, int32_t nsets, uint32_t flags,
                         int32_t* changed_counts);
/* Views of the rows product i reported in the last run (valid until the next
 * run or mutating call on that product). */
dsg_status dsg_batch_rows(dsg_batch* b, int32_t i, dsg_rows* out);
/* Counters and host-clock time totals of the runs so far. */
typedef struct {
  int64_t captures;   /* graph captures (first run, or after arrays or storage changed) */
  int64_t replays;
  int64_t deferred;   /* products with rows completed after the replay */
  double prepare_ms;  /* validation round trip and room reservation */
  double capture_ms;  /* capture and instantiation */
  double replay_ms;   /* launch until the results were read back (the direct products run meanwhile) */
  double finish_ms;   /* completion of rows that waited for room */
  int64_t direct;     /* product updates that took the plain path (a large C, or a Bloom matrix) */
  double direct_ms;   /* their time (apply and update), beside the replay */
} dsg_batch_stats;
dsg_status dsg_batch_info(const dsg_batch* b, dsg_batch_stats* out);
/* Free the batched form's graph and buffers; its products are untouched. */
dsg_status dsg_batch_destroy(dsg_batch* b);

/* ---- served form: a request loop over resident A, B and C ----
 *
 * A server owns a product (and its context) from dsg_server_create to
 * dsg_server_destroy and answers requests in arrival order, so every result
 * is the one the requests would get one at a time, in that order: an update
 * request is dsg_mat_apply of its entries followed by dsg_prod_update; a
 * query sees every update submitted before it and none submitted after it.
 * Inside, requests that arrive while others are on the device are admitted
 * as staging slots and memory free up (continuous batching): consecutive
 * update requests are merged into one batch in arrival order (the batch
 * semantics of dsg_mat_apply -- entries take effect in order -- make the
 * merged batch equal to the sequence), consecutive queries are answered by
 * one gather, and the host-to-device copy of the next group overlaps the
 * device work of the current one.  Memory admission: a group is admitted when
 * its estimated staging and workspace bytes fit the budget next to the groups
 * in flight (a group larger than the whole budget is admitted alone).
 * While a server lives, other calls on its context, matrices and products
 * return DSG_E_STATE; the server calls are thread safe. */
typedef struct dsg_server dsg_server;
typedef struct {
  size_t mem_budget;       /* bytes for in-flight groups; 0: 4 GiB */
  int64_t max_coalesce;    /* most update entries merged into one batch; 0: 1 << 20 */
  int32_t max_query_rows;  /* most rows gathered for one query group; 0: 65536 */
  int32_t slots;           /* groups staged or running at once, 1..8; 0: 2 */
} dsg_server_cfg;

#define DSG_PENDING (-1)
typedef struct {
  int32_t status;          /* DSG_PENDING, DSG_OK, or the error that ended the request */
  int32_t kind;            /* 0: update, 1: query */
  double latency_ms;       /* submission to completion (host clock) */
  int64_t group;           /* sequence number of the group that carried it */
  int32_t group_requests;  /* requests merged into that group */
  int32_t changed_rows;    /* update: rows of C the group changed */
  int32_t nq;              /* query: rows asked for */
  int64_t nnz;             /* query: entries of the answer */
} dsg_server_result;

typedef struct {
  int64_t update_requests, query_requests, update_entries;
  int64_t update_groups, query_groups;
  double update_p50_ms, update_p99_ms, update_mean_ms;
  double query_p50_ms, query_p99_ms, query_mean_ms;
  double busy_ms;           /* first submission to last completion */
  double updates_per_s;     /* update entries / busy_ms */
  size_t peak_inflight_bytes;
} dsg_server_stats;

/* cfg may be NULL (defaults).  The product must not be in a batched executor. */
dsg_status dsg_server_create(dsg_ctx* ctx, dsg_prod* p, const dsg_server_cfg* cfg, dsg_server** out);
/* Host arrays, as for dsg_mat_apply; copied before the call returns.  mat is
 * the product's A or B.  Bad indices or op codes: DSG_E_RANGE / DSG_E_ARG and
 * nothing is queued. */
dsg_status dsg_server_submit_update(dsg_server* s, dsg_mat* mat, const int32_t* rows, const int32_t* cols,
                                    const void* vals, const uint8_t* ops, int64_t n, uint64_t* ticket);
/* Host row ids (copied; repeats allowed).  DSG_E_RANGE for a bad row id. */
dsg_status dsg_server_submit_query(dsg_server* s, const int32_t* rows, int32_t nq, uint64_t* ticket);
/* State of a request; wait != 0 blocks until it completes. */
dsg_status dsg_server_poll(dsg_server* s, uint64_t ticket, int32_t wait, dsg_server_result* out);
/* Answer of a completed query: row_ptr[nq + 1] and, when col is not NULL, the
 * entries of each asked row sorted by column (cap entries of room; DSG_E_ARG
 * if fewer than the answer holds).  *nnz_out receives the entry count. */
dsg_status dsg_server_query_result(dsg_server* s, uint64_t ticket, int64_t* row_ptr, int32_t* col, void* val,
                                   int64_t cap, int64_t* nnz_out);
/* Forget a completed request (its answer is freed). */
dsg_status dsg_server_release(dsg_server* s, uint64_t ticket);
/* Block until every submitted request has completed. */
dsg_status dsg_server_drain(dsg_server* s);
dsg_status dsg_server_stats_get(dsg_server* s, dsg_server_stats* out);
/* Drains, stops the server and returns the context to the caller. */
dsg_status dsg_server_destroy(dsg_server* s);

#ifdef __cplusplus
}
#endif
#endif
