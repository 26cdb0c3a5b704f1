/* CPU oracle for batch-dynamic SpGEMM -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct reference for what the GPU library
 * computes.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code with the GPU path.
 *
 * What it computes (Fast Dynamic Updates and Dynamic SpGEMM on MPI-Distributed
 * Graphs, arXiv 2202.08808):
 *   - matrices over a semiring whose additive neutral element is the implicit
 *     value of every absent entry; a present entry is a structural non-zero
 *     even if its value equals that element (Section 3);
 *   - update semantics insert/change ("merge"), delete ("mask") and algebraic
 *     add, applied one by one in batch order (Section 4.1);
 *   - the dynamic product's defining result C' = A' B' (Section 5, problem
 *     statement), computed from scratch with row-wise Gustavson and a dense
 *     accumulator (Section 6.1 names Gustavson's algorithm).
 *
 * Matrices are CSR with each row sorted by column and no duplicate keys.
 * Pins: dense brute force, 2-walk enumeration, scipy, closed forms and
 * invariants, all in the CPU tests.
 */
#ifndef DSG_ORACLE_H
#define DSG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_PLUS_TIMES_I64 = 0, ORC_MIN_PLUS_F32 = 1, ORC_PLUS_TIMES_F64 = 2 };
enum { ORC_OP_SET = 0, ORC_OP_DELETE = 1, ORC_OP_ADD = 2 };

/* Value size in bytes of a semiring, or 0 for an unknown id. */
int orc_value_size(int semiring);

/* Apply a batch of b updates to the sorted CSR (rp, ci, v) of shape
 * nrows x ncols, strictly one update after the other in batch order.
 *   SET    : overwrite if present, else insert          (merge)
 *   DELETE : remove if present, else nothing            (mask)
 *   ADD    : v <- v (+) x if present, else insert x     (algebraic)
 * Output: sorted CSR (orp[nrows+1], oci, ov) with capacity nnz_in + b;
 * changed[nrows] (may be NULL) is set to 1 for every row whose stored content
 * (set of column/value-bit pairs) differs from before, else 0.
 * Returns nnz_out, or -1 if an index is out of range or an op is unknown
 * (the output is then undefined). */
int64_t orc_apply(int semiring, int32_t nrows, int32_t ncols,
                  const int64_t* rp, const int32_t* ci, const void* v,
                  const int32_t* brow, const int32_t* bcol, const void* bval,
                  const uint8_t* bop, int64_t b,
                  int64_t* orp, int32_t* oci, void* ov, uint8_t* changed);

/* Row-wise Gustavson C = A (x) B, A nrows x ninner, B ninner x ncols.
 * rows == NULL: every row of A, output row q is row q of C;
 * else the nq listed rows, output row q is row rows[q] of C.
 * Phase 1 (cv == NULL and cci == NULL): fills crp[nq+1] with row pointers.
 * Phase 2: fills cci / cv from crp.  Output rows are sorted by column.
 * nthreads <= 1 runs single-threaded, else an OpenMP loop over rows.
 * Returns 0, or -1 on bad arguments. */
int orc_spgemm(int semiring, int32_t nrows, int32_t ninner, int32_t ncols,
               const int64_t* arp, const int32_t* aci, const void* av,
               const int64_t* brp, const int32_t* bci, const void* bv,
               const int32_t* rows, int32_t nq,
               int64_t* crp, int32_t* cci, void* cv, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
