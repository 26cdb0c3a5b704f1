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
 *     accumulator (Section 6.1 names Gustavson's algorithm);
 *   - the Boolean (or, and) semiring that Section 3 lists, applied bitwise to
 *     32-bit words (32 Boolean semirings side by side; values 0/1 give the
 *     plain Boolean product);
 *   - transposed operands and C = alpha A B + beta X, the general form of the
 *     problem in Section 3 (transposition: Section 5, "Handling
 *     Transposition").
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

enum { ORC_PLUS_TIMES_I64 = 0, ORC_MIN_PLUS_F32 = 1, ORC_PLUS_TIMES_F64 = 2, ORC_OR_AND_U32 = 3 };
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

/* Transpose: T = A^T, t_ji = a_ij, for the sorted CSR A (nrows x ncols) with
 * values of vs bytes.  T is ncols x nrows: trp[ncols+1], tci / tv with room
 * for nnz(A) entries, each row sorted by column.  Returns nnz, or -1 on bad
 * arguments. */
int64_t orc_transpose(int32_t nrows, int32_t ncols, int vs,
                      const int64_t* rp, const int32_t* ci, const void* v,
                      int64_t* trp, int32_t* tci, void* tv);

/* D = (alpha (x) C) (+) (beta (x) X), entry by entry, for C and X of the same
 * shape (Section 3: C = alpha A B + beta X with the product in place of A B).
 * D holds an entry wherever C or X does: alpha (x) c where only C has one,
 * beta (x) x where only X has one, (alpha (x) c) (+) (beta (x) x) where
 * both do (an absent entry is the neutral element, which (x) maps to itself
 * and (+) ignores).  alpha and beta point to one value each.  Output:
 * drp[nrows+1], dci / dv with room for nnz(C) + nnz(X).  Returns nnz(D), or
 * -1 on bad arguments. */
int64_t orc_axpby(int semiring, int32_t nrows, const void* alpha,
                  const int64_t* crp, const int32_t* cci, const void* cv,
                  const void* beta, const int64_t* xrp, const int32_t* xci, const void* xv,
                  int64_t* drp, int32_t* dci, void* dv);

/* ---- general updates filtered by a Bloom matrix (Section 5.2, Algorithm 2)
 * on one process: the steps of the algorithm in its order, each on sorted
 * CSR structures.  l = 64 (bit k mod 64 stands for column / row k).  Every
 * two-phase function fills the row pointers when its column output is NULL
 * and the columns (and values) on a second call. */

/* A*: entries present in exactly one of A and A', or in both with different
 * value bits (vs bytes per value). */
int orc_changed_entries(int32_t nrows, int vs,
                        const int64_t* rp, const int32_t* ci, const void* v,
                        const int64_t* rp2, const int32_t* ci2, const void* v2,
                        int64_t* srp, int32_t* sci);

/* F, the Bloom matrix of C = A B: C's structure, and for each entry the bits
 * (k mod 64) of the k with a_ik and b_kj present. */
int orc_bloom(int32_t nrows, int32_t ncols,
              const int64_t* arp, const int32_t* aci, const int64_t* brp, const int32_t* bci,
              int64_t* frp, int32_t* fci, uint64_t* fv);

/* computePattern: C* = A* B' + A B* (Eq. 1) as a structure; fs[e] = f*_ij,
 * the bits of the k with a*_ik b'_kj or a'_ik b*_kj present. */
int orc_pattern(int32_t nrows, int32_t ncols,
                const int64_t* arp, const int32_t* aci, const int64_t* asrp, const int32_t* asci,
                const int64_t* a2rp, const int32_t* a2ci, const int64_t* bsrp, const int32_t* bsci,
                const int64_t* b2rp, const int32_t* b2ci,
                int64_t* csrp, int32_t* csci, uint64_t* fs);

/* E = (F | F*) masked at C*, and r_i = bitwise or of row i of E. */
int orc_row_filter(int32_t nrows, const int64_t* csrp, const int32_t* csci, const uint64_t* fs,
                   const int64_t* frp, const int32_t* fci, const uint64_t* fv, uint64_t* r);

/* Z, H = A^R B' masked at C*: per entry of C*, the semiring sum (ascending k)
 * over the k of A' row i whose bit is in r_i, with b'_kj present (zv, zp = 1
 * when there is one) and the bits of those k (hv). */
int orc_masked_product(int sr, int32_t nrows, int32_t ncols,
                       const int64_t* a2rp, const int32_t* a2ci, const void* a2v, const uint64_t* r,
                       const int64_t* b2rp, const int32_t* b2ci, const void* b2v,
                       const int64_t* csrp, const int32_t* csci,
                       void* zv, uint8_t* zp, uint64_t* hv);

/* Merge masked at C*: X outside C*; z where zp, nothing where !zp, on C*. */
int orc_masked_merge(int32_t nrows, int vs,
                     const int64_t* xrp, const int32_t* xci, const void* xv,
                     const int64_t* csrp, const int32_t* csci, const void* zv, const uint8_t* zp,
                     int64_t* orp, int32_t* oci, void* ov);

#ifdef __cplusplus
}
#endif
#endif
