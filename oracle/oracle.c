/* CPU oracle for batch-dynamic SpGEMM -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain C, built with -O2 -ffp-contract=off -fno-fast-math so that every
 * fp64 product and sum is one IEEE-754 rounding, with no fused multiply-add.
 * Loaded only by the tests, the smoke check and the benchmark's CPU-baseline
 * leg; it shares no code with the GPU library.
 *
 * Readings of the paper that this file fixes (Section numbers of arXiv
 * 2202.08808):
 *  - absent entries equal the semiring's additive neutral element and present
 *    entries stay present whatever their value (Section 3);
 *  - SET on a present entry overwrites it, on an absent one inserts it (the
 *    "merge" procedure, Section 4.1); DELETE removes a present entry and is a
 *    no-op on an absent one ("mask", Section 4.1); ADD folds x into a present
 *    entry with the semiring's addition and inserts x where absent (algebraic
 *    update, Section 4.1 and Section 5);
 *  - a batch is the sequence of its updates applied in batch order, so
 *    repeated keys resolve last-one-wins with later ADDs folded on top;
 *  - a row is "changed" when its stored set of (column, value bits) differs;
 *  - C' = A' B' over the semiring (Section 5, problem statement): c_ij is
 *    present iff some k has both a_ik and b_kj present, and its value is the
 *    semiring sum over those k, taken in ascending k, of a_ik (x) b_kj;
 *  - (min,+) on fp32: (x) is the rounded fp32 sum; (+) is the minimum with
 *    -0 ordered below +0; (+,x) on int64 wraps around (two's complement);
 *  - the Boolean semiring (Section 3 lists (or, and)) on 32-bit words: (+)
 *    is bitwise or, (x) bitwise and, 0 the neutral element, so each bit is
 *    one Boolean semiring;
 *  - a transposed operand is the matrix with t_ji = a_ij (Section 3 allows
 *    either operand transposed; Section 5, "Handling Transposition");
 *  - C = alpha A B + beta X (Section 3) scales with the semiring's (x) and
 *    adds with its (+); an entry present in either term is present.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_value_size(int semiring) {
  switch (semiring) {
    case ORC_PLUS_TIMES_I64: return 8;
    case ORC_MIN_PLUS_F32: return 4;
    case ORC_PLUS_TIMES_F64: return 8;
    case ORC_OR_AND_U32: return 4;
    default: return 0;
  }
}

/* ---- semiring arithmetic (Section 3: semirings, neutral element) ---- */

static float mp_add(float a, float b) {
  if (a < b) return a;
  if (b < a) return b;
  return signbit(a) ? a : b; /* equal: prefer -0 over +0, else either */
}

/* dst <- x (+) y */
static void sr_add(int sr, void* dst, const void* x, const void* y) {
  if (sr == ORC_PLUS_TIMES_I64) {
    uint64_t a, b, r;
    memcpy(&a, x, 8); memcpy(&b, y, 8);
    r = a + b;
    memcpy(dst, &r, 8);
  } else if (sr == ORC_MIN_PLUS_F32) {
    float a, b, r;
    memcpy(&a, x, 4); memcpy(&b, y, 4);
    r = mp_add(a, b);
    memcpy(dst, &r, 4);
  } else if (sr == ORC_OR_AND_U32) {
    uint32_t a, b, r;
    memcpy(&a, x, 4); memcpy(&b, y, 4);
    r = a | b;
    memcpy(dst, &r, 4);
  } else {
    double a, b, r;
    memcpy(&a, x, 8); memcpy(&b, y, 8);
    r = a + b;
    memcpy(dst, &r, 8);
  }
}

/* dst <- x (x) y */
static void sr_mul(int sr, void* dst, const void* x, const void* y) {
  if (sr == ORC_PLUS_TIMES_I64) {
    uint64_t a, b, r;
    memcpy(&a, x, 8); memcpy(&b, y, 8);
    r = a * b;
    memcpy(dst, &r, 8);
  } else if (sr == ORC_MIN_PLUS_F32) {
    float a, b, r;
    memcpy(&a, x, 4); memcpy(&b, y, 4);
    r = a + b;
    memcpy(dst, &r, 4);
  } else if (sr == ORC_OR_AND_U32) {
    uint32_t a, b, r;
    memcpy(&a, x, 4); memcpy(&b, y, 4);
    r = a & b;
    memcpy(dst, &r, 4);
  } else {
    double a, b, r;
    memcpy(&a, x, 8); memcpy(&b, y, 8);
    r = a * b;
    memcpy(dst, &r, 8);
  }
}

/* ---- updates (Section 4.1) ---- */

/* first position in cols[0..len) whose column is >= c */
static int64_t lower_bound(const int32_t* cols, int64_t len, int32_t c) {
  int64_t lo = 0, hi = len;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (cols[mid] < c) lo = mid + 1; else hi = mid;
  }
  return lo;
}

int64_t orc_apply(int sr, int32_t nrows, int32_t ncols,
                  const int64_t* rp, const int32_t* ci, const void* v,
                  const int32_t* brow, const int32_t* bcol, const void* bval,
                  const uint8_t* bop, int64_t b,
                  int64_t* orp, int32_t* oci, void* ov, uint8_t* changed) {
  const int vs = orc_value_size(sr);
  if (vs == 0 || nrows < 0 || ncols < 0 || b < 0) return -1;
  for (int64_t t = 0; t < b; ++t) {
    if (brow[t] < 0 || brow[t] >= nrows || bcol[t] < 0 || bcol[t] >= ncols) return -1;
    if (bop[t] > ORC_OP_ADD) return -1;
  }
  /* The updates of one row, in batch order: rows do not interact, so applying
   * each row's updates in their batch order is the sequential application. */
  int64_t* first = (int64_t*)calloc((size_t)nrows + 1, sizeof(int64_t));
  int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(b > 0 ? b : 1));
  for (int64_t t = 0; t < b; ++t) first[brow[t] + 1]++;
  for (int32_t i = 0; i < nrows; ++i) first[i + 1] += first[i];
  {
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ((size_t)nrows + 1));
    memcpy(fill, first, sizeof(int64_t) * ((size_t)nrows + 1));
    for (int64_t t = 0; t < b; ++t) order[fill[brow[t]]++] = t;
    free(fill);
  }
  const char* vin = (const char*)v;
  const char* bv = (const char*)bval;
  char* vout = (char*)ov;
  int64_t maxrow = 0;
  for (int32_t i = 0; i < nrows; ++i) {
    int64_t need = rp[i + 1] - rp[i] + (first[i + 1] - first[i]);
    if (need > maxrow) maxrow = need;
  }
  int32_t* wc = (int32_t*)malloc(sizeof(int32_t) * (size_t)(maxrow > 0 ? maxrow : 1));
  char* wv = (char*)malloc((size_t)vs * (size_t)(maxrow > 0 ? maxrow : 1));
  int64_t out = 0;
  orp[0] = 0;
  for (int32_t i = 0; i < nrows; ++i) {
    int64_t len0 = rp[i + 1] - rp[i];
    int64_t len = len0;
    memcpy(wc, ci + rp[i], sizeof(int32_t) * (size_t)len);
    memcpy(wv, vin + (size_t)vs * (size_t)rp[i], (size_t)vs * (size_t)len);
    for (int64_t u = first[i]; u < first[i + 1]; ++u) {
      int64_t t = order[u];
      int32_t c = bcol[t];
      const char* x = bv + (size_t)vs * (size_t)t;
      int64_t pos = lower_bound(wc, len, c);
      int present = pos < len && wc[pos] == c;
      if (bop[t] == ORC_OP_DELETE) {
        if (present) {
          memmove(wc + pos, wc + pos + 1, sizeof(int32_t) * (size_t)(len - pos - 1));
          memmove(wv + (size_t)vs * pos, wv + (size_t)vs * (pos + 1), (size_t)vs * (size_t)(len - pos - 1));
          --len;
        }
      } else if (present) {
        if (bop[t] == ORC_OP_SET) memcpy(wv + (size_t)vs * pos, x, (size_t)vs);
        else sr_add(sr, wv + (size_t)vs * pos, wv + (size_t)vs * pos, x);
      } else { /* SET or ADD on an absent entry inserts x */
        memmove(wc + pos + 1, wc + pos, sizeof(int32_t) * (size_t)(len - pos));
        memmove(wv + (size_t)vs * (pos + 1), wv + (size_t)vs * pos, (size_t)vs * (size_t)(len - pos));
        wc[pos] = c;
        memcpy(wv + (size_t)vs * pos, x, (size_t)vs);
        ++len;
      }
    }
    if (changed) {
      int diff = len != len0;
      if (!diff) diff = memcmp(wc, ci + rp[i], sizeof(int32_t) * (size_t)len) != 0;
      if (!diff) diff = memcmp(wv, vin + (size_t)vs * (size_t)rp[i], (size_t)vs * (size_t)len) != 0;
      changed[i] = (uint8_t)diff;
    }
    memcpy(oci + out, wc, sizeof(int32_t) * (size_t)len);
    memcpy(vout + (size_t)vs * (size_t)out, wv, (size_t)vs * (size_t)len);
    out += len;
    orp[i + 1] = out;
  }
  free(wc); free(wv); free(order); free(first);
  return out;
}

/* ---- Gustavson product (Section 5 problem statement; Section 6.1) ---- */

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

typedef struct {
  int64_t* mark;   /* mark[j] == q  <=>  column j already touched for output row q */
  char* acc;       /* dense accumulator, one value per column */
  int32_t* touched;
} spa_t;

static int spa_init(spa_t* s, int32_t ncols, int vs) {
  size_t n = (size_t)(ncols > 0 ? ncols : 1);
  s->mark = (int64_t*)malloc(sizeof(int64_t) * n);
  s->acc = (char*)malloc((size_t)vs * n);
  s->touched = (int32_t*)malloc(sizeof(int32_t) * n);
  if (!s->mark || !s->acc || !s->touched) return -1;
  for (size_t j = 0; j < n; ++j) s->mark[j] = -1;
  return 0;
}

static void spa_free(spa_t* s) { free(s->mark); free(s->acc); free(s->touched); }

/* Accumulate output row q (= row i of A times B) into the SPA; returns the
 * number of touched columns, sorted ascending in s->touched. */
static int64_t gustavson_row(int sr, int vs, int64_t q, int32_t i,
                             const int64_t* arp, const int32_t* aci, const char* av,
                             const int64_t* brp, const int32_t* bci, const char* bv,
                             spa_t* s) {
  int64_t nt = 0;
  char p[8];
  for (int64_t ea = arp[i]; ea < arp[i + 1]; ++ea) {     /* ascending k */
    int32_t k = aci[ea];
    const char* a = av + (size_t)vs * (size_t)ea;
    for (int64_t eb = brp[k]; eb < brp[k + 1]; ++eb) {   /* ascending j */
      int32_t j = bci[eb];
      char* slot = s->acc + (size_t)vs * (size_t)j;
      sr_mul(sr, p, a, bv + (size_t)vs * (size_t)eb);
      if (s->mark[j] != q) {
        s->mark[j] = q;
        memcpy(slot, p, (size_t)vs);
        s->touched[nt++] = j;
      } else {
        sr_add(sr, slot, slot, p);
      }
    }
  }
  qsort(s->touched, (size_t)nt, sizeof(int32_t), cmp_i32);
  return nt;
}

int orc_spgemm(int sr, int32_t nrows, int32_t ninner, int32_t ncols,
               const int64_t* arp, const int32_t* aci, const void* av,
               const int64_t* brp, const int32_t* bci, const void* bv,
               const int32_t* rows, int32_t nq,
               int64_t* crp, int32_t* cci, void* cv, int nthreads) {
  const int vs = orc_value_size(sr);
  (void)ninner;
  if (vs == 0 || nrows < 0 || ncols < 0) return -1;
  const int64_t nout = rows ? nq : nrows;
  if (rows)
    for (int32_t q = 0; q < nq; ++q)
      if (rows[q] < 0 || rows[q] >= nrows) return -1;
  const int numeric = (cci != NULL || cv != NULL);
  int bad = 0;
#ifdef _OPENMP
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
#endif
  {
    spa_t s;
    if (spa_init(&s, ncols, vs) != 0) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
      bad = 1;
    } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
      for (int64_t q = 0; q < nout; ++q) {
        int32_t i = rows ? rows[q] : (int32_t)q;
        int64_t nt = gustavson_row(sr, vs, q, i, arp, aci, (const char*)av, brp, bci,
                                   (const char*)bv, &s);
        if (!numeric) {
          crp[q + 1] = nt;
        } else {
          int64_t o = crp[q];
          for (int64_t t = 0; t < nt; ++t) {
            int32_t j = s.touched[t];
            cci[o + t] = j;
            memcpy((char*)cv + (size_t)vs * (size_t)(o + t), s.acc + (size_t)vs * (size_t)j,
                   (size_t)vs);
          }
        }
      }
    }
    spa_free(&s);
  }
  if (bad) return -1;
  if (!numeric) {
    crp[0] = 0;
    for (int64_t q = 0; q < nout; ++q) crp[q + 1] += crp[q];
  }
  return 0;
}

/* ---- transposition (Section 3; Section 5, "Handling Transposition") ---- */

int64_t orc_transpose(int32_t nrows, int32_t ncols, int vs,
                      const int64_t* rp, const int32_t* ci, const void* v,
                      int64_t* trp, int32_t* tci, void* tv) {
  if (nrows < 0 || ncols < 0 || vs <= 0) return -1;
  const int64_t nnz = rp[nrows];
  for (int64_t e = 0; e < nnz; ++e)
    if (ci[e] < 0 || ci[e] >= ncols) return -1;
  /* row j of T holds the entries of column j of A: count them ... */
  for (int32_t j = 0; j <= ncols; ++j) trp[j] = 0;
  for (int64_t e = 0; e < nnz; ++e) trp[ci[e] + 1]++;
  for (int32_t j = 0; j < ncols; ++j) trp[j + 1] += trp[j];
  /* ... then place a_ij at t_ji, visiting i in ascending order so that each
   * row of T comes out sorted by its column i */
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ((size_t)ncols + 1));
  memcpy(fill, trp, sizeof(int64_t) * ((size_t)ncols + 1));
  for (int32_t i = 0; i < nrows; ++i) {
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      int64_t o = fill[ci[e]]++;
      tci[o] = i;
      memcpy((char*)tv + (size_t)vs * (size_t)o, (const char*)v + (size_t)vs * (size_t)e, (size_t)vs);
    }
  }
  free(fill);
  return nnz;
}

/* ---- C = alpha A B + beta X (Section 3) ---- */

int64_t orc_axpby(int sr, int32_t nrows, const void* alpha,
                  const int64_t* crp, const int32_t* cci, const void* cv,
                  const void* beta, const int64_t* xrp, const int32_t* xci, const void* xv,
                  int64_t* drp, int32_t* dci, void* dv) {
  const int vs = orc_value_size(sr);
  if (vs == 0 || nrows < 0) return -1;
  char t1[8], t2[8];
  int64_t out = 0;
  drp[0] = 0;
  for (int32_t i = 0; i < nrows; ++i) {
    /* walk the two sorted rows together */
    int64_t a = crp[i], b = xrp[i];
    while (a < crp[i + 1] || b < xrp[i + 1]) {
      const int take_c = a < crp[i + 1] && (b >= xrp[i + 1] || cci[a] <= xci[b]);
      const int take_x = b < xrp[i + 1] && (a >= crp[i + 1] || xci[b] <= cci[a]);
      char* d = (char*)dv + (size_t)vs * (size_t)out;
      if (take_c && take_x) {
        sr_mul(sr, t1, alpha, (const char*)cv + (size_t)vs * (size_t)a);
        sr_mul(sr, t2, beta, (const char*)xv + (size_t)vs * (size_t)b);
        sr_add(sr, d, t1, t2);
        dci[out] = cci[a];
        ++a; ++b;
      } else if (take_c) {
        sr_mul(sr, d, alpha, (const char*)cv + (size_t)vs * (size_t)a);
        dci[out] = cci[a];
        ++a;
      } else {
        sr_mul(sr, d, beta, (const char*)xv + (size_t)vs * (size_t)b);
        dci[out] = xci[b];
        ++b;
      }
      ++out;
    }
    drp[i + 1] = out;
  }
  return out;
}

/* ---- general updates filtered by a Bloom matrix (Section 5.2, Algorithm 2)
 *
 * One process holds every block, so the algorithm's broadcasts, sends and
 * aggregations over the process grid are the identity here; what remains is
 * its local arithmetic, step by step in the algorithm's order:
 *   computePattern   C* = A* B' + A B* (Eq. 1) as a structure, and F* with
 *                    bit (k mod l) of f*_ij set when a*_ik b'_kj or
 *                    a'_ik b*_kj is a term of c*_ij;
 *   E                F (+) F* (bitwise or), masked at C*;
 *   R                the bitwise or of E over each row;
 *   A^R              A' keeping, in row i, the columns k with bit (k mod l)
 *                    of r_i set;
 *   Z, H             A^R B' masked at C*: for (i,j) in C*, z_ij is the
 *                    semiring sum over those k (ascending) with b'_kj present
 *                    and h_ij the Bloom bits of those k;
 *   merge            C' = C outside C*, z_ij on C* where some term exists,
 *                    no entry where none does; F' likewise from F and H.
 * F is the Bloom matrix of C = A B: on C's structure, bit (k mod l) of f_ij
 * is set iff a_ik and b_kj are both present.  l = 64, the width the paper
 * uses.  A* (and B*) mark the changed entries: present in exactly one of A
 * and A', or in both with different value bits (deletions included). */

#define ORC_BLOOM_L 64

static uint64_t bloom_bit(int32_t k) { return (uint64_t)1 << ((uint32_t)k % ORC_BLOOM_L); }

/* Structure of the changed entries between two sorted CSR matrices of the
 * same shape (values of vs bytes).  Two phases as orc_spgemm: srp only when
 * sci == NULL, then sci. */
int orc_changed_entries(int32_t nrows, int vs,
                        const int64_t* rp, const int32_t* ci, const void* v,
                        const int64_t* rp2, const int32_t* ci2, const void* v2,
                        int64_t* srp, int32_t* sci) {
  if (nrows < 0 || vs <= 0) return -1;
  if (sci == NULL) srp[0] = 0;
  for (int32_t i = 0; i < nrows; ++i) {
    int64_t a = rp[i], b = rp2[i], n = 0;
    while (a < rp[i + 1] || b < rp2[i + 1]) {
      int32_t j;
      int changed;
      if (b >= rp2[i + 1] || (a < rp[i + 1] && ci[a] < ci2[b])) {
        j = ci[a++]; changed = 1;                           /* deleted */
      } else if (a >= rp[i + 1] || ci2[b] < ci[a]) {
        j = ci2[b++]; changed = 1;                          /* inserted */
      } else {
        j = ci[a];                                          /* in both: compare value bits */
        changed = memcmp((const char*)v + (size_t)vs * (size_t)a,
                         (const char*)v2 + (size_t)vs * (size_t)b, (size_t)vs) != 0;
        ++a; ++b;
      }
      if (!changed) continue;
      if (sci) sci[srp[i] + n] = j;
      ++n;
    }
    if (sci == NULL) srp[i + 1] = srp[i] + n;
  }
  return 0;
}

/* Bloom matrix F of C = A B (structures only): frp / fci are C's structure,
 * fv[e] the bits of the k's contributing to that entry.  Two phases. */
int orc_bloom(int32_t nrows, int32_t ncols,
              const int64_t* arp, const int32_t* aci, const int64_t* brp, const int32_t* bci,
              int64_t* frp, int32_t* fci, uint64_t* fv) {
  if (nrows < 0 || ncols < 0) return -1;
  size_t nc = (size_t)(ncols > 0 ? ncols : 1);
  int32_t* mark = (int32_t*)malloc(sizeof(int32_t) * nc);
  uint64_t* bits = (uint64_t*)malloc(sizeof(uint64_t) * nc);
  int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * nc);
  if (!mark || !bits || !touched) { free(mark); free(bits); free(touched); return -1; }
  for (size_t j = 0; j < nc; ++j) mark[j] = -1;
  if (fci == NULL) frp[0] = 0;
  for (int32_t i = 0; i < nrows; ++i) {
    int64_t nt = 0;
    for (int64_t ea = arp[i]; ea < arp[i + 1]; ++ea) {
      int32_t k = aci[ea];
      for (int64_t eb = brp[k]; eb < brp[k + 1]; ++eb) {
        int32_t j = bci[eb];
        if (mark[j] != i) { mark[j] = i; bits[j] = 0; touched[nt++] = j; }
        bits[j] |= bloom_bit(k);
      }
    }
    qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
    if (fci == NULL) {
      frp[i + 1] = frp[i] + nt;
    } else {
      for (int64_t t = 0; t < nt; ++t) {
        fci[frp[i] + t] = touched[t];
        fv[frp[i] + t] = bits[touched[t]];
      }
    }
  }
  free(mark); free(bits); free(touched);
  return 0;
}

/* computePattern: C* = A* B' + A B* as a structure, with F* (see above).
 * A, A*, A' are nrows x ninner, B', B* ninner x ncols, all structures sorted
 * by column.  Output: C* (csrp, csci) and fs[e] = f*_ij.  Two phases. */
int orc_pattern(int32_t nrows, int32_t ncols,
                const int64_t* arp, const int32_t* aci,       /* A  */
                const int64_t* asrp, const int32_t* asci,     /* A* */
                const int64_t* a2rp, const int32_t* a2ci,     /* A' */
                const int64_t* bsrp, const int32_t* bsci,     /* B* */
                const int64_t* b2rp, const int32_t* b2ci,     /* B' */
                int64_t* csrp, int32_t* csci, uint64_t* fs) {
  if (nrows < 0 || ncols < 0) return -1;
  size_t nc = (size_t)(ncols > 0 ? ncols : 1);
  int32_t* mark = (int32_t*)malloc(sizeof(int32_t) * nc);   /* j holds an entry of C* in row i */
  int32_t* seen = (int32_t*)malloc(sizeof(int32_t) * nc);   /* bits[j] belongs to row i */
  uint64_t* bits = (uint64_t*)malloc(sizeof(uint64_t) * nc);
  int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * nc);
  if (!mark || !seen || !bits || !touched) { free(mark); free(seen); free(bits); free(touched); return -1; }
  for (size_t j = 0; j < nc; ++j) mark[j] = seen[j] = -1;
  if (csci == NULL) csrp[0] = 0;
  for (int32_t i = 0; i < nrows; ++i) {
    int64_t nt = 0;
#define ORC_BITS(j, k) do { if (seen[j] != i) { seen[j] = i; bits[j] = 0; } bits[j] |= bloom_bit(k); } while (0)
    /* A* B': pattern and bits */
    for (int64_t e = asrp[i]; e < asrp[i + 1]; ++e) {
      int32_t k = asci[e];
      for (int64_t f = b2rp[k]; f < b2rp[k + 1]; ++f) {
        int32_t j = b2ci[f];
        if (mark[j] != i) { mark[j] = i; touched[nt++] = j; }
        ORC_BITS(j, k);
      }
    }
    /* A B*: pattern */
    for (int64_t e = arp[i]; e < arp[i + 1]; ++e) {
      int32_t k = aci[e];
      for (int64_t f = bsrp[k]; f < bsrp[k + 1]; ++f) {
        int32_t j = bsci[f];
        if (mark[j] != i) { mark[j] = i; touched[nt++] = j; }
      }
    }
    /* A' B*: bits */
    for (int64_t e = a2rp[i]; e < a2rp[i + 1]; ++e) {
      int32_t k = a2ci[e];
      for (int64_t f = bsrp[k]; f < bsrp[k + 1]; ++f) ORC_BITS(bsci[f], k);
    }
#undef ORC_BITS
    qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
    if (csci == NULL) {
      csrp[i + 1] = csrp[i] + nt;
    } else {
      for (int64_t t = 0; t < nt; ++t) {
        int32_t j = touched[t];
        csci[csrp[i] + t] = j;
        fs[csrp[i] + t] = seen[j] == i ? bits[j] : 0;
      }
    }
  }
  free(mark); free(seen); free(bits); free(touched);
  return 0;
}

/* E and R: r_i = bitwise or over (i, j) in C* of f_ij | f*_ij, with f_ij = 0
 * where C (structure frp / fci, bits fv) has no entry (i, j). */
int orc_row_filter(int32_t nrows,
                   const int64_t* csrp, const int32_t* csci, const uint64_t* fs,
                   const int64_t* frp, const int32_t* fci, const uint64_t* fv,
                   uint64_t* r) {
  if (nrows < 0) return -1;
  for (int32_t i = 0; i < nrows; ++i) {
    uint64_t acc = 0;
    int64_t f = frp[i];
    for (int64_t e = csrp[i]; e < csrp[i + 1]; ++e) {
      const int32_t j = csci[e];
      uint64_t x = fs[e];                                   /* f*_ij */
      while (f < frp[i + 1] && fci[f] < j) ++f;
      if (f < frp[i + 1] && fci[f] == j) x |= fv[f];        /* f_ij */
      acc |= x;                                             /* e_ij into r_i */
    }
    r[i] = acc;
  }
  return 0;
}

/* Z and H: A^R B' masked at C*.  For every entry e = (i, j) of C*: zp[e] = 1
 * and zv[e] = the semiring sum, over k ascending in A' row i with bit
 * (k mod l) of r_i set and b'_kj present, of a'_ik (x) b'_kj, and hv[e] the
 * bits of those k; zp[e] = 0 and hv[e] = 0 where there is no such k. */
int orc_masked_product(int sr, int32_t nrows, int32_t ncols,
                       const int64_t* a2rp, const int32_t* a2ci, const void* a2v, const uint64_t* r,
                       const int64_t* b2rp, const int32_t* b2ci, const void* b2v,
                       const int64_t* csrp, const int32_t* csci,
                       void* zv, uint8_t* zp, uint64_t* hv) {
  const int vs = orc_value_size(sr);
  if (vs == 0 || nrows < 0 || ncols < 0) return -1;
  size_t nc = (size_t)(ncols > 0 ? ncols : 1);
  int64_t* where = (int64_t*)malloc(sizeof(int64_t) * nc);  /* position in C* of (i, j), or -1 */
  if (!where) return -1;
  for (size_t j = 0; j < nc; ++j) where[j] = -1;
  char p[8];
  for (int32_t i = 0; i < nrows; ++i) {
    for (int64_t e = csrp[i]; e < csrp[i + 1]; ++e) {
      where[csci[e]] = e;
      zp[e] = 0;
      hv[e] = 0;
    }
    for (int64_t ea = a2rp[i]; ea < a2rp[i + 1]; ++ea) {    /* ascending k */
      const int32_t k = a2ci[ea];
      if (!(r[i] & bloom_bit(k))) continue;                 /* not in A^R */
      const char* a = (const char*)a2v + (size_t)vs * (size_t)ea;
      for (int64_t eb = b2rp[k]; eb < b2rp[k + 1]; ++eb) {
        const int64_t e = where[b2ci[eb]];
        if (e < 0) continue;                                /* masked out */
        char* z = (char*)zv + (size_t)vs * (size_t)e;
        sr_mul(sr, p, a, (const char*)b2v + (size_t)vs * (size_t)eb);
        if (!zp[e]) { memcpy(z, p, (size_t)vs); zp[e] = 1; }
        else sr_add(sr, z, z, p);
        hv[e] |= bloom_bit(k);
      }
    }
    for (int64_t e = csrp[i]; e < csrp[i + 1]; ++e) where[csci[e]] = -1;
  }
  free(where);
  return 0;
}

/* Merge masked at C*: out = X outside C*; on C*, the entry z (present where
 * zp) and no entry where !zp.  X: sorted CSR with values of vs bytes.  Two
 * phases (orp only when oci == NULL). */
int orc_masked_merge(int32_t nrows, int vs,
                     const int64_t* xrp, const int32_t* xci, const void* xv,
                     const int64_t* csrp, const int32_t* csci, const void* zv, const uint8_t* zp,
                     int64_t* orp, int32_t* oci, void* ov) {
  if (nrows < 0 || vs <= 0) return -1;
  if (oci == NULL) orp[0] = 0;
  for (int32_t i = 0; i < nrows; ++i) {
    int64_t a = xrp[i], b = csrp[i], n = 0;
    while (a < xrp[i + 1] || b < csrp[i + 1]) {
      const void* src = NULL;
      int32_t j;
      if (b >= csrp[i + 1] || (a < xrp[i + 1] && xci[a] < csci[b])) {
        j = xci[a]; src = (const char*)xv + (size_t)vs * (size_t)a; ++a;     /* outside C*: kept */
      } else {
        j = csci[b];
        if (zp[b]) src = (const char*)zv + (size_t)vs * (size_t)b;         /* on C*: z, or nothing */
        if (a < xrp[i + 1] && xci[a] == j) ++a;
        ++b;
      }
      if (!src) continue;
      if (oci) {
        oci[orp[i] + n] = j;
        memcpy((char*)ov + (size_t)vs * (size_t)(orp[i] + n), src, (size_t)vs);
      }
      ++n;
    }
    if (oci == NULL) orp[i + 1] = orp[i] + n;
  }
  return 0;
}
