// D = (alpha (x) C) (+) (beta (x) X) for a product's C: Section 3 states the
// SpGEMM problem as C = alpha A B + beta X, with the maintained product in
// place of A B here.
//
// D starts as C's rows in canonical order with every value multiplied by
// alpha.  X's entries, multiplied by beta, are then applied to D as
// algebraic additions (Section 4.1): where D holds the column, the two
// values are combined with the semiring's addition; elsewhere the entry is
// inserted.  That is the entrywise sum over the union of the two structures,
// an absent entry being the neutral element.
#include <algorithm>
#include <cstring>

#include "internal.h"
#include "kernel_common.h"

namespace {

template <int SR>
__global__ void k_scale(int64_t n, typename Sem<SR>::V* val, uint64_t sbits) {
  using S = Sem<SR>;
  using V = typename S::V;
  V s;
  if constexpr (sizeof(V) == 8) s = __builtin_bit_cast(V, sbits);
  else s = __builtin_bit_cast(V, (uint32_t)sbits);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    val[i] = S::from_acc(S::mul(s, val[i]));
}

// row index of every entry of a CSR, one wavefront per row
__global__ __launch_bounds__(256) void k_row_ids(int32_t n, const int64_t* rp, int32_t* rows) {
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  for (int64_t e = rp[i] + lane; e < rp[i + 1]; e += 64) rows[e] = (int32_t)i;
}

__global__ void k_fill_ops(int64_t n, uint8_t* ops, uint8_t op) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) ops[i] = op;
}

// device memory of one call, released on every exit
struct Tmp {
  Ctx* c;
  void* p = nullptr;
  size_t bytes = 0;
  Tmp(Ctx* ctx, size_t b) : c(ctx), bytes(b ? b : 8) { p = ctx_alloc(c, bytes); }
  ~Tmp() {
    (void)hipStreamSynchronize(c->stream);
    ctx_free(c, p, bytes);
  }
  Tmp(const Tmp&) = delete;
  Tmp& operator=(const Tmp&) = delete;
};

unsigned grid_for(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 4096); }

int64_t read_count(Ctx* c, const int64_t* d) {
  int64_t* h = (int64_t*)c->pinned;
  DSG_HIP(hipMemcpyAsync(h, d, 8, hipMemcpyDeviceToHost, c->stream));
  DSG_HIP(hipStreamSynchronize(c->stream));
  return *h;
}

void scale(Ctx* c, int sr, void* val, int64_t n, uint64_t sbits) {
  if (n == 0) return;
  hipStream_t s = c->stream;
  switch (sr) {
    case 0: hipLaunchKernelGGL(k_scale<0>, dim3(grid_for(n)), dim3(256), 0, s, n, (int64_t*)val, sbits); break;
    case 1: hipLaunchKernelGGL(k_scale<1>, dim3(grid_for(n)), dim3(256), 0, s, n, (float*)val, sbits); break;
    case 2: hipLaunchKernelGGL(k_scale<2>, dim3(grid_for(n)), dim3(256), 0, s, n, (double*)val, sbits); break;
    default: hipLaunchKernelGGL(k_scale<3>, dim3(grid_for(n)), dim3(256), 0, s, n, (uint32_t*)val, sbits); break;
  }
  DSG_HIP(hipGetLastError());
}

// canonical row pointers of m and their entry count
int64_t canonical_rows(DMat* m, int64_t* d_rp) {
  mat_export_device(m, d_rp, nullptr, nullptr, nullptr, m->ctx->stream);
  return read_count(m->ctx, d_rp + m->nrows);
}

}  // namespace

DMat* prod_scale_add(DProd* p, const void* alpha, DMat* X, const void* beta) {
  Ctx* c = p->ctx;
  hipStream_t s = c->stream;
  DMat* C = p->C;
  const int32_t n = C->nrows;
  const int vs = C->vsz;
  uint64_t abits = 0, bbits = 0;
  std::memcpy(&abits, alpha, (size_t)vs);
  if (X) std::memcpy(&bbits, beta, (size_t)vs);
  // alpha (x) C, canonical
  Tmp rp(c, ((size_t)n + 1) * 8);
  const int64_t nnz = canonical_rows(C, (int64_t*)rp.p);
  Tmp col(c, (size_t)nnz * 4), val(c, (size_t)nnz * vs);
  if (nnz > 0) mat_export_device(C, (int64_t*)rp.p, (int32_t*)col.p, val.p, nullptr, s);
  scale(c, C->sr, val.p, nnz, abits);
  DMat* D = mat_create(c, n, C->ncols, C->sr, (const int64_t*)rp.p, (const int32_t*)col.p, val.p);
  if (!X) return D;
  try {
    // (+) beta (x) X, as algebraic additions
    Tmp xrp(c, ((size_t)n + 1) * 8);
    const int64_t nx = canonical_rows(X, (int64_t*)xrp.p);
    if (nx == 0) return D;
    Tmp xcol(c, (size_t)nx * 4), xval(c, (size_t)nx * vs), xrow(c, (size_t)nx * 4), xop(c, (size_t)nx);
    mat_export_device(X, (int64_t*)xrp.p, (int32_t*)xcol.p, xval.p, nullptr, s);
    scale(c, C->sr, xval.p, nx, bbits);
    hipLaunchKernelGGL(k_row_ids, dim3((unsigned)(((int64_t)n * 64 + 255) / 256)), dim3(256), 0, s, n,
                       (const int64_t*)xrp.p, (int32_t*)xrow.p);
    hipLaunchKernelGGL(k_fill_ops, dim3(grid_for(nx)), dim3(256), 0, s, nx, (uint8_t*)xop.p, (uint8_t)DSG_OP_ADD);
    DSG_HIP(hipGetLastError());
    mat_apply_device(D, (const int32_t*)xrow.p, (const int32_t*)xcol.p, xval.p, (const uint8_t*)xop.p, nx);
    DSG_HIP(hipStreamSynchronize(s));
  } catch (...) {
    mat_destroy(D);
    throw;
  }
  return D;
}
