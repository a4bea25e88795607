// Column-major (CSC) copy of a sparse A, for the two-pass form of the
// per-iteration product A^T(Ap) of Algorithm 2 step 4 when n is too large
// for a per-workgroup accumulator of n values in LDS. The first pass forms
// t = A u row by row, the second q_j = sum_i a_ij t_i column by column from
// this copy; no atomics, and every q_j is summed in ascending row order, so
// the result does not depend on scheduling.
//
// Built once at setup: the entries' column indices are sorted as keys with
// their CSR positions as values by a stable radix sort (rows stay ascending
// within a column), then the row index and the value of each entry are
// gathered into column order.
#include <rocprim/device/device_radix_sort.hpp>

#include "common.h"

namespace lsq {

static unsigned grid_for(int64_t items) {
  int64_t b = (items + 255) / 256;
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return (unsigned)b;
}

__global__ void k_entry_keys(int64_t nnz, const int32_t *__restrict__ ci, uint32_t *__restrict__ key,
                             int64_t *__restrict__ pos) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x) {
    key[k] = (uint32_t)ci[k];
    pos[k] = k;
  }
}

// row index of every stored entry
__global__ void k_entry_rows(int64_t m, const int64_t *__restrict__ rp, int32_t *__restrict__ row) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) row[k] = (int32_t)i;
}

// column pointers from the sorted column keys: cp[j] = first position with
// key >= j, cp[n] = nnz
__global__ void k_col_ptr(int64_t nnz, int64_t n, const uint32_t *__restrict__ skey, int64_t *__restrict__ cp) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p <= nnz; p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t prev = p == 0 ? -1 : (int64_t)skey[p - 1];
    const int64_t cur = p == nnz ? n : (int64_t)skey[p];
    for (int64_t j = prev + 1; j <= cur; ++j) cp[j] = p;
  }
}

template <typename TA>
__global__ void k_csc_gather(int64_t nnz, const int64_t *__restrict__ spos, const int32_t *__restrict__ row,
                             const TA *__restrict__ v, const float *__restrict__ v32, int32_t *__restrict__ ri,
                             TA *__restrict__ cv, float *__restrict__ cv32) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = spos[p];
    ri[p] = row[k];
    cv[p] = v[k];
    if (cv32) cv32[p] = v32[k];
  }
}

int build_csc(lsq_ctx *ctx) {
  hipStream_t st = ctx->stream;
  const int64_t m = ctx->m, n = ctx->n, nnz = ctx->nnz;
  const size_t vb = ctx->dtype == LSQ_F64 ? 8 : 4;
  // float32 values beside float64 ones when the inner solve reads a float32 copy
  const bool want32 = ctx->A32own != nullptr;
  uint32_t *key = (uint32_t *)lsq_alloc(ctx, (size_t)(nnz + 1) * 4);
  uint32_t *skey = (uint32_t *)lsq_alloc(ctx, (size_t)(nnz + 1) * 4);
  int64_t *pos = (int64_t *)lsq_alloc(ctx, (size_t)(nnz + 1) * 8);
  int64_t *spos = (int64_t *)lsq_alloc(ctx, (size_t)(nnz + 1) * 8);
  int32_t *row = (int32_t *)lsq_alloc(ctx, (size_t)(nnz + 1) * 4);
  ctx->csc_cp = (int64_t *)lsq_alloc(ctx, (size_t)(n + 1) * 8);
  ctx->csc_ri = (int32_t *)lsq_alloc(ctx, (size_t)(nnz + 1) * 4);
  ctx->csc_v = lsq_alloc(ctx, (size_t)(nnz + 1) * vb);
  ctx->csc_v32 = want32 ? (float *)lsq_alloc(ctx, (size_t)(nnz + 1) * 4) : (float *)ctx->csc_v;
  ctx->tvec = (double *)lsq_alloc(ctx, (size_t)(m + 1) * 8);
  if (!key || !skey || !pos || !spos || !row || !ctx->csc_cp || !ctx->csc_ri || !ctx->csc_v || !ctx->csc_v32 ||
      !ctx->tvec)
    return LSQ_ENOMEM;
  k_entry_keys<<<grid_for(nnz), 256, 0, st>>>(nnz, ctx->ci, key, pos);
  k_entry_rows<<<grid_for(m), 256, 0, st>>>(m, ctx->rp, row);
  int bits = 1;
  while (bits < 32 && ((int64_t)1 << bits) < n) ++bits;
  size_t tmp_bytes = 0;
  LSQ_HIP_CHECK(rocprim::radix_sort_pairs(nullptr, tmp_bytes, key, skey, pos, spos, (size_t)nnz, 0, bits, st));
  void *tmp = lsq_alloc(ctx, tmp_bytes + 16);
  if (!tmp) return LSQ_ENOMEM;
  LSQ_HIP_CHECK(rocprim::radix_sort_pairs(tmp, tmp_bytes, key, skey, pos, spos, (size_t)nnz, 0, bits, st));
  k_col_ptr<<<grid_for(nnz + 1), 256, 0, st>>>(nnz, n, skey, ctx->csc_cp);
  if (ctx->dtype == LSQ_F64)
    k_csc_gather<double><<<grid_for(nnz), 256, 0, st>>>(nnz, spos, row, (const double *)ctx->A, ctx->A32,
                                                         ctx->csc_ri, (double *)ctx->csc_v,
                                                         want32 ? ctx->csc_v32 : nullptr);
  else
    k_csc_gather<float><<<grid_for(nnz), 256, 0, st>>>(nnz, spos, row, (const float *)ctx->A, nullptr, ctx->csc_ri,
                                                        (float *)ctx->csc_v, nullptr);
  LSQ_HIP_CHECK(hipGetLastError());
  LSQ_HIP_CHECK(hipStreamSynchronize(st));
  lsq_free_one(ctx, tmp);
  lsq_free_one(ctx, row);
  lsq_free_one(ctx, spos);
  lsq_free_one(ctx, pos);
  lsq_free_one(ctx, skey);
  lsq_free_one(ctx, key);
  return LSQ_OK;
}

}  // namespace lsq
