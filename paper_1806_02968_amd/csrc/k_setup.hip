// Setup kernels of Algorithm 2: column norms (step 1), row weights of the
// normalised matrix (Eq. R2P), the inclusive CDF of the weights, the i.i.d.
// draws of Algorithm 1 from a Philox4x64-10 counter generator, and the
// compaction of the drawn rows into (row, multiplicity) pairs.
#include <algorithm>
#include <type_traits>

#include "common.h"

namespace lsq {

// ---------------------------------------------------------------------------
// fills

template <typename T>
__global__ void k_fill(T *x, int64_t n, T v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

static unsigned grid256(int64_t n, int64_t cap = 8192) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

void launch_fill_f64(double *x, int64_t n, double v, hipStream_t st) { k_fill<double><<<grid256(n), 256, 0, st>>>(x, n, v); }
void launch_fill_f32(float *x, int64_t n, float v, hipStream_t st) { k_fill<float><<<grid256(n), 256, 0, st>>>(x, n, v); }
void launch_fill_i32(int32_t *x, int64_t n, int32_t v, hipStream_t st) { k_fill<int32_t><<<grid256(n), 256, 0, st>>>(x, n, v); }

// ---------------------------------------------------------------------------
// Algorithm 2 step 1: D_j = ||a^j||_2, accumulated in float64

constexpr int kCnCols = 4;  // columns per thread per pass

template <typename TA>
__global__ __launch_bounds__(256) void k_colnorm_dense(int64_t m, int64_t n, int64_t ld, const TA *__restrict__ A,
                                                       double *__restrict__ part, int64_t rows_per_blk) {
  const int64_t r0 = blockIdx.x * rows_per_blk;
  int64_t r1 = r0 + rows_per_blk;
  if (r1 > m) r1 = m;
  for (int64_t j0 = 0; j0 < n; j0 += 256 * kCnCols) {
    double acc[kCnCols];
#pragma unroll
    for (int c = 0; c < kCnCols; ++c) acc[c] = 0.0;
    for (int64_t i = r0; i < r1; ++i) {
      const TA *row = A + i * ld;
#pragma unroll
      for (int c = 0; c < kCnCols; ++c) {
        int64_t j = j0 + threadIdx.x + c * 256;
        if (j < n) {
          double a = (double)row[j];
          acc[c] += a * a;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < kCnCols; ++c) {
      int64_t j = j0 + threadIdx.x + c * 256;
      if (j < n) part[blockIdx.x * n + j] = acc[c];
    }
  }
}

// 16-byte loads for rows whose length and stride are multiples of a vector:
// thread t owns the column vectors t, t + 256, ..., NC of them, and requests
// RB rows of them before adding any (clamped row index; the row loop bound is
// uniform). Each column still adds its rows in ascending order.
template <typename TA>
using Vec16 = typename std::conditional<sizeof(TA) == 4, float4, double2>::type;

template <typename TA, int NC>
__global__ __launch_bounds__(256) void k_colnorm_dense_vec(int64_t m, int64_t n, int64_t ld,
                                                           const TA *__restrict__ A, double *__restrict__ part,
                                                           int64_t rows_per_blk) {
  constexpr int V = 16 / sizeof(TA), RB = 4;
  typedef Vec16<TA> VT;
  const int64_t r0 = blockIdx.x * rows_per_blk;
  const int64_t r1 = r0 + rows_per_blk < m ? r0 + rows_per_blk : m;
  const int64_t nv = n / V;
  int64_t gi[NC];
  double acc[NC][V];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int64_t g = threadIdx.x + 256 * c;
    gi[c] = g < nv ? g : 0;
#pragma unroll
    for (int k = 0; k < V; ++k) acc[c][k] = 0.0;
  }
  for (int64_t i0 = r0; i0 < r1; i0 += RB) {
    VT x[RB][NC];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int64_t i = i0 + r < r1 ? i0 + r : r1 - 1;
      const VT *row = (const VT *)(A + i * ld);
#pragma unroll
      for (int c = 0; c < NC; ++c) x[r][c] = row[gi[c]];
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      if (i0 + r >= r1) break;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const TA *e = (const TA *)&x[r][c];
#pragma unroll
        for (int k = 0; k < V; ++k) {
          const double a = (double)e[k];
          acc[c][k] += a * a;
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int64_t g = threadIdx.x + 256 * c;
    if (g < nv)
#pragma unroll
      for (int k = 0; k < V; ++k) part[blockIdx.x * n + g * V + k] = acc[c][k];
  }
}

template <typename TA>
__global__ void k_colnorm_csr(int64_t nnz, const int32_t *__restrict__ ci, const TA *__restrict__ v,
                              double *__restrict__ sumsq) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x) {
    double a = (double)v[k];
    atomicAdd(&sumsq[ci[k]], a * a);
  }
}

__global__ void k_colnorm_finish(int64_t n, const double *__restrict__ part, int nblk, double *__restrict__ D,
                                 double *__restrict__ invD, float *__restrict__ invD32, int32_t *flags) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * n + j];
    double d = sqrt(s);
    D[j] = d;
    double inv = 1.0 / d;
    invD[j] = inv;
    if (invD32) invD32[j] = (float)inv;
    if (!isfinite(d)) atomicOr(&flags[0], 2);
    else if (d == 0.0) atomicOr(&flags[0], 1);
  }
}

template <typename TA>
static bool vec16_ok(const lsq_ctx *c) {
  constexpr int V = 16 / sizeof(TA);
  return c->n % V == 0 && c->ld % V == 0 && ((uintptr_t)c->A % 16) == 0;
}

template <typename TA>
static void colnorm_dense_t(const lsq_ctx *c, double *part, int nblk, int64_t rpb, hipStream_t st) {
  constexpr int V = 16 / sizeof(TA);
  const TA *A = (const TA *)c->A;
  const int64_t nc = (c->n / V + 255) / 256;
  if (vec16_ok<TA>(c) && nc <= 8) {
    // 2 million x 2000 float32: 7.35 ms with one 4-byte load per column and row
    if (nc <= 1) k_colnorm_dense_vec<TA, 1><<<nblk, 256, 0, st>>>(c->m, c->n, c->ld, A, part, rpb);
    else if (nc <= 2) k_colnorm_dense_vec<TA, 2><<<nblk, 256, 0, st>>>(c->m, c->n, c->ld, A, part, rpb);
    else if (nc <= 4) k_colnorm_dense_vec<TA, 4><<<nblk, 256, 0, st>>>(c->m, c->n, c->ld, A, part, rpb);
    else k_colnorm_dense_vec<TA, 8><<<nblk, 256, 0, st>>>(c->m, c->n, c->ld, A, part, rpb);
    return;
  }
  k_colnorm_dense<TA><<<nblk, 256, 0, st>>>(c->m, c->n, c->ld, A, part, rpb);
}

void launch_colnorm_dense(const lsq_ctx *c, double *part, int nblk, hipStream_t st) {
  int64_t rpb = (c->m + nblk - 1) / nblk;
  if (c->dtype == LSQ_F64) colnorm_dense_t<double>(c, part, nblk, rpb, st);
  else colnorm_dense_t<float>(c, part, nblk, rpb, st);
}

// column sums of squares of a CSR A into per-workgroup partial rows: block b
// adds the entries of its nnz range into an LDS row of n sums (no contention
// on global memory) and writes it to part row b
template <typename TA>
__global__ __launch_bounds__(1024) void k_colnorm_csr_lds(int64_t nnz, int n, const int32_t *__restrict__ ci,
                                                          const TA *__restrict__ v, double *__restrict__ part) {
  extern __shared__ __align__(16) unsigned char smem[];
  double *acc = (double *)smem;
  for (int j = threadIdx.x; j < n; j += blockDim.x) acc[j] = 0.0;
  __syncthreads();
  const int64_t per = (nnz + gridDim.x - 1) / gridDim.x;
  const int64_t k0 = blockIdx.x * per, k1 = k0 + per < nnz ? k0 + per : nnz;
  for (int64_t k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
    const double a = (double)v[k];
    atomicAdd(&acc[ci[k]], a * a);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += blockDim.x) part[blockIdx.x * (int64_t)n + j] = acc[j];
}

// returns the number of partial rows written to part
int launch_colnorm_csr_part(const lsq_ctx *c, double *part, hipStream_t st) {
  const int64_t n = c->n;
  if (n * 8 > 128 * 1024 || c->part_bytes < (size_t)256 * n * sizeof(double)) {
    launch_colnorm_csr(c, part, st);
    return 1;
  }
  const int nblk = (int)std::max<int64_t>(1, std::min<int64_t>(256, c->nnz / 4096));
  const size_t lds = n * sizeof(double);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void *)k_colnorm_csr_lds<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              128 * 1024);
    (void)hipFuncSetAttribute((const void *)k_colnorm_csr_lds<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              128 * 1024);
    (void)hipGetLastError();
    attr = true;
  }
  if (c->dtype == LSQ_F64)
    k_colnorm_csr_lds<double><<<nblk, 1024, lds, st>>>(c->nnz, (int)n, c->ci, (const double *)c->A, part);
  else
    k_colnorm_csr_lds<float><<<nblk, 1024, lds, st>>>(c->nnz, (int)n, c->ci, (const float *)c->A, part);
  return nblk;
}

void launch_colnorm_csr(const lsq_ctx *c, double *sumsq, hipStream_t st) {
  launch_fill_f64(sumsq, c->n, 0.0, st);
  if (c->dtype == LSQ_F64)
    k_colnorm_csr<double><<<grid256(c->nnz, 16384), 256, 0, st>>>(c->nnz, c->ci, (const double *)c->A, sumsq);
  else
    k_colnorm_csr<float><<<grid256(c->nnz, 16384), 256, 0, st>>>(c->nnz, c->ci, (const float *)c->A, sumsq);
}

void launch_colnorm_finish(int64_t n, const double *part, int nblk, double *D, double *invD, float *invD32,
                           int32_t *flags, hipStream_t st) {
  k_colnorm_finish<<<grid256(n), 256, 0, st>>>(n, part, nblk, D, invD, invD32, flags);
}

// ---------------------------------------------------------------------------
// Eq. (R2P) numerator on the normalised rows: w_i = sum_j (a_ij / D_j)^2

template <typename TA>
__global__ __launch_bounds__(256) void k_rowweight_dense(int64_t m, int64_t n, int64_t ld, const TA *__restrict__ A,
                                                         const double *__restrict__ invD, double *__restrict__ w,
                                                         int32_t *flags) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < m; i += nwaves) {
    const TA *row = A + i * ld;
    double acc = 0.0;
    for (int64_t j = lane; j < n; j += 64) {
      double a = (double)row[j] * invD[j];
      acc += a * a;
    }
    acc = wave_sum(acc);
    if (lane == 0) {
      w[i] = acc;
      if (!isfinite(acc)) atomicOr(&flags[0], 2);
    }
  }
}

// one wave per pair of rows with 16-byte loads, U vectors per lane per row
// requested before any is used (clamped indices)
template <typename TA>
__global__ __launch_bounds__(256) void k_rowweight_dense_vec(int64_t m, int64_t n, int64_t ld,
                                                             const TA *__restrict__ A,
                                                             const double *__restrict__ invD, double *__restrict__ w,
                                                             int32_t *flags) {
  constexpr int V = 16 / sizeof(TA), RW = 2, U = 2;
  typedef Vec16<TA> VT;
  const int lane = threadIdx.x & 63;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t nv = n / V;
  for (int64_t i0 = wave * RW; i0 < m; i0 += nwaves * RW) {
    double acc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) acc[r] = 0.0;
    for (int64_t g0 = 0; g0 < nv; g0 += 64 * U) {
      VT x[RW][U];
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        const int64_t i = i0 + r < m ? i0 + r : m - 1;
        const VT *row = (const VT *)(A + i * ld);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t g = g0 + lane + 64 * u;
          x[r][u] = row[g < nv ? g : 0];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t g = g0 + lane + 64 * u;
        if (g >= nv) continue;
#pragma unroll
        for (int k = 0; k < V; ++k) {
          const double d = invD[g * V + k];
#pragma unroll
          for (int r = 0; r < RW; ++r) {
            const double a = (double)((const TA *)&x[r][u])[k] * d;
            acc[r] += a * a;
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const double t = wave_sum(acc[r]);
      if (lane == 0 && i0 + r < m) {
        w[i0 + r] = t;
        if (!isfinite(t)) atomicOr(&flags[0], 2);
      }
    }
  }
}

template <typename TA, int G>
__global__ __launch_bounds__(256) void k_rowweight_csr(int64_t m, const int64_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci, const TA *__restrict__ v,
                                                       const double *__restrict__ invD, double *__restrict__ w,
                                                       int32_t *flags) {
  const int gl = threadIdx.x & (G - 1);
  const int64_t grp = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) / G;
  // every group runs the same number of iterations so that the group
  // reduction is always executed by whole groups
  const int64_t iters = (m + ngrp - 1) / ngrp;
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t i = grp + it * ngrp;
    double acc = 0.0;
    if (i < m) {
      for (int64_t k = rp[i] + gl; k < rp[i + 1]; k += G) {
        double a = (double)v[k] * invD[ci[k]];
        acc += a * a;
      }
    }
    acc = group_sum<G>(acc);
    if (i < m && gl == 0) {
      w[i] = acc;
      if (!isfinite(acc)) atomicOr(&flags[0], 2);
    }
  }
}

template <typename TA>
static void rowweight_csr_dispatch(const lsq_ctx *c, double *w, int32_t *flags, hipStream_t st) {
  double avg = (double)c->nnz / (double)(c->m > 0 ? c->m : 1);
  const TA *v = (const TA *)c->A;
  unsigned grid = grid256(c->m * 16, 16384);
  if (avg <= 4) k_rowweight_csr<TA, 4><<<grid, 256, 0, st>>>(c->m, c->rp, c->ci, v, c->invD, w, flags);
  else if (avg <= 8) k_rowweight_csr<TA, 8><<<grid, 256, 0, st>>>(c->m, c->rp, c->ci, v, c->invD, w, flags);
  else if (avg <= 16) k_rowweight_csr<TA, 16><<<grid, 256, 0, st>>>(c->m, c->rp, c->ci, v, c->invD, w, flags);
  else if (avg <= 32) k_rowweight_csr<TA, 32><<<grid, 256, 0, st>>>(c->m, c->rp, c->ci, v, c->invD, w, flags);
  else k_rowweight_csr<TA, 64><<<grid, 256, 0, st>>>(c->m, c->rp, c->ci, v, c->invD, w, flags);
}

void launch_rowweight(const lsq_ctx *c, double *w, int32_t *flags, hipStream_t st) {
  if (c->fmt == LSQ_DENSE) {
    unsigned grid = grid256(c->m * 64, 16384);
    if (c->dtype == LSQ_F64) {
      if (vec16_ok<double>(c))
        k_rowweight_dense_vec<double><<<grid, 256, 0, st>>>(c->m, c->n, c->ld, (const double *)c->A, c->invD, w,
                                                             flags);
      else
        k_rowweight_dense<double><<<grid, 256, 0, st>>>(c->m, c->n, c->ld, (const double *)c->A, c->invD, w, flags);
    } else {
      // 2 million x 2000 float32: 4.6 ms with 4-byte loads
      if (vec16_ok<float>(c))
        k_rowweight_dense_vec<float><<<grid, 256, 0, st>>>(c->m, c->n, c->ld, (const float *)c->A, c->invD, w,
                                                            flags);
      else
        k_rowweight_dense<float><<<grid, 256, 0, st>>>(c->m, c->n, c->ld, (const float *)c->A, c->invD, w, flags);
    }
  } else {
    if (c->dtype == LSQ_F64) rowweight_csr_dispatch<double>(c, w, flags, st);
    else rowweight_csr_dispatch<float>(c, w, flags, st);
  }
}

// ---------------------------------------------------------------------------
// scans: each thread owns 16 consecutive elements and sums them in order, so
// the CDF is non-decreasing within a thread's run

constexpr int kScanT = 256, kScanE = 16, kScanChunk = kScanT * kScanE;

size_t scan_scratch_elems(int64_t m) { return (size_t)((m + kScanChunk - 1) / kScanChunk) + 1; }

template <typename T>
__global__ __launch_bounds__(kScanT) void k_scan_blocksum(int64_t m, const T *__restrict__ x, T *__restrict__ bs) {
  __shared__ T red[kScanT / kWave];
  const int64_t base = blockIdx.x * (int64_t)kScanChunk + threadIdx.x * (int64_t)kScanE;
  T acc = 0;
  for (int e = 0; e < kScanE; ++e)
    if (base + e < m) acc += x[base + e];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) bs[blockIdx.x] = acc;
}

template <typename T>
__global__ void k_scan_offsets(int64_t nb, T *bs) {  // exclusive, sequential
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    T run = 0;
    for (int64_t b = 0; b < nb; ++b) {
      T v = bs[b];
      bs[b] = run;
      run += v;
    }
    bs[nb] = run;
  }
}

template <typename T, bool INCLUSIVE>
__global__ __launch_bounds__(kScanT) void k_scan_local(int64_t m, const T *__restrict__ x, const T *__restrict__ boff,
                                                       T *__restrict__ y) {
  __shared__ T ts[kScanT];
  const int64_t base = blockIdx.x * (int64_t)kScanChunk + threadIdx.x * (int64_t)kScanE;
  T v[kScanE];
  T acc = 0;
#pragma unroll
  for (int e = 0; e < kScanE; ++e) {
    v[e] = (base + e < m) ? x[base + e] : (T)0;
    acc += v[e];
  }
  ts[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T run = 0;
    for (int t = 0; t < kScanT; ++t) {
      T a = ts[t];
      ts[t] = run;
      run += a;
    }
  }
  __syncthreads();
  T run = boff[blockIdx.x] + ts[threadIdx.x];
#pragma unroll
  for (int e = 0; e < kScanE; ++e) {
    if (base + e < m) {
      if (INCLUSIVE) {
        run += v[e];
        y[base + e] = run;
      } else {
        y[base + e] = run;
        run += v[e];
      }
    }
  }
}

void launch_scan_cdf(int64_t m, const double *w, double *cdf, double *bs, hipStream_t st) {
  int64_t nb = (m + kScanChunk - 1) / kScanChunk;
  k_scan_blocksum<double><<<(unsigned)nb, kScanT, 0, st>>>(m, w, bs);
  k_scan_offsets<double><<<1, 64, 0, st>>>(nb, bs);
  k_scan_local<double, true><<<(unsigned)nb, kScanT, 0, st>>>(m, w, bs, cdf);
}

// ---------------------------------------------------------------------------
// Algorithm 1: s i.i.d. trials, Pr{i_t = k} = p_k = w_k / W.
// u_t is word (t mod 4) of Philox4x64-10 (Salmon et al., SC'11) with counter
// (t div 4, 0, 0, 0) and key (seed, 0), top 53 bits scaled by 2^-53; the
// trial picks the first row whose CDF value exceeds u_t W.

__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__global__ __launch_bounds__(256) void k_draw(int64_t m, const double *__restrict__ w, const double *__restrict__ cdf,
                                              int64_t s, uint64_t seed, int64_t *__restrict__ idx,
                                              double *__restrict__ gap, int32_t *__restrict__ cnt) {
  const double W = cdf[m - 1];
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < s; t += (int64_t)gridDim.x * blockDim.x) {
    uint64_t c[4] = {(uint64_t)t >> 2, 0, 0, 0};
    philox4x64_10(c, seed, 0);
    uint64_t word = c[t & 3];
    double u = (double)(word >> 11) * 0x1.0p-53;
    double tau = u * W;
    int64_t lo = 0, hi = m;
    while (lo < hi) {
      int64_t mid = lo + ((hi - lo) >> 1);
      if (cdf[mid] > tau) hi = mid;
      else lo = mid + 1;
    }
    int64_t i = lo;
    bool adjusted = false;
    if (i == m) {
      i = m - 1;
      while (i > 0 && !(w[i] > 0.0)) --i;
      adjusted = true;
    } else if (!(w[i] > 0.0)) {
      int64_t k = i;
      while (k < m && !(w[k] > 0.0)) ++k;
      if (k == m) {
        k = i;
        while (k > 0 && !(w[k] > 0.0)) --k;
      }
      i = k;
      adjusted = true;
    }
    double g = 0.0;
    if (!adjusted) {
      double below = i > 0 ? cdf[i - 1] : 0.0;
      double g1 = tau - below, g2 = cdf[i] - tau;
      g = (g1 < g2 ? g1 : g2) / W;
    }
    idx[t] = i;
    gap[t] = g;
    atomicAdd(&cnt[i], 1);
  }
}

void launch_draw(int64_t m, const double *w, const double *cdf, int64_t s, uint64_t seed, int64_t *idx,
                 double *gap, int32_t *cnt, hipStream_t st) {
  k_draw<<<grid256(s, 8192), 256, 0, st>>>(m, w, cdf, s, seed, idx, gap, cnt);
}

// ---------------------------------------------------------------------------
// distinct drawn rows (ascending) and their multiplicities

__global__ void k_flag_counts(int64_t m, const int32_t *__restrict__ cnt, int64_t *__restrict__ f) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    f[i] = cnt[i] > 0 ? 1 : 0;
}

__global__ void k_scatter_rows(int64_t m, const int32_t *__restrict__ cnt, const int64_t *__restrict__ pos,
                               int64_t *__restrict__ urow, int32_t *__restrict__ ucnt) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    if (cnt[i] > 0) {
      urow[pos[i]] = i;
      ucnt[pos[i]] = cnt[i];
    }
}

// scratch: m + scan_scratch_elems(m) int64
void launch_compact_counts(int64_t m, const int32_t *cnt, int64_t *scratch, int64_t *urow, int32_t *ucnt,
                           int64_t *dcount, hipStream_t st) {
  int64_t nb = (m + kScanChunk - 1) / kScanChunk;
  int64_t *f = scratch, *bs = scratch + m;
  k_flag_counts<<<grid256(m), 256, 0, st>>>(m, cnt, f);
  k_scan_blocksum<int64_t><<<(unsigned)nb, kScanT, 0, st>>>(m, f, bs);
  k_scan_offsets<int64_t><<<1, 64, 0, st>>>(nb, bs);
  k_scan_local<int64_t, false><<<(unsigned)nb, kScanT, 0, st>>>(m, f, bs, f);
  k_scatter_rows<<<grid256(m), 256, 0, st>>>(m, cnt, f, urow, ucnt);
  (void)hipMemcpyAsync(dcount, bs + nb, sizeof(int64_t), hipMemcpyDeviceToDevice, st);
}

}  // namespace lsq
