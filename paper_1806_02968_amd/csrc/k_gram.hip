// Sampled Gram matrix of Section 3.3, M = sum_t (1/(s p_{i_t})) a_{i_t}^T a_{i_t}
// over the normalised rows (Algorithm 2 step 3). Duplicate draws are merged:
// a row drawn c_r times enters once with weight c_r W / (s w_r).
//
// Dense A: the distinct rows are gathered into A_s (s_d x n), each scaled by
// sqrt(c_r W / (s w_r)), and M = A_s^T A_s is formed by an MFMA SYRK
// (float64 v_mfma_f64_16x16x4f64, or float32 v_mfma_f32_16x16x4f32 for the
// float32 preconditioner) over the upper tiles, mirrored.
//
// CSR A: an expand-sort-reduce product. Every (column j, sampled row r) pair
// expands row r into keys (l, r) with values coef_r * a_rj * a_rl, grouped by
// output row j; each row's keys are sorted (bitonic, in LDS) and equal columns
// summed in increasing r, which makes M exactly symmetric and the build
// deterministic.
#include <algorithm>

#include "common.h"

namespace lsq {

// ---------------------------------------------------------------------------
// dense gather

template <typename TA, typename TO>
__global__ __launch_bounds__(256) void k_gather_dense(int64_t sd, int64_t n, int64_t ld, const TA *__restrict__ A,
                                                      const int64_t *__restrict__ urow, const int32_t *__restrict__ ucnt,
                                                      const double *__restrict__ w, const double *__restrict__ invD,
                                                      const double *__restrict__ Wp, double s, TO *__restrict__ As) {
  const double W = *Wp;
  const int lane = threadIdx.x & 63;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t r = wave; r < sd; r += nwaves) {
    const int64_t i = urow[r];
    const double sc = sqrt((double)ucnt[r] * W / (s * w[i]));
    const TA *row = A + i * ld;
    for (int64_t j = lane; j < n; j += 64) As[r * n + j] = (TO)(sc * ((double)row[j] * invD[j]));
  }
}

static unsigned grid_rows(int64_t rows) {
  int64_t b = (rows * 64 + 255) / 256;
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return (unsigned)b;
}

void launch_gather_dense_f64(const lsq_ctx *c, double *As, hipStream_t st) {
  if (c->dtype == LSQ_F64)
    k_gather_dense<double, double><<<grid_rows(c->s_d), 256, 0, st>>>(c->s_d, c->n, c->ld, (const double *)c->A, c->urow,
                                                                       c->ucnt, c->w, c->invD, c->cdf + c->m - 1,
                                                                       (double)c->s, As);
  else
    k_gather_dense<float, double><<<grid_rows(c->s_d), 256, 0, st>>>(c->s_d, c->n, c->ld, (const float *)c->A, c->urow,
                                                                      c->ucnt, c->w, c->invD, c->cdf + c->m - 1,
                                                                      (double)c->s, As);
}

void launch_gather_dense_f32(const lsq_ctx *c, float *As, hipStream_t st) {
  if (c->dtype == LSQ_F64)
    k_gather_dense<double, float><<<grid_rows(c->s_d), 256, 0, st>>>(c->s_d, c->n, c->ld, (const double *)c->A, c->urow,
                                                                      c->ucnt, c->w, c->invD, c->cdf + c->m - 1,
                                                                      (double)c->s, As);
  else
    k_gather_dense<float, float><<<grid_rows(c->s_d), 256, 0, st>>>(c->s_d, c->n, c->ld, (const float *)c->A, c->urow,
                                                                     c->ucnt, c->w, c->invD, c->cdf + c->m - 1,
                                                                     (double)c->s, As);
}

// ---------------------------------------------------------------------------
// MFMA SYRK: M = As^T As, 64x64 output tiles over the upper triangle of tiles.
// Four waves per tile, each a 32x32 quadrant of 2x2 16x16 MFMA blocks. A_s
// rows are staged through LDS 16 at a time. For a 16x16x4 MFMA lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; its four results are column l%16 of rows
// l/16 + 4i (float64) or 4(l/16) + i (float32), i < 4.

constexpr int kTile = 64, kKc = 32;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T>
struct Acc4;
template <>
struct Acc4<double> {
  typedef d4 type;
  static __device__ __forceinline__ int row(int lane, int i) { return (lane >> 4) + 4 * i; }
};
template <>
struct Acc4<float> {
  typedef f4 type;
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

// tile index -> (tj, tl), tj <= tl, upper tiles in row order
__device__ __forceinline__ void syrk_tile(int b, int nt, int *tj, int *tl) {
  int t = 0;
  while (b >= nt - t) {
    b -= nt - t;
    ++t;
  }
  *tj = t;
  *tl = t + b;
}

// One 64 x 64 upper tile of A_s^T A_s per workgroup (4 waves, 32 x 32 each,
// 2 x 2 MFMA 16 x 16 blocks), over the sampled rows of its split: kKc rows
// per stage through LDS, the next stage's rows requested into registers
// before the current stage's products (clamped indices, zeroed when stored).
// With one split the tile is written to both triangles of M; with several,
// each split writes its partial tile and k_syrk_reduce adds them in split
// order.
template <typename T>
__global__ __launch_bounds__(256) void k_syrk(int64_t sd, int64_t n, const T *__restrict__ As, T *__restrict__ M,
                                              int nt, int64_t chunk, T *__restrict__ part) {
  typedef typename Acc4<T>::type acc_t;
  constexpr int PER = kKc * kTile / 256;
  __shared__ T sj[kKc][kTile];
  __shared__ T sl[kKc][kTile];
  const int ntiles = nt * (nt + 1) / 2;
  const int tile = blockIdx.x % ntiles, split = blockIdx.x / ntiles;
  int tj, tl;
  syrk_tile(tile, nt, &tj, &tl);
  const int64_t J0 = (int64_t)tj * kTile, L0 = (int64_t)tl * kTile;
  const int64_t rb = split * chunk, re = rb + chunk < sd ? rb + chunk : sd;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wj = wv >> 1, wl = wv & 1;
  acc_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = acc_t{0, 0, 0, 0};
  T rj[PER], rl[PER];
  auto fetch = [&](int64_t r0) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * 256;
      const int64_t r = r0 + e / kTile;
      const int cc = e % kTile;
      const int64_t rr = r < re ? r : rb;
      const int64_t jj = J0 + cc < n ? J0 + cc : 0, ll = L0 + cc < n ? L0 + cc : 0;
      rj[q] = As[rr * n + jj];
      rl[q] = As[rr * n + ll];
    }
  };
  if (rb < re) fetch(rb);
  for (int64_t r0 = rb; r0 < re; r0 += kKc) {
    __syncthreads();  // the previous stage's products are done with LDS
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * 256;
      const int rr = e / kTile, cc = e % kTile;
      const bool okr = r0 + rr < re;
      sj[rr][cc] = okr && J0 + cc < n ? rj[q] : (T)0;
      sl[rr][cc] = okr && L0 + cc < n ? rl[q] : (T)0;
    }
    __syncthreads();
    if (r0 + kKc < re) fetch(r0 + kKc);
#pragma unroll
    for (int ks = 0; ks < kKc / 4; ++ks) {
      const int kr = ks * 4 + (lane >> 4);
      T a0 = sj[kr][wj * 32 + (lane & 15)];
      T a1 = sj[kr][wj * 32 + 16 + (lane & 15)];
      T b0 = sl[kr][wl * 32 + (lane & 15)];
      T b1 = sl[kr][wl * 32 + 16 + (lane & 15)];
      acc[0][0] = mfma16(a0, b0, acc[0][0]);
      acc[0][1] = mfma16(a0, b1, acc[0][1]);
      acc[1][0] = mfma16(a1, b0, acc[1][0]);
      acc[1][1] = mfma16(a1, b1, acc[1][1]);
    }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int jl = wj * 32 + x * 16 + Acc4<T>::row(lane, i);
        const int ll = wl * 32 + y * 16 + (lane & 15);
        const T v = acc[x][y][i];
        if (part) {
          part[((int64_t)split * ntiles + tile) * (kTile * kTile) + jl * kTile + ll] = v;
        } else {
          const int64_t j = J0 + jl, l = L0 + ll;
          if (j < n && l < n && l >= j) {
            M[j * n + l] = v;
            M[l * n + j] = v;
          }
        }
      }
}

// M from the splits' partial tiles, added in split order (one workgroup per tile)
template <typename T>
__global__ __launch_bounds__(256) void k_syrk_reduce(int64_t n, int nt, int nsplit, const T *__restrict__ part,
                                                     T *__restrict__ M) {
  const int ntiles = nt * (nt + 1) / 2, tile = blockIdx.x;
  int tj, tl;
  syrk_tile(tile, nt, &tj, &tl);
  const int64_t J0 = (int64_t)tj * kTile, L0 = (int64_t)tl * kTile;
  for (int loc = threadIdx.x; loc < kTile * kTile; loc += 256) {
    const int64_t j = J0 + loc / kTile, l = L0 + loc % kTile;
    if (j >= n || l >= n || l < j) continue;
    T v = part[(int64_t)tile * (kTile * kTile) + loc];
    for (int s = 1; s < nsplit; ++s) v += part[((int64_t)s * ntiles + tile) * (kTile * kTile) + loc];
    M[j * n + l] = v;
    M[l * n + j] = v;
  }
}

// splits of the sampled rows so that the launch has about eight workgroups
// per CU, at most 8 splits of at least 8 stages each (float64, n = 2000: 29.3
// TFLOP/s at two workgroups per CU, 33.6 at four, 36.7 at eight; n = 1000,
// 136 tiles: 28.2, 32.4, 32.6)
int syrk_splits(int64_t sd, int64_t n, int ncu) {
  const int64_t nt = (n + kTile - 1) / kTile, ntiles = nt * (nt + 1) / 2;
  int64_t S = (8 * (int64_t)std::max(ncu, 1) + ntiles - 1) / ntiles;
  S = std::max<int64_t>(1, std::min<int64_t>({S, 8, sd / (8 * kKc)}));
  return (int)S;
}
size_t syrk_scratch_elems(int64_t n, int nsplit) {
  if (nsplit <= 1) return 0;
  const int64_t nt = (n + kTile - 1) / kTile;
  return (size_t)nsplit * (size_t)(nt * (nt + 1) / 2) * kTile * kTile;
}

template <typename T>
static void launch_syrk_t(int64_t sd, int64_t n, const T *As, T *M, int nsplit, T *part, hipStream_t st) {
  const int nt = (int)((n + kTile - 1) / kTile), ntiles = nt * (nt + 1) / 2;
  if (nsplit <= 1 || !part) {
    k_syrk<T><<<ntiles, 256, 0, st>>>(sd, n, As, M, nt, std::max<int64_t>(sd, 1), nullptr);
    return;
  }
  int64_t chunk = (sd + nsplit - 1) / nsplit;
  chunk = (chunk + kKc - 1) / kKc * kKc;
  k_syrk<T><<<ntiles * nsplit, 256, 0, st>>>(sd, n, As, M, nt, chunk, part);
  k_syrk_reduce<T><<<ntiles, 256, 0, st>>>(n, nt, nsplit, part, M);
}
void launch_syrk_f64(int64_t sd, int64_t n, const double *As, double *M, int nsplit, double *part,
                     hipStream_t st) {
  launch_syrk_t<double>(sd, n, As, M, nsplit, part, st);
}
void launch_syrk_f32(int64_t sd, int64_t n, const float *As, float *M, int nsplit, float *part, hipStream_t st) {
  launch_syrk_t<float>(sd, n, As, M, nsplit, part, st);
}

template <typename T>
__global__ void k_dense_diag_guard(int64_t n, T *M, int32_t *flags) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    if (M[j * n + j] == (T)0) {
      M[j * n + j] = (T)1;
      atomicAdd(&flags[1], 1);
    }
}
void launch_dense_diag_guard_f64(int64_t n, double *M, int32_t *flags, hipStream_t st) {
  k_dense_diag_guard<double><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, M, flags);
}
void launch_dense_diag_guard_f32(int64_t n, float *M, int32_t *flags, hipStream_t st) {
  k_dense_diag_guard<float><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, M, flags);
}

__global__ void k_cast(const double *__restrict__ x, float *__restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}
void launch_cast_f64_f32(const double *x, float *y, int64_t n, hipStream_t st) {
  int64_t b = (n + 255) / 256;
  if (b > 16384) b = 16384;
  if (b < 1) b = 1;
  k_cast<<<(unsigned)b, 256, 0, st>>>(x, y, n);
}

// ---------------------------------------------------------------------------
// sparse Gram (CSR A)

__global__ void k_col_counts(int64_t sd, const int64_t *__restrict__ urow, const int64_t *__restrict__ rp,
                             const int32_t *__restrict__ ci, int64_t *__restrict__ ccnt) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t r = wave; r < sd; r += nwaves) {
    const int64_t i = urow[r];
    for (int64_t k = rp[i] + lane; k < rp[i + 1]; k += 64) atomicAdd((unsigned long long *)&ccnt[ci[k]], 1ull);
  }
}

__global__ void k_csc_fill(int64_t sd, const int64_t *__restrict__ urow, const int64_t *__restrict__ rp,
                           const int32_t *__restrict__ ci, const int64_t *__restrict__ cptr,
                           int64_t *__restrict__ cfill, int32_t *__restrict__ csc_r, int64_t *__restrict__ csc_k,
                           int64_t *__restrict__ plen) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t r = wave; r < sd; r += nwaves) {
    const int64_t i = urow[r];
    const int64_t len = rp[i + 1] - rp[i];
    for (int64_t k = rp[i] + lane; k < rp[i + 1]; k += 64) {
      const int32_t j = ci[k];
      const int64_t pos = cptr[j] + (int64_t)atomicAdd((unsigned long long *)&cfill[j], 1ull);
      csc_r[pos] = (int32_t)r;
      csc_k[pos] = k;
      plen[pos] = len;
    }
  }
}

// G lanes per CSC entry (column j of sampled row r): lane t forms the
// products with the row's entries t, t + G, ..., so a group reads the row and
// writes its products contiguously
template <typename TA, int G>
__global__ void k_expand(int64_t E, const int32_t *__restrict__ csc_r, const int64_t *__restrict__ csc_k,
                         const int64_t *__restrict__ poff, const int64_t *__restrict__ urow,
                         const int32_t *__restrict__ ucnt, const int64_t *__restrict__ rp,
                         const int32_t *__restrict__ ci, const TA *__restrict__ v, const double *__restrict__ w,
                         const double *__restrict__ invD, const double *__restrict__ Wp, double s,
                         uint64_t *__restrict__ key, double *__restrict__ val) {
  const double W = *Wp;
  const int t = threadIdx.x % G;
  const int64_t g0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int64_t ng = (int64_t)gridDim.x * blockDim.x / G;
  for (int64_t e = g0; e < E; e += ng) {
    const int32_t r = csc_r[e];
    const int64_t k = csc_k[e];
    const int64_t i = urow[r];
    const int32_t j = ci[k];
    const double coef = (double)ucnt[r] * W / (s * w[i]);
    const double aj = (double)v[k] * invD[j];
    const int64_t q0 = rp[i], q1 = rp[i + 1];
    const int64_t o = poff[e] - q0;
    for (int64_t q = q0 + t; q < q1; q += G) {
      const int32_t l = ci[q];
      const double al = (double)v[q] * invD[l];
      key[o + q] = ((uint64_t)(uint32_t)l << 32) | (uint32_t)r;
      val[o + q] = coef * (aj * al);
    }
  }
}

constexpr int kSortCap = 2048, kSortT = 256;

// bitonic sort of N (power of two) key/value pairs at (k, v), ascending keys;
// the caller synchronises before and after
__device__ void bitonic_block(uint64_t *k, double *v, int N) {
  for (int size = 2; size <= N; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < N / 2; t += blockDim.x) {
        int lo = 2 * t - (t & (stride - 1));
        int hi = lo + stride;
        bool up = ((lo & size) == 0);
        uint64_t a = k[lo], b = k[hi];
        if ((a > b) == up) {
          k[lo] = b;
          k[hi] = a;
          double x = v[lo];
          v[lo] = v[hi];
          v[hi] = x;
        }
      }
      __syncthreads();
    }
  }
}

// reduce a sorted row (P entries at k, v) by column, insert/guard the
// diagonal, and write cols/vals to (oc, ov); returns the count in *cnt_out.
// heads: LDS int array of >= P + 1 entries. Executed by the whole block.
// NT: the block's threads.
template <int NT>
__device__ void reduce_sorted_row(const uint64_t *k, const double *v, int64_t P, int32_t j, int32_t *oc,
                                  double *ov, int *heads, int64_t *cnt_out, int32_t *flags) {
  __shared__ int wcnt[NT / kWave], wbelow[NT / kWave], wdiag[NT / kWave];
  // head flags (first entry of each column) and their exclusive positions:
  // thread t scans a contiguous chunk, the chunk counts are scanned over the
  // block in thread order
  const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave, nw = NT / kWave;
  const int chunk = (int)((P + NT - 1) / NT);
  const int t0 = (int)min<int64_t>(P, (int64_t)tid * chunk), t1 = (int)min<int64_t>(P, (int64_t)t0 + chunk);
  auto col = [&](int t) -> uint32_t { return (uint32_t)(k[t] >> 32); };
  int cnt = 0, below = 0, hd = 0;
  for (int t = t0; t < t1; ++t) {
    const uint32_t c = col(t);
    const bool h = t == 0 || col(t - 1) != c;
    cnt += h;
    below += h && (int32_t)c < j;
    hd |= h && (int32_t)c == j;
  }
  int incl = cnt;  // inclusive scan over the wave
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  const int wb = wave_sum(below);
  const bool wd = __ballot(hd != 0) != 0;
  if (lane == kWave - 1) {
    wcnt[wid] = incl;
    wbelow[wid] = wb;
    wdiag[wid] = wd;
  }
  __syncthreads();
  int base = 0, nh = 0, ins = 0, has_diag = 0;
  for (int w = 0; w < nw; ++w) {
    base += w < wid ? wcnt[w] : 0;
    nh += wcnt[w];
    ins += wbelow[w];
    has_diag |= wdiag[w];
  }
  int run = base + incl - cnt;
  for (int t = t0; t < t1; ++t) {
    const bool h = t == 0 || col(t - 1) != col(t);
    heads[t] = h ? run++ : -1;
  }
  __syncthreads();
  const int shift_from = has_diag ? 0x7fffffff : ins;
  for (int64_t t = threadIdx.x; t < P; t += blockDim.x) {
    int pos = heads[t];
    if (pos < 0) continue;
    uint32_t c = (uint32_t)(k[t] >> 32);
    double acc = v[t];
    for (int64_t q = t + 1; q < P && (uint32_t)(k[q] >> 32) == c; ++q) acc += v[q];
    if ((int32_t)c == j && acc == 0.0) {
      acc = 1.0;
      atomicAdd(&flags[1], 1);
    }
    int o = pos >= shift_from ? pos + 1 : pos;
    oc[o] = (int32_t)c;
    ov[o] = acc;
  }
  if (threadIdx.x == 0) {
    if (!has_diag) {
      oc[ins] = j;
      ov[ins] = 1.0;
      atomicAdd(&flags[1], 1);
    }
    *cnt_out = nh + (has_diag ? 0 : 1);
  }
  __syncthreads();
}

// one block per output row j whose product segment fits in LDS; longer rows
// get ucount = -1 and are handled by k_row_big
__global__ __launch_bounds__(kSortT) void k_row_small(int64_t n, const int64_t *__restrict__ cptr,
                                                      const int64_t *__restrict__ poff, uint64_t *__restrict__ key,
                                                      double *__restrict__ val, int32_t *__restrict__ ocol,
                                                      double *__restrict__ oval, int64_t *__restrict__ ucount,
                                                      int32_t *flags) {
  __shared__ uint64_t sk[kSortCap];
  __shared__ double sv[kSortCap];
  __shared__ int heads[kSortCap + 1];
  for (int64_t j = blockIdx.x; j < n; j += gridDim.x) {
    const int64_t S = poff[cptr[j]], P = poff[cptr[j + 1]] - S;
    if (P > kSortCap) {
      if (threadIdx.x == 0) ucount[j] = -1;
      continue;
    }
    int N = 1;
    while (N < P) N <<= 1;
    __syncthreads();
    for (int t = threadIdx.x; t < N; t += blockDim.x) {
      sk[t] = t < P ? key[S + t] : ~0ull;
      sv[t] = t < P ? val[S + t] : 0.0;
    }
    __syncthreads();
    bitonic_block(sk, sv, N);
    // output positions are offset by the row's own index so that a row
    // with P products can hold P + 1 entries (the inserted diagonal)
    reduce_sorted_row<kSortT>(sk, sv, P, (int32_t)j, ocol + S + j, oval + S + j, heads, &ucount[j], flags);
  }
}

// rows with more products than fit in LDS: global-memory bitonic sort in a
// padded scratch copy, one block per row, rows taken from a host list
__global__ __launch_bounds__(1024) void k_row_big(int64_t j, const int64_t *__restrict__ cptr,
                                                  const int64_t *__restrict__ poff, const uint64_t *__restrict__ key,
                                                  const double *__restrict__ val, uint64_t *__restrict__ sk,
                                                  double *__restrict__ sv, int *__restrict__ heads, int N,
                                                  int32_t *__restrict__ ocol, double *__restrict__ oval,
                                                  int64_t *__restrict__ ucount, int32_t *flags) {
  const int64_t S = poff[cptr[j]], P = poff[cptr[j + 1]] - S;
  for (int t = threadIdx.x; t < N; t += blockDim.x) {
    sk[t] = t < P ? key[S + t] : ~0ull;
    sv[t] = t < P ? val[S + t] : 0.0;
  }
  __syncthreads();
  bitonic_block(sk, sv, N);
  reduce_sorted_row<1024>(sk, sv, P, (int32_t)j, ocol + S + j, oval + S + j, heads, &ucount[j], flags);
}

__global__ void k_gather_M(int64_t n, const int64_t *__restrict__ cptr, const int64_t *__restrict__ poff,
                           const int64_t *__restrict__ mptr, const int32_t *__restrict__ ocol,
                           const double *__restrict__ oval, int32_t *__restrict__ Mrp, int32_t *__restrict__ Mci,
                           double *__restrict__ Mv, int32_t *__restrict__ Mdiag) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t j = wave; j < n; j += nwaves) {
    const int64_t src = poff[cptr[j]] + j, dst = mptr[j], cntj = mptr[j + 1] - mptr[j];
    for (int64_t q = lane; q < cntj; q += 64) {
      int32_t c = ocol[src + q];
      Mci[dst + q] = c;
      Mv[dst + q] = oval[src + q];
      if (c == (int32_t)j) Mdiag[j] = (int32_t)(dst + q);
    }
    if (lane == 0) Mrp[j] = (int32_t)dst;
    if (lane == 0 && j == n - 1) Mrp[n] = (int32_t)mptr[n];
  }
}

// exclusive int64 scan of x (in place) with a trailing total at x[n]; uses
// the scan kernels of the setup via a small host helper
static void scan_i64_inplace(int64_t *x, int64_t n, int64_t *tmp, hipStream_t st);

}  // namespace lsq

// ---------------------------------------------------------------------------
// host driver of the sparse Gram build

namespace lsq {

// simple exclusive scan for int64 arrays (block sums -> offsets -> local)
__global__ __launch_bounds__(256) void k_i64_blocksum(int64_t n, const int64_t *__restrict__ x, int64_t *__restrict__ bs) {
  __shared__ int64_t red[4];
  const int64_t base = blockIdx.x * 4096ll + threadIdx.x * 16ll;
  int64_t acc = 0;
  for (int e = 0; e < 16; ++e)
    if (base + e < n) acc += x[base + e];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) bs[blockIdx.x] = acc;
}
__global__ void k_i64_offsets(int64_t nb, int64_t *bs) {
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int64_t b = 0; b < nb; ++b) {
      int64_t v = bs[b];
      bs[b] = run;
      run += v;
    }
    bs[nb] = run;
  }
}
__global__ __launch_bounds__(256) void k_i64_local(int64_t n, int64_t *__restrict__ x, const int64_t *__restrict__ bs) {
  __shared__ int64_t ts[256];
  const int64_t base = blockIdx.x * 4096ll + threadIdx.x * 16ll;
  int64_t v[16];
  int64_t acc = 0;
  for (int e = 0; e < 16; ++e) {
    v[e] = base + e < n ? x[base + e] : 0;
    acc += v[e];
  }
  ts[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int t = 0; t < 256; ++t) {
      int64_t a = ts[t];
      ts[t] = run;
      run += a;
    }
  }
  __syncthreads();
  int64_t run = bs[blockIdx.x] + ts[threadIdx.x];
  for (int e = 0; e < 16; ++e)
    if (base + e < n) {
      x[base + e] = run;
      run += v[e];
    }
}
__global__ void k_i64_total(int64_t n, int64_t *x, const int64_t *bs, int64_t nb) { x[n] = bs[nb]; }

// tmp must hold n/4096 + 2 entries; x must hold n + 1
static void scan_i64_inplace(int64_t *x, int64_t n, int64_t *tmp, hipStream_t st) {
  int64_t nb = (n + 4095) / 4096;
  if (nb < 1) nb = 1;
  k_i64_blocksum<<<(unsigned)nb, 256, 0, st>>>(n, x, tmp);
  k_i64_offsets<<<1, 64, 0, st>>>(nb, tmp);
  k_i64_local<<<(unsigned)nb, 256, 0, st>>>(n, x, tmp);
  k_i64_total<<<1, 1, 0, st>>>(n, x, tmp, nb);
}

static unsigned waves_grid(int64_t items) {
  int64_t b = (items * 64 + 255) / 256;
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return (unsigned)b;
}

int build_sparse_gram(lsq_ctx *ctx) {
  hipStream_t st = ctx->stream;
  const int64_t n = ctx->n, sd = ctx->s_d;
  int64_t *cptr = (int64_t *)lsq_alloc(ctx, (n + 1) * sizeof(int64_t));
  int64_t *cfill = (int64_t *)lsq_alloc(ctx, (n + 1) * sizeof(int64_t));
  int64_t *tmp = (int64_t *)lsq_alloc(ctx, ((n + 4095) / 4096 + 2) * sizeof(int64_t));
  if (!cptr || !cfill || !tmp) return LSQ_ENOMEM;
  LSQ_HIP_CHECK(hipMemsetAsync(cptr, 0, (n + 1) * sizeof(int64_t), st));
  LSQ_HIP_CHECK(hipMemsetAsync(cfill, 0, (n + 1) * sizeof(int64_t), st));
  k_col_counts<<<waves_grid(sd), 256, 0, st>>>(sd, ctx->urow, ctx->rp, ctx->ci, cptr);
  scan_i64_inplace(cptr, n, tmp, st);
  int64_t E = 0;
  LSQ_HIP_CHECK(hipMemcpyAsync(&E, cptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  LSQ_HIP_CHECK(hipStreamSynchronize(st));

  int32_t *csc_r = (int32_t *)lsq_alloc(ctx, (E + 1) * sizeof(int32_t));
  int64_t *csc_k = (int64_t *)lsq_alloc(ctx, (E + 1) * sizeof(int64_t));
  int64_t *poff = (int64_t *)lsq_alloc(ctx, (E + 1) * sizeof(int64_t));
  int64_t *tmp2 = (int64_t *)lsq_alloc(ctx, ((E + 4095) / 4096 + 2) * sizeof(int64_t));
  if (!csc_r || !csc_k || !poff || !tmp2) return LSQ_ENOMEM;
  k_csc_fill<<<waves_grid(sd), 256, 0, st>>>(sd, ctx->urow, ctx->rp, ctx->ci, cptr, cfill, csc_r, csc_k, poff);
  scan_i64_inplace(poff, E, tmp2, st);
  int64_t P = 0;
  LSQ_HIP_CHECK(hipMemcpyAsync(&P, poff + E, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  LSQ_HIP_CHECK(hipStreamSynchronize(st));

  uint64_t *key = (uint64_t *)lsq_alloc(ctx, (P + 1) * sizeof(uint64_t));
  double *val = (double *)lsq_alloc(ctx, (P + 1) * sizeof(double));
  // reduced rows: each row's segment may grow by one (the diagonal)
  int32_t *ocol = (int32_t *)lsq_alloc(ctx, (P + n + 1) * sizeof(int32_t));
  double *oval = (double *)lsq_alloc(ctx, (P + n + 1) * sizeof(double));
  int64_t *ucount = (int64_t *)lsq_alloc(ctx, (n + 1) * sizeof(int64_t));
  if (!key || !val || !ocol || !oval || !ucount) return LSQ_ENOMEM;
  {
    // lanes per CSC entry from the average row length of A
    const double avg = (double)ctx->nnz / (double)std::max<int64_t>(1, ctx->m);
    const int G = avg <= 2 ? 2 : avg <= 4 ? 4 : avg <= 8 ? 8 : avg <= 16 ? 16 : 32;
    int64_t b = (E * G + 255) / 256;
    if (b > 16384) b = 16384;
    if (b < 1) b = 1;
    const double *Wp = ctx->cdf + ctx->m - 1;
#define LSQ_EXPAND(TA, GG)                                                                                        \
  k_expand<TA, GG><<<(unsigned)b, 256, 0, st>>>(E, csc_r, csc_k, poff, ctx->urow, ctx->ucnt, ctx->rp, ctx->ci, \
                                                (const TA *)ctx->A, ctx->w, ctx->invD, Wp, (double)ctx->s, key, val)
    if (ctx->dtype == LSQ_F64) {
      switch (G) {
        case 2: LSQ_EXPAND(double, 2); break;
        case 4: LSQ_EXPAND(double, 4); break;
        case 8: LSQ_EXPAND(double, 8); break;
        case 16: LSQ_EXPAND(double, 16); break;
        default: LSQ_EXPAND(double, 32); break;
      }
    } else {
      switch (G) {
        case 2: LSQ_EXPAND(float, 2); break;
        case 4: LSQ_EXPAND(float, 4); break;
        case 8: LSQ_EXPAND(float, 8); break;
        case 16: LSQ_EXPAND(float, 16); break;
        default: LSQ_EXPAND(float, 32); break;
      }
    }
#undef LSQ_EXPAND
  }
  // the product offset of column j's first CSC entry: poff[cptr[j]]
  {
    int64_t g = n < 65536 ? n : 65536;
    k_row_small<<<(unsigned)(g > 0 ? g : 1), kSortT, 0, st>>>(n, cptr, poff, key, val, ocol, oval, ucount,
                                                                ctx->flags);
  }
  // rows too long for LDS
  std::vector<int64_t> hcount(n);
  LSQ_HIP_CHECK(hipMemcpyAsync(hcount.data(), ucount, n * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  LSQ_HIP_CHECK(hipStreamSynchronize(st));
  std::vector<int64_t> big;
  for (int64_t j = 0; j < n; ++j)
    if (hcount[j] < 0) big.push_back(j);
  if (!big.empty()) {
    std::vector<int64_t> hcptr(n + 1);
    LSQ_HIP_CHECK(hipMemcpy(hcptr.data(), cptr, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
    int64_t maxP = 0;
    std::vector<int64_t> bigP(big.size());
    for (size_t q = 0; q < big.size(); ++q) {
      int64_t a = 0, bb = 0;
      LSQ_HIP_CHECK(hipMemcpy(&a, poff + hcptr[big[q]], sizeof(int64_t), hipMemcpyDeviceToHost));
      LSQ_HIP_CHECK(hipMemcpy(&bb, poff + hcptr[big[q] + 1], sizeof(int64_t), hipMemcpyDeviceToHost));
      bigP[q] = bb - a;
      maxP = std::max(maxP, bb - a);
    }
    int64_t N = 1;
    while (N < maxP) N <<= 1;
    if (N > (int64_t)1 << 30) return LSQ_EINVAL;
    uint64_t *sk = (uint64_t *)lsq_alloc(ctx, N * sizeof(uint64_t));
    double *sv = (double *)lsq_alloc(ctx, N * sizeof(double));
    int *heads = (int *)lsq_alloc(ctx, (N + 1) * sizeof(int));
    if (!sk || !sv || !heads) return LSQ_ENOMEM;
    for (size_t q = 0; q < big.size(); ++q) {
      int Nq = 1;
      while (Nq < bigP[q]) Nq <<= 1;
      k_row_big<<<1, 1024, 0, st>>>(big[q], cptr, poff, key, val, sk, sv, heads, Nq, ocol, oval, ucount, ctx->flags);
    }
  }
  // row pointers of M
  int64_t *mptr = (int64_t *)lsq_alloc(ctx, (n + 1) * sizeof(int64_t));
  if (!mptr) return LSQ_ENOMEM;
  LSQ_HIP_CHECK(hipMemcpyAsync(mptr, ucount, n * sizeof(int64_t), hipMemcpyDeviceToDevice, st));
  scan_i64_inplace(mptr, n, tmp, st);
  int64_t nnzM = 0;
  LSQ_HIP_CHECK(hipMemcpyAsync(&nnzM, mptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  LSQ_HIP_CHECK(hipStreamSynchronize(st));
  if (nnzM >= ((int64_t)1 << 31)) {
    ctx->err = "M has more than 2^31 entries";
    return LSQ_EINVAL;
  }
  ctx->nnzM = nnzM;
  ctx->Mrp = (int32_t *)lsq_alloc(ctx, (n + 1) * sizeof(int32_t));
  ctx->Mci = (int32_t *)lsq_alloc(ctx, (nnzM + 1) * sizeof(int32_t));
  ctx->Md = (double *)lsq_alloc(ctx, (nnzM + 1) * sizeof(double));
  ctx->Mdiag = (int32_t *)lsq_alloc(ctx, n * sizeof(int32_t));
  if (!ctx->Mrp || !ctx->Mci || !ctx->Md || !ctx->Mdiag) return LSQ_ENOMEM;
  k_gather_M<<<waves_grid(n), 256, 0, st>>>(n, cptr, poff, mptr, ocol, oval, ctx->Mrp, ctx->Mci, ctx->Md, ctx->Mdiag);
  LSQ_HIP_CHECK(hipGetLastError());
  return LSQ_OK;
}

}  // namespace lsq
