// The per-iteration product of Algorithm 2 step 4: only Ax and A^T(Ax) are
// needed (Section 4.2), here fused into one pass over A. For each row a_i the
// pass forms t_i = hb*b_i - a_i . u and accumulates t_i a_i^T into the output,
// so A is read once per product:
//   K p = D^{-1} A^T A D^{-1} p   (u = D^{-1} p, hb = 0, output scaled by D^{-1})
//   g   = A^T (b - A x)           (u = x, hb = 1: the float64 refinement residual)
//
// Dense A (row-major): one wave per row; lane l holds columns l, l+64, ...,
// so every load instruction moves 64 consecutive elements; the row dot is a
// wave reduction and the rank-1 update stays in registers; each block writes
// one partial output row and a second kernel sums the partial rows in a fixed
// order.
//
// CSR A: G lanes per row; the scatter of t_i a_i goes to global memory with
// atomic adds, or (n small enough) to a per-block LDS accumulator flushed
// once per block.
#include <algorithm>

#include "common.h"

namespace lsq {

constexpr int kAtThreads = 256, kAtWaves = kAtThreads / kWave;
constexpr int kDenseLdsBlocks = 512;  // two per CU

template <typename TA, typename CT, int NC, bool HAS_B>
__global__ __launch_bounds__(kAtThreads) void k_atap_dense(int64_t m, int n, int64_t ld, const TA *__restrict__ A,
                                                           const CT *__restrict__ u, const double *__restrict__ b,
                                                           CT *__restrict__ part, int64_t rows_per_blk) {
  __shared__ CT red[64 * NC];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  CT ur[NC], acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int j = lane + 64 * c;
    ur[c] = j < n ? u[j] : (CT)0;
    acc[c] = 0;
  }
  const int64_t r0 = blockIdx.x * rows_per_blk;
  int64_t r1 = r0 + rows_per_blk;
  if (r1 > m) r1 = m;
  int64_t i = r0 + wave;
  // two rows per step keep twice the loads in flight
  for (; i + kAtWaves < r1; i += 2 * kAtWaves) {
    const TA *row0 = A + i * ld;
    const TA *row1 = A + (i + kAtWaves) * ld;
    CT a0[NC], a1[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int j = lane + 64 * c;
      a0[c] = j < n ? (CT)row0[j] : (CT)0;
      a1[c] = j < n ? (CT)row1[j] : (CT)0;
    }
    CT d0 = 0, d1 = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      d0 += a0[c] * ur[c];
      d1 += a1[c] * ur[c];
    }
    d0 = wave_sum(d0);
    d1 = wave_sum(d1);
    if (HAS_B) {
      d0 = (CT)b[i] - d0;
      d1 = (CT)b[i + kAtWaves] - d1;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] += d0 * a0[c] + d1 * a1[c];
  }
  if (i < r1) {
    const TA *row0 = A + i * ld;
    CT a0[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int j = lane + 64 * c;
      a0[c] = j < n ? (CT)row0[j] : (CT)0;
    }
    CT d0 = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) d0 += a0[c] * ur[c];
    d0 = wave_sum(d0);
    if (HAS_B) d0 = (CT)b[i] - d0;
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] += d0 * a0[c];
  }
  // combine the four waves in a fixed order
  for (int w = 0; w < kAtWaves; ++w) {
    if (wave == w) {
#pragma unroll
      for (int c = 0; c < NC; ++c) red[lane + 64 * c] = (w == 0 ? (CT)0 : red[lane + 64 * c]) + acc[c];
    }
    __syncthreads();
  }
  for (int j = threadIdx.x; j < n; j += kAtThreads) part[blockIdx.x * (int64_t)n + j] = red[j];
}

// Dense A, one wave per row with VEC-wide loads: lane l holds columns
// VEC*l + 64*VEC*c + e (e < VEC), so one load instruction moves 64*VEC
// consecutive elements (16 bytes per lane). Needs n % VEC == 0 and rows aligned
// to VEC elements. Otherwise as k_atap_dense.
template <typename T, int V>
struct VecT;
template <>
struct VecT<float, 4> {
  typedef float4 type;
};
template <>
struct VecT<double, 2> {
  typedef double2 type;
};
template <typename TA, int V>
__device__ __forceinline__ void vload(const TA *p, TA (&out)[V]) {
  typedef typename VecT<TA, V>::type VT;
  const VT v = *(const VT *)p;
  if constexpr (V == 4) {
    out[0] = v.x;
    out[1] = v.y;
    out[2] = v.z;
    out[3] = v.w;
  } else {
    out[0] = v.x;
    out[1] = v.y;
  }
}

template <typename TA, typename CT, int NC, int V, bool HAS_B>
__global__ __launch_bounds__(kAtThreads) void k_atap_dense_vec(int64_t m, int n, int64_t ld, const TA *__restrict__ A,
                                                               const CT *__restrict__ u, const double *__restrict__ b,
                                                               CT *__restrict__ part, int64_t rows_per_blk) {
  __shared__ CT red[64 * NC * V];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  CT ur[NC][V], acc[NC][V];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const int j = V * lane + kWave * V * c + e;
      ur[c][e] = j < n ? u[j] : (CT)0;
      acc[c][e] = 0;
    }
  const int64_t r0 = blockIdx.x * rows_per_blk;
  int64_t r1 = r0 + rows_per_blk;
  if (r1 > m) r1 = m;
  for (int64_t i = r0 + wave; i < r1; i += 2 * kAtWaves) {
    const bool two = i + kAtWaves < r1;
    const TA *row0 = A + i * ld;
    const TA *row1 = A + (two ? i + kAtWaves : i) * ld;
    TA a0[NC][V], a1[NC][V];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int j = V * lane + kWave * V * c;
      if (j < n) {
        vload<TA, V>(row0 + j, a0[c]);
        vload<TA, V>(row1 + j, a1[c]);
      } else {
#pragma unroll
        for (int e = 0; e < V; ++e) a0[c][e] = a1[c][e] = 0;
      }
    }
    CT d0 = 0, d1 = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int e = 0; e < V; ++e) {
        d0 += (CT)a0[c][e] * ur[c][e];
        d1 += (CT)a1[c][e] * ur[c][e];
      }
    d0 = wave_sum(d0);
    d1 = wave_sum(d1);
    if (HAS_B) {
      d0 = (CT)b[i] - d0;
      d1 = two ? (CT)b[i + kAtWaves] - d1 : (CT)0;
    }
    if (!two) d1 = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int e = 0; e < V; ++e) acc[c][e] += d0 * (CT)a0[c][e] + d1 * (CT)a1[c][e];
  }
  // combine the four waves in a fixed order
  for (int w = 0; w < kAtWaves; ++w) {
    if (wave == w) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int e = 0; e < V; ++e) {
          const int k = V * lane + kWave * V * c + e;
          red[k] = (w == 0 ? (CT)0 : red[k]) + acc[c][e];
        }
    }
    __syncthreads();
  }
  for (int j = threadIdx.x; j < n; j += kAtThreads) part[blockIdx.x * (int64_t)n + j] = red[j];
}

// Dense A, LDS-staged batches: a block takes R consecutive rows at a time.
// Phase 1: wave w streams rows w, w+4, ... of the batch from HBM (64
// consecutive elements per load instruction), forms t_r = a_r . u, or
// b_r - a_r . u for the residual form (u staged in LDS once), and copies the
// row into LDS. Phase 2: thread t adds
// sum_r t_r a_r[j] for its columns j = t, t+256, ... from LDS. A is read from
// HBM once, the per-thread state is NC accumulators, and each block writes
// one partial output row.
template <typename TA, typename CT, int NC, bool HAS_B>
__global__ __launch_bounds__(kAtThreads) void k_atap_dense_lds(int64_t m, int n, int64_t ld, const TA *__restrict__ A,
                                                               const CT *__restrict__ u, const double *__restrict__ b,
                                                               CT *__restrict__ part, int64_t rows_per_blk, int R) {
  extern __shared__ __align__(16) unsigned char smem[];
  CT *us = (CT *)smem;   // n
  CT *ts = us + n;       // R
  TA *rows = (TA *)(ts + R + (R & 1));  // R x n
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  for (int j = threadIdx.x; j < n; j += kAtThreads) us[j] = u[j];
  CT acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = 0;
  const int64_t r0 = blockIdx.x * rows_per_blk;
  const int64_t r1 = r0 + rows_per_blk < m ? r0 + rows_per_blk : m;
  __syncthreads();
  constexpr int NR = 4 * NC;  // elements per lane of one row (n <= 256 NC)
  constexpr int RW = sizeof(TA) * NR <= 128 ? 2 : 1;  // rows in flight per wave
  for (int64_t rb = r0; rb < r1; rb += R) {
    const int nr = (int)(r1 - rb < R ? r1 - rb : R);
    // RW rows per wave at a time, each loaded in one burst of NR loads
    for (int r = wave; r < nr; r += RW * kAtWaves) {
      TA a[RW][NR];
#pragma unroll
      for (int w = 0; w < RW; ++w) {
        const int rr = r + w * kAtWaves < nr ? r + w * kAtWaves : r;
        const TA *row = A + (rb + rr) * ld;
#pragma unroll
        for (int c = 0; c < NR; ++c) {
          const int j = lane + kWave * c;
          a[w][c] = j < n ? row[j] : (TA)0;
        }
      }
#pragma unroll
      for (int w = 0; w < RW; ++w) {
        const int rr = r + w * kAtWaves;
        if (rr >= nr) break;  // wave-uniform
        TA *dst = rows + (int64_t)rr * n;
        CT d = 0;
#pragma unroll
        for (int c = 0; c < NR; ++c) {
          const int j = lane + kWave * c;
          if (j < n) {
            d += (CT)a[w][c] * us[j];
            dst[j] = a[w][c];
          }
        }
        d = wave_sum(d);
        if (lane == 0) ts[rr] = HAS_B ? (CT)b[rb + rr] - d : d;
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int j = threadIdx.x + kAtThreads * c;
      if (j < n) {
        CT sacc = 0;
        for (int r = 0; r < nr; ++r) sacc += ts[r] * (CT)rows[(int64_t)r * n + j];
        acc[c] += sacc;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int j = threadIdx.x + kAtThreads * c;
    if (j < n) part[blockIdx.x * (int64_t)n + j] = acc[c];
  }
}

// Dense A, column-owned row batches: thread t of the block owns the V-element
// groups t, t + 256, ... of every row (16-byte loads, consecutive threads on
// consecutive groups), so A goes from HBM straight to registers and each
// thread keeps its columns' output sums in registers. A batch of RB rows is
// requested while the previous batch is reduced: each thread forms its part
// of every row dot, the parts are summed over the wave (DPP) and over the
// four waves (LDS, one barrier per batch, fixed order), and each thread adds
// t_r a_r for its columns. Needs n % V == 0 and rows aligned to 16 bytes.
template <typename TA, typename CT, int NC, int V, int RB, bool HAS_B>
__global__ __launch_bounds__(kAtThreads) void k_atap_dense_cols(int64_t m, int n, int64_t ld,
                                                                const TA *__restrict__ A, const CT *__restrict__ u,
                                                                const double *__restrict__ b, CT *__restrict__ part,
                                                                int64_t rows_per_blk) {
  __shared__ CT red[2][kAtWaves][RB];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int ng = n / V;  // V-element groups per row
  int gi[NC];            // this thread's groups, clamped in range
  bool gon[NC];
  CT uv[NC][V], acc[NC][V];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int g = threadIdx.x + kAtThreads * c;
    gon[c] = g < ng;
    gi[c] = gon[c] ? g : ng - 1;
#pragma unroll
    for (int e = 0; e < V; ++e) {
      uv[c][e] = gon[c] ? u[gi[c] * V + e] : (CT)0;
      acc[c][e] = 0;
    }
  }
  const int64_t r0 = blockIdx.x * rows_per_blk;
  const int64_t r1 = r0 + rows_per_blk < m ? r0 + rows_per_blk : m;
  const int nbatch = (int)((r1 - r0 + RB - 1) / RB);
  TA a[2][RB][NC][V];
  auto load = [&](int k, TA (&dst)[RB][NC][V]) {
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      int64_t row = r0 + (int64_t)k * RB + r;
      row = row < r1 ? row : r1 - 1;
      const TA *p = A + row * ld;
#pragma unroll
      for (int c = 0; c < NC; ++c) vload<TA, V>(p + gi[c] * V, dst[r][c]);
    }
  };
  auto consume = [&](int k, const TA (&src)[RB][NC][V]) {
    CT d[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      CT s = 0;
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int e = 0; e < V; ++e) s += gon[c] ? (CT)src[r][c][e] * uv[c][e] : (CT)0;
      d[r] = dpp_group_sum<kWave>(s);
    }
    if (lane == dpp_sum_lane<kWave>())
#pragma unroll
      for (int r = 0; r < RB; ++r) red[k & 1][wave][r] = d[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int64_t row = r0 + (int64_t)k * RB + r;
      CT t = 0;
#pragma unroll
      for (int w = 0; w < kAtWaves; ++w) t += red[k & 1][w][r];
      if (HAS_B) t = (CT)b[row < r1 ? row : r1 - 1] - t;
      t = row < r1 ? t : (CT)0;
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int e = 0; e < V; ++e) acc[c][e] += t * (CT)src[r][c][e];
    }
  };
  if (nbatch > 0) load(0, a[0]);
  for (int k = 0; k < nbatch; k += 2) {
    if (k + 1 < nbatch) load(k + 1, a[1]);
    consume(k, a[0]);
    if (k + 1 >= nbatch) break;
    if (k + 2 < nbatch) load(k + 2, a[0]);
    consume(k + 1, a[1]);
  }
#pragma unroll
  for (int c = 0; c < NC; ++c)
    if (gon[c])
#pragma unroll
      for (int e = 0; e < V; ++e) part[blockIdx.x * (int64_t)n + gi[c] * V + e] = acc[c][e];
}

// first level of the partial-row reduction: blockIdx.y sums rows
// [y*seg, (y+1)*seg) of part into row y of out (fixed order)
template <typename CT>
__global__ void k_part_reduce(int64_t n, const CT *__restrict__ part, int nblk, int seg, CT *__restrict__ out) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int b0 = blockIdx.y * seg;
  int b1 = b0 + seg;
  if (b1 > nblk) b1 = nblk;
  CT s = 0;
  for (int b = b0; b < b1; ++b) s += part[(int64_t)b * n + j];
  out[blockIdx.y * n + j] = s;
}

template <typename CT>
__global__ void k_atap_finish(int64_t n, const CT *__restrict__ part, int nblk, const CT *__restrict__ s_out,
                              CT *__restrict__ q) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    CT s = 0;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * n + j];
    q[j] = s_out ? s * s_out[j] : s;
  }
}

// generic dense fallback for n > 2048: y = hb*b - A u, then per-block column
// partials of A^T y
template <typename TA, typename CT, bool HAS_B>
__global__ __launch_bounds__(kAtThreads) void k_gemv_rows(int64_t m, int64_t n, int64_t ld, const TA *__restrict__ A,
                                                          const CT *__restrict__ u, const double *__restrict__ b,
                                                          CT *__restrict__ y) {
  const int lane = threadIdx.x % kWave;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t i = wave; i < m; i += nw) {
    CT d = 0;
    for (int64_t j = lane; j < n; j += 64) d += (CT)A[i * ld + j] * u[j];
    d = wave_sum(d);
    if (lane == 0) y[i] = HAS_B ? (CT)b[i] - d : d;
  }
}

template <typename TA, typename CT>
__global__ __launch_bounds__(kAtThreads) void k_gemv_t_part(int64_t m, int64_t n, int64_t ld, const TA *__restrict__ A,
                                                            const CT *__restrict__ y, CT *__restrict__ part,
                                                            int64_t rows_per_blk) {
  const int64_t r0 = blockIdx.x * rows_per_blk;
  int64_t r1 = r0 + rows_per_blk;
  if (r1 > m) r1 = m;
  for (int64_t j = threadIdx.x; j < n; j += kAtThreads) {
    CT s = 0;
    for (int64_t i = r0; i < r1; ++i) s += (CT)A[i * ld + j] * y[i];
    part[blockIdx.x * n + j] = s;
  }
}

// ---------------------------------------------------------------------------
// CSR

// One pass over rows [r0, r1) of a CSR matrix by groups of G lanes: group g
// takes rows r0 + (it*U + u)*ngrp + g, U rows at a time, so the row pointers,
// entries and b values of U rows are requested before any of them is used
// (enough bytes in flight to cover the memory latency), and at each u the
// groups of a block read one contiguous stretch of entries. For each row it
// forms d = a_i . u (d = b_i - a_i . u with HAS_B), calls emit(i, d) on the
// row's first lane and, with SCATTER, add(j, d a_ij) for its entries.
template <typename TA, typename CT, int G, int U, bool HAS_B, bool SCATTER, int NT, typename Gather, typename Add,
          typename Emit>
__device__ __forceinline__ void csr_rows_pass(int64_t r0, int64_t r1, const int64_t *__restrict__ rp,
                                              const int32_t *__restrict__ ci, const TA *__restrict__ v,
                                              const double *__restrict__ b, Gather uget, Add add, Emit emit) {
  constexpr int ngrp = NT / G;
  const int gl = threadIdx.x % G;
  const int grp = threadIdx.x / G;
  for (int64_t base = r0; base < r1; base += (int64_t)ngrp * U) {
    TA av[U];
    int32_t aj[U];
    double bv[U];
    int onrows = 0;    // rows with an entry in this lane
    int longrows = 0;  // rows with more than G entries (their rest is read again below)
    // loads are issued unconditionally from clamped indices and their
    // results selected afterwards: a guarded load becomes a branch with a
    // wait for every earlier load
    int64_t k0[U], k1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + u * ngrp + grp;
      const int64_t ic = i < r1 ? i : r0;
      k0[u] = rp[ic];
      k1[u] = rp[ic + 1];
      if (HAS_B) bv[u] = b[ic];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = base + u * ngrp + grp < r1;
      const int64_t len = (k1[u] - k0[u]) & -(int64_t)ok;
      const bool on = gl < len;
      const int64_t k = on ? k0[u] + gl : 0;
      av[u] = v[k];
      aj[u] = ci[k];
      onrows |= on ? 1 << u : 0;
      longrows |= len > G ? 1 << u : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      av[u] = (onrows >> u) & 1 ? av[u] : (TA)0;
      aj[u] = (onrows >> u) & 1 ? aj[u] : 0;
    }
    CT d[U];
#pragma unroll
    for (int u = 0; u < U; ++u) d[u] = (CT)av[u] * uget(aj[u]);
    if (longrows) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (!((longrows >> u) & 1)) continue;
        const int64_t i = base + u * ngrp + grp;
        const int64_t k1 = i < r1 ? rp[i + 1] : 0;
        for (int64_t k = (i < r1 ? rp[i] : 0) + G + gl; k < k1; k += G) d[u] += (CT)v[k] * uget(ci[k]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      d[u] = group_sum<G>(d[u]);
      if (HAS_B) d[u] = (CT)bv[u] - d[u];
      const int64_t i = base + u * ngrp + grp;
      if (gl == 0 && i < r1) emit(i, d[u]);
    }
    if (!SCATTER) continue;
#pragma unroll
    for (int u = 0; u < U; ++u)
      if ((onrows >> u) & 1) add(aj[u], d[u] * (CT)av[u]);
    if (longrows) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (!((longrows >> u) & 1)) continue;
        const int64_t i = base + u * ngrp + grp;
        const int64_t k1 = i < r1 ? rp[i + 1] : 0;
        for (int64_t k = (i < r1 ? rp[i] : 0) + G + gl; k < k1; k += G) add(ci[k], d[u] * (CT)v[k]);
      }
    }
  }
}

// rows in flight per group: enough that a block has tens of KB of A requested
template <int G>
constexpr int csr_unroll() {
  return G <= 16 ? 8 : (G == 32 ? 4 : 2);
}

template <typename TA, typename CT, int G, bool HAS_B>
__global__ __launch_bounds__(kAtThreads) void k_atap_csr(int64_t m, int n, const int64_t *__restrict__ rp,
                                                         const int32_t *__restrict__ ci, const TA *__restrict__ v,
                                                         const CT *__restrict__ u, const double *__restrict__ b,
                                                         CT *__restrict__ q, int64_t rows_per_blk) {
  const int64_t r0 = blockIdx.x * rows_per_blk;
  const int64_t r1 = r0 + rows_per_blk < m ? r0 + rows_per_blk : m;
  csr_rows_pass<TA, CT, G, csr_unroll<G>(), HAS_B, true, kAtThreads>(
      r0, r1, rp, ci, v, b, [&](int j) -> CT { return u[j]; }, [&](int j, CT a) { atomicAdd(&q[j], a); },
      [](int64_t, CT) {});
}

// per-workgroup accumulation in LDS; each workgroup writes one partial output
// row, summed over workgroups in a fixed order by k_atap_finish
constexpr int kLdsThreads = 1024, kLdsBlocks = 256;

template <typename TA, typename CT, int G, bool HAS_B, bool USTAGE>
__global__ __launch_bounds__(kLdsThreads) void k_atap_csr_lds(int64_t m, int n, const int64_t *__restrict__ rp,
                                                              const int32_t *__restrict__ ci,
                                                              const TA *__restrict__ v, const CT *__restrict__ ug,
                                                              const double *__restrict__ b, CT *__restrict__ part,
                                                              int64_t rows_per_blk) {
  extern __shared__ __align__(16) unsigned char smem[];
  CT *qs = (CT *)smem;
  CT *us = qs + n;  // a copy of u when it fits beside the accumulator
  for (int j = threadIdx.x; j < n; j += kLdsThreads) {
    qs[j] = 0;
    if (USTAGE) us[j] = ug[j];
  }
  __syncthreads();
  const CT *u = USTAGE ? us : ug;
  const int64_t r0 = blockIdx.x * rows_per_blk;
  const int64_t r1 = r0 + rows_per_blk < m ? r0 + rows_per_blk : m;
  csr_rows_pass<TA, CT, G, csr_unroll<G>(), HAS_B, true, kLdsThreads>(
      r0, r1, rp, ci, v, b, [&](int j) -> CT { return u[j]; }, [&](int j, CT a) { atomicAdd(&qs[j], a); },
      [](int64_t, CT) {});
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += kLdsThreads) part[blockIdx.x * (int64_t)n + j] = qs[j];
}

// one row pass without scatter: out_i = scale_i * (hb b_i - a_i . u), for the
// two-pass product (rows of A with u = D^{-1} p, then rows of the CSC copy,
// i.e. columns of A, with u = t)
template <typename TA, typename CT, typename UT, int G, bool HAS_B>
__global__ __launch_bounds__(kAtThreads) void k_csr_dot(int64_t m, const int64_t *__restrict__ rp,
                                                        const int32_t *__restrict__ ci, const TA *__restrict__ v,
                                                        const UT *__restrict__ u, const double *__restrict__ b,
                                                        const CT *__restrict__ scale, UT *__restrict__ out,
                                                        int64_t rows_per_blk) {
  const int64_t r0 = blockIdx.x * rows_per_blk;
  const int64_t r1 = r0 + rows_per_blk < m ? r0 + rows_per_blk : m;
  csr_rows_pass<TA, CT, G, csr_unroll<G>(), HAS_B, false, kAtThreads>(
      r0, r1, rp, ci, v, b, [&](int j) -> CT { return (CT)u[j]; }, [](int, CT) {},
      [&](int64_t i, CT d) { out[i] = (UT)(scale ? scale[i] * d : d); });
}

template <typename CT>
__global__ void k_scale_inplace(int64_t n, const CT *__restrict__ s, CT *__restrict__ q) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    q[j] *= s[j];
}

// ---------------------------------------------------------------------------
// dispatch

void atap_f64_impl(lsq_ctx *c, const double *s_in, const double *p, const double *b, double *q,
                   const double *s_out);

static int dense_blocks(int64_t m) {
  int64_t b = m / 64;
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return (int)b;
}

template <typename TA, typename CT, bool HAS_B>
static void atap_dense_t(lsq_ctx *c, const TA *A, const CT *u, const double *b, CT *q, const CT *s_out) {
  const int64_t m = c->m, n = c->n;
  CT *part = (CT *)c->part;
  hipStream_t st = c->stream;
  const int nb = (int)n;
  const int seg = 16;
  // 16-byte loads: VEC elements per lane per load
  constexpr int V = 16 / sizeof(TA);
  const bool vec_ok = n % V == 0 && c->ld % V == 0 && ((uintptr_t)A % 16) == 0 && n <= kWave * V * 8;
  // LDS-staged batches while a batch of at least 4 rows fits in 64 KB
  const int64_t lds_budget = 64 * 1024 - 64;
  const int64_t R = std::min<int64_t>(64, (lds_budget - (n + 2) * (int64_t)sizeof(CT)) / (n * (int64_t)sizeof(TA)));
  const bool lds_ok = n <= 256 * 16 && R >= 4;
  int algo = c->opt.atap_algo;
  // column-owned batches: two groups of V columns per thread at most
  const bool cols_ok = vec_ok && n <= 2 * kAtThreads * V;
  if (algo == 4 && !cols_ok) algo = 0;
  if (algo == 0 || (algo == 3 && !vec_ok) || (algo == 2 && !lds_ok)) {
    // registers hold u, the output row and two rows of A per lane; the
    // LDS-staged form takes over when that does not fit (float storage,
    // float64 arithmetic, long rows)
    const int64_t per_lane = (n + kWave - 1) / kWave * (2 * sizeof(TA) + 2 * sizeof(CT)) / 4;
    algo = per_lane <= 128 ? (vec_ok ? 3 : 1) : (lds_ok ? 2 : 1);
    // column-owned batches for long float32 rows (2 million x 2000: 5.9 TB/s
    // against 3.1 for the LDS form with float64 arithmetic, 6.0 against 5.3
    // for one wave per row in float32) and for rows too long for registers
    if (cols_ok && n > 512 && (sizeof(TA) == 4 || per_lane > 128)) algo = 4;
  }
  if (algo == 4) {
    const int nblk = dense_blocks(m);
    const int64_t rpb = (m + nblk - 1) / nblk;
    // rows per batch: two batches of RB rows in registers (8 KB per wave each)
    if (n <= kAtThreads * V)
      k_atap_dense_cols<TA, CT, 1, V, 8, HAS_B><<<nblk, kAtThreads, 0, st>>>(m, nb, c->ld, A, u, b, part, rpb);
    else
      k_atap_dense_cols<TA, CT, 2, V, 4, HAS_B><<<nblk, kAtThreads, 0, st>>>(m, nb, c->ld, A, u, b, part, rpb);
    const int nseg = (nblk + seg - 1) / seg;
    CT *part2 = part + (int64_t)nblk * n;
    const int64_t fb = (n + 255) / 256;
    k_part_reduce<CT><<<dim3((unsigned)fb, (unsigned)nseg), 256, 0, st>>>(n, part, nblk, seg, part2);
    k_atap_finish<CT><<<(unsigned)fb, 256, 0, st>>>(n, part2, nseg, s_out, q);
    return;
  }
  if (algo == 3) {
    const int nblk = dense_blocks(m);
    const int64_t rpb = (m + nblk - 1) / nblk;
    const int nc = (int)((n + kWave * V - 1) / (kWave * V));
    if (nc <= 1) k_atap_dense_vec<TA, CT, 1, V, HAS_B><<<nblk, kAtThreads, 0, st>>>(m, nb, c->ld, A, u, b, part, rpb);
    else if (nc <= 2) k_atap_dense_vec<TA, CT, 2, V, HAS_B><<<nblk, kAtThreads, 0, st>>>(m, nb, c->ld, A, u, b, part, rpb);
    else if (nc <= 4) k_atap_dense_vec<TA, CT, 4, V, HAS_B><<<nblk, kAtThreads, 0, st>>>(m, nb, c->ld, A, u, b, part, rpb);
    else k_atap_dense_vec<TA, CT, 8, V, HAS_B><<<nblk, kAtThreads, 0, st>>>(m, nb, c->ld, A, u, b, part, rpb);
    const int nseg = (nblk + seg - 1) / seg;
    CT *part2 = part + (int64_t)nblk * n;
    const int64_t fb = (n + 255) / 256;
    k_part_reduce<CT><<<dim3((unsigned)fb, (unsigned)nseg), 256, 0, st>>>(n, part, nblk, seg, part2);
    k_atap_finish<CT><<<(unsigned)fb, 256, 0, st>>>(n, part2, nseg, s_out, q);
    return;
  }
  if (algo == 2) {
    const int nblk = (int)std::max<int64_t>(1, std::min<int64_t>(kDenseLdsBlocks, (m + R - 1) / R));
    const int64_t rpb = (m + nblk - 1) / nblk;
    const size_t lds = (n + R + 2) * sizeof(CT) + R * n * sizeof(TA);
    const int r = (int)R;
    if (n <= 256)
      k_atap_dense_lds<TA, CT, 1, HAS_B><<<nblk, kAtThreads, lds, st>>>(m, nb, c->ld, A, u, b, part, rpb, r);
    else if (n <= 512)
      k_atap_dense_lds<TA, CT, 2, HAS_B><<<nblk, kAtThreads, lds, st>>>(m, nb, c->ld, A, u, b, part, rpb, r);
    else if (n <= 1024)
      k_atap_dense_lds<TA, CT, 4, HAS_B><<<nblk, kAtThreads, lds, st>>>(m, nb, c->ld, A, u, b, part, rpb, r);
    else if (n <= 2048)
      k_atap_dense_lds<TA, CT, 8, HAS_B><<<nblk, kAtThreads, lds, st>>>(m, nb, c->ld, A, u, b, part, rpb, r);
    else
      k_atap_dense_lds<TA, CT, 16, HAS_B><<<nblk, kAtThreads, lds, st>>>(m, nb, c->ld, A, u, b, part, rpb, r);
    const int nseg = (nblk + seg - 1) / seg;
    CT *part2 = part + (int64_t)nblk * n;
    const int64_t fb = (n + 255) / 256;
    k_part_reduce<CT><<<dim3((unsigned)fb, (unsigned)nseg), 256, 0, st>>>(n, part, nblk, seg, part2);
    k_atap_finish<CT><<<(unsigned)fb, 256, 0, st>>>(n, part2, nseg, s_out, q);
    return;
  }
  const int nblk = dense_blocks(m);
  const int64_t rpb = (m + nblk - 1) / nblk;
  if (n <= 64) k_atap_dense<TA, CT, 1, HAS_B><<<nblk, kAtThreads, 0, st>>>(m, nb, c->ld, A, u, b, part, rpb);
  else if (n <= 128) k_atap_dense<TA, CT, 2, HAS_B><<<nblk, kAtThreads, 0, st>>>(m, nb, c->ld, A, u, b, part, rpb);
  else if (n <= 256) k_atap_dense<TA, CT, 4, HAS_B><<<nblk, kAtThreads, 0, st>>>(m, nb, c->ld, A, u, b, part, rpb);
  else if (n <= 512) k_atap_dense<TA, CT, 8, HAS_B><<<nblk, kAtThreads, 0, st>>>(m, nb, c->ld, A, u, b, part, rpb);
  else if (n <= 1024) k_atap_dense<TA, CT, 16, HAS_B><<<nblk, kAtThreads, 0, st>>>(m, nb, c->ld, A, u, b, part, rpb);
  else if (n <= 2048) k_atap_dense<TA, CT, 32, HAS_B><<<nblk, kAtThreads, 0, st>>>(m, nb, c->ld, A, u, b, part, rpb);
  else {
    CT *y = (CT *)c->vm;
    k_gemv_rows<TA, CT, HAS_B><<<8192, kAtThreads, 0, st>>>(m, n, c->ld, A, u, b, y);
    k_gemv_t_part<TA, CT><<<nblk, kAtThreads, 0, st>>>(m, n, c->ld, A, y, part, rpb);
  }
  const int nseg = (nblk + seg - 1) / seg;
  CT *part2 = part + (int64_t)nblk * n;
  const int64_t fb = (n + 255) / 256;
  k_part_reduce<CT><<<dim3((unsigned)(fb > 0 ? fb : 1), (unsigned)nseg), 256, 0, st>>>(n, part, nblk, seg, part2);
  k_atap_finish<CT><<<(unsigned)(fb > 0 ? fb : 1), 256, 0, st>>>(n, part2, nseg, s_out, q);
}

template <typename TA, typename CT, bool HAS_B, int G>
static void atap_csr_g(lsq_ctx *c, const TA *v, const CT *u, const double *b, CT *q, bool lds, const CT *s_out) {
  const int64_t m = c->m;
  const int n = (int)c->n;
  hipStream_t st = c->stream;
  if (lds) {
    const int64_t nblk = std::min<int64_t>(kLdsBlocks, std::max<int64_t>(1, m / 64));
    const int64_t rpb = (m + nblk - 1) / nblk;
    const bool ustage = 2 * (int64_t)n * (int64_t)sizeof(CT) <= 160 * 1024;
    auto kern = ustage ? k_atap_csr_lds<TA, CT, G, HAS_B, true> : k_atap_csr_lds<TA, CT, G, HAS_B, false>;
    static bool attr = false;
    if (!attr) {
      (void)hipFuncSetAttribute((const void *)k_atap_csr_lds<TA, CT, G, HAS_B, true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipGetLastError();
      (void)hipFuncSetAttribute((const void *)k_atap_csr_lds<TA, CT, G, HAS_B, false>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipGetLastError();
      attr = true;
    }
    CT *part = (CT *)c->part;
    const size_t lds = (size_t)n * sizeof(CT) * (ustage ? 2 : 1);
    kern<<<(unsigned)nblk, kLdsThreads, lds, st>>>(m, n, c->rp, c->ci, v, u, b, part, rpb);
    // partial rows: 16-row segments in parallel, then the segment sums
    const int seg = 16;
    const int nseg = (int)((nblk + seg - 1) / seg);
    CT *part2 = part + nblk * (int64_t)n;
    const int64_t fb = (n + 255) / 256;
    k_part_reduce<CT><<<dim3((unsigned)(fb > 0 ? fb : 1), (unsigned)nseg), 256, 0, st>>>(n, part, (int)nblk, seg, part2);
    k_atap_finish<CT><<<(unsigned)(fb > 0 ? fb : 1), 256, 0, st>>>(n, part2, nseg, s_out, q);
  } else {
    const int64_t rows_per_blk_iter = (kAtThreads / G) * csr_unroll<G>();
    int64_t nblk = (m + rows_per_blk_iter - 1) / rows_per_blk_iter;
    if (nblk > 65536) nblk = 65536;
    if (nblk < 1) nblk = 1;
    const int64_t rpb = (m + nblk - 1) / nblk;
    k_atap_csr<TA, CT, G, HAS_B><<<(unsigned)nblk, kAtThreads, 0, st>>>(m, n, c->rp, c->ci, v, u, b, q, rpb);
  }
}

template <typename TA, typename CT, bool HAS_B, int G>
static void csr_dot_g(int64_t rows, const int64_t *rp, const int32_t *ci, const TA *v, const CT *u, const double *b,
                      const CT *scale, CT *out, hipStream_t st) {
  const int64_t rows_per_blk_iter = (kAtThreads / G) * csr_unroll<G>();
  int64_t nblk = (rows + rows_per_blk_iter - 1) / rows_per_blk_iter;
  if (nblk > 65536) nblk = 65536;
  if (nblk < 1) nblk = 1;
  const int64_t rpb = (rows + nblk - 1) / nblk;
  k_csr_dot<TA, CT, CT, G, HAS_B><<<(unsigned)nblk, kAtThreads, 0, st>>>(rows, rp, ci, v, u, b, scale, out, rpb);
}

// out_i = scale_i (hb b_i - a_i . u) over the rows of a CSR matrix, G lanes
// per row chosen by the average row length
template <typename TA, typename CT, bool HAS_B>
static void csr_dot(int64_t rows, int64_t nnz, const int64_t *rp, const int32_t *ci, const TA *v, const CT *u,
                    const double *b, const CT *scale, CT *out, hipStream_t st) {
  const double avg = (double)nnz / (double)(rows > 0 ? rows : 1);
  if (avg <= 2) csr_dot_g<TA, CT, HAS_B, 2>(rows, rp, ci, v, u, b, scale, out, st);
  else if (avg <= 4) csr_dot_g<TA, CT, HAS_B, 4>(rows, rp, ci, v, u, b, scale, out, st);
  else if (avg <= 8) csr_dot_g<TA, CT, HAS_B, 8>(rows, rp, ci, v, u, b, scale, out, st);
  else if (avg <= 16) csr_dot_g<TA, CT, HAS_B, 16>(rows, rp, ci, v, u, b, scale, out, st);
  else if (avg <= 32) csr_dot_g<TA, CT, HAS_B, 32>(rows, rp, ci, v, u, b, scale, out, st);
  else csr_dot_g<TA, CT, HAS_B, 64>(rows, rp, ci, v, u, b, scale, out, st);
}

template <typename TA, typename CT, bool HAS_B>
static void atap_csr_t(lsq_ctx *c, const TA *v, const CT *u, const double *b, CT *q, const CT *s_out) {
  hipStream_t st = c->stream;
  if (c->atap_algo == 3) {
    // two passes: t = hb b - A u over the rows, q = s_out (A^T t) over the
    // columns (the CSC copy of the values that v points at)
    const TA *cv = (const void *)v == c->A ? (const TA *)c->csc_v : (const TA *)(const void *)c->csc_v32;
    CT *t = (CT *)(void *)c->tvec;
    csr_dot<TA, CT, HAS_B>(c->m, c->nnz, c->rp, c->ci, v, u, b, nullptr, t, st);
    csr_dot<TA, CT, false>(c->n, c->nnz, c->csc_cp, c->csc_ri, cv, t, nullptr, s_out, q, st);
    return;
  }
  const bool lds = c->atap_algo == 2;
  if (!lds) {
    if (sizeof(CT) == 8) launch_fill_f64((double *)q, c->n, 0.0, st);
    else launch_fill_f32((float *)q, c->n, 0.0f, st);
  }
  const double avg = (double)c->nnz / (double)c->m;
  // the LDS form scales its output in the finishing pass
  const CT *fs = lds ? s_out : nullptr;
  if (avg <= 2) atap_csr_g<TA, CT, HAS_B, 2>(c, v, u, b, q, lds, fs);
  else if (avg <= 4) atap_csr_g<TA, CT, HAS_B, 4>(c, v, u, b, q, lds, fs);
  else if (avg <= 8) atap_csr_g<TA, CT, HAS_B, 8>(c, v, u, b, q, lds, fs);
  else if (avg <= 16) atap_csr_g<TA, CT, HAS_B, 16>(c, v, u, b, q, lds, fs);
  else if (avg <= 32) atap_csr_g<TA, CT, HAS_B, 32>(c, v, u, b, q, lds, fs);
  else atap_csr_g<TA, CT, HAS_B, 64>(c, v, u, b, q, lds, fs);
  if (s_out && !lds) {
    int64_t fb = (c->n + 255) / 256;
    k_scale_inplace<CT><<<(unsigned)(fb > 0 ? fb : 1), 256, 0, st>>>(c->n, s_out, q);
  }
}

// algorithmic bytes of one fused pass: every stored entry of A once (value,
// plus column index and row pointers for CSR), the input vector, b when used,
// and the output vector
static double atap_bytes(const lsq_ctx *c, size_t ta, size_t ct, bool has_b) {
  const double n = (double)c->n, m = (double)c->m;
  double by = 2 * n * ct + (has_b ? 8 * m : 0);
  if (c->fmt == LSQ_DENSE) by += m * n * ta;
  else by += (double)c->nnz * (ta + 4) + (m + 1) * 8;
  return by;
}

void atap_f64(lsq_ctx *c, const double *s_in, const double *p, const double *b, double *q, const double *s_out) {
  const int slot = prof_begin(c, KC_ATAP);
  atap_f64_impl(c, s_in, p, b, q, s_out);
  prof_end(c, slot, atap_bytes(c, c->dtype == LSQ_F64 ? 8 : 4, 8, b != nullptr));
}

void atap_f64_impl(lsq_ctx *c, const double *s_in, const double *p, const double *b, double *q,
                   const double *s_out) {
  const double *u = p;
  if (s_in) {
    Vec<double>::scale(c->n, s_in, p, c->vu, c->stream);
    u = c->vu;
  }
  if (c->fmt == LSQ_DENSE) {
    if (c->dtype == LSQ_F64) {
      if (b) atap_dense_t<double, double, true>(c, (const double *)c->A, u, b, q, s_out);
      else atap_dense_t<double, double, false>(c, (const double *)c->A, u, b, q, s_out);
    } else {
      if (b) atap_dense_t<float, double, true>(c, (const float *)c->A, u, b, q, s_out);
      else atap_dense_t<float, double, false>(c, (const float *)c->A, u, b, q, s_out);
    }
  } else {
    if (c->dtype == LSQ_F64) {
      if (b) atap_csr_t<double, double, true>(c, (const double *)c->A, u, b, q, s_out);
      else atap_csr_t<double, double, false>(c, (const double *)c->A, u, b, q, s_out);
    } else {
      if (b) atap_csr_t<float, double, true>(c, (const float *)c->A, u, b, q, s_out);
      else atap_csr_t<float, double, false>(c, (const float *)c->A, u, b, q, s_out);
    }
  }
}

void atap_f32(lsq_ctx *c, const float *s_in, const float *p, float *q, const float *s_out) {
  const int slot = prof_begin(c, KC_ATAP);
  const float *u = p;
  if (s_in) {
    Vec<float>::scale(c->n, s_in, p, c->fu, c->stream);
    u = c->fu;
  }
  if (c->fmt == LSQ_DENSE) atap_dense_t<float, float, false>(c, c->A32, u, nullptr, q, s_out);
  else atap_csr_t<float, float, false>(c, c->A32, u, nullptr, q, s_out);
  prof_end(c, slot, atap_bytes(c, 4, 4, false));
}

void resid64(lsq_ctx *c, const double *x, const double *b, double *g) {
  if (b) {
    atap_f64(c, nullptr, x, b, g, nullptr);
  } else {
    atap_f64(c, nullptr, x, nullptr, g, nullptr);
  }
}

// ---------------------------------------------------------------------------
// backward pass over A

template <typename TA>
__global__ __launch_bounds__(256) void k_grad_dense(int64_t m, int64_t n, int64_t ld, const TA *__restrict__ A,
                                                    const double *__restrict__ b, const double *__restrict__ x,
                                                    const double *__restrict__ lam, double *__restrict__ gb,
                                                    TA *__restrict__ gA) {
  const int lane = threadIdx.x % kWave;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t i = wave; i < m; i += nw) {
    const TA *row = A + i * ld;
    double dv = 0, dx = 0;
    for (int64_t j = lane; j < n; j += 64) {
      const double a = (double)row[j];
      dv += a * lam[j];
      dx += a * x[j];
    }
    dv = wave_sum(dv);
    dx = wave_sum(dx);
    const double ri = b[i] - dx;
    if (gb && lane == 0) gb[i] = dv;
    if (gA)
      for (int64_t j = lane; j < n; j += 64) gA[i * ld + j] = (TA)(ri * lam[j] - dv * x[j]);
  }
}

template <typename TA, int G>
__global__ __launch_bounds__(256) void k_grad_csr(int64_t m, const int64_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci, const TA *__restrict__ v,
                                                  const double *__restrict__ b, const double *__restrict__ x,
                                                  const double *__restrict__ lam, double *__restrict__ gb,
                                                  TA *__restrict__ gA) {
  const int gl = threadIdx.x % G;
  const int64_t grp = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) / G;
  const int64_t iters = (m + ngrp - 1) / ngrp;
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t i = grp + it * ngrp;
    double dv = 0, dx = 0;
    if (i < m)
      for (int64_t k = rp[i] + gl; k < rp[i + 1]; k += G) {
        const double a = (double)v[k];
        dv += a * lam[ci[k]];
        dx += a * x[ci[k]];
      }
    dv = group_sum<G>(dv);
    dx = group_sum<G>(dx);
    if (i < m) {
      const double ri = b[i] - dx;
      if (gb && gl == 0) gb[i] = dv;
      if (gA)
        for (int64_t k = rp[i] + gl; k < rp[i + 1]; k += G) gA[k] = (TA)(ri * lam[ci[k]] - dv * x[ci[k]]);
    }
  }
}

template <typename TA>
static void grad_t(lsq_ctx *c, const double *x, const double *lam, double *gb, TA *gA) {
  hipStream_t st = c->stream;
  if (c->fmt == LSQ_DENSE) {
    int64_t blk = (c->m * 64 + 255) / 256;
    if (blk > 16384) blk = 16384;
    k_grad_dense<TA><<<(unsigned)blk, 256, 0, st>>>(c->m, c->n, c->ld, (const TA *)c->A, c->b, x, lam, gb, gA);
  } else {
    const double avg = (double)c->nnz / (double)c->m;
    const int64_t G = avg <= 2 ? 2 : avg <= 4 ? 4 : avg <= 8 ? 8 : avg <= 16 ? 16 : avg <= 32 ? 32 : 64;
    int64_t blk = (c->m * G + 255) / 256;
    if (blk > 16384) blk = 16384;
    const TA *v = (const TA *)c->A;
    switch (G) {
      case 2: k_grad_csr<TA, 2><<<(unsigned)blk, 256, 0, st>>>(c->m, c->rp, c->ci, v, c->b, x, lam, gb, gA); break;
      case 4: k_grad_csr<TA, 4><<<(unsigned)blk, 256, 0, st>>>(c->m, c->rp, c->ci, v, c->b, x, lam, gb, gA); break;
      case 8: k_grad_csr<TA, 8><<<(unsigned)blk, 256, 0, st>>>(c->m, c->rp, c->ci, v, c->b, x, lam, gb, gA); break;
      case 16: k_grad_csr<TA, 16><<<(unsigned)blk, 256, 0, st>>>(c->m, c->rp, c->ci, v, c->b, x, lam, gb, gA); break;
      case 32: k_grad_csr<TA, 32><<<(unsigned)blk, 256, 0, st>>>(c->m, c->rp, c->ci, v, c->b, x, lam, gb, gA); break;
      default: k_grad_csr<TA, 64><<<(unsigned)blk, 256, 0, st>>>(c->m, c->rp, c->ci, v, c->b, x, lam, gb, gA); break;
    }
  }
}

void grad_pass(lsq_ctx *c, const double *x, const double *lam, double *grad_b, void *grad_A) {
  if (c->dtype == LSQ_F64) grad_t<double>(c, x, lam, grad_b, (double *)grad_A);
  else grad_t<float>(c, x, lam, grad_b, (float *)grad_A);
}

}  // namespace lsq
