// Algorithm 3: t forward then t backward Gauss-Seidel steps on M from e = 0.
// Each step e <- e + B^{-1}(r - M e) (B = lower part of M with its diagonal)
// is evaluated in the equivalent form e <- B^{-1}(r - U e) (U = strict upper
// part), and each backward step as e <- B^{-T}(r - L e) (L = strict lower
// part); the first forward step has e = 0 and needs no product.
//
// Triangular solves keep the paper's natural row order. Rows are grouped into
// level sets (a row's level is one more than the largest level of the rows it
// depends on) and a single workgroup of 16 waves walks the level-ordered rows:
// wave w takes batches w, w+16, ..., each batch a few rows of one level, and a
// row waits only for the entries of x it reads, which are published in LDS
// (or global memory for large n) by overwriting a NaN sentinel. A batch's
// dependencies all lie in strictly lower levels, i.e. in earlier batches, so
// the walk always makes progress without workgroup barriers.
#include <algorithm>
#include <vector>

#include "common.h"

namespace lsq {

template <typename T>
struct Bits;
template <>
struct Bits<double> {
  typedef unsigned long long U;
  static constexpr U kSent = 0x7FF4DEADBEEF0001ull;  // a signalling NaN no arithmetic produces
};
template <>
struct Bits<float> {
  typedef unsigned int U;
  static constexpr U kSent = 0x7FA0BEEFu;
};

template <typename T>
__device__ __forceinline__ T from_bits(typename Bits<T>::U u) {
  return __builtin_bit_cast(T, u);
}
template <typename T>
__device__ __forceinline__ typename Bits<T>::U to_bits(T v) {
  return __builtin_bit_cast(typename Bits<T>::U, v);
}

constexpr int kTrsvThreads = 1024, kTrsvWaves = kTrsvThreads / kWave;
constexpr int kSpinLimit = 1 << 24;

// One row of a solve: the row, its entry range [k0, k1) in the triangle being
// solved (CSR positions, or positions in the dense row-major M) and the
// position of its diagonal.
struct RowTask {
  int row;
  int64_t k0, k1, dpos;
};

template <bool DENSE, bool UPPER, int R>
__device__ __forceinline__ RowTask get_task(int b, int g, int nbatch, int n, const int4 *__restrict__ task,
                                            const int32_t *__restrict__ ord) {
  RowTask t{-1, 0, 0, 0};
  if (b >= nbatch) return t;
  if (DENSE) {
    const int row = ord[b * R + g];
    t.row = row;
    if (row >= 0) {
      const int64_t base = (int64_t)row * n;
      t.dpos = base + row;
      t.k0 = UPPER ? t.dpos + 1 : base;
      t.k1 = UPPER ? base + n : t.dpos;
    }
  } else {
    const int4 q = task[b * R + g];
    t.row = q.x;
    t.k0 = q.y;
    t.k1 = q.z;
    t.dpos = q.w;
  }
  return t;
}

// E entries per lane are loaded into registers in one burst (G*E per row per
// chunk); the next batch's row is loaded while the current row waits for its
// dependencies, so the global-memory latency overlaps the dependency chain.
template <typename T, bool DENSE, bool UPPER, bool LDSX, int G, int E>
__global__ __launch_bounds__(kTrsvThreads) void k_trsv(int n, const int4 *__restrict__ task,
                                                       const int32_t *__restrict__ ord,
                                                       const int32_t *__restrict__ ci, const T *__restrict__ val,
                                                       const T *__restrict__ rhs, T *__restrict__ x, int nbatch,
                                                       int32_t *__restrict__ err) {
  typedef typename Bits<T>::U U;
  constexpr int R = kWave / G;
  constexpr int scope = LDSX ? __HIP_MEMORY_SCOPE_WORKGROUP : __HIP_MEMORY_SCOPE_AGENT;
  extern __shared__ __align__(16) unsigned char smem[];
  U *xs = LDSX ? (U *)smem : (U *)x;
  for (int i = threadIdx.x; i < n; i += kTrsvThreads) __hip_atomic_store(&xs[i], Bits<T>::kSent, __ATOMIC_RELAXED, scope);
  __syncthreads();
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int g = lane / G, gl = lane % G;
  bool failed = false;

  auto load = [&](const RowTask &t, int64_t kb, int (&jj)[E], T (&vv)[E]) {
    const int64_t base = DENSE && t.row >= 0 ? (int64_t)t.row * n : 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t k = kb + gl + (int64_t)G * e;
      if (t.row >= 0 && k < t.k1) {
        jj[e] = DENSE ? (int)(k - base) : ci[k];
        vv[e] = val[k];
      } else {
        jj[e] = -1;
        vv[e] = 0;
      }
    }
  };
  // all E reads are issued together; only entries still holding the sentinel
  // are read again
  auto consume = [&](const int (&jj)[E], const T (&vv)[E], T acc) -> T {
    U u[E];
#pragma unroll
    for (int e = 0; e < E; ++e) u[e] = jj[e] >= 0 ? __hip_atomic_load(&xs[jj[e]], __ATOMIC_RELAXED, scope) : (U)0;
    int spins = 0;  // bounded wait: a schedule error is reported, never a hang
    bool pending = true;
    while (pending) {
      pending = false;
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (u[e] == Bits<T>::kSent) {
          u[e] = __hip_atomic_load(&xs[jj[e]], __ATOMIC_RELAXED, scope);
          pending = pending || (u[e] == Bits<T>::kSent);
        }
      if (pending && ++spins > kSpinLimit) {
        failed = true;
#pragma unroll
        for (int e = 0; e < E; ++e)
          if (u[e] == Bits<T>::kSent) u[e] = 0;
        pending = false;
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) acc += vv[e] * from_bits<T>(u[e]);
    return acc;
  };

  // the task records run two rows ahead of the data, so the data loads of the
  // next row never wait for their own task record
  int b = wave;
  RowTask cur = get_task<DENSE, UPPER, R>(b, g, nbatch, n, task, ord);
  RowTask nx = get_task<DENSE, UPPER, R>(b + kTrsvWaves, g, nbatch, n, task, ord);
  int cj[E];
  T cv[E];
  load(cur, cur.k0, cj, cv);
  T crhs = cur.row >= 0 ? rhs[cur.row] : (T)0, cdg = cur.row >= 0 ? val[cur.dpos] : (T)1;
  for (; b < nbatch; b += kTrsvWaves) {
    const RowTask nx2 = get_task<DENSE, UPPER, R>(b + 2 * kTrsvWaves, g, nbatch, n, task, ord);
    // prefetch the wave's next row
    int nj[E];
    T nv[E];
    load(nx, nx.k0, nj, nv);
    const T nrhs = nx.row >= 0 ? rhs[nx.row] : (T)0, ndg = nx.row >= 0 ? val[nx.dpos] : (T)1;

    T acc = consume(cj, cv, (T)0);
    for (int64_t kb = cur.k0 + (int64_t)G * E; kb < cur.k1; kb += (int64_t)G * E) {  // long rows
      int tj[E];
      T tv[E];
      load(cur, kb, tj, tv);
      acc = consume(tj, tv, acc);
    }
    acc = dpp_group_sum<G>(acc);
    if (cur.row >= 0 && gl == dpp_sum_lane<G>()) {
      const T xi = (crhs - acc) / cdg;
      __hip_atomic_store(&xs[cur.row], to_bits<T>(xi), __ATOMIC_RELAXED, scope);
    }
    cur = nx;
    nx = nx2;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      cj[e] = nj[e];
      cv[e] = nv[e];
    }
    crhs = nrhs;
    cdg = ndg;
  }
  if (failed) atomicOr(err, 1);
  if (LDSX) {
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kTrsvThreads) x[i] = from_bits<T>(xs[i]);
  }
}

// out_i = r_i - sum over the strict upper (UPPER_PART) or strict lower part of
// row i of M_ij e_j
template <typename T, bool DENSE, bool UPPER_PART, int G>
__global__ __launch_bounds__(256) void k_sgs_rhs(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                 const T *__restrict__ val, const int32_t *__restrict__ dg,
                                                 const T *__restrict__ r, const T *__restrict__ e, T *__restrict__ out) {
  const int gl = threadIdx.x % G;
  const int64_t grp = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) / G;
  const int64_t iters = (n + ngrp - 1) / ngrp;
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t row = grp + it * ngrp;
    T acc = 0;
    if (row < n) {
      int64_t k0, k1, base = 0;
      if (DENSE) {
        base = row * (int64_t)n;
        k0 = UPPER_PART ? base + row + 1 : base;
        k1 = UPPER_PART ? base + n : base + row;
      } else {
        k0 = UPPER_PART ? (int64_t)dg[row] + 1 : rp[row];
        k1 = UPPER_PART ? rp[row + 1] : dg[row];
      }
      for (int64_t k = k0 + gl; k < k1; k += G) {
        const int j = DENSE ? (int)(k - base) : ci[k];
        acc += val[k] * e[j];
      }
    }
    acc = group_sum<G>(acc);
    if (row < n && gl == 0) out[row] = r[row] - acc;
  }
}

// ---------------------------------------------------------------------------
// level analysis (host): natural order, forward on the lower part, backward on
// the upper part; rows sorted by level, each level padded to whole batches

int build_levels(lsq_ctx *ctx) {
  const int64_t n = ctx->n;
  std::vector<int32_t> lev_f(n, 0), lev_b(n, 0);
  std::vector<int32_t> rp_h, dg_h;
  if (ctx->Mdense) {
    for (int64_t i = 0; i < n; ++i) {
      lev_f[i] = (int32_t)i;
      lev_b[i] = (int32_t)(n - 1 - i);
    }
    ctx->G = 64;
  } else {
    std::vector<int32_t> &rp = rp_h, &dg = dg_h;
    rp.resize(n + 1);
    dg.resize(n);
    std::vector<int32_t> ci(ctx->nnzM);
    LSQ_HIP_CHECK(hipMemcpyAsync(rp.data(), ctx->Mrp, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    LSQ_HIP_CHECK(hipMemcpyAsync(ci.data(), ctx->Mci, ctx->nnzM * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    LSQ_HIP_CHECK(hipMemcpyAsync(dg.data(), ctx->Mdiag, n * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    LSQ_HIP_CHECK(hipStreamSynchronize(ctx->stream));
    for (int64_t i = 0; i < n; ++i) {
      int32_t lv = 0;
      for (int32_t k = rp[i]; k < dg[i]; ++k) lv = std::max(lv, lev_f[ci[k]] + 1);
      lev_f[i] = lv;
    }
    for (int64_t i = n - 1; i >= 0; --i) {
      int32_t lv = 0;
      for (int32_t k = dg[i] + 1; k < rp[i + 1]; ++k) lv = std::max(lv, lev_b[ci[k]] + 1);
      lev_b[i] = lv;
    }
    double avg = (double)(ctx->nnzM - n) / (2.0 * (double)n);
    int G = 4;
    while (G < 64 && G < avg) G <<= 1;
    ctx->G = G;
  }
  const int R = 64 / ctx->G;
  auto order = [&](const std::vector<int32_t> &lev, bool reverse, int64_t *nlev, int64_t *nbatch,
                   std::vector<int32_t> &ord) {
    int32_t L = 0;
    for (int64_t i = 0; i < n; ++i) L = std::max(L, lev[i] + 1);
    std::vector<int64_t> cnt(L + 1, 0);
    for (int64_t i = 0; i < n; ++i) cnt[lev[i] + 1]++;
    std::vector<int64_t> bstart(L + 1, 0);  // batch offsets per level
    for (int32_t l = 0; l < L; ++l) bstart[l + 1] = bstart[l] + (cnt[l + 1] + R - 1) / R;
    *nlev = L;
    *nbatch = bstart[L];
    ord.assign((size_t)(*nbatch) * R, -1);
    std::vector<int64_t> fill(L, 0);
    for (int64_t q = 0; q < n; ++q) {
      const int64_t i = reverse ? n - 1 - q : q;
      const int32_t l = lev[i];
      ord[bstart[l] * R + fill[l]++] = (int32_t)i;
    }
  };
  std::vector<int32_t> of, ob;
  order(lev_f, false, &ctx->nlev_f, &ctx->nbatch_f, of);
  order(lev_b, true, &ctx->nlev_b, &ctx->nbatch_b, ob);
  if (!ctx->Mdense) {
    // per-row tasks in level order: row, entry range of its triangle, diagonal
    auto tasks = [&](const std::vector<int32_t> &ord, bool upper, int4 **out) -> int {
      std::vector<int4> t(ord.size());
      for (size_t q = 0; q < ord.size(); ++q) {
        const int32_t i = ord[q];
        if (i < 0) {
          t[q] = make_int4(-1, 0, 0, 0);
        } else if (upper) {
          t[q] = make_int4(i, dg_h[i] + 1, rp_h[i + 1], dg_h[i]);
        } else {
          t[q] = make_int4(i, rp_h[i], dg_h[i], dg_h[i]);
        }
      }
      *out = (int4 *)lsq_alloc(ctx, t.size() * sizeof(int4) + 16);
      if (!*out) return LSQ_ENOMEM;
      LSQ_HIP_CHECK(hipMemcpy(*out, t.data(), t.size() * sizeof(int4), hipMemcpyHostToDevice));
      return LSQ_OK;
    };
    int rc = tasks(of, false, &ctx->task_f);
    if (rc != LSQ_OK) return rc;
    rc = tasks(ob, true, &ctx->task_b);
    if (rc != LSQ_OK) return rc;
  }
  ctx->ord_f = (int32_t *)lsq_alloc(ctx, of.size() * sizeof(int32_t) + 4);
  ctx->ord_b = (int32_t *)lsq_alloc(ctx, ob.size() * sizeof(int32_t) + 4);
  if (!ctx->ord_f || !ctx->ord_b) return LSQ_ENOMEM;
  LSQ_HIP_CHECK(hipMemcpyAsync(ctx->ord_f, of.data(), of.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
  LSQ_HIP_CHECK(hipMemcpyAsync(ctx->ord_b, ob.data(), ob.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
  LSQ_HIP_CHECK(hipStreamSynchronize(ctx->stream));
  return LSQ_OK;
}

// ---------------------------------------------------------------------------
// launch helpers

template <typename T>
static bool lds_fits(int64_t n) {
  return n * (int64_t)sizeof(T) <= 131072;
}

template <typename T, bool DENSE, bool UPPER, bool LDSX, int G>
static void launch_trsv_g(lsq_ctx *c, const T *val, const T *rhs, T *x) {
  constexpr int E = G >= 32 ? 8 : 4;
  auto kern = k_trsv<T, DENSE, UPPER, LDSX, G, E>;
  size_t lds = LDSX ? (size_t)c->n * sizeof(T) : 0;
  static bool attr_set = false;
  if (LDSX && !attr_set) {
    (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
  const int32_t *ord = UPPER ? c->ord_b : c->ord_f;
  const int nb = (int)(UPPER ? c->nbatch_b : c->nbatch_f);
  const int4 *task = UPPER ? c->task_b : c->task_f;
  kern<<<1, kTrsvThreads, lds, c->stream>>>((int)c->n, task, ord, c->Mci, val, rhs, x, nb, c->flags + 3);
}

template <typename T, bool DENSE, bool UPPER, bool LDSX>
static void launch_trsv_l(lsq_ctx *c, const T *val, const T *rhs, T *x) {
  switch (c->G) {
    case 4: launch_trsv_g<T, DENSE, UPPER, LDSX, 4>(c, val, rhs, x); break;
    case 8: launch_trsv_g<T, DENSE, UPPER, LDSX, 8>(c, val, rhs, x); break;
    case 16: launch_trsv_g<T, DENSE, UPPER, LDSX, 16>(c, val, rhs, x); break;
    case 32: launch_trsv_g<T, DENSE, UPPER, LDSX, 32>(c, val, rhs, x); break;
    default: launch_trsv_g<T, DENSE, UPPER, LDSX, 64>(c, val, rhs, x); break;
  }
}

template <typename T, bool UPPER>
static void launch_trsv(lsq_ctx *c, const T *val, const T *rhs, T *x) {
  const bool lds = lds_fits<T>(c->n);
  if (c->Mdense) {
    if (lds) launch_trsv_g<T, true, UPPER, true, 64>(c, val, rhs, x);
    else launch_trsv_g<T, true, UPPER, false, 64>(c, val, rhs, x);
  } else {
    if (lds) launch_trsv_l<T, false, UPPER, true>(c, val, rhs, x);
    else launch_trsv_l<T, false, UPPER, false>(c, val, rhs, x);
  }
}

template <typename T, bool UPPER_PART>
static void launch_rhs(lsq_ctx *c, const T *val, const T *r, const T *e, T *out) {
  const int64_t n = c->n;
  int64_t b = (n * (c->Mdense ? 64 : c->G) + 255) / 256;
  if (b < 1) b = 1;
  if (b > 8192) b = 8192;
  if (c->Mdense) {
    k_sgs_rhs<T, true, UPPER_PART, 64><<<(unsigned)b, 256, 0, c->stream>>>((int)n, c->Mrp, c->Mci, val, c->Mdiag, r, e, out);
    return;
  }
  switch (c->G) {
    case 4: k_sgs_rhs<T, false, UPPER_PART, 4><<<(unsigned)b, 256, 0, c->stream>>>((int)n, c->Mrp, c->Mci, val, c->Mdiag, r, e, out); break;
    case 8: k_sgs_rhs<T, false, UPPER_PART, 8><<<(unsigned)b, 256, 0, c->stream>>>((int)n, c->Mrp, c->Mci, val, c->Mdiag, r, e, out); break;
    case 16: k_sgs_rhs<T, false, UPPER_PART, 16><<<(unsigned)b, 256, 0, c->stream>>>((int)n, c->Mrp, c->Mci, val, c->Mdiag, r, e, out); break;
    case 32: k_sgs_rhs<T, false, UPPER_PART, 32><<<(unsigned)b, 256, 0, c->stream>>>((int)n, c->Mrp, c->Mci, val, c->Mdiag, r, e, out); break;
    default: k_sgs_rhs<T, false, UPPER_PART, 64><<<(unsigned)b, 256, 0, c->stream>>>((int)n, c->Mrp, c->Mci, val, c->Mdiag, r, e, out); break;
  }
}

// algorithmic bytes of one triangular solve and of one strict-part product:
// every stored entry read once (value, plus column index when sparse), the
// row pointers, the level order, the right-hand side and the output
template <typename T>
static double trsv_bytes(const lsq_ctx *c) {
  const double n = (double)c->n;
  if (c->Mdense) return (n * (n - 1) / 2 + n) * sizeof(T) + n * (4 + 2 * sizeof(T));
  const double strict = ((double)c->nnzM - n) / 2;
  return (strict + n) * (sizeof(T) + 4) + n * (4 + 8 + 2 * sizeof(T));
}
template <typename T>
static double rhs_bytes(const lsq_ctx *c) {
  const double n = (double)c->n;
  if (c->Mdense) return n * (n - 1) / 2 * sizeof(T) + 3 * n * sizeof(T);
  const double strict = ((double)c->nnzM - n) / 2;
  return strict * (sizeof(T) + 4) + n * (8 + 3 * sizeof(T));
}

template <typename T>
static void sgs_apply(lsq_ctx *c, const T *val, const T *r, T *z, T *tmp) {
  const int t = c->sweeps;
  if (t == 0) {
    Vec<T>::copy(c->n, r, z, c->stream);
    return;
  }
  const double tb = trsv_bytes<T>(c), rb = rhs_bytes<T>(c);
  int slot = prof_begin(c, KC_TRSV);
  launch_trsv<T, false>(c, val, r, z);  // first forward step from e = 0
  prof_end(c, slot, tb);
  for (int k = 1; k < t; ++k) {
    slot = prof_begin(c, KC_SGS_RHS);
    launch_rhs<T, true>(c, val, r, z, tmp);
    prof_end(c, slot, rb);
    slot = prof_begin(c, KC_TRSV);
    launch_trsv<T, false>(c, val, tmp, z);
    prof_end(c, slot, tb);
  }
  for (int k = 0; k < t; ++k) {
    slot = prof_begin(c, KC_SGS_RHS);
    launch_rhs<T, false>(c, val, r, z, tmp);
    prof_end(c, slot, rb);
    slot = prof_begin(c, KC_TRSV);
    launch_trsv<T, true>(c, val, tmp, z);
    prof_end(c, slot, tb);
  }
}

void sgs_apply_f64(lsq_ctx *c, const double *r, double *z) { sgs_apply<double>(c, c->Md, r, z, c->vrhs); }
void sgs_apply_f32(lsq_ctx *c, const float *r, float *z) { sgs_apply<float>(c, c->Mf, r, z, c->frhs); }

}  // namespace lsq
