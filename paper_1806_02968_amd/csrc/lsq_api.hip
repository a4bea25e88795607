// C ABI of liblsq (declared in include/lsq.h): Algorithm 2 of Chen & Wu
// (arXiv:1806.02968) on one MI355X, plus the adjoint solve of the
// differentiable form and the float32-inner / float64-refinement mode.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <vector>

#include "common.h"

using namespace lsq;

int lsq_hip_fail(lsq_ctx *ctx, hipError_t e, const char *what) {
  if (ctx) {
    ctx->err = std::string("HIP error ") + hipGetErrorString(e) + " in " + what;
    ctx->info.status = LSQ_EHIP;
  }
  return LSQ_EHIP;
}

// Device memory: a process-wide cache of freed blocks, keyed by device and
// rounded size (a request takes the smallest fitting block up to 25 % larger). A context's blocks return to the cache when it is destroyed
// (after its stream has drained) or when a temporary is released (after a
// stream synchronisation), so repeated setups reuse the same blocks instead of
// paying hipMalloc/hipFree every time. Blocks stay allocated until the process
// ends.
static std::mutex g_pool_mu;
static std::map<std::pair<int, size_t>, std::vector<void *>> g_blocks;

static size_t round_size(size_t bytes) {
  if (bytes <= (1u << 20)) {
    size_t r = 4096;
    while (r < bytes) r <<= 1;
    return r;
  }
  return (bytes + (1u << 20) - 1) & ~(size_t)((1u << 20) - 1);
}

void *lsq_alloc(lsq_ctx *ctx, size_t bytes) {
  const size_t rb = round_size(bytes < 16 ? 16 : bytes);
  void *p = nullptr;
  size_t got = rb;
  {
    // the smallest cached block of at least rb and at most rb + rb/4 bytes:
    // sizes that depend on the data (the sample, the Gram pattern) change
    // from one setup to the next
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (auto it = g_blocks.lower_bound({ctx->device, rb});
         it != g_blocks.end() && it->first.first == ctx->device && it->first.second <= rb + rb / 4; ++it)
      if (!it->second.empty()) {
        p = it->second.back();
        it->second.pop_back();
        got = it->first.second;
        break;
      }
  }
  if (!p && hipMalloc(&p, rb) != hipSuccess) {
    (void)hipGetLastError();
    ctx->err = "device allocation of " + std::to_string(bytes) + " bytes failed";
    return nullptr;
  }
  ctx->allocs.push_back(Dev{p, got});
  return p;
}

static void release_blocks(int device, const std::vector<Dev> &blocks) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  for (const Dev &d : blocks) g_blocks[{device, d.bytes}].push_back(d.p);
}

void lsq_free_one(lsq_ctx *ctx, void *p) {
  for (size_t i = 0; i < ctx->allocs.size(); ++i)
    if (ctx->allocs[i].p == p) {
      (void)hipStreamSynchronize(ctx->stream);  // no queued kernel still uses it
      release_blocks(ctx->device, {ctx->allocs[i]});
      ctx->allocs.erase(ctx->allocs.begin() + i);
      return;
    }
}

// pinned host scalars and timing events are kept in process-wide free lists
static std::vector<double *> g_pinned;
static std::vector<hipEvent_t> g_events;

static double *take_pinned(size_t count) {
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (!g_pinned.empty()) {
      double *p = g_pinned.back();
      g_pinned.pop_back();
      return p;
    }
  }
  double *p = nullptr;
  if (hipHostMalloc((void **)&p, count * sizeof(double), hipHostMallocDefault) != hipSuccess) return nullptr;
  return p;
}
static void give_pinned(double *p) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  g_pinned.push_back(p);
}
static hipError_t take_event(hipEvent_t *e) {
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (!g_events.empty()) {
      *e = g_events.back();
      g_events.pop_back();
      return hipSuccess;
    }
  }
  return hipEventCreate(e);
}
static void give_event(hipEvent_t e) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  g_events.push_back(e);
}

#define RET(code)                 \
  do {                            \
    int rc_ = (code);             \
    ctx->info.status = rc_;       \
    return rc_;                   \
  } while (0)

#define TRY(expr)                    \
  do {                               \
    int rc_ = (expr);                \
    if (rc_ != LSQ_OK) RET(rc_);     \
  } while (0)

#define ALLOC(ptr, type, count)                                   \
  do {                                                            \
    (ptr) = (type *)lsq_alloc(ctx, (size_t)(count) * sizeof(type)); \
    if (!(ptr)) RET(LSQ_ENOMEM);                                  \
  } while (0)

// ---------------------------------------------------------------------------
// small kernels of the driver

__global__ void k_validate_csr(int64_t m, int64_t n, int64_t nnz, const int64_t *__restrict__ rp,
                               const int32_t *__restrict__ ci, int32_t *flags) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = rp[i], b = rp[i + 1];
    if (a < 0 || b < a || b > nnz || (i == 0 && a != 0) || (i == m - 1 && b != nnz)) {
      atomicOr(&flags[0], 4);
      continue;
    }
    for (int64_t k = a; k < b; ++k) {
      const int32_t c = ci[k];
      if (c < 0 || c >= n || (k > a && ci[k - 1] >= c)) {
        atomicOr(&flags[0], 4);
        break;
      }
    }
  }
}

__global__ void k_check_finite(int64_t m, const double *__restrict__ b, int32_t *flags) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(b[i])) atomicOr(&flags[0], 2);
}

__global__ void k_count_ties(int64_t s, const double *__restrict__ gap, double eps, int32_t *flags) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < s; t += (int64_t)gridDim.x * blockDim.x)
    if (gap[t] <= eps) atomicAdd(&flags[2], 1);
}

// the triangular solves raise flags[3] when a wait for an entry of x exceeds
// its spin limit (a scheduling fault); report it instead of a wrong result
static int check_wait_flag(lsq_ctx *ctx, int rc) {
  int32_t f = 0;
  if (hipMemcpy(&f, ctx->flags + 3, sizeof(f), hipMemcpyDeviceToHost) != hipSuccess) return LSQ_EHIP;
  if (f) {
    ctx->err = "triangular solve wait limit exceeded";
    return LSQ_EHIP;
  }
  return rc;
}

// ---------------------------------------------------------------------------
// kernel timing

namespace lsq {
int prof_begin(lsq_ctx *c, int cls) {
  if (!c->opt.profile) return -1;
  if (!c->prof_ready) {
    for (int i = 0; i < 2 * lsq_ctx::kProfSlots; ++i)
      if (take_event(&c->prof_ev[i]) != hipSuccess) return -1;
    c->prof_ready = true;
  }
  if (c->prof_used == lsq_ctx::kProfSlots) {
    if (hipStreamSynchronize(c->stream) != hipSuccess) return -1;
    prof_harvest(c);
  }
  const int slot = c->prof_used++;
  c->prof_cls[slot] = cls;
  c->prof_alias[slot] = -1;
  (void)hipEventRecord(c->prof_ev[2 * slot], c->stream);
  return slot;
}
int prof_switch(lsq_ctx *c, int slot, double bytes, int cls) {
  if (slot < 0) return prof_begin(c, cls);
  if (c->prof_used == lsq_ctx::kProfSlots) {
    prof_end(c, slot, bytes);
    return prof_begin(c, cls);
  }
  c->prof_bytes[slot] = bytes;
  (void)hipEventRecord(c->prof_ev[2 * slot + 1], c->stream);
  const int next = c->prof_used++;
  c->prof_cls[next] = cls;
  c->prof_alias[next] = 2 * slot + 1;
  return next;
}
void prof_end(lsq_ctx *c, int slot, double bytes) {
  if (slot < 0) return;
  c->prof_bytes[slot] = bytes;
  (void)hipEventRecord(c->prof_ev[2 * slot + 1], c->stream);
}
void prof_harvest(lsq_ctx *c) {
  for (int i = 0; i < c->prof_used; ++i) {
    float ms = 0.0f;
    const hipEvent_t start = c->prof_alias[i] >= 0 ? c->prof_ev[c->prof_alias[i]] : c->prof_ev[2 * i];
    if (hipEventElapsedTime(&ms, start, c->prof_ev[2 * i + 1]) != hipSuccess) continue;
    const int k = c->prof_cls[i];
    c->kstats.launches[k] += 1;
    c->kstats.ms[k] += ms;
    c->kstats.bytes[k] += c->prof_bytes[i];
  }
  c->prof_used = 0;
}
void prof_harvest_ready(lsq_ctx *c) {
  int done = 0;
  while (done < c->prof_used && hipEventQuery(c->prof_ev[2 * done + 1]) == hipSuccess) ++done;
  // a remaining slot that starts at a harvested slot's end keeps that slot
  while (done > 0 && done < c->prof_used && c->prof_alias[done] >= 0) --done;
  if (done == 0) return;
  const int used = c->prof_used;
  c->prof_used = done;
  prof_harvest(c);
  // the launches still running move to the front, with their events
  for (int i = done; i < used; ++i) {
    std::swap(c->prof_ev[2 * (i - done)], c->prof_ev[2 * i]);
    std::swap(c->prof_ev[2 * (i - done) + 1], c->prof_ev[2 * i + 1]);
    c->prof_cls[i - done] = c->prof_cls[i];
    c->prof_bytes[i - done] = c->prof_bytes[i];
    c->prof_alias[i - done] = c->prof_alias[i] >= 0 ? c->prof_alias[i] - 2 * done : -1;
  }
  c->prof_used = used - done;
}
}  // namespace lsq

extern "C" int lsq_get_kernel_stats(lsq_ctx *ctx, lsq_kernel_stats *stats, int32_t reset) {
  if (!ctx || !stats) return LSQ_EINVAL;
  LSQ_HIP_CHECK(hipStreamSynchronize(ctx->stream));
  prof_harvest(ctx);
  *stats = ctx->kstats;
  if (reset) ctx->kstats = lsq_kernel_stats{};
  return LSQ_OK;
}

static unsigned grid_n(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > 8192) b = 8192;
  return (unsigned)b;
}

static double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

static int read_scalars(lsq_ctx *ctx) {
  LSQ_HIP_CHECK(hipMemcpyAsync(ctx->hscal, ctx->scal, Scal::COUNT * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
  LSQ_HIP_CHECK(hipStreamSynchronize(ctx->stream));
  prof_harvest(ctx);
  return LSQ_OK;
}

template <typename T>
static double dev_dot(lsq_ctx *ctx, int64_t n, const T *x, const T *y, const double *d, int slot) {
  int np = Vec<T>::dot_partials(n, x, y, d, ctx->part, ctx->stream);
  launch_finish(ctx->part, np, ctx->scal, slot, 0, ctx->stream);
  if (read_scalars(ctx) != LSQ_OK) return NAN;
  return ctx->hscal[slot];
}

// ---------------------------------------------------------------------------
// options

extern "C" void lsq_default_options(lsq_options *o) {
  memset(o, 0, sizeof(*o));
  o->mode = LSQ_MODE_FP64;
  o->tol = 1e-10;
  o->max_iter = 0;
  o->fixed_iters = -1;
  o->max_replace = 3;
  o->inner_tol = 1e-5;
  o->max_inner = 0;
  o->max_outer = 30;
  o->tie_eps = 0x1.0p-44;
  o->atap_algo = 0;
  o->near_levels = 48;
  o->chain_levels = 0;
}

extern "C" const char *lsq_strerror(int code) {
  switch (code) {
    case LSQ_OK: return "ok";
    case LSQ_ENOCONV: return "tolerance not reached";
    case LSQ_EINVAL: return "invalid argument";
    case LSQ_ESINGULAR: return "zero column (rank-deficient matrix)";
    case LSQ_ENONFINITE: return "non-finite input";
    case LSQ_ENOMEM: return "device allocation failed";
    case LSQ_EHIP: return "HIP runtime error";
    case LSQ_EBREAKDOWN: return "PCG breakdown";
    case LSQ_ESTATE: return "invalid state";
    default: return "unknown error";
  }
}

extern "C" const char *lsq_last_error(const lsq_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

extern "C" void lsq_destroy(lsq_ctx *ctx) {
  if (!ctx) return;
  if (ctx->prof_ready) {
    (void)hipStreamSynchronize(ctx->stream);
    for (int i = 0; i < 2 * lsq_ctx::kProfSlots; ++i) give_event(ctx->prof_ev[i]);
  }
  if (ctx->scal_ev) {
    (void)hipStreamSynchronize(ctx->stream);
    give_event(ctx->scal_ev);
  }
  (void)hipStreamSynchronize(ctx->stream);  // nothing queued still uses the blocks or the pinned scalars
  release_blocks(ctx->device, ctx->allocs);
  if (ctx->hscal) give_pinned(ctx->hscal);
  delete ctx;
}

static int64_t sample_size(double C, int64_t n) {
  if (n <= 1) return 1;
  double v = ceil(C * (double)n * log((double)n));
  int64_t s = (int64_t)v;
  return s < n ? n : s;
}

// ---------------------------------------------------------------------------
// setup: Algorithm 2 steps 1-3

static int setup_impl(lsq_ctx *ctx) {
  hipStream_t st = ctx->stream;
  const int64_t m = ctx->m, n = ctx->n;
  const bool fp32 = ctx->opt.mode == LSQ_MODE_FP32_REFINE;

  ALLOC(ctx->flags, int32_t, 16);  // [8]: arrival count of the fused reductions
  ALLOC(ctx->scal, double, Scal::COUNT);
  ctx->hscal = take_pinned(Scal::COUNT);
  if (!ctx->hscal) RET(LSQ_ENOMEM);
  ALLOC(ctx->D, double, n);
  ALLOC(ctx->invD, double, n);
  if (fp32) ALLOC(ctx->invD32, float, n);
  ALLOC(ctx->w, double, m);
  ALLOC(ctx->cdf, double, m);
  // reduction partials and dense A^T(Ap) partial rows
  // sparse A^T(Ap): per-workgroup LDS partial rows when a row of n values fits
  // in LDS, otherwise two passes over A (rows, then a CSC copy), or global
  // atomics on request
  const bool csc_ok = ctx->fmt == LSQ_CSR && m < INT32_MAX;
  if (ctx->opt.atap_algo == 0 && ctx->fmt == LSQ_CSR) ctx->atap_algo = n * 8 <= 131072 ? 2 : (csc_ok ? 3 : 1);
  if (ctx->opt.atap_algo == 0 && ctx->fmt == LSQ_DENSE) ctx->atap_algo = n * 8 <= 131072 ? 2 : 1;
  if (ctx->fmt == LSQ_CSR && ctx->atap_algo == 2 && n * 8 > 131072) ctx->atap_algo = csc_ok ? 3 : 1;
  if (ctx->fmt == LSQ_CSR && ctx->atap_algo == 3 && !csc_ok) ctx->atap_algo = 1;
  const int64_t part_elems = std::max<int64_t>(
      ctx->fmt == LSQ_DENSE ? (1024 + 64) * n : (ctx->atap_algo == 2 ? (256 + 16) * n : n), 4096);
  ALLOC(ctx->part, double, part_elems);
  ctx->part_bytes = part_elems * sizeof(double);
  if (ctx->fmt == LSQ_DENSE && n > 2048) ALLOC(ctx->vm, double, m);
  launch_fill_i32(ctx->flags, 16, 0, st);

  // argument checks that need the device; nothing indexes with A's column
  // indices before they have been validated
  if (ctx->fmt == LSQ_CSR) k_validate_csr<<<grid_n(m), 256, 0, st>>>(m, n, ctx->nnz, ctx->rp, ctx->ci, ctx->flags);
  k_check_finite<<<grid_n(m), 256, 0, st>>>(m, ctx->b, ctx->flags);
  int32_t hflags[8];
  LSQ_HIP_CHECK(hipMemcpyAsync(hflags, ctx->flags, sizeof(hflags), hipMemcpyDeviceToHost, st));
  LSQ_HIP_CHECK(hipStreamSynchronize(st));
  if (hflags[0] & 4) {
    ctx->err = "CSR structure invalid (row pointers or unsorted/duplicate/out-of-range columns)";
    RET(LSQ_EINVAL);
  }

  // step 1: column norms
  if (ctx->fmt == LSQ_DENSE) {
    int nblk = (int)std::min<int64_t>(1024, std::max<int64_t>(1, m / 64));
    launch_colnorm_dense(ctx, ctx->part, nblk, st);
    launch_colnorm_finish(n, ctx->part, nblk, ctx->D, ctx->invD, ctx->invD32, ctx->flags, st);
  } else {
    const int nblk = launch_colnorm_csr_part(ctx, ctx->part, st);
    launch_colnorm_finish(n, ctx->part, nblk, ctx->D, ctx->invD, ctx->invD32, ctx->flags, st);
  }
  LSQ_HIP_CHECK(hipMemcpyAsync(hflags, ctx->flags, sizeof(hflags), hipMemcpyDeviceToHost, st));
  LSQ_HIP_CHECK(hipStreamSynchronize(st));
  if (hflags[0] & 2) {
    ctx->err = "A or b contains NaN or Inf";
    RET(LSQ_ENONFINITE);
  }
  if (hflags[0] & 1) {
    ctx->err = "A has a zero column";
    RET(LSQ_ESINGULAR);
  }
  // Eq. (R2P) weights of the normalised rows
  launch_rowweight(ctx, ctx->w, ctx->flags, st);
  LSQ_HIP_CHECK(hipMemcpyAsync(hflags, ctx->flags, sizeof(hflags), hipMemcpyDeviceToHost, st));
  LSQ_HIP_CHECK(hipStreamSynchronize(st));
  if (hflags[0] & 2) {
    ctx->err = "A or b contains NaN or Inf";
    RET(LSQ_ENONFINITE);
  }
  if (hflags[0] & 1) {
    ctx->err = "A has a zero column";
    RET(LSQ_ESINGULAR);
  }

  // step 2 with Algorithm 1
  double *bs;
  ALLOC(bs, double, scan_scratch_elems(m) + 1);
  launch_scan_cdf(m, ctx->w, ctx->cdf, bs, st);
  ctx->s = sample_size(ctx->C, n);
  const int64_t s = ctx->s;
  ALLOC(ctx->idx, int64_t, s);
  ALLOC(ctx->gap, double, s);
  ALLOC(ctx->cnt, int32_t, m);
  launch_fill_i32(ctx->cnt, m, 0, st);
  launch_draw(m, ctx->w, ctx->cdf, s, ctx->seed, ctx->idx, ctx->gap, ctx->cnt, st);
  k_count_ties<<<grid_n(s), 256, 0, st>>>(s, ctx->gap, ctx->opt.tie_eps, ctx->flags);
  int64_t *scr, *dcount;
  ALLOC(scr, int64_t, m + scan_scratch_elems(m) + 1);
  ALLOC(dcount, int64_t, 1);
  ALLOC(ctx->urow, int64_t, m);
  ALLOC(ctx->ucnt, int32_t, m);
  launch_compact_counts(m, ctx->cnt, scr, ctx->urow, ctx->ucnt, dcount, st);
  LSQ_HIP_CHECK(hipMemcpyAsync(&ctx->s_d, dcount, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  LSQ_HIP_CHECK(hipMemcpyAsync(&ctx->W, ctx->cdf + m - 1, sizeof(double), hipMemcpyDeviceToHost, st));
  LSQ_HIP_CHECK(hipStreamSynchronize(st));
  LSQ_HIP_CHECK(hipGetLastError());
  lsq_free_one(ctx, scr);
  lsq_free_one(ctx, bs);

  // step 3: M = A_s^T A_s
  if (ctx->fmt == LSQ_DENSE) {
    ctx->Mdense = true;
    ctx->nnzM = n * n;
    if (fp32) {
      float *As;
      ALLOC(As, float, std::max<int64_t>(ctx->s_d, 1) * n);
      ALLOC(ctx->Mf, float, n * n);
      launch_gather_dense_f32(ctx, As, st);
      const int ns = syrk_splits(ctx->s_d, n, ctx->ncu);
      float *sp = nullptr;
      if (ns > 1) ALLOC(sp, float, syrk_scratch_elems(n, ns));
      const int gslot = prof_begin(ctx, KC_GRAM);
      launch_syrk_f32(ctx->s_d, n, As, ctx->Mf, ns, sp, st);
      prof_end(ctx, gslot, (double)ctx->s_d * (double)n * (double)(n + 1));
      launch_dense_diag_guard_f32(n, ctx->Mf, ctx->flags, st);
      LSQ_HIP_CHECK(hipStreamSynchronize(st));
      if (sp) lsq_free_one(ctx, sp);
      lsq_free_one(ctx, As);
    } else {
      double *As;
      ALLOC(As, double, std::max<int64_t>(ctx->s_d, 1) * n);
      ALLOC(ctx->Md, double, n * n);
      launch_gather_dense_f64(ctx, As, st);
      const int ns = syrk_splits(ctx->s_d, n, ctx->ncu);
      double *sp = nullptr;
      if (ns > 1) ALLOC(sp, double, syrk_scratch_elems(n, ns));
      const int gslot = prof_begin(ctx, KC_GRAM);
      launch_syrk_f64(ctx->s_d, n, As, ctx->Md, ns, sp, st);
      prof_end(ctx, gslot, (double)ctx->s_d * (double)n * (double)(n + 1));
      launch_dense_diag_guard_f64(n, ctx->Md, ctx->flags, st);
      LSQ_HIP_CHECK(hipStreamSynchronize(st));
      if (sp) lsq_free_one(ctx, sp);
      lsq_free_one(ctx, As);
    }
  } else {
    ctx->Mdense = false;
    TRY(build_sparse_gram(ctx));
    if (fp32) {
      ALLOC(ctx->Mf, float, ctx->nnzM + 1);
      launch_cast_f64_f32(ctx->Md, ctx->Mf, ctx->nnzM, st);
    }
  }
  LSQ_HIP_CHECK(hipGetLastError());
  // level sets of the two triangular solves of Algorithm 3
  TRY(build_levels(ctx));

  // float32 operator copies
  if (fp32) {
    if (ctx->dtype == LSQ_F32) {
      ctx->A32 = (const float *)ctx->A;
    } else {
      const int64_t cnt = ctx->fmt == LSQ_DENSE ? m * ctx->ld : ctx->nnz;
      ALLOC(ctx->A32own, float, cnt);
      launch_cast_f64_f32((const double *)ctx->A, ctx->A32own, cnt, st);
      ctx->A32 = ctx->A32own;
    }
  }
  if (ctx->fmt == LSQ_CSR && ctx->atap_algo == 3) TRY(build_csc(ctx));

  // work vectors
  ALLOC(ctx->vy, double, n);
  ALLOC(ctx->vr, double, n);
  ALLOC(ctx->vz, double, n);
  ALLOC(ctx->vp, double, n);
  ALLOC(ctx->vq, double, n);
  ALLOC(ctx->vu, double, n);
  ALLOC(ctx->vg, double, n);
  ALLOC(ctx->vrhs, double, n);
  ALLOC(ctx->vx, double, n);
  ALLOC(ctx->vz2, double, n);
  if (fp32) {
    ALLOC(ctx->fy, float, n);
    ALLOC(ctx->fr, float, n);
    ALLOC(ctx->fz, float, n);
    ALLOC(ctx->fp, float, n);
    ALLOC(ctx->fq, float, n);
    ALLOC(ctx->fu, float, n);
    ALLOC(ctx->frhs, float, n);
    ALLOC(ctx->fz2, float, n);
  }
  LSQ_HIP_CHECK(hipMemcpyAsync(hflags, ctx->flags, sizeof(hflags), hipMemcpyDeviceToHost, st));
  LSQ_HIP_CHECK(hipStreamSynchronize(st));
  LSQ_HIP_CHECK(hipGetLastError());
  ctx->info.s = s;
  ctx->info.s_distinct = ctx->s_d;
  ctx->info.nnz_M = ctx->nnzM;
  ctx->info.levels_fwd = ctx->nlev_f;
  ctx->info.levels_bwd = ctx->nlev_b;
  ctx->info.atap_algo = ctx->fmt == LSQ_CSR ? ctx->atap_algo : ctx->opt.atap_algo;
  ctx->info.ties = hflags[2];
  ctx->info.diag_fixes = hflags[1];
  ctx->info.W = ctx->W;
  return LSQ_OK;
}

extern "C" int lsq_setup(const lsq_matrix *A, const double *b, double C, int32_t sweeps, uint64_t seed,
                         const lsq_options *opt, void *stream, lsq_ctx **out) {
  if (!out) return LSQ_EINVAL;
  *out = nullptr;
  if (!A || !b || !A->values || A->m < 1 || A->n < 1 || A->m < A->n || !(C > 0.0) || sweeps < 0) return LSQ_EINVAL;
  if (A->format != LSQ_DENSE && A->format != LSQ_CSR) return LSQ_EINVAL;
  if (A->dtype != LSQ_F64 && A->dtype != LSQ_F32) return LSQ_EINVAL;
  if (A->format == LSQ_DENSE && A->ld < A->n) return LSQ_EINVAL;
  if (A->format == LSQ_CSR && (!A->row_ptr || !A->col_idx || A->nnz < 0 || A->n >= ((int64_t)1 << 31)))
    return LSQ_EINVAL;
  if (((uintptr_t)A->values | (uintptr_t)b) % 4 != 0) return LSQ_EINVAL;
  lsq_options o;
  lsq_default_options(&o);
  if (opt) o = *opt;
  if (o.mode != LSQ_MODE_FP64 && o.mode != LSQ_MODE_FP32_REFINE) return LSQ_EINVAL;
  if (!(o.tol >= 0.0) || o.max_replace < 0) return LSQ_EINVAL;
  if (!(o.tie_eps >= 0.0)) o.tie_eps = 0x1.0p-44;
  if (!(o.inner_tol > 0.0)) o.inner_tol = 1e-5;
  if (o.max_outer <= 0) o.max_outer = 30;
  if (o.near_levels <= 0) o.near_levels = 48;
  if (o.near_levels > 1024) return LSQ_EINVAL;
  if (o.chain_levels > 64 || o.chain_levels < -1) return LSQ_EINVAL;

  lsq_ctx *ctx = new lsq_ctx();
  ctx->fmt = A->format;
  ctx->dtype = A->dtype;
  ctx->m = A->m;
  ctx->n = A->n;
  ctx->ld = A->format == LSQ_DENSE ? A->ld : A->n;
  ctx->nnz = A->format == LSQ_CSR ? A->nnz : A->m * A->n;
  ctx->A = A->values;
  ctx->rp = A->row_ptr;
  ctx->ci = A->col_idx;
  ctx->b = b;
  ctx->stream = (hipStream_t)stream;
  ctx->opt = o;
  ctx->C = C;
  ctx->sweeps = sweeps;
  ctx->seed = seed;
  ctx->atap_algo = o.atap_algo;
  if (hipGetDevice(&ctx->device) != hipSuccess ||
      hipDeviceGetAttribute(&ctx->ncu, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess) {
    delete ctx;
    return LSQ_EHIP;
  }
  const double t0 = now_ms();
  int rc = setup_impl(ctx);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->info.setup_ms = now_ms() - t0;
  if (rc != LSQ_OK) {
    lsq_destroy(ctx);
    return rc;
  }
  ctx->info.status = LSQ_OK;
  *out = ctx;
  return LSQ_OK;
}

// ---------------------------------------------------------------------------
// PCG (Algorithm 2 step 4) on K y = f, K = D^{-1} A^T A D^{-1}, for float64
// (T = double) or the float32 inner solve. On entry r holds the initial
// residual and y the initial iterate; the loop stops when (fixed < 0) the
// recursive ratio ||d.*r|| / nf is <= tol, at k == fixed (fixed >= 0), or at
// k == max_iter.

enum PcgEnd { END_CONVERGED = 0, END_MAXITER = 1, END_FIXED = 2, END_BREAKDOWN = 3, END_ERROR = 4 };

template <typename T>
struct Ops;
template <>
struct Ops<double> {
  static void P(lsq_ctx *c, const double *r, double *z) { sgs_apply_f64(c, r, z); }
  static void K(lsq_ctx *c, const double *p, double *q) { atap_f64(c, c->invD, p, nullptr, q, c->invD); }
  // K from an input already scaled by invD (u = invD p)
  static void K_pre(lsq_ctx *c, const double *u, double *q) { atap_f64(c, nullptr, u, nullptr, q, c->invD); }
  static const double *s(lsq_ctx *c) { return c->invD; }
  static double *u(lsq_ctx *c) { return c->vu; }
  static double *y(lsq_ctx *c) { return c->vy; }
  static double *r(lsq_ctx *c) { return c->vr; }
  static double *z(lsq_ctx *c) { return c->vz; }
  static double *p(lsq_ctx *c) { return c->vp; }
  static double *q(lsq_ctx *c) { return c->vq; }
};
template <>
struct Ops<float> {
  static void P(lsq_ctx *c, const float *r, float *z) { sgs_apply_f32(c, r, z); }
  static void K(lsq_ctx *c, const float *p, float *q) { atap_f32(c, c->invD32, p, q, c->invD32); }
  static void K_pre(lsq_ctx *c, const float *u, float *q) { atap_f32(c, nullptr, u, q, c->invD32); }
  static const float *s(lsq_ctx *c) { return c->invD32; }
  static float *u(lsq_ctx *c) { return c->fu; }
  static float *y(lsq_ctx *c) { return c->fy; }
  static float *r(lsq_ctx *c) { return c->fr; }
  static float *z(lsq_ctx *c) { return c->fz; }
  static float *p(lsq_ctx *c) { return c->fp; }
  static float *q(lsq_ctx *c) { return c->fq; }
};

// PCG iterations from the current (y, r); the next iteration's
// preconditioner application is queued ahead while the residual is above
// kSpecMargin times the tolerance
constexpr double kSpecMargin = 20.0;

template <typename T>
static int pcg_run(lsq_ctx *ctx, const double *dscale, double nf, double tol, int64_t max_iter, int64_t fixed,
                   int64_t *k, double *rel) {
  hipStream_t st = ctx->stream;
  const int64_t n = ctx->n;
  T *y = Ops<T>::y(ctx), *r = Ops<T>::r(ctx), *z = Ops<T>::z(ctx), *p = Ops<T>::p(ctx), *q = Ops<T>::q(ctx);
  bool restart = true, have_z = false;
  if (!ctx->scal_ev && take_event(&ctx->scal_ev) != hipSuccess) {
    ctx->scal_ev = nullptr;
    return END_ERROR;
  }
  for (;;) {
    if (fixed >= 0) {
      if (*k >= fixed) return END_FIXED;
    } else if (*rel <= tol) {
      return END_CONVERGED;
    }
    if (*k >= max_iter) return END_MAXITER;
    if (!have_z) Ops<T>::P(ctx, r, z);
    have_z = false;
    // reductions finish in their own last workgroup (fixed order); the count
    // of arrived workgroups lives in flags[8]
    const Fin fin_rz{ctx->scal, restart ? 0 : Scal::RHO_NEW, restart ? 2 : 3, (unsigned *)(ctx->flags + 8)};
    Vec<T>::dot_partials(n, r, z, nullptr, ctx->part, st, &fin_rz);
    // p = z + beta p, with the operator's scaled input u = invD p in the same pass
    T *u = Ops<T>::u(ctx);
    Vec<T>::update_p_scaled(n, restart ? nullptr : ctx->scal + Scal::BETA, z, p, Ops<T>::s(ctx), u, st);
    restart = false;
    Ops<T>::K_pre(ctx, u, q);
    const Fin fin_pq{ctx->scal, 0, 1, (unsigned *)(ctx->flags + 8)};
    Vec<T>::dot_partials(n, p, q, nullptr, ctx->part, st, &fin_pq);
    const Fin fin_rn{ctx->scal, Scal::RNORM2, 0, (unsigned *)(ctx->flags + 8)};
    Vec<T>::update_yr(n, ctx->scal + Scal::ALPHA, p, q, y, r, dscale, ctx->part, st, &fin_rn);
    // the scalars go to the host; unless this iteration may end the loop, the
    // next iteration's P r (which needs only the new r) is queued before the
    // host waits for them, so the GPU does not idle through the round trip.
    // Unneeded only when the residual falls more than kSpecMargin-fold in one
    // iteration; the arithmetic is the same either way
    if (hipMemcpyAsync(ctx->hscal, ctx->scal, Scal::COUNT * sizeof(double), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipEventRecord(ctx->scal_ev, st) != hipSuccess)
      return END_ERROR;
    const bool may_end = fixed >= 0 ? *k + 1 >= fixed : *rel <= kSpecMargin * tol;
    if (!may_end && *k + 1 < max_iter) {
      Ops<T>::P(ctx, r, z);
      have_z = true;
    }
    if (hipEventSynchronize(ctx->scal_ev) != hipSuccess) return END_ERROR;
    prof_harvest_ready(ctx);
    const double pq = ctx->hscal[Scal::PQ], rho = ctx->hscal[Scal::RHO];
    if (!(pq > 0.0) || !(rho > 0.0)) return END_BREAKDOWN;
    ++*k;
    *rel = sqrt(ctx->hscal[Scal::RNORM2]) / nf;
  }
}

// residual of the normal equation in float64 at the current x (original
// scaling): forward g = A^T(b - A x); adjoint g = gx - A^T A x
static void true_residual(lsq_ctx *ctx, const double *x, const double *gx, double *g) {
  if (!gx) {
    resid64(ctx, x, ctx->b, g);
  } else {
    atap_f64(ctx, nullptr, x, nullptr, ctx->vu, nullptr);
    launch_sub_f64(ctx->n, gx, ctx->vu, g, ctx->stream);
  }
}

// float64 PCG with residual replacement. g0 = right-hand side of the
// normal equation in original scaling (A^T b, or gx for the adjoint).
static int solve_fp64(lsq_ctx *ctx, const double *g0, const double *gx, double *x) {
  hipStream_t st = ctx->stream;
  const int64_t n = ctx->n;
  const lsq_options &o = ctx->opt;
  const int64_t max_iter = o.max_iter > 0 ? o.max_iter : std::min<int64_t>(10 * n, 100000);
  launch_fill_f64(ctx->vy, n, 0.0, st);
  Vec<double>::scale(n, ctx->invD, g0, ctx->vr, st);
  const double nf = sqrt(dev_dot<double>(ctx, n, g0, g0, nullptr, Scal::FNORM2));
  int64_t k = 0, repl = 0;
  double rel = 0.0, rel_true = 0.0;
  bool have_true = false;
  int status = LSQ_OK;
  if (nf == 0.0) {
    launch_fill_f64(x, n, 0.0, st);
    ctx->info.iters = 0;
    ctx->info.replacements = 0;
    ctx->info.relres = 0.0;
    ctx->info.relres_true = 0.0;
    ctx->info.converged = 1;
    LSQ_HIP_CHECK(hipStreamSynchronize(st));
    return LSQ_OK;
  }
  rel = sqrt(dev_dot<double>(ctx, n, ctx->vr, (const double *)nullptr, ctx->D, Scal::TMP0)) / nf;
  for (;;) {
    int end = pcg_run<double>(ctx, ctx->D, nf, o.tol, max_iter, o.fixed_iters, &k, &rel);
    have_true = false;
    if (end == END_ERROR) return LSQ_EHIP;
    if (end == END_BREAKDOWN) {
      status = LSQ_EBREAKDOWN;
      break;
    }
    if (end != END_CONVERGED) break;
    Vec<double>::scale(n, ctx->invD, ctx->vy, x, st);
    true_residual(ctx, x, gx, ctx->vg);
    rel_true = sqrt(dev_dot<double>(ctx, n, ctx->vg, ctx->vg, nullptr, Scal::TMP1)) / nf;
    have_true = true;
    if (rel_true <= o.tol || repl >= o.max_replace || k >= max_iter) break;
    // residual replacement: restart from the true residual
    Vec<double>::scale(n, ctx->invD, ctx->vg, ctx->vr, st);
    rel = rel_true;
    ++repl;
  }
  Vec<double>::scale(n, ctx->invD, ctx->vy, x, st);
  if (!have_true) {
    true_residual(ctx, x, gx, ctx->vg);
    rel_true = sqrt(dev_dot<double>(ctx, n, ctx->vg, ctx->vg, nullptr, Scal::TMP1)) / nf;
  }
  if (status == LSQ_OK && o.fixed_iters < 0 && !(rel_true <= o.tol)) status = LSQ_ENOCONV;
  ctx->info.iters = k;
  ctx->info.outer_iters = 0;
  ctx->info.replacements = repl;
  ctx->info.relres = rel;
  ctx->info.relres_true = rel_true;
  ctx->info.converged = rel_true <= o.tol;
  LSQ_HIP_CHECK(hipStreamSynchronize(st));
  LSQ_HIP_CHECK(hipGetLastError());
  return status;
}

// float32 inner PCG inside float64 iterative refinement of x
static int solve_refine(lsq_ctx *ctx, const double *g0, const double *gx, double *x) {
  hipStream_t st = ctx->stream;
  const int64_t n = ctx->n;
  const lsq_options &o = ctx->opt;
  const int64_t max_iter = o.max_iter > 0 ? o.max_iter : std::min<int64_t>(10 * n, 100000);
  const int64_t max_inner = o.max_inner > 0 ? o.max_inner : max_iter;
  launch_fill_f64(x, n, 0.0, st);
  const double nf = sqrt(dev_dot<double>(ctx, n, g0, g0, nullptr, Scal::FNORM2));
  if (nf == 0.0) {
    ctx->info.iters = 0;
    ctx->info.outer_iters = 0;
    ctx->info.relres = ctx->info.relres_true = 0.0;
    ctx->info.converged = 1;
    LSQ_HIP_CHECK(hipStreamSynchronize(st));
    return LSQ_OK;
  }
  // g = residual at x = 0
  Vec<double>::copy(n, g0, ctx->vg, st);
  double rel = 1.0;
  int64_t total = 0, outer = 0;
  int status = LSQ_OK;
  for (;;) {
    if (rel <= o.tol) break;
    if (outer >= o.max_outer || total >= max_iter) {
      status = LSQ_ENOCONV;
      break;
    }
    // h = D^{-1} g, solved in float32 at unit scale
    Vec<double>::scale(n, ctx->invD, ctx->vg, ctx->vu, st);
    const double nu = sqrt(dev_dot<double>(ctx, n, ctx->vu, ctx->vu, nullptr, Scal::TMP0));
    if (!(nu > 0.0)) break;
    launch_f64_to_f32_scaled(n, ctx->vu, nullptr, 1.0 / nu, ctx->fr, st);
    launch_fill_f32(ctx->fy, n, 0.0f, st);
    const double nf32 = sqrt(dev_dot<float>(ctx, n, ctx->fr, ctx->fr, nullptr, Scal::TMP1));
    int64_t k = 0;
    double rel32 = 1.0;
    const int64_t cap = std::min<int64_t>(max_inner, max_iter - total);
    int end = pcg_run<float>(ctx, nullptr, nf32, o.inner_tol, cap, -1, &k, &rel32);
    if (end == END_ERROR) return LSQ_EHIP;
    total += k;
    ++outer;
    // x += D^{-1} (nu d) in float64
    launch_axpy_scaled_f64(n, nu, ctx->invD, ctx->fy, x, st);
    true_residual(ctx, x, gx, ctx->vg);
    rel = sqrt(dev_dot<double>(ctx, n, ctx->vg, ctx->vg, nullptr, Scal::TMP1)) / nf;
    if (end == END_BREAKDOWN && k == 0) {
      status = LSQ_EBREAKDOWN;
      break;
    }
  }
  ctx->info.iters = total;
  ctx->info.outer_iters = outer;
  ctx->info.replacements = 0;
  ctx->info.relres = rel;
  ctx->info.relres_true = rel;
  ctx->info.converged = rel <= o.tol;
  LSQ_HIP_CHECK(hipStreamSynchronize(st));
  LSQ_HIP_CHECK(hipGetLastError());
  return status;
}

extern "C" int lsq_solve(lsq_ctx *ctx, double *x, lsq_info *info) {
  if (!ctx) return LSQ_EINVAL;
  if (!x) RET(LSQ_EINVAL);
  const double t0 = now_ms();
  // A^T b in float64: the residual pass at x = 0
  launch_fill_f64(ctx->vx, ctx->n, 0.0, ctx->stream);
  resid64(ctx, ctx->vx, ctx->b, ctx->vg);
  double *g0 = ctx->vx;  // A^T b, kept in vx for the solve
  Vec<double>::copy(ctx->n, ctx->vg, g0, ctx->stream);
  int rc = ctx->opt.mode == LSQ_MODE_FP32_REFINE ? solve_refine(ctx, g0, nullptr, x) : solve_fp64(ctx, g0, nullptr, x);
  (void)hipStreamSynchronize(ctx->stream);
  rc = check_wait_flag(ctx, rc);
  ctx->info.solve_ms = now_ms() - t0;
  ctx->info.status = rc;
  if (rc >= 0) ctx->solved = true;
  if (info) *info = ctx->info;
  return rc;
}

// several right-hand sides on one setup: the sample, M and its level sets do
// not depend on b (Algorithm 2 steps 1-3 read A only), so each column only
// repeats step 4
extern "C" int lsq_solve_many(lsq_ctx *ctx, int32_t nrhs, const double *B, int64_t ldb, double *X, int64_t ldx,
                              lsq_info *infos) {
  if (!ctx) return LSQ_EINVAL;
  if (nrhs < 0 || (nrhs > 0 && (!B || !X || ldb < ctx->m || ldx < ctx->n))) RET(LSQ_EINVAL);
  if (nrhs == 0) return LSQ_OK;
  hipStream_t st = ctx->stream;
  // every column is checked before any is solved
  launch_fill_i32(ctx->flags, 1, 0, st);
  for (int32_t j = 0; j < nrhs; ++j)
    k_check_finite<<<grid_n(ctx->m), 256, 0, st>>>(ctx->m, B + (int64_t)j * ldb, ctx->flags);
  int32_t f0 = 0;
  LSQ_HIP_CHECK(hipMemcpyAsync(&f0, ctx->flags, sizeof(f0), hipMemcpyDeviceToHost, st));
  LSQ_HIP_CHECK(hipStreamSynchronize(st));
  if (f0 & 2) {
    ctx->err = "B contains NaN or Inf";
    RET(LSQ_ENONFINITE);
  }
  const double *b0 = ctx->b;
  int worst = LSQ_OK;
  for (int32_t j = 0; j < nrhs; ++j) {
    ctx->b = B + (int64_t)j * ldb;
    lsq_info inf;
    const int rc = lsq_solve(ctx, X + (int64_t)j * ldx, &inf);
    if (infos) infos[j] = inf;
    if (rc < 0) {
      worst = rc;
      break;
    }
    if (rc != LSQ_OK) worst = rc;
  }
  ctx->b = b0;
  return worst;
}

extern "C" int lsq_backward(lsq_ctx *ctx, const double *x, const double *grad_x, double *lambda, double *grad_b,
                            void *grad_A, lsq_info *info) {
  if (!ctx) return LSQ_EINVAL;
  if (!x || !grad_x) RET(LSQ_EINVAL);
  const double t0 = now_ms();
  double *lam = lambda;
  if (!lam) lam = ctx->vx;
  // keep grad_x in a private buffer (the solve overwrites vx when lam is vx)
  double *gx;
  ALLOC(gx, double, ctx->n);
  Vec<double>::copy(ctx->n, grad_x, gx, ctx->stream);
  int rc = ctx->opt.mode == LSQ_MODE_FP32_REFINE ? solve_refine(ctx, gx, gx, lam) : solve_fp64(ctx, gx, gx, lam);
  if (rc >= 0 && (grad_b || grad_A)) grad_pass(ctx, x, lam, grad_b, grad_A);
  (void)hipStreamSynchronize(ctx->stream);
  rc = check_wait_flag(ctx, rc);
  lsq_free_one(ctx, gx);
  if (hipGetLastError() != hipSuccess && rc >= 0) rc = LSQ_EHIP;
  ctx->info.solve_ms = now_ms() - t0;
  ctx->info.status = rc;
  if (info) *info = ctx->info;
  return rc;
}

// ---------------------------------------------------------------------------
// inspection

extern "C" int lsq_get_setup(const lsq_ctx *cctx, double *D_host, double *w_host, int64_t *idx_host, double *gap_host) {
  lsq_ctx *ctx = const_cast<lsq_ctx *>(cctx);
  if (!ctx) return LSQ_EINVAL;
  hipStream_t st = ctx->stream;
  if (D_host) LSQ_HIP_CHECK(hipMemcpyAsync(D_host, ctx->D, ctx->n * sizeof(double), hipMemcpyDeviceToHost, st));
  if (w_host) LSQ_HIP_CHECK(hipMemcpyAsync(w_host, ctx->w, ctx->m * sizeof(double), hipMemcpyDeviceToHost, st));
  if (idx_host) LSQ_HIP_CHECK(hipMemcpyAsync(idx_host, ctx->idx, ctx->s * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  if (gap_host) LSQ_HIP_CHECK(hipMemcpyAsync(gap_host, ctx->gap, ctx->s * sizeof(double), hipMemcpyDeviceToHost, st));
  LSQ_HIP_CHECK(hipStreamSynchronize(st));
  return LSQ_OK;
}

extern "C" int64_t lsq_get_M_nnz(const lsq_ctx *ctx) { return ctx ? ctx->nnzM : -1; }

extern "C" int lsq_get_M(const lsq_ctx *cctx, int64_t *rp_host, int32_t *ci_host, double *v_host) {
  lsq_ctx *ctx = const_cast<lsq_ctx *>(cctx);
  if (!ctx || !rp_host || !ci_host || !v_host) return LSQ_EINVAL;
  hipStream_t st = ctx->stream;
  const int64_t n = ctx->n, nnz = ctx->nnzM;
  std::vector<float> tmpf;
  if (ctx->Mdense) {
    for (int64_t j = 0; j <= n; ++j) rp_host[j] = j * n;
    for (int64_t j = 0; j < n; ++j)
      for (int64_t l = 0; l < n; ++l) ci_host[j * n + l] = (int32_t)l;
  } else {
    std::vector<int32_t> rp(n + 1);
    LSQ_HIP_CHECK(hipMemcpyAsync(rp.data(), ctx->Mrp, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    LSQ_HIP_CHECK(hipMemcpyAsync(ci_host, ctx->Mci, nnz * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    LSQ_HIP_CHECK(hipStreamSynchronize(st));
    for (int64_t j = 0; j <= n; ++j) rp_host[j] = rp[j];
  }
  if (ctx->Md) {
    LSQ_HIP_CHECK(hipMemcpyAsync(v_host, ctx->Md, nnz * sizeof(double), hipMemcpyDeviceToHost, st));
    LSQ_HIP_CHECK(hipStreamSynchronize(st));
  } else {
    tmpf.resize(nnz);
    LSQ_HIP_CHECK(hipMemcpyAsync(tmpf.data(), ctx->Mf, nnz * sizeof(float), hipMemcpyDeviceToHost, st));
    LSQ_HIP_CHECK(hipStreamSynchronize(st));
    for (int64_t q = 0; q < nnz; ++q) v_host[q] = tmpf[q];
  }
  return LSQ_OK;
}

extern "C" int lsq_apply_P(lsq_ctx *ctx, const double *r, double *z) {
  if (!ctx || !r || !z) return LSQ_EINVAL;
  hipStream_t st = ctx->stream;
  if (ctx->opt.mode == LSQ_MODE_FP32_REFINE) {
    launch_f64_to_f32_scaled(ctx->n, r, nullptr, 1.0, ctx->fr, st);
    sgs_apply_f32(ctx, ctx->fr, ctx->fz);
    launch_f32_to_f64(ctx->n, ctx->fz, z, st);
  } else {
    sgs_apply_f64(ctx, r, z);
  }
  LSQ_HIP_CHECK(hipStreamSynchronize(st));
  LSQ_HIP_CHECK(hipGetLastError());
  return check_wait_flag(ctx, LSQ_OK);
}

extern "C" int lsq_apply_K(lsq_ctx *ctx, const double *p, double *q) {
  if (!ctx || !p || !q) return LSQ_EINVAL;
  atap_f64(ctx, ctx->invD, p, nullptr, q, ctx->invD);
  LSQ_HIP_CHECK(hipStreamSynchronize(ctx->stream));
  LSQ_HIP_CHECK(hipGetLastError());
  return LSQ_OK;
}

extern "C" int lsq_get_info(const lsq_ctx *ctx, lsq_info *info) {
  if (!ctx || !info) return LSQ_EINVAL;
  *info = ctx->info;
  return LSQ_OK;
}
