// Internal header of liblsq: device helpers, the context layout and the
// host-side launchers of every kernel. Not part of the public ABI (lsq.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "lsq.h"

namespace lsq {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// device helpers

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// sum over aligned groups of G lanes (G a power of two <= 64)
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

// Sums over groups of G lanes with DPP moves (no LDS traffic). G <= 16: every
// lane of the group holds the sum; G == 32: lane 31 of each half-wave; G == 64:
// lane 63. dpp_sum_lane<G>() names a lane holding the result.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_take(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int tlo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWMASK, 0xF, false);
  const int thi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWMASK, 0xF, false);
  return __hiloint2double(thi, tlo);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_take(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xF, false));
}

template <int G, typename T>
__device__ __forceinline__ T dpp_group_sum(T v) {
  // quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror
  if (G >= 2) v += dpp_take<0xB1, 0xF>(v);
  if (G >= 4) v += dpp_take<0x4E, 0xF>(v);
  if (G >= 8) v += dpp_take<0x141, 0xF>(v);
  if (G >= 16) v += dpp_take<0x140, 0xF>(v);
  // row_bcast:15 into rows 1 and 3, then row_bcast:31 into rows 2 and 3
  if (G >= 32) v += dpp_take<0x142, 0xA>(v);
  if (G >= 64) v += dpp_take<0x143, 0xC>(v);
  return v;
}
template <int G>
__device__ __forceinline__ int dpp_sum_lane() {
  return G == 64 ? 63 : (G == 32 ? 31 : 0);
}

// block-wide sum, result valid in every thread; red must hold blockDim/64 T
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *red) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  T t = 0;
  for (int k = 0; k < nw; ++k) t += red[k];
  return t;
}

// ---------------------------------------------------------------------------
// context

struct Dev {
  void *p = nullptr;
  size_t bytes = 0;
};

struct Scal {
  // device scalars of the PCG loop (float64 slots; the float32 loop uses the
  // float slots of the same layout through a second array)
  enum { RHO = 0, PQ, ALPHA, BETA, RNORM2, RHO_NEW, FNORM2, TMP0, TMP1, COUNT = 16 };
};

}  // namespace lsq

// device-side tasks and entries of one triangular solve
struct TriDev {
  int4 *ta = nullptr, *tb = nullptr, *ft = nullptr;
  int32_t *mci = nullptr, *fci = nullptr;
  void *mval = nullptr, *fval = nullptr;
  int64_t nbatch = 0, nft = 0, nslot = 0;
  // chain mode: per pass and lane the row and the chain entries
  int32_t *crow = nullptr, *cj = nullptr;
  void *cv = nullptr;
  int64_t npass = 0;
};

struct lsq_ctx {
  // problem (borrowed)
  int32_t fmt = 0, dtype = 0;
  int64_t m = 0, n = 0, ld = 0, nnz = 0;
  const void *A = nullptr;
  const int64_t *rp = nullptr;
  const int32_t *ci = nullptr;
  const double *b = nullptr;
  hipStream_t stream = nullptr;
  lsq_options opt{};
  double C = 4.0;
  int32_t sweeps = 1;
  uint64_t seed = 0;
  int device = 0;
  int ncu = 1;  // compute units of the device

  // setup results
  double *D = nullptr, *invD = nullptr, *w = nullptr, *cdf = nullptr;
  float *invD32 = nullptr;
  int64_t s = 0, s_d = 0;
  int64_t *idx = nullptr;
  double *gap = nullptr;
  int32_t *cnt = nullptr;
  int64_t *urow = nullptr;  // distinct drawn rows, ascending
  int32_t *ucnt = nullptr;  // multiplicity of each
  double W = 0.0;

  // M: dense (n*n row-major) or CSR with int32 offsets
  bool Mdense = false;
  bool dense_blk = false;  // dense M: blocked triangular solves
  int64_t nnzM = 0;
  double *Md = nullptr;   // float64 values (dense n*n or CSR nnz)
  float *Mf = nullptr;    // float32 values (FP32_REFINE)
  int32_t *Mrp = nullptr, *Mci = nullptr, *Mdiag = nullptr;

  // triangular solves: main-block task slots (row, near range, late count)
  // and (rows of lower levels, far slots), helper far-chunk tasks, and the
  // triangle's entries copied in task order (values in the solve's precision)
  int G = 64;  // lanes per row in the strict-part products
  int trsv_e = 4;  // near entries per lane of the triangular solves' main block
  bool trsv_chain = false;  // chain mode of the triangular solves
  bool trsv_preset = false;  // the next solve's sentinel slots were set by the kernel before it
  int trsv_ec = 2;          // chain entries per lane (chain mode)
  TriDev tri_f, tri_b;
  void *tdg = nullptr;     // diagonal of M
  void *farbuf = nullptr;  // far-sum slots
  int64_t nlev_f = 0, nlev_b = 0;

  // float32 copy of A when A is stored in float64 (FP32_REFINE)
  const float *A32 = nullptr;
  float *A32own = nullptr;

  // work vectors
  double *vy = nullptr, *vr = nullptr, *vz = nullptr, *vp = nullptr, *vq = nullptr, *vu = nullptr,
         *vg = nullptr, *vrhs = nullptr, *vx = nullptr, *vz2 = nullptr;
  float *fy = nullptr, *fr = nullptr, *fz = nullptr, *fp = nullptr, *fq = nullptr, *fu = nullptr,
        *frhs = nullptr, *fe = nullptr, *fz2 = nullptr;
  double *part = nullptr;  // reduction partials / dense A^T(Ap) partial rows
  size_t part_bytes = 0;
  double *scal = nullptr;  // device scalars (float64)
  float *scalf = nullptr;  // device scalars (float32)
  int32_t *flags = nullptr;  // device status flags
  double *hscal = nullptr;   // pinned host scalars
  double *vm = nullptr;      // m-length float64 scratch

  // sparse A^T(Ap) algorithm in use
  int atap_algo = 1;
  // CSC copy of a sparse A (two-pass A^T(Ap), atap_algo 3): column pointers,
  // row indices, values in A's storage type and, when the float32 inner solve
  // reads a float32 copy of A, in float32; t = A u between the passes
  int64_t *csc_cp = nullptr;
  int32_t *csc_ri = nullptr;
  void *csc_v = nullptr;
  float *csc_v32 = nullptr;
  double *tvec = nullptr;

  // kernel timing (opt.profile)
  static constexpr int kProfSlots = 64;
  hipEvent_t prof_ev[2 * kProfSlots] = {};
  int prof_cls[kProfSlots] = {};
  double prof_bytes[kProfSlots] = {};
  int prof_alias[kProfSlots] = {};  // >= 0: the slot starts at that event (a predecessor's end)
  int prof_used = 0;
  bool prof_ready = false;
  hipEvent_t scal_ev = nullptr;  // marks the PCG scalars' copy to the host
  lsq_kernel_stats kstats{};

  lsq_info info{};
  std::string err;
  std::vector<lsq::Dev> allocs;
  bool solved = false;
};

namespace lsq {

// ---------------------------------------------------------------------------
// launchers (each enqueues on `st`; no host synchronisation)

// setup (k_setup.hip)
void launch_fill_f64(double *x, int64_t n, double v, hipStream_t st);
void launch_fill_f32(float *x, int64_t n, float v, hipStream_t st);
void launch_fill_i32(int32_t *x, int64_t n, int32_t v, hipStream_t st);
void launch_colnorm_dense(const lsq_ctx *c, double *part, int nblk, hipStream_t st);
void launch_colnorm_csr(const lsq_ctx *c, double *sumsq, hipStream_t st);
int launch_colnorm_csr_part(const lsq_ctx *c, double *part, hipStream_t st);
void launch_colnorm_finish(int64_t n, const double *part, int nblk, double *D, double *invD,
                           float *invD32, int32_t *flags, hipStream_t st);
void launch_rowweight(const lsq_ctx *c, double *w, int32_t *flags, hipStream_t st);
void launch_scan_cdf(int64_t m, const double *w, double *cdf, double *blocksum, hipStream_t st);
void launch_draw(int64_t m, const double *w, const double *cdf, int64_t s, uint64_t seed,
                 int64_t *idx, double *gap, int32_t *cnt, hipStream_t st);
// distinct rows: returns device count in *dcount (int64); urow/ucnt sized m
void launch_compact_counts(int64_t m, const int32_t *cnt, int64_t *scratch, int64_t *urow,
                           int32_t *ucnt, int64_t *dcount, hipStream_t st);
size_t scan_scratch_elems(int64_t m);

// Gram (k_gram.hip)
// dense: gathers the scaled distinct rows into As (s_d x n, row-major) then
// M = As^T As (upper tiles by MFMA, mirrored)
void launch_gather_dense_f64(const lsq_ctx *c, double *As, hipStream_t st);
void launch_gather_dense_f32(const lsq_ctx *c, float *As, hipStream_t st);
// M = A_s^T A_s on MFMA; nsplit > 1 splits the sampled rows, with a scratch
// of syrk_scratch_elems(n, nsplit) values for the partial tiles
int syrk_splits(int64_t sd, int64_t n, int ncu);
size_t syrk_scratch_elems(int64_t n, int nsplit);
void launch_syrk_f64(int64_t sd, int64_t n, const double *As, double *M, int nsplit, double *part,
                     hipStream_t st);
void launch_syrk_f32(int64_t sd, int64_t n, const float *As, float *M, int nsplit, float *part, hipStream_t st);
void launch_dense_diag_guard_f64(int64_t n, double *M, int32_t *flags, hipStream_t st);
void launch_dense_diag_guard_f32(int64_t n, float *M, int32_t *flags, hipStream_t st);
// sparse Gram (several passes with host-read sizes); returns LSQ code
int build_sparse_gram(lsq_ctx *c);
void launch_cast_f64_f32(const double *x, float *y, int64_t n, hipStream_t st);

// SGS (k_sgs.hip)
int build_levels(lsq_ctx *c);
void sgs_apply_f64(lsq_ctx *c, const double *r, double *z);
void sgs_apply_f32(lsq_ctx *c, const float *r, float *z);

// A^T(Ap) and friends (k_atap.hip)
// q = s_out .* A^T( hb*b - A (s_in .* p) ), with hb in {0,1}; s_in/s_out may be null
void atap_f64(lsq_ctx *c, const double *s_in, const double *p, const double *b, double *q,
              const double *s_out);
void atap_f32(lsq_ctx *c, const float *s_in, const float *p, float *q, const float *s_out);
int build_csc(lsq_ctx *ctx);  // k_transpose.hip
// float64 residual pass: g = A^T (b - A x) (b may be null: g = -A^T A x)
void resid64(lsq_ctx *c, const double *x, const double *b, double *g);
// backward pass over A: grad_b = A lam, grad_A = (b - A x) lam^T - (A lam) x^T
void grad_pass(lsq_ctx *c, const double *x, const double *lam, double *grad_b, void *grad_A);

// vector ops (k_vec.hip)
// a reduction finished in the kernel that forms its partials: scal[dst] and
// the op of launch_finish; cnt counts the workgroups that have arrived (zero
// between reductions)
struct Fin {
  double *scal;
  int dst, op;
  unsigned *cnt;
};

template <typename T>
struct Vec {
  static void scale(int64_t n, const T *a, const T *x, T *y, hipStream_t st);  // y = a.*x
  static void copy(int64_t n, const T *x, T *y, hipStream_t st);
  // dot partials: part[nb] = partial sums of x.*y (or (d.*x)^2 when d != null and y == null);
  // with fin, the last workgroup also finishes the sum (launch_finish's op)
  static int dot_partials(int64_t n, const T *x, const T *y, const double *d, double *part,
                          hipStream_t st, const Fin *fin = nullptr);
  // y += alpha p; r -= alpha q; partial sums of (d .* r)^2 (d may be null)
  static int update_yr(int64_t n, const double *alpha, const T *p, const T *q, T *y, T *r,
                       const double *d, double *part, hipStream_t st, const Fin *fin = nullptr);
  // p = z + beta p  (beta == null: p = z)
  static void update_p(int64_t n, const double *beta, const T *z, T *p, hipStream_t st);
  // the same, also writing u = s .* p (the scaled input of the operator product)
  static void update_p_scaled(int64_t n, const double *beta, const T *z, T *p, const T *s, T *u, hipStream_t st);
};
// single-block finisher over `np` partials (fixed order, deterministic):
// op 0: scal[dst] = sum; op 1: scal[PQ] = sum, scal[ALPHA] = scal[RHO] / sum;
// op 2: scal[RHO] = scal[RHO_NEW] = sum; op 3: scal[RHO_NEW] = sum,
// scal[BETA] = sum / scal[RHO], scal[RHO] = sum
void launch_finish(const double *part, int np, double *scal, int dst, int op, hipStream_t st);
// x = a .* y in float64 (x = D^-1 y) and float32->float64 axpy helpers
void launch_axpy_scaled_f64(int64_t n, double nu, const double *invD, const float *d, double *x,
                            hipStream_t st);
void launch_f64_to_f32_scaled(int64_t n, const double *x, const double *s, double mul, float *y,
                              hipStream_t st);
void launch_f32_to_f64(int64_t n, const float *x, double *y, hipStream_t st);
void launch_sub_f64(int64_t n, const double *a, const double *b, double *y, hipStream_t st);

}  // namespace lsq

namespace lsq {
// kernel timing around launches of one class; no-ops unless opt.profile
int prof_begin(lsq_ctx *c, int cls);
void prof_end(lsq_ctx *c, int slot, double bytes);
// ends `slot` and begins a slot of class cls at the same event (for launches
// queued back to back: one timing event between them instead of two)
int prof_switch(lsq_ctx *c, int slot, double bytes, int cls);
void prof_harvest(lsq_ctx *c);  // call after the stream has been synchronised
void prof_harvest_ready(lsq_ctx *c);  // harvests the launches already complete
enum { KC_TRSV = LSQ_KC_TRSV, KC_SGS_RHS = LSQ_KC_SGS_RHS, KC_ATAP = LSQ_KC_ATAP, KC_VEC = LSQ_KC_VEC, KC_GRAM = LSQ_KC_GRAM };
}  // namespace lsq

#define LSQ_HIP_CHECK(expr)                                   \
  do {                                                        \
    hipError_t e_ = (expr);                                   \
    if (e_ != hipSuccess) return lsq_hip_fail(ctx, e_, #expr); \
  } while (0)

int lsq_hip_fail(lsq_ctx *ctx, hipError_t e, const char *what);
void *lsq_alloc(lsq_ctx *ctx, size_t bytes);
void lsq_free_one(lsq_ctx *ctx, void *p);
