/*
 * lsq.h -- C ABI of the MI355X (gfx950) row-sampling preconditioned
 * least-squares solver.
 *
 * The method is Algorithm 2 of Chen & Wu, "A Preconditioner based on
 * Non-uniform Row Sampling for Linear Least Squares Problems"
 * (arXiv:1806.02968): for an overdetermined full-rank A (m x n, m >= n) it
 * solves the normal equation A^T A x = A^T b (Section 1, Eq. NOR) by
 * preconditioned CG, where the preconditioner is a few symmetric Gauss-Seidel
 * sweeps (Algorithm 3) on the Gram matrix M = A_s^T A_s of s = ceil(C n ln n)
 * rows drawn with probability proportional to their squared norm
 * (Algorithm 1, Eq. R2P) from the column-normalised matrix (Algorithm 2
 * step 1).
 *
 * Conventions shared by every entry point:
 *  - All array arguments are DEVICE pointers unless the name ends in _host.
 *    Device arrays must be 16-byte aligned; the library never frees them.
 *  - All GPU work is enqueued on the HIP stream given to lsq_setup
 *    (hipStream_t passed as void*; NULL = the null stream). Entry points
 *    return once their outputs are final on that stream (each one reads a
 *    few scalars back to the host, which synchronises the stream).
 *  - Return codes: 0 = LSQ_OK; a positive code is a warning whose outputs are
 *    still written; a negative code is an error. lsq_strerror() names a code,
 *    lsq_last_error() gives the context's last message.
 *  - A context is not thread safe; use one per host thread.
 */
#ifndef LSQ_H
#define LSQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define LSQ_OK 0
#define LSQ_ENOCONV 1      /* tolerance not reached within max_iter; x written  */
#define LSQ_EINVAL (-1)    /* bad argument (null pointer, m < n, n < 1, C <= 0,
                              sweeps < 0, unknown format/dtype/mode, bad CSR)  */
#define LSQ_ESINGULAR (-2) /* a column of A is zero (rank(A) < n)               */
#define LSQ_ENONFINITE (-3)/* A or b holds NaN or Inf                           */
#define LSQ_ENOMEM (-4)    /* device allocation failed                          */
#define LSQ_EHIP (-5)      /* a HIP runtime call failed                         */
#define LSQ_EBREAKDOWN (-6)/* PCG breakdown: p^T A^T A p <= 0 or r^T P r <= 0    */
#define LSQ_ESTATE (-7)    /* call not valid in the context's state             */

/* ---- matrix description ------------------------------------------------ */
#define LSQ_DENSE 0 /* row-major, element (i,j) at values[i*ld + j]           */
#define LSQ_CSR 1   /* row_ptr[m+1] (int64), col_idx[nnz] (int32, ascending
                       and unique within each row), values[nnz]               */
#define LSQ_F64 0
#define LSQ_F32 1

typedef struct {
  int32_t format;         /* LSQ_DENSE or LSQ_CSR                              */
  int32_t dtype;          /* storage type of values: LSQ_F64 or LSQ_F32        */
  int64_t m, n;           /* rows, columns; m >= n >= 1                        */
  int64_t ld;             /* dense: row stride in elements, ld >= n            */
  int64_t nnz;            /* CSR: number of stored entries                     */
  const void *values;     /* device; borrowed until lsq_destroy                */
  const int64_t *row_ptr; /* device (CSR)                                      */
  const int32_t *col_idx; /* device (CSR)                                      */
} lsq_matrix;

/* ---- options ----------------------------------------------------------- */
#define LSQ_MODE_FP64 0        /* every step in float64                         */
#define LSQ_MODE_FP32_REFINE 1 /* float32 inner PCG (float32 A and M, float32
                                  Gram product) inside float64 iterative
                                  refinement of x (residual, A^T r, update and
                                  stopping norms in float64)                  */

typedef struct {
  int32_t mode;        /* LSQ_MODE_*; fixed at setup                         */
  double tol;          /* stop when ||A^T(b - A x)|| / ||A^T b|| <= tol (1e-10) */
  int64_t max_iter;    /* PCG iteration cap (0: min(10 n, 100000))           */
  int64_t fixed_iters; /* >= 0: run exactly this many PCG iterations, no stop
                          test, no residual replacement (-1: off)            */
  int32_t max_replace; /* residual replacements after convergence of the
                          recursive residual (3)                             */
  double inner_tol;    /* FP32_REFINE: inner relative tolerance (1e-5)       */
  int64_t max_inner;   /* FP32_REFINE: inner iteration cap per outer step (0: max_iter) */
  int32_t max_outer;   /* FP32_REFINE: refinement steps cap (30)             */
  double tie_eps;      /* CDF-boundary tie band for reporting draws (2^-44)  */
  int32_t atap_algo;   /* A^T(Ap) kernel: 0 auto; sparse A: 1 global atomics,
                          2 workgroup partial sums in LDS, 3 a row pass then a
                          pass over a column-major copy of A; dense A: 1 one
                          wave per row, 2 row batches staged in LDS, 3 one
                          wave per row with 16-byte loads, 4 column groups
                          owned by threads, row batches in registers (n a
                          multiple of 4 / 2 for float32 / float64 storage,
                          n <= 2048 / 1024, rows 16-byte aligned)            */
  int32_t profile;     /* nonzero: time every hot-kernel launch with HIP
                          events on the context's stream (lsq_get_kernel_stats) */
  int32_t near_levels; /* triangular solves: entries reading rows at most this
                          many levels below their own row's level are summed on
                          the dependency chain, older ones ahead of time on
                          other CUs (0: 48; at most 1024)                    */
  int32_t chain_levels; /* triangular solves: when x and the rows' partial sums
                          fit in LDS and levels hold at most 32 rows on
                          average (any rows when
                          set explicitly), one wave sums
                          the entries reading rows at most this many levels
                          below (0: automatic, the most levels from 6 down to
                          3 that keep at most 8 such entries per row, else 3
                          when it keeps at most 32, else 2 when that does;
                          -1: off; at most 64)                               */
} lsq_options;

/* Fills *opt with the defaults above. */
void lsq_default_options(lsq_options *opt);

/* ---- statistics -------------------------------------------------------- */
typedef struct {
  int64_t s;            /* draws, ceil(C n ln n) (at least n)                 */
  int64_t s_distinct;   /* distinct rows among the draws                      */
  int64_t nnz_M;        /* stored entries of M (n*n when M is dense)          */
  int64_t levels_fwd;   /* level sets of the forward (lower) solve            */
  int64_t levels_bwd;   /* level sets of the backward (upper) solve           */
  int64_t ties;         /* draws whose CDF gap is <= tie_eps                  */
  int64_t diag_fixes;   /* zero diagonal entries of M replaced by 1           */
  int64_t iters;        /* PCG iterations (FP64) / total inner iterations     */
  int64_t outer_iters;  /* refinement steps (FP32_REFINE)                     */
  int64_t replacements; /* residual replacements                              */
  double W;             /* total row weight of the normalised matrix (= n)    */
  double relres;        /* recursive residual ratio at exit                   */
  double relres_true;   /* true ||A^T(b-Ax)|| / ||A^T b|| (float64) at exit   */
  double setup_ms;      /* lsq_setup wall time                                */
  double solve_ms;      /* last lsq_solve / lsq_backward wall time            */
  int32_t converged;    /* 1 if relres_true <= tol                            */
  int32_t status;       /* return code of the last call                       */
  int32_t trsv_mode;    /* triangular solves: 0 one main workgroup with x in
                           LDS, 1 chain mode, 2 main workgroups with x in
                           global memory, 3 dense M in 64-row blocks, one
                           workgroup per block                                */
  int32_t atap_algo;    /* sparse A: the A^T(Ap) kernel in use (values of
                           lsq_options.atap_algo); dense A: the option as
                           given (0: chosen per call by the vector length)    */
  int32_t chain_levels; /* chain mode: the levels below a row whose entries
                           are summed on the chain (0 outside chain mode)     */
  int32_t chain_max;    /* chain mode: the most such entries in one row (the
                           chain wave holds 4 rows of 16 lanes' worth: the
                           smallest power of two >= 2 and >= chain_max / 4
                           entries per lane); 0 outside chain mode            */
} lsq_info;

typedef struct lsq_ctx lsq_ctx;

/* Algorithm 2 steps 1-3 (Section 4.1): column norms D, row weights
 * w_i = ||a_i D^{-1}||^2 (Eq. R2P), s draws with replacement (Algorithm 1)
 * from a Philox4x64-10 counter generator keyed by seed, the Gram matrix
 * M = sum_t (1/(s p_{i_t})) a_{i_t}^T a_{i_t} of the normalised rows
 * (Section 3.3), and the level sets of its triangular solves (Algorithm 3).
 *   A      matrix (borrowed, must stay valid and unchanged until lsq_destroy)
 *   b      device float64[m] right-hand side (borrowed likewise)
 *   C      sample-size factor (> 0; the paper uses 4)
 *   sweeps Gauss-Seidel sweeps t of Algorithm 3 (>= 0; 0 gives plain CG on
 *          the normalised system, the paper's "CG" comparison)
 *   seed   key of the counter generator
 *   opt    options (NULL: defaults)
 *   stream hipStream_t for all work
 *   out    receives the context; NULL on error
 * Errors: LSQ_EINVAL, LSQ_ESINGULAR, LSQ_ENONFINITE, LSQ_ENOMEM, LSQ_EHIP. */
int lsq_setup(const lsq_matrix *A, const double *b, double C, int32_t sweeps, uint64_t seed,
              const lsq_options *opt, void *stream, lsq_ctx **out);

/* Algorithm 2 step 4: PCG on A^T A x = A^T b with the sampled SGS
 * preconditioner, iterating on the normalised unknown y = D x.
 *   x     device float64[n]; output (the iteration starts from x = 0)
 *   info  host, nullable
 * Returns LSQ_OK, LSQ_ENOCONV (x still written), LSQ_EBREAKDOWN, LSQ_EHIP. */
int lsq_solve(lsq_ctx *ctx, double *x, lsq_info *info);

/* Several right-hand sides on one setup (not in the paper): Algorithm 2
 * steps 1-3 read A only, so the sample, M and the level sets of lsq_setup
 * serve every b; step 4 (PCG) runs once per column, in column order, each
 * exactly as lsq_solve with that column in place of the setup's b.
 *   nrhs   number of columns (>= 0; 0 returns LSQ_OK and touches nothing)
 *   B      device float64, column j at B + j*ldb (m entries), ldb >= m;
 *          borrowed for the call only
 *   X      device float64, column j at X + j*ldx (n entries), ldx >= n;
 *          output, columns must not overlap B
 *   infos  host lsq_info[nrhs], nullable: one record per column
 * Every column of B is checked for NaN/Inf before any is solved
 * (LSQ_ENONFINITE, nothing written). Returns LSQ_OK; LSQ_ENOCONV if some
 * column missed the tolerance (all columns still solved and written); the
 * first negative status (LSQ_EBREAKDOWN, LSQ_EHIP), after which later
 * columns are not solved. The setup's own b is kept for later lsq_solve.
 * Each column's work is that of one lsq_solve: the per-iteration kernels are
 * not batched across columns. */
int lsq_solve_many(lsq_ctx *ctx, int32_t nrhs, const double *B, int64_t ldb, double *X, int64_t ldx,
                   lsq_info *infos);

/* Differentiable form (not in the paper): given the solution x of lsq_solve
 * and grad_x = dL/dx, solves the adjoint A^T A lambda = grad_x with the same
 * preconditioner and mode, then forms
 *   grad_b = A lambda                    (device float64[m], nullable)
 *   grad_A = (b - A x) lambda^T - (A lambda) x^T restricted to A's pattern
 *            (device, A's dtype: m*ld for dense, nnz for CSR; nullable)
 *   lambda                               (device float64[n], nullable)
 * Returns as lsq_solve. */
int lsq_backward(lsq_ctx *ctx, const double *x, const double *grad_x, double *lambda,
                 double *grad_b, void *grad_A, lsq_info *info);

/* ---- inspection of the set-up state (used by parity checks) ----------- */

/* Copies of the setup's quantities to HOST memory:
 *   D_host[n] column norms; w_host[m] row weights;
 *   idx_host[s] drawn row of each draw t; gap_host[s] its CDF gap / W.
 * Null pointers are skipped.                                               */
int lsq_get_setup(const lsq_ctx *ctx, double *D_host, double *w_host, int64_t *idx_host,
                  double *gap_host);

/* M to HOST memory as float64 (in FP32_REFINE mode the float32 M, widened).
 * lsq_get_M_nnz gives the number of stored entries (n*n when dense).
 * rp_host[n+1], ci_host[nnz], v_host[nnz]; for dense M the CSR lists every
 * entry of each row.                                                       */
int64_t lsq_get_M_nnz(const lsq_ctx *ctx);
int lsq_get_M(const lsq_ctx *ctx, int64_t *rp_host, int32_t *ci_host, double *v_host);

/* One application of the preconditioner z = P r (Algorithm 3 from e = 0;
 * FP32_REFINE contexts apply their float32 M and widen the result) and of
 * the normalised normal-equation operator q = D^{-1}A^T A D^{-1} p (float64
 * arithmetic on A's storage in both modes). Device float64[n] in and out.  */
int lsq_apply_P(lsq_ctx *ctx, const double *r, double *z);
int lsq_apply_K(lsq_ctx *ctx, const double *p, double *q);

/* Per-kernel-class launch statistics accumulated while opt.profile is set:
 * class 0 = triangular solve of Algorithm 3, 1 = its strict-part product,
 * 2 = the fused A^T(A p) pass (with its reduction), 3 = vector kernels,
 * 4 = the dense Gram product M = A_s^T A_s (MFMA; setup, Section 3.3).
 * bytes[] are ALGORITHMIC bytes: one read of every stored entry the kernel
 * needs (value + column index) and of its vectors, one write of its output;
 * for class 4 it holds floating-point operations instead (2 per
 * multiply-add of the n(n+1)/2 distinct entries of M).
 * reset != 0 clears the counters after copying them.                       */
#define LSQ_KC_TRSV 0
#define LSQ_KC_SGS_RHS 1
#define LSQ_KC_ATAP 2
#define LSQ_KC_VEC 3
#define LSQ_KC_GRAM 4
#define LSQ_KCLASSES 5
typedef struct {
  int64_t launches[LSQ_KCLASSES];
  double ms[LSQ_KCLASSES];
  double bytes[LSQ_KCLASSES];
} lsq_kernel_stats;
int lsq_get_kernel_stats(lsq_ctx *ctx, lsq_kernel_stats *stats, int32_t reset);

/* Copies the statistics of the last call into *info. */
int lsq_get_info(const lsq_ctx *ctx, lsq_info *info);

/* Frees everything the context owns (not A, b or caller outputs). NULL ok. */
void lsq_destroy(lsq_ctx *ctx);

const char *lsq_strerror(int code);
const char *lsq_last_error(const lsq_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* LSQ_H */
