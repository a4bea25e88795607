/*
 * CPU oracle for the row-sampling preconditioned least-squares solver of
 * Chen & Wu, "A Preconditioner based on Non-uniform Row Sampling for Linear
 * Least Squares Problems" (arXiv:1806.02968).
 *
 * TEST INFRASTRUCTURE ONLY. This library is the slow, sequential, float64
 * reference that the GPU library is checked against. Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the GPU
 * library never links or calls it, and the two share no source.
 *
 * Every routine follows the paper's definitions in the paper's order:
 *   Algorithm 2 step 1   column normalisation A <- A D^{-1}
 *   Eq. (R2P)            sampling density p_k = ||a_k||^2 / ||A||_F^2
 *   Algorithm 1          s i.i.d. draws with replacement, scale 1/sqrt(s p)
 *   Section 3.3 (EATA)   M = A_s^T A_s = (1/s) sum_t a_{i_t}^T a_{i_t} / p_{i_t}
 *   Algorithm 3          t forward then t backward Gauss-Seidel steps on M
 *   Algorithm 2 step 4   PCG on the normal equation (Eq. NOR)
 * plus the adjoint solve and gradient formulas of the differentiable form.
 */
#ifndef LSQ_ORACLE_H
#define LSQ_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t fmt;   /* 0: dense row-major, 1: CSR                         */
  int32_t dtype; /* 0: float64 values, 1: float32 values                */
  int64_t m, n;  /* rows, columns                                       */
  int64_t ld;    /* dense: row stride in elements (>= n)               */
  int64_t nnz;   /* CSR: number of stored entries                       */
  const void *values;
  const int64_t *row_ptr; /* CSR: m+1 */
  const int32_t *col_idx; /* CSR: nnz, ascending and unique per row */
} orc_matrix;

typedef struct {
  int64_t s;            /* number of draws                                   */
  int64_t iters;        /* PCG iterations                                    */
  int64_t replacements; /* residual replacements performed                   */
  int64_t ties;         /* draws whose CDF gap is <= tie_eps                 */
  int64_t diag_fixes;   /* zero diagonal entries of M replaced by 1          */
  int64_t nnz_M;        /* stored entries of M (CSR) or n*n (dense)          */
  double W;             /* total row weight (the CDF's last entry)           */
  double relres;        /* recursive ||D r|| / ||D f|| at exit               */
  double relres_true;   /* true residual norm ratio at exit                  */
  int32_t status;       /* 0 ok, 1 not converged, <0 error                   */
} orc_info;

typedef struct orc_state orc_state;

/* ---- building blocks (each also used on its own by the tests) ---------- */

/* Philox4x64-10 block function (Salmon et al., SC'11). */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
/* Uniform u_t in [0,1) for draw t: word (t mod 4) of Philox4x64-10 with
 * counter (t div 4, 0, 0, 0) and key (seed, 0), top 53 bits times 2^-53.   */
double orc_uniform(uint64_t seed, int64_t t);
/* s = max(n, ceil(C n ln n)); 1 when n == 1.                               */
int64_t orc_sample_size(double C, int64_t n);
/* D_j = sqrt(sum_i a_ij^2). Returns 0, -2 if some D_j == 0, -3 if not finite */
int orc_column_norms(const orc_matrix *A, double *D);
/* w_i = sum_j (a_ij * invD_j)^2                                             */
void orc_row_weights(const orc_matrix *A, const double *invD, double *w);
/* inclusive prefix sums of w; returns the total W = cdf[m-1]                */
double orc_cdf(int64_t m, const double *w, double *cdf);
/* draw index for tau: first i with cdf_i > tau among rows with w_i > 0;
 * writes the relative distance of tau to the nearest bracketing CDF value. */
int64_t orc_draw(int64_t m, const double *w, const double *cdf, double tau, double *gap);

/* ---- the method ---------------------------------------------------------- */

/* Algorithm 2 steps 1-3. idx_override (nullable) replaces the s draws.     */
orc_state *orc_setup(const orc_matrix *A, double C, int32_t sweeps, uint64_t seed,
                     double tie_eps, const int64_t *idx_override, int64_t s_override,
                     int32_t *status);
void orc_free(orc_state *st);

int64_t orc_n(const orc_state *st);
int64_t orc_s(const orc_state *st);
void orc_get_D(const orc_state *st, double *D);
void orc_get_w(const orc_state *st, double *w);
void orc_get_samples(const orc_state *st, int64_t *idx, double *gap);
void orc_get_info(const orc_state *st, orc_info *info);
/* M as dense n x n (works for both storages; small n only)                 */
void orc_get_M_dense(const orc_state *st, double *M);
/* M as CSR: sizes first (nnz), then arrays                                  */
int64_t orc_M_nnz(const orc_state *st);
void orc_get_M_csr(const orc_state *st, int64_t *rp, int32_t *ci, double *v);
/* one entry M_jl computed from the draws (independent of the stored M)     */
double orc_M_entry(const orc_state *st, int64_t j, int64_t l);

/* z = P r, Algorithm 3 from e = 0 (literal form e <- e + B^{-1}(r - M e)) */
void orc_apply_P(const orc_state *st, const double *r, double *z);
/* q = D^{-1} A^T A D^{-1} p                                                  */
void orc_apply_K(const orc_state *st, const double *p, double *q);

/* Algorithm 2 step 4. x: out (n). fixed_iters >= 0 runs exactly that many
 * iterations with no stopping test and no residual replacement.            */
int orc_solve(orc_state *st, const double *b, double tol, int64_t max_iter,
              int64_t fixed_iters, int32_t max_replace, double *x, orc_info *info);

/* Adjoint solve A^T A lambda = gx (same preconditioner), then
 * grad_b = A lambda and grad_A = (b - A x) lambda^T - (A lambda) x^T on A's
 * pattern (dense: m*ld array, CSR: nnz array). Null outputs are skipped.   */
int orc_backward(orc_state *st, const double *b, const double *x, const double *gx,
                 double tol, int64_t max_iter, int64_t fixed_iters, int32_t max_replace,
                 double *lambda, double *grad_b, double *grad_A, orc_info *info);

#ifdef __cplusplus
}
#endif
#endif
