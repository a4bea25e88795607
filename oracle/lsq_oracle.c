/*
 * CPU oracle (float64, sequential) for the row-sampling preconditioned
 * least-squares solver of Chen & Wu (arXiv:1806.02968).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the GPU library. It shares no source
 * with the GPU path.
 *
 * Plain loops in the order the paper states the method. The only numerical
 * refinements over a naive transcription are compensated (Neumaier) sums for
 * the column norms and row weights and a double-double running sum for the
 * sampling CDF, so that the oracle's own rounding stays well inside the
 * CDF-boundary tie band used when comparing drawn indices.
 */
#include "lsq_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): 10 rounds of two 64x64->128 multiplies with    */
/* a Weyl-sequence key schedule.                                             */

#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL
#define PHILOX_W1 0xBB67AE8584CAA73BULL

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(PHILOX_M0, x0, &hi0, &lo0);
    mulhilo64(PHILOX_M1, x2, &hi1, &lo1);
    uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

double orc_uniform(uint64_t seed, int64_t t) {
  uint64_t ctr[4] = {(uint64_t)t >> 2, 0, 0, 0};
  uint64_t key[2] = {seed, 0};
  uint64_t out[4];
  orc_philox4x64_10(ctr, key, out);
  return (double)(out[t & 3] >> 11) * 0x1.0p-53;
}

/* ------------------------------------------------------------------------ */
/* matrix access                                                            */

static double dense_at(const orc_matrix *A, int64_t i, int64_t j) {
  if (A->dtype == 0) return ((const double *)A->values)[i * A->ld + j];
  return (double)((const float *)A->values)[i * A->ld + j];
}

static double csr_val(const orc_matrix *A, int64_t k) {
  if (A->dtype == 0) return ((const double *)A->values)[k];
  return (double)((const float *)A->values)[k];
}

/* a_ij of a CSR matrix (0 when not stored); binary search within row i */
static double csr_at(const orc_matrix *A, int64_t i, int64_t j) {
  int64_t lo = A->row_ptr[i], hi = A->row_ptr[i + 1];
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (A->col_idx[mid] < j) lo = mid + 1; else hi = mid;
  }
  if (lo < A->row_ptr[i + 1] && A->col_idx[lo] == j) return csr_val(A, lo);
  return 0.0;
}

static double mat_at(const orc_matrix *A, int64_t i, int64_t j) {
  return A->fmt == 0 ? dense_at(A, i, j) : csr_at(A, i, j);
}

/* Neumaier compensated summation state */
typedef struct { double s, c; } ksum;
static void ksum_add(ksum *k, double x) {
  double t = k->s + x;
  if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x; else k->c += (x - t) + k->s;
  k->s = t;
}
static double ksum_get(const ksum *k) { return k->s + k->c; }

/* ------------------------------------------------------------------------ */
/* Algorithm 2 step 1: D_jj = ||a^j||_2                                     */

int orc_column_norms(const orc_matrix *A, double *D) {
  int64_t m = A->m, n = A->n;
  ksum *acc = (ksum *)calloc((size_t)n, sizeof(ksum));
  if (A->fmt == 0) {
    for (int64_t i = 0; i < m; ++i)
      for (int64_t j = 0; j < n; ++j) {
        double a = dense_at(A, i, j);
        ksum_add(&acc[j], a * a);
      }
  } else {
    for (int64_t i = 0; i < m; ++i)
      for (int64_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k) {
        double a = csr_val(A, k);
        ksum_add(&acc[A->col_idx[k]], a * a);
      }
  }
  int status = 0;
  for (int64_t j = 0; j < n; ++j) {
    D[j] = sqrt(ksum_get(&acc[j]));
    if (!isfinite(D[j])) status = -3;
    else if (D[j] == 0.0 && status == 0) status = -2;
  }
  free(acc);
  return status;
}

/* Eq. (R2P) numerator on the normalised matrix: w_i = ||a_i D^{-1}||^2    */
void orc_row_weights(const orc_matrix *A, const double *invD, double *w) {
  for (int64_t i = 0; i < A->m; ++i) {
    ksum k = {0.0, 0.0};
    if (A->fmt == 0) {
      for (int64_t j = 0; j < A->n; ++j) {
        double a = dense_at(A, i, j) * invD[j];
        ksum_add(&k, a * a);
      }
    } else {
      for (int64_t q = A->row_ptr[i]; q < A->row_ptr[i + 1]; ++q) {
        double a = csr_val(A, q) * invD[A->col_idx[q]];
        ksum_add(&k, a * a);
      }
    }
    w[i] = ksum_get(&k);
  }
}

/* Algorithm 2 step 2: s = C n log n, natural log, rounded up, at least n  */
int64_t orc_sample_size(double C, int64_t n) {
  if (n <= 1) return 1;
  double v = ceil(C * (double)n * log((double)n));
  int64_t s = (int64_t)v;
  return s < n ? n : s;
}

/* inclusive CDF of the (unnormalised) density, double-double running sum */
double orc_cdf(int64_t m, const double *w, double *cdf) {
  double hi = 0.0, lo = 0.0, prev = 0.0;
  for (int64_t k = 0; k < m; ++k) {
    double s = hi + w[k];
    double bb = s - hi;
    double err = (hi - (s - bb)) + (w[k] - bb);
    lo += err;
    hi = s + lo;
    lo = lo - (hi - s);
    double c = hi + lo;
    if (c < prev) c = prev;
    cdf[k] = c;
    prev = c;
  }
  return m > 0 ? cdf[m - 1] : 0.0;
}

/* Algorithm 1, one trial: Pr{i = k} = p_k realised as the first index whose
 * CDF value exceeds tau = u W. Rows of zero weight have p_k = 0 and are
 * never returned.                                                          */
int64_t orc_draw(int64_t m, const double *w, const double *cdf, double tau, double *gap) {
  int64_t lo = 0, hi = m;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (cdf[mid] > tau) hi = mid; else lo = mid + 1;
  }
  int64_t i = lo;
  int adjusted = 0;
  if (i == m) { /* tau at or past the total: last row of positive weight */
    i = m - 1;
    while (i > 0 && !(w[i] > 0.0)) --i;
    adjusted = 1;
  } else if (!(w[i] > 0.0)) {
    int64_t k = i;
    while (k < m && !(w[k] > 0.0)) ++k;
    if (k == m) { k = i; while (k > 0 && !(w[k] > 0.0)) --k; }
    i = k;
    adjusted = 1;
  }
  double W = cdf[m - 1];
  if (adjusted) {
    *gap = 0.0;
  } else {
    double below = i > 0 ? cdf[i - 1] : 0.0;
    double g1 = tau - below, g2 = cdf[i] - tau;
    *gap = (g1 < g2 ? g1 : g2) / W;
  }
  return i;
}

/* ------------------------------------------------------------------------ */
/* state                                                                    */

struct orc_state {
  orc_matrix A;
  int64_t m, n, s;
  int32_t sweeps;
  double *D, *invD, *w, W;
  int64_t *idx;
  double *gap;
  double *coef; /* W / (s w_{i_t}) = 1 / (s p_{i_t}) */
  int64_t ties, diag_fixes;
  int32_t have_gram;
  /* M: dense n*n, or CSR */
  double *Md;
  int64_t *Mrp;
  int32_t *Mci;
  double *Mv;
  int64_t *Mdiag; /* CSR position of each diagonal entry */
  orc_info last;
};

int64_t orc_n(const orc_state *st) { return st->n; }
int64_t orc_s(const orc_state *st) { return st->s; }
void orc_get_D(const orc_state *st, double *D) { memcpy(D, st->D, (size_t)st->n * sizeof(double)); }
void orc_get_w(const orc_state *st, double *w) { memcpy(w, st->w, (size_t)st->m * sizeof(double)); }
void orc_get_samples(const orc_state *st, int64_t *idx, double *gap) {
  if (idx) memcpy(idx, st->idx, (size_t)st->s * sizeof(int64_t));
  if (gap) memcpy(gap, st->gap, (size_t)st->s * sizeof(double));
}
void orc_get_info(const orc_state *st, orc_info *info) { *info = st->last; }

void orc_free(orc_state *st) {
  if (!st) return;
  free(st->D); free(st->invD); free(st->w); free(st->idx); free(st->gap); free(st->coef);
  free(st->Md); free(st->Mrp); free(st->Mci); free(st->Mv); free(st->Mdiag);
  free(st);
}

/* row i of the normalised matrix, dense scratch of length n */
static void normalised_row_dense(const orc_state *st, int64_t i, double *out) {
  for (int64_t j = 0; j < st->n; ++j) out[j] = dense_at(&st->A, i, j) * st->invD[j];
}

/* Section 3.3: M = A_s^T A_s = sum_t (1/(s p_{i_t})) a_{i_t}^T a_{i_t}, the
 * rows already normalised (Algorithm 2 step 3 uses the normalised A).     */
static void gram_dense(orc_state *st) {
  int64_t n = st->n;
  st->Md = (double *)calloc((size_t)(n * n), sizeof(double));
  double *row = (double *)malloc((size_t)n * sizeof(double));
  for (int64_t t = 0; t < st->s; ++t) {
    normalised_row_dense(st, st->idx[t], row);
    double c = st->coef[t];
    for (int64_t j = 0; j < n; ++j)
      for (int64_t l = j; l < n; ++l) st->Md[j * n + l] += c * (row[j] * row[l]);
  }
  for (int64_t j = 0; j < n; ++j)
    for (int64_t l = j + 1; l < n; ++l) st->Md[l * n + j] = st->Md[j * n + l];
  for (int64_t j = 0; j < n; ++j)
    if (st->Md[j * n + j] == 0.0) { st->Md[j * n + j] = 1.0; st->diag_fixes++; }
  free(row);
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* same sum for a CSR matrix; row j of M collects, over the draws t (in
 * increasing t) whose row has an entry in column j, coef_t * a_j * a_l.  */
static void gram_csr(orc_state *st) {
  const orc_matrix *A = &st->A;
  int64_t n = st->n, s = st->s;
  /* column -> list of (draw t, position k of column j in row i_t) */
  int64_t *cnt = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
  for (int64_t t = 0; t < s; ++t) {
    int64_t i = st->idx[t];
    for (int64_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k) cnt[A->col_idx[k] + 1]++;
  }
  for (int64_t j = 0; j < n; ++j) cnt[j + 1] += cnt[j];
  int64_t tot = cnt[n];
  int64_t *lt = (int64_t *)malloc((size_t)(tot > 0 ? tot : 1) * sizeof(int64_t));
  int64_t *lk = (int64_t *)malloc((size_t)(tot > 0 ? tot : 1) * sizeof(int64_t));
  int64_t *fill = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  memcpy(fill, cnt, (size_t)n * sizeof(int64_t));
  for (int64_t t = 0; t < s; ++t) {
    int64_t i = st->idx[t];
    for (int64_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k) {
      int64_t j = A->col_idx[k];
      lt[fill[j]] = t;
      lk[fill[j]] = k;
      fill[j]++;
    }
  }
  double *acc = (double *)calloc((size_t)n, sizeof(double));
  char *mark = (char *)calloc((size_t)n, 1);
  int32_t *touched = (int32_t *)malloc((size_t)(n + 1) * sizeof(int32_t));
  int64_t cap = 1024, nnz = 0;
  st->Mrp = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
  st->Mci = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
  st->Mv = (double *)malloc((size_t)cap * sizeof(double));
  st->Mdiag = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  st->Mrp[0] = 0;
  for (int64_t j = 0; j < n; ++j) {
    int64_t nt = 0;
    for (int64_t e = cnt[j]; e < cnt[j + 1]; ++e) {
      int64_t t = lt[e], i = st->idx[t];
      double aj = csr_val(A, lk[e]) * st->invD[j];
      double c = st->coef[t];
      for (int64_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k) {
        int32_t l = A->col_idx[k];
        double al = csr_val(A, k) * st->invD[l];
        acc[l] += c * (aj * al);
        if (!mark[l]) { mark[l] = 1; touched[nt++] = l; }
      }
    }
    if (!mark[j]) { /* column j never drawn: empty row; diagonal guard below */
      mark[j] = 1; touched[nt++] = (int32_t)j; acc[j] = 0.0;
    }
    qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
    if (nnz + nt > cap) {
      while (nnz + nt > cap) cap *= 2;
      st->Mci = (int32_t *)realloc(st->Mci, (size_t)cap * sizeof(int32_t));
      st->Mv = (double *)realloc(st->Mv, (size_t)cap * sizeof(double));
    }
    for (int64_t q = 0; q < nt; ++q) {
      int32_t l = touched[q];
      double v = acc[l];
      if (l == j) {
        st->Mdiag[j] = nnz;
        if (v == 0.0) { v = 1.0; st->diag_fixes++; }
      }
      st->Mci[nnz] = l;
      st->Mv[nnz] = v;
      nnz++;
      acc[l] = 0.0;
      mark[l] = 0;
    }
    st->Mrp[j + 1] = nnz;
  }
  free(cnt); free(lt); free(lk); free(fill); free(acc); free(mark); free(touched);
}

orc_state *orc_setup(const orc_matrix *A, double C, int32_t sweeps, uint64_t seed, double tie_eps,
                     const int64_t *idx_override, int64_t s_override, int32_t *status) {
  *status = 0;
  if (A->m < 1 || A->n < 1 || A->m < A->n || sweeps < 0 || !(C > 0.0)) { *status = -1; return NULL; }
  orc_state *st = (orc_state *)calloc(1, sizeof(orc_state));
  st->A = *A;
  st->m = A->m;
  st->n = A->n;
  st->sweeps = sweeps;
  int64_t m = st->m, n = st->n;
  st->D = (double *)malloc((size_t)n * sizeof(double));
  st->invD = (double *)malloc((size_t)n * sizeof(double));
  st->w = (double *)malloc((size_t)m * sizeof(double));

  /* Algorithm 2 step 1 */
  int rc = orc_column_norms(A, st->D);
  if (rc != 0) { *status = rc; orc_free(st); return NULL; }
  for (int64_t j = 0; j < n; ++j) st->invD[j] = 1.0 / st->D[j];

  /* Eq. (R2P) on the normalised rows */
  orc_row_weights(A, st->invD, st->w);
  for (int64_t i = 0; i < m; ++i)
    if (!isfinite(st->w[i])) { *status = -3; orc_free(st); return NULL; }
  double *cdf = (double *)malloc((size_t)m * sizeof(double));
  st->W = orc_cdf(m, st->w, cdf);

  /* Algorithm 2 step 2 with Algorithm 1 */
  st->s = idx_override ? s_override : orc_sample_size(C, n);
  st->idx = (int64_t *)malloc((size_t)st->s * sizeof(int64_t));
  st->gap = (double *)malloc((size_t)st->s * sizeof(double));
  st->coef = (double *)malloc((size_t)st->s * sizeof(double));
  for (int64_t t = 0; t < st->s; ++t) {
    if (idx_override) {
      st->idx[t] = idx_override[t];
      st->gap[t] = 1.0;
      if (st->idx[t] < 0 || st->idx[t] >= m || !(st->w[st->idx[t]] > 0.0)) {
        *status = -1; free(cdf); orc_free(st); return NULL;
      }
    } else {
      double tau = orc_uniform(seed, t) * st->W;
      st->idx[t] = orc_draw(m, st->w, cdf, tau, &st->gap[t]);
      if (st->gap[t] <= tie_eps) st->ties++;
    }
    /* S_{t,i_t} = 1/sqrt(s p_{i_t}), so each draw enters M with 1/(s p) */
    st->coef[t] = st->W / ((double)st->s * st->w[st->idx[t]]);
  }
  free(cdf);

  /* Algorithm 2 step 3 (Section 3.3) */
  if (A->fmt == 0) gram_dense(st); else gram_csr(st);
  st->have_gram = 1;
  st->last.s = st->s;
  st->last.ties = st->ties;
  st->last.diag_fixes = st->diag_fixes;
  st->last.W = st->W;
  st->last.nnz_M = A->fmt == 0 ? n * n : st->Mrp[n];
  return st;
}

void orc_get_M_dense(const orc_state *st, double *M) {
  int64_t n = st->n;
  if (st->A.fmt == 0) { memcpy(M, st->Md, (size_t)(n * n) * sizeof(double)); return; }
  memset(M, 0, (size_t)(n * n) * sizeof(double));
  for (int64_t j = 0; j < n; ++j)
    for (int64_t q = st->Mrp[j]; q < st->Mrp[j + 1]; ++q) M[j * n + st->Mci[q]] = st->Mv[q];
}

int64_t orc_M_nnz(const orc_state *st) { return st->A.fmt == 0 ? st->n * st->n : st->Mrp[st->n]; }

void orc_get_M_csr(const orc_state *st, int64_t *rp, int32_t *ci, double *v) {
  int64_t n = st->n;
  if (st->A.fmt == 0) {
    for (int64_t j = 0; j <= n; ++j) rp[j] = j * n;
    for (int64_t j = 0; j < n; ++j)
      for (int64_t l = 0; l < n; ++l) { ci[j * n + l] = (int32_t)l; v[j * n + l] = st->Md[j * n + l]; }
    return;
  }
  memcpy(rp, st->Mrp, (size_t)(n + 1) * sizeof(int64_t));
  memcpy(ci, st->Mci, (size_t)st->Mrp[n] * sizeof(int32_t));
  memcpy(v, st->Mv, (size_t)st->Mrp[n] * sizeof(double));
}

double orc_M_entry(const orc_state *st, int64_t j, int64_t l) {
  double acc = 0.0;
  for (int64_t t = 0; t < st->s; ++t) {
    int64_t i = st->idx[t];
    double aj = mat_at(&st->A, i, j), al = mat_at(&st->A, i, l);
    if (aj == 0.0 || al == 0.0) continue;
    acc += st->coef[t] * ((aj * st->invD[j]) * (al * st->invD[l]));
  }
  return acc;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 3                                                               */

/* res = r - M e */
static void residual_M(const orc_state *st, const double *r, const double *e, double *res) {
  int64_t n = st->n;
  for (int64_t j = 0; j < n; ++j) {
    double acc = 0.0;
    if (st->A.fmt == 0) {
      for (int64_t l = 0; l < n; ++l) acc += st->Md[j * n + l] * e[l];
    } else {
      for (int64_t q = st->Mrp[j]; q < st->Mrp[j + 1]; ++q) acc += st->Mv[q] * e[st->Mci[q]];
    }
    res[j] = r[j] - acc;
  }
}

/* solve B d = res, B the lower triangular part of M including the diagonal */
static void solve_lower(const orc_state *st, const double *res, double *d) {
  int64_t n = st->n;
  for (int64_t j = 0; j < n; ++j) {
    double acc = res[j], diag;
    if (st->A.fmt == 0) {
      for (int64_t l = 0; l < j; ++l) acc -= st->Md[j * n + l] * d[l];
      diag = st->Md[j * n + j];
    } else {
      for (int64_t q = st->Mrp[j]; q < st->Mdiag[j]; ++q) acc -= st->Mv[q] * d[st->Mci[q]];
      diag = st->Mv[st->Mdiag[j]];
    }
    d[j] = acc / diag;
  }
}

/* solve B^T d = res, B^T the upper triangular part of M including the diagonal */
static void solve_upper(const orc_state *st, const double *res, double *d) {
  int64_t n = st->n;
  for (int64_t j = n - 1; j >= 0; --j) {
    double acc = res[j], diag;
    if (st->A.fmt == 0) {
      for (int64_t l = j + 1; l < n; ++l) acc -= st->Md[j * n + l] * d[l];
      diag = st->Md[j * n + j];
    } else {
      for (int64_t q = st->Mdiag[j] + 1; q < st->Mrp[j + 1]; ++q) acc -= st->Mv[q] * d[st->Mci[q]];
      diag = st->Mv[st->Mdiag[j]];
    }
    d[j] = acc / diag;
  }
}

void orc_apply_P(const orc_state *st, const double *r, double *z) {
  int64_t n = st->n;
  double *e = (double *)calloc((size_t)n, sizeof(double));
  double *res = (double *)malloc((size_t)n * sizeof(double));
  double *d = (double *)malloc((size_t)n * sizeof(double));
  if (st->sweeps == 0) {
    memcpy(z, r, (size_t)n * sizeof(double));
  } else {
    for (int32_t it = 0; it < st->sweeps; ++it) { /* e <- e + B^{-1}(r - M e) */
      residual_M(st, r, e, res);
      solve_lower(st, res, d);
      for (int64_t j = 0; j < n; ++j) e[j] += d[j];
    }
    for (int32_t it = 0; it < st->sweeps; ++it) { /* e <- e + B^{-T}(r - M e) */
      residual_M(st, r, e, res);
      solve_upper(st, res, d);
      for (int64_t j = 0; j < n; ++j) e[j] += d[j];
    }
    memcpy(z, e, (size_t)n * sizeof(double));
  }
  free(e); free(res); free(d);
}

/* ------------------------------------------------------------------------ */
/* products with A                                                          */

static void mul_A(const orc_matrix *A, const double *x, double *y) { /* y = A x */
  for (int64_t i = 0; i < A->m; ++i) {
    double acc = 0.0;
    if (A->fmt == 0) {
      for (int64_t j = 0; j < A->n; ++j) acc += dense_at(A, i, j) * x[j];
    } else {
      for (int64_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k) acc += csr_val(A, k) * x[A->col_idx[k]];
    }
    y[i] = acc;
  }
}

static void mul_At(const orc_matrix *A, const double *y, double *x) { /* x = A^T y */
  memset(x, 0, (size_t)A->n * sizeof(double));
  for (int64_t i = 0; i < A->m; ++i) {
    if (A->fmt == 0) {
      for (int64_t j = 0; j < A->n; ++j) x[j] += dense_at(A, i, j) * y[i];
    } else {
      for (int64_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k) x[A->col_idx[k]] += csr_val(A, k) * y[i];
    }
  }
}

void orc_apply_K(const orc_state *st, const double *p, double *q) {
  int64_t n = st->n;
  double *u = (double *)calloc((size_t)n, sizeof(double));
  double *v = (double *)calloc((size_t)st->m, sizeof(double));
  for (int64_t j = 0; j < n; ++j) u[j] = st->invD[j] * p[j];
  mul_A(&st->A, u, v);
  mul_At(&st->A, v, q);
  for (int64_t j = 0; j < n; ++j) q[j] *= st->invD[j];
  free(u); free(v);
}

static double dot(int64_t n, const double *a, const double *b) {
  double s = 0.0;
  for (int64_t j = 0; j < n; ++j) s += a[j] * b[j];
  return s;
}

static double scaled_norm(int64_t n, const double *D, const double *r) { /* ||D r|| */
  double s = 0.0;
  for (int64_t j = 0; j < n; ++j) { double v = D[j] * r[j]; s += v * v; }
  return sqrt(s);
}

/* true residual of the normal equation in original scaling:
 * forward (b != NULL): g = A^T (b - A x); adjoint: g = gx - A^T (A x)      */
static void true_residual(const orc_state *st, const double *b, const double *gx, const double *x,
                          double *g) {
  int64_t m = st->m, n = st->n;
  double *v = (double *)malloc((size_t)m * sizeof(double));
  mul_A(&st->A, x, v);
  if (b) {
    for (int64_t i = 0; i < m; ++i) v[i] = b[i] - v[i];
    mul_At(&st->A, v, g);
  } else {
    mul_At(&st->A, v, g);
    for (int64_t j = 0; j < n; ++j) g[j] = gx[j] - g[j];
  }
  free(v);
}

static double norm2(int64_t n, const double *v) { return sqrt(dot(n, v, v)); }

/* Algorithm 2 step 4: preconditioned CG on K y = f, K = D^{-1} A^T A D^{-1},
 * f = D^{-1} g0, x = D^{-1} y; the stopping test uses the original scaling
 * ||D r|| / ||g0||, i.e. ||A^T(b - A x)|| / ||A^T b|| for the forward solve. */
static int pcg(orc_state *st, const double *b, const double *gx, const double *g0, double tol,
               int64_t max_iter, int64_t fixed_iters, int32_t max_replace, double *x, orc_info *info) {
  int64_t n = st->n;
  double *y = (double *)calloc((size_t)n, sizeof(double));
  double *r = (double *)malloc((size_t)n * sizeof(double));
  double *z = (double *)malloc((size_t)n * sizeof(double));
  double *p = (double *)calloc((size_t)n, sizeof(double));
  double *q = (double *)malloc((size_t)n * sizeof(double));
  double *g = (double *)malloc((size_t)n * sizeof(double));
  if (max_iter <= 0) max_iter = 10 * n < 100000 ? 10 * n : 100000;
  for (int64_t j = 0; j < n; ++j) r[j] = st->invD[j] * g0[j];
  double nf = norm2(n, g0);
  int64_t k = 0, repl = 0;
  int restart = 1, status = 0, have_true = 0;
  double rho = 0.0, rel_true = 0.0;
  double rel = nf > 0.0 ? scaled_norm(n, st->D, r) / nf : 0.0;
  if (nf == 0.0) { /* zero right-hand side: the solution is 0 */
    max_iter = 0;
    fixed_iters = -1;
  }
  for (;;) {
    if (fixed_iters >= 0) {
      if (k >= fixed_iters) break;
    } else if (rel <= tol) {
      for (int64_t j = 0; j < n; ++j) x[j] = st->invD[j] * y[j];
      if (nf > 0.0) {
        true_residual(st, b, gx, x, g);
        rel_true = norm2(n, g) / nf;
      }
      have_true = 1;
      if (rel_true <= tol || repl >= max_replace || k >= max_iter) break;
      /* residual replacement: continue from the true residual */
      for (int64_t j = 0; j < n; ++j) r[j] = st->invD[j] * g[j];
      rel = rel_true;
      repl++;
      restart = 1;
      have_true = 0;
      continue;
    }
    if (k >= max_iter) break;
    have_true = 0;
    orc_apply_P(st, r, z);
    double rho_new = dot(n, r, z);
    if (restart) {
      memcpy(p, z, (size_t)n * sizeof(double));
      restart = 0;
    } else {
      double beta = rho_new / rho;
      for (int64_t j = 0; j < n; ++j) p[j] = z[j] + beta * p[j];
    }
    rho = rho_new;
    orc_apply_K(st, p, q);
    double pq = dot(n, p, q);
    if (!(pq > 0.0) || !(rho > 0.0)) { status = -6; break; }
    double alpha = rho / pq;
    for (int64_t j = 0; j < n; ++j) { y[j] += alpha * p[j]; r[j] -= alpha * q[j]; }
    k++;
    rel = scaled_norm(n, st->D, r) / nf;
  }
  for (int64_t j = 0; j < n; ++j) x[j] = st->invD[j] * y[j];
  if (!have_true) {
    if (nf > 0.0) {
      true_residual(st, b, gx, x, g);
      rel_true = norm2(n, g) / nf;
    } else {
      rel_true = 0.0;
    }
  }
  if (status == 0 && fixed_iters < 0 && !(rel_true <= tol)) status = 1;
  info->iters = k;
  info->replacements = repl;
  info->relres = rel;
  info->relres_true = rel_true;
  info->status = status;
  free(y); free(r); free(z); free(p); free(q); free(g);
  return status;
}

int orc_solve(orc_state *st, const double *b, double tol, int64_t max_iter, int64_t fixed_iters,
              int32_t max_replace, double *x, orc_info *info) {
  double *g0 = (double *)malloc((size_t)st->n * sizeof(double));
  mul_At(&st->A, b, g0); /* A^T b */
  orc_info inf = st->last;
  int rc = pcg(st, b, NULL, g0, tol, max_iter, fixed_iters, max_replace, x, &inf);
  st->last = inf;
  if (info) *info = inf;
  free(g0);
  return rc;
}

int orc_backward(orc_state *st, const double *b, const double *x, const double *gx, double tol,
                 int64_t max_iter, int64_t fixed_iters, int32_t max_replace, double *lambda,
                 double *grad_b, double *grad_A, orc_info *info) {
  int64_t m = st->m, n = st->n;
  orc_info inf = st->last;
  /* adjoint normal equation A^T A lambda = gx with the same preconditioner */
  int rc = pcg(st, NULL, gx, gx, tol, max_iter, fixed_iters, max_replace, lambda, &inf);
  double *v = (double *)malloc((size_t)m * sizeof(double));
  double *res = (double *)malloc((size_t)m * sizeof(double));
  mul_A(&st->A, lambda, v); /* A lambda */
  mul_A(&st->A, x, res);
  for (int64_t i = 0; i < m; ++i) res[i] = b[i] - res[i]; /* b - A x */
  if (grad_b) memcpy(grad_b, v, (size_t)m * sizeof(double));
  if (grad_A) {
    if (st->A.fmt == 0) {
      for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) grad_A[i * st->A.ld + j] = res[i] * lambda[j] - v[i] * x[j];
    } else {
      for (int64_t i = 0; i < m; ++i)
        for (int64_t k = st->A.row_ptr[i]; k < st->A.row_ptr[i + 1]; ++k) {
          int32_t j = st->A.col_idx[k];
          grad_A[k] = res[i] * lambda[j] - v[i] * x[j];
        }
    }
  }
  free(v); free(res);
  if (info) *info = inf;
  return rc;
}
