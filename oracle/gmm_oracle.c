/*
 * gmm_oracle.c -- plain FP64 CPU oracle for Gaussian-mixture training
 * (k-means seeding + EM), written from Sanderson & Curtin,
 * "An Open Source C++ Implementation of Multi-Threaded Gaussian Mixture
 * Models, k-Means and Expectation Maximisation" (arXiv:1707.09094).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or constant with the
 * GPU path.
 *
 * What it computes is the plain definition of each step, in double precision,
 * one definition per loop, no tiling, no algebraic expansion:
 *   - E-step: log-domain Gaussian (Sec. 2.2, Eq. 15), log-sum-exp of the
 *     weighted log-densities (Sec. 2.2, Eqs. 16-18; max-shifted form, same
 *     value as the paper's pairwise log-add), responsibilities (Sec. 2, Eq. 3).
 *   - M-step: Eqs. 4-7 of Sec. 2 directly, with the covariance two-pass and
 *     centred on the NEW mean (Eq. 7; Appendix A summary), followed by the
 *     diagonal variance floor (end of Sec. 2.2).
 *   - k-means: Lloyd iteration as hard-assignment EM (Sec. 3, Eq. 19) with
 *     squared Euclidean or global-diagonal Mahalanobis distance (Sec. 3.1,
 *     Eq. 20) and dead-mean resurrection (end of Sec. 3.1).
 *
 * Threading: OpenMP is used only where the work items are independent and no
 * sum changes order -- the per-sample E-step/assignment rows, and one thread
 * per (component) for the M-step sums, each of which is still a plain
 * sequential loop over samples i = 0..N-1.  Results are therefore bit-identical
 * for any thread count.
 *
 * Data layout (Sec. 4 API: one sample per column): X is D x N column-major,
 * sample i at X + i*ldx, float32 (oracle_*) or float64 (oracle_*_f64, the
 * gmm_diag precision); float32 samples are promoted exactly to double.
 * Parameters are double: hefts[G], means[g*D + d], dcovs[g*D + d] (diagonal),
 * covs[g*D*D + e*D + d] (full, column-major per component).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define LOG_2PI 1.8378770664093454835606594728112353 /* log(2*pi) */

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_NOTPD = 2, ORC_NONFINITE = 1 };

static int g_threads = 0; /* 0 = OpenMP default */

void oracle_set_threads(int n) { g_threads = n; }

int oracle_get_threads(void) {
#ifdef _OPENMP
  return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
  return 1;
#endif
}

#ifdef _OPENMP
#define NTHR (g_threads > 0 ? g_threads : omp_get_max_threads())
#endif

/* Samples are FP32 (the fgmm_diag precision, Sec. 4) or FP64 (gmm_diag, and
 * the precision of the speed-up experiment, Sec. 5.1).  FP32 values are
 * promoted exactly to double where they are read, so every computation below
 * is the same FP64 arithmetic for both, and FP32 data given as FP64 gives
 * bit-identical results. */
typedef struct {
  const float* f;  /* FP32 samples, or NULL */
  const double* d; /* FP64 samples when f is NULL */
  int64_t ldx;
} samples_t;

static inline double xval(const samples_t* S, int64_t i, int d) {
  return S->f ? (double)S->f[i * S->ldx + d] : S->d[i * S->ldx + d];
}

/* ------------------------------------------------------------------------ */
/* Gaussian log-density, Sec. 2.2 Eq. 15.                                    */
/* ------------------------------------------------------------------------ */

/* Diagonal covariance: log|Sigma| = sum log sigma2_d and Sigma^-1 = 1/sigma2_d
 * (Sec. 4, items (i) and (ii)). */
static double log_det_diag(const double* s2, int D) {
  double logdet = 0.0;
  for (int d = 0; d < D; ++d) logdet += log(s2[d]);
  return logdet;
}

static double log_gauss_diag(const samples_t* S, int64_t i, const double* mu, const double* s2,
                             double logdet, int D) {
  double maha = 0.0;
  if (S->f) {
    const float* x = S->f + i * S->ldx;
    for (int d = 0; d < D; ++d) {
      double t = (double)x[d] - mu[d];
      maha += t * t / s2[d];
    }
  } else {
    const double* x = S->d + i * S->ldx;
    for (int d = 0; d < D; ++d) {
      double t = x[d] - mu[d];
      maha += t * t / s2[d];
    }
  }
  return -0.5 * ((double)D * LOG_2PI + logdet) - 0.5 * maha;
}

/* Textbook Cholesky Sigma = L L^T (lower, column-major, L[e*D + d] = L_{d,e}).
 * Returns 0 on success, ORC_NOTPD if a pivot is not positive. */
static int cholesky(const double* S, double* L, int D) {
  memset(L, 0, sizeof(double) * (size_t)D * D);
  for (int j = 0; j < D; ++j) {
    double s = S[j * D + j];
    for (int k = 0; k < j; ++k) s -= L[k * D + j] * L[k * D + j];
    if (!(s > 0.0)) return ORC_NOTPD;
    double ljj = sqrt(s);
    L[j * D + j] = ljj;
    for (int i = j + 1; i < D; ++i) {
      double t = S[j * D + i];
      for (int k = 0; k < j; ++k) t -= L[k * D + i] * L[k * D + j];
      L[j * D + i] = t / ljj;
    }
  }
  return 0;
}

/* Full covariance Eq. 15 with log|Sigma| = 2 sum log L_dd and the Mahalanobis
 * term as ||z||^2, L z = x - mu (forward substitution). */
static double log_gauss_full(const samples_t* S, int64_t i, const double* mu, const double* L,
                             double logdet, int D, double* z) {
  double maha = 0.0;
  for (int d = 0; d < D; ++d) {
    double t = xval(S, i, d) - mu[d];
    for (int k = 0; k < d; ++k) t -= L[k * D + d] * z[k];
    z[d] = t / L[d * D + d];
    maha += z[d] * z[d];
  }
  return -0.5 * ((double)D * LOG_2PI + logdet) - 0.5 * maha;
}

/* log sum_g exp(a_g), max-shifted (Sec. 2.2, Eqs. 16-18). */
static double log_sum_exp(const double* a, int G) {
  double m = -INFINITY;
  for (int g = 0; g < G; ++g)
    if (a[g] > m) m = a[g];
  if (m == -INFINITY) return -INFINITY;
  if (!isfinite(m)) return m;
  double s = 0.0;
  for (int g = 0; g < G; ++g) s += exp(a[g] - m);
  return m + log(s);
}

/* ------------------------------------------------------------------------ */
/* E-step: a[i*G+g] = log w_g + log N(x_i | g), lse[i] = log p(x_i | lambda). */
/* ------------------------------------------------------------------------ */

static int estep_diag(const samples_t* S, int64_t N, int D, int G, const double* hefts,
                      const double* means, const double* dcovs, double* a, double* lse) {
  double* logdet = (double*)malloc(sizeof(double) * G);
  if (!logdet) return ORC_ENOMEM;
  for (int g = 0; g < G; ++g) logdet[g] = log_det_diag(dcovs + (size_t)g * D, D);
#pragma omp parallel for schedule(static) num_threads(NTHR)
  for (int64_t i = 0; i < N; ++i) {
    double* ai = a + i * G;
    for (int g = 0; g < G; ++g)
      ai[g] = log(hefts[g]) + log_gauss_diag(S, i, means + (size_t)g * D,
                                             dcovs + (size_t)g * D, logdet[g], D);
    lse[i] = log_sum_exp(ai, G);
  }
  free(logdet);
  return 0;
}

static int estep_full(const samples_t* S, int64_t N, int D, int G, const double* hefts,
                      const double* means, const double* covs, double* a, double* lse) {
  size_t DD = (size_t)D * D;
  double* L = (double*)malloc(sizeof(double) * DD * G);
  double* logdet = (double*)malloc(sizeof(double) * G);
  if (!L || !logdet) {
    free(L);
    free(logdet);
    return ORC_ENOMEM;
  }
  int rc = 0;
  for (int g = 0; g < G && rc == 0; ++g) {
    rc = cholesky(covs + DD * g, L + DD * g, D);
    if (rc == 0) {
      double s = 0.0;
      for (int d = 0; d < D; ++d) s += log(L[DD * g + (size_t)d * D + d]);
      logdet[g] = 2.0 * s;
    }
  }
  if (rc == 0) {
#pragma omp parallel num_threads(NTHR)
    {
      double* z = (double*)malloc(sizeof(double) * D);
#pragma omp for schedule(static)
      for (int64_t i = 0; i < N; ++i) {
        double* ai = a + i * G;
        for (int g = 0; g < G; ++g)
          ai[g] = log(hefts[g]) + log_gauss_full(S, i, means + (size_t)g * D, L + DD * g,
                                                 logdet[g], D, z);
        lse[i] = log_sum_exp(ai, G);
      }
      free(z);
    }
  }
  free(L);
  free(logdet);
  return rc;
}

static double mean_of(const double* v, int64_t N) {
  double s = 0.0;
  for (int64_t i = 0; i < N; ++i) s += v[i];
  return s / (double)N;
}

/* ------------------------------------------------------------------------ */
/* Public: log-likelihood (Sec. 4 API: log_p(X) per sample, avg_log_p(X)).   */
/* ------------------------------------------------------------------------ */

static int loglik_s(const samples_t* S, int64_t N, int D, int G, int full,
                  const double* hefts, const double* means, const double* covs,
                  double* mean_loglik, double* per_sample /* N or NULL */) {
  if (N < 1 || D < 1 || G < 1 || S->ldx < D) return ORC_EINVAL;
  double* a = (double*)malloc(sizeof(double) * (size_t)N * G);
  double* lse = (double*)malloc(sizeof(double) * (size_t)N);
  if (!a || !lse) {
    free(a);
    free(lse);
    return ORC_ENOMEM;
  }
  int rc = full ? estep_full(S, N, D, G, hefts, means, covs, a, lse)
                : estep_diag(S, N, D, G, hefts, means, covs, a, lse);
  if (rc == 0) {
    *mean_loglik = mean_of(lse, N);
    if (per_sample) memcpy(per_sample, lse, sizeof(double) * (size_t)N);
    if (!isfinite(*mean_loglik)) rc = ORC_NONFINITE;
  }
  free(a);
  free(lse);
  return rc;
}

/* Per-Gaussian log-likelihood log N(x_i | g) without the weight
 * (Sec. 4 API: log_p(X, g)). */
static int log_p_g_s(const samples_t* S, int64_t N, int D, int G, const double* means,
                   const double* dcovs, int g, double* out /* N */) {
  if (N < 1 || D < 1 || G < 1 || S->ldx < D || g < 0 || g >= G) return ORC_EINVAL;
  double logdet = log_det_diag(dcovs + (size_t)g * D, D);
#pragma omp parallel for schedule(static) num_threads(NTHR)
  for (int64_t i = 0; i < N; ++i)
    out[i] = log_gauss_diag(S, i, means + (size_t)g * D, dcovs + (size_t)g * D, logdet, D);
  return 0;
}

/* Seeding of the initial means (Sec. 4 API seed modes static_spread /
 * random_spread: "a maximally spread subset of the training samples"), read as
 * farthest-first traversal.  The first seed is sample `first` (0 for
 * static_spread, a caller-drawn index for random_spread); seed k+1 is the
 * sample whose distance to its nearest already-chosen seed is largest, the
 * lowest index on ties.  Distance: sum_d lam_d (x_d - y_d)^2 with lam = NULL
 * meaning lam_d = 1 (Euclidean), each term lam_d * (u * u) added in order
 * d = 0..D-1.  idx_out[G] receives the chosen sample indices, means_out[G*D]
 * their coordinates. */
static int seed_spread_s(const samples_t* S, int64_t N, int D, int G, const double* lam,
                       int64_t first, int64_t* idx_out, double* means_out) {
  if (N < 1 || D < 1 || G < 1 || S->ldx < D || first < 0 || first >= N) return ORC_EINVAL;
  double* dmin = (double*)malloc(sizeof(double) * (size_t)N);
  if (!dmin) return ORC_ENOMEM;
  int64_t s = first;
  for (int k = 0; k < G; ++k) {
    idx_out[k] = s;
    for (int d = 0; d < D; ++d) means_out[(size_t)k * D + d] = xval(S, s, d);
    const double* y = means_out + (size_t)k * D;
#pragma omp parallel for schedule(static) num_threads(NTHR)
    for (int64_t i = 0; i < N; ++i) {
      double q = 0.0;
      for (int d = 0; d < D; ++d) {
        const double u = xval(S, i, d) - y[d];
        q += (lam ? lam[d] : 1.0) * (u * u);
      }
      dmin[i] = (k == 0 || q < dmin[i]) ? q : dmin[i];
    }
    double best = -1.0;
    int64_t bi = 0;
    for (int64_t i = 0; i < N; ++i)
      if (dmin[i] > best) {
        best = dmin[i];
        bi = i;
      }
    s = bi;
  }
  free(dmin);
  return 0;
}

/* Responsibilities l_{g,i} (Sec. 2, Eq. 3), exposed for tests: out[i*G+g]. */
static int responsibilities_s(const samples_t* S, int64_t N, int D, int G, int full,
                            const double* hefts, const double* means, const double* covs,
                            double* out) {
  if (N < 1 || D < 1 || G < 1 || S->ldx < D) return ORC_EINVAL;
  double* lse = (double*)malloc(sizeof(double) * (size_t)N);
  if (!lse) return ORC_ENOMEM;
  int rc = full ? estep_full(S, N, D, G, hefts, means, covs, out, lse)
                : estep_diag(S, N, D, G, hefts, means, covs, out, lse);
  if (rc == 0) {
#pragma omp parallel for schedule(static) num_threads(NTHR)
    for (int64_t i = 0; i < N; ++i)
      for (int g = 0; g < G; ++g) out[i * G + g] = exp(out[i * G + g] - lse[i]);
  }
  free(lse);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Public: one EM iteration (Sec. 2, Eqs. 3-7; variance floor, Sec. 2.2).     */
/*                                                                            */
/* Outputs the new parameters and the mean log-likelihood of the INPUT        */
/* parameters (the E-step by-product).  A component whose L_g is exactly 0   */
/* gets weight 0 and keeps its previous mean and covariance (the paper does  */
/* not say; any value maximises the Q-function then).  L_out (G, optional)    */
/* returns L_g.                                                               */
/* ------------------------------------------------------------------------ */

static int em_iter_s(const samples_t* S, int64_t N, int D, int G, int full,
                   const double* hefts, const double* means, const double* covs, double var_floor,
                   double* hefts_out, double* means_out, double* covs_out, double* mean_loglik,
                   double* L_out) {
  if (N < 1 || D < 1 || G < 1 || S->ldx < D) return ORC_EINVAL;
  size_t csz = full ? (size_t)D * D : (size_t)D;
  double* l = (double*)malloc(sizeof(double) * (size_t)N * G);
  double* lse = (double*)malloc(sizeof(double) * (size_t)N);
  if (!l || !lse) {
    free(l);
    free(lse);
    return ORC_ENOMEM;
  }
  int rc = full ? estep_full(S, N, D, G, hefts, means, covs, l, lse)
                : estep_diag(S, N, D, G, hefts, means, covs, l, lse);
  if (rc != 0) {
    free(l);
    free(lse);
    return rc;
  }
  *mean_loglik = mean_of(lse, N);

  /* Eq. 3: l_{g,i} = w_g N(x_i|g) / sum_k w_k N(x_i|k), in the log domain. */
#pragma omp parallel for schedule(static) num_threads(NTHR)
  for (int64_t i = 0; i < N; ++i)
    for (int g = 0; g < G; ++g) l[i * G + g] = exp(l[i * G + g] - lse[i]);

#pragma omp parallel for schedule(static) num_threads(NTHR)
  for (int g = 0; g < G; ++g) {
    /* Eq. 4 */
    double Lg = 0.0;
    for (int64_t i = 0; i < N; ++i) Lg += l[i * G + g];
    if (L_out) L_out[g] = Lg;
    /* Eq. 5 */
    hefts_out[g] = Lg / (double)N;
    double* mu = means_out + (size_t)g * D;
    double* C = covs_out + csz * g;
    if (Lg == 0.0) {
      memcpy(mu, means + (size_t)g * D, sizeof(double) * D);
      memcpy(C, covs + csz * g, sizeof(double) * csz);
      continue;
    }
    /* Each accumulator below is a plain sequential sum over i = 0..N-1; the
       loop nest only visits the samples once per pass. */
    double* s = (double*)malloc(sizeof(double) * csz);
    if (!s) abort();
    /* Eq. 6 */
    for (int d = 0; d < D; ++d) s[d] = 0.0;
    for (int64_t i = 0; i < N; ++i) {
      double li = l[i * G + g];
      for (int d = 0; d < D; ++d) s[d] += xval(S, i, d) * li;
    }
    for (int d = 0; d < D; ++d) mu[d] = s[d] / Lg;
    /* Eq. 7, centred on the new mean; second pass over the samples. */
    if (!full) {
      for (int d = 0; d < D; ++d) s[d] = 0.0;
      for (int64_t i = 0; i < N; ++i) {
        double li = l[i * G + g];
        for (int d = 0; d < D; ++d) {
          double t = xval(S, i, d) - mu[d];
          s[d] += t * t * li;
        }
      }
      for (int d = 0; d < D; ++d) {
        double v = s[d] / Lg;
        C[d] = v > var_floor ? v : var_floor; /* floor on the diagonal, Sec. 2.2 */
      }
    } else {
      for (size_t k = 0; k < csz; ++k) s[k] = 0.0;
      for (int64_t i = 0; i < N; ++i) {
        double li = l[i * G + g];
        for (int e = 0; e < D; ++e) {
          double te = xval(S, i, e) - mu[e];
          for (int d = e; d < D; ++d)
            s[(size_t)e * D + d] += (xval(S, i, d) - mu[d]) * te * li;
        }
      }
      for (int e = 0; e < D; ++e)
        for (int d = e; d < D; ++d) {
          C[(size_t)e * D + d] = s[(size_t)e * D + d] / Lg;
          C[(size_t)d * D + e] = s[(size_t)e * D + d] / Lg;
        }
      for (int d = 0; d < D; ++d) {
        double v = C[(size_t)d * D + d];
        C[(size_t)d * D + d] = v > var_floor ? v : var_floor;
      }
    }
    free(s);
  }
  free(l);
  free(lse);
  return isfinite(*mean_loglik) ? 0 : ORC_NONFINITE;
}

/* ------------------------------------------------------------------------ */
/* Public: global diagonal statistics for the Mahalanobis k-means distance   */
/* (Sec. 3.1: a global diagonal covariance estimated from all the data).     */
/* Population variance (divide by N), two-pass.                              */
/* ------------------------------------------------------------------------ */

static int global_stats_s(const samples_t* S, int64_t N, int D, double* mean,
                        double* var) {
  if (N < 1 || D < 1 || S->ldx < D) return ORC_EINVAL;
  /* Sequential sums over i for each dimension; the sample loop is outermost so
     memory is read in order. */
  for (int d = 0; d < D; ++d) mean[d] = 0.0;
  for (int64_t i = 0; i < N; ++i)
    for (int d = 0; d < D; ++d) mean[d] += xval(S, i, d);
  for (int d = 0; d < D; ++d) mean[d] /= (double)N;
  for (int d = 0; d < D; ++d) var[d] = 0.0;
  for (int64_t i = 0; i < N; ++i)
    for (int d = 0; d < D; ++d) {
      double t = xval(S, i, d) - mean[d];
      var[d] += t * t;
    }
  for (int d = 0; d < D; ++d) var[d] /= (double)N;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Public: one k-means iteration (Sec. 3, Eq. 19; Sec. 3.1, Eq. 20).          */
/*                                                                            */
/* dist(x, mu_g) = sum_d lam[d] (x_d - mu_gd)^2, lam = 1 for the Euclidean    */
/* distance, lam = 1/var_global for the Mahalanobis one.  assign_i = lowest-  */
/* index argmin.  New mean = average of the assigned samples.                 */
/*                                                                            */
/* Dead means (no samples): resurrected (end of Sec. 3.1) as one of the       */
/* vectors of the most popular mean.  Reading used here: dead clusters in     */
/* increasing g; the donor is the cluster with the largest remaining count   */
/* (ties -> lowest g), which must be at least 2; each donation lowers the    */
/* donor's remaining count by one; the k-th donation from a donor takes its   */
/* k-th lowest-index sample.  A dead cluster with no eligible donor keeps its */
/* mean.                                                                      */
/*                                                                            */
/* Hand-off statistics (Sec. 3: parameters as Eqs. 5-7 with hard l):          */
/* hefts = count/N, dcovs = max(mean squared deviation about the new mean,    */
/* floor); a cluster with count 0 gets dcov 1 (the reset() convention of the  */
/* Sec. 4 API) and heft 0.                                                    */
/*                                                                            */
/* inertia = sum_i dist(x_i, mu_assign(i)) under the INPUT means.             */
/* gap[i] (optional) = (d2 - d1)/max(d1, 1e-300): the relative gap between    */
/* the best and second-best distance (+inf when G == 1).                      */
/* ------------------------------------------------------------------------ */

static int kmeans_iter_s(const samples_t* S, int64_t N, int D, int G, const double* lam,
                       const double* means, double var_floor, double* means_out,
                       double* dcovs_out, double* hefts_out, int64_t* counts_out,
                       int32_t* assign_out, double* inertia, double* gap /* N or NULL */) {
  if (N < 1 || D < 1 || G < 1 || S->ldx < D) return ORC_EINVAL;
  double* best = (double*)malloc(sizeof(double) * (size_t)N);
  int64_t* rem = (int64_t*)malloc(sizeof(int64_t) * (size_t)G);
  int64_t* taken = (int64_t*)calloc((size_t)G, sizeof(int64_t));
  if (!best || !rem || !taken) {
    free(best);
    free(rem);
    free(taken);
    return ORC_ENOMEM;
  }

  /* Eq. 19: hard assignment to the nearest mean. */
#pragma omp parallel for schedule(static) num_threads(NTHR)
  for (int64_t i = 0; i < N; ++i) {
    double d1 = INFINITY, d2 = INFINITY;
    int arg = 0;
    for (int g = 0; g < G; ++g) {
      double s = 0.0;
      for (int d = 0; d < D; ++d) {
        double t = xval(S, i, d) - means[(size_t)g * D + d];
        s += lam[d] * t * t;
      }
      if (s < d1) {
        d2 = d1;
        d1 = s;
        arg = g;
      } else if (s < d2) {
        d2 = s;
      }
    }
    assign_out[i] = arg;
    best[i] = d1;
    if (gap) gap[i] = (G == 1) ? INFINITY : (d2 - d1) / (d1 > 1e-300 ? d1 : 1e-300);
  }

  double in = 0.0;
  for (int64_t i = 0; i < N; ++i) in += best[i];
  *inertia = in;

  for (int g = 0; g < G; ++g) counts_out[g] = 0;
  for (int64_t i = 0; i < N; ++i) counts_out[assign_out[i]] += 1;

  /* New means (Eq. 6 with l in {0,1}) and hand-off variances (Eq. 7). */
#pragma omp parallel for schedule(static) num_threads(NTHR)
  for (int g = 0; g < G; ++g) {
    double* mu = means_out + (size_t)g * D;
    int64_t c = counts_out[g];
    if (c == 0) {
      memcpy(mu, means + (size_t)g * D, sizeof(double) * D);
      for (int d = 0; d < D; ++d) dcovs_out[(size_t)g * D + d] = 1.0;
      hefts_out[g] = 0.0;
      continue;
    }
    /* Sequential sums over the cluster's samples in increasing i. */
    double* s = (double*)malloc(sizeof(double) * D);
    if (!s) abort();
    for (int d = 0; d < D; ++d) s[d] = 0.0;
    for (int64_t i = 0; i < N; ++i)
      if (assign_out[i] == g)
        for (int d = 0; d < D; ++d) s[d] += xval(S, i, d);
    for (int d = 0; d < D; ++d) mu[d] = s[d] / (double)c;
    for (int d = 0; d < D; ++d) s[d] = 0.0;
    for (int64_t i = 0; i < N; ++i)
      if (assign_out[i] == g)
        for (int d = 0; d < D; ++d) {
          double t = xval(S, i, d) - mu[d];
          s[d] += t * t;
        }
    for (int d = 0; d < D; ++d) {
      double v = s[d] / (double)c;
      dcovs_out[(size_t)g * D + d] = v > var_floor ? v : var_floor;
    }
    free(s);
    hefts_out[g] = (double)c / (double)N;
  }

  /* Dead-mean resurrection (end of Sec. 3.1). */
  for (int g = 0; g < G; ++g) rem[g] = counts_out[g];
  for (int g = 0; g < G; ++g) {
    if (counts_out[g] != 0) continue;
    int q = 0;
    for (int k = 1; k < G; ++k)
      if (rem[k] > rem[q]) q = k;
    if (rem[q] < 2) continue;
    int64_t want = taken[q], seen = 0, pick = -1;
    for (int64_t i = 0; i < N; ++i)
      if (assign_out[i] == q) {
        if (seen == want) {
          pick = i;
          break;
        }
        ++seen;
      }
    if (pick < 0) continue;
    for (int d = 0; d < D; ++d) means_out[(size_t)g * D + d] = xval(S, pick, d);
    taken[q] += 1;
    rem[q] -= 1;
  }

  free(best);
  free(rem);
  free(taken);
  return isfinite(*inertia) ? 0 : ORC_NONFINITE;
}

/* ------------------------------------------------------------------------ */
/* Public: every k-means distance (Sec. 3, Eq. 19's argument; Sec. 3.1,       */
/* Eq. 20's weights): out[i*G + g] = sum_d lam[d] (x_di - mu_gd)^2.          */
/* ------------------------------------------------------------------------ */

static int kmeans_dists_s(const samples_t* S, int64_t N, int D, int G, const double* lam,
                        const double* means, double* out) {
  if (N < 1 || D < 1 || G < 1 || S->ldx < D) return ORC_EINVAL;
#pragma omp parallel for schedule(static) num_threads(NTHR)
  for (int64_t i = 0; i < N; ++i)
    for (int g = 0; g < G; ++g) {
      double s = 0.0;
      for (int d = 0; d < D; ++d) {
        double t = xval(S, i, d) - means[(size_t)g * D + d];
        s += lam[d] * t * t;
      }
      out[i * G + g] = s;
    }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Public: closest Gaussian per sample (Sec. 4 API: assign(X, dist_mode)).    */
/* mode 0 = Euclidean distance to the means; mode 1 = probabilistic:          */
/* the Gaussian with the largest weighted likelihood.  Lowest index on ties. */
/* ------------------------------------------------------------------------ */

static int assign_s(const samples_t* S, int64_t N, int D, int G, int mode,
                  const double* hefts, const double* means, const double* dcovs,
                  int32_t* out) {
  if (N < 1 || D < 1 || G < 1 || S->ldx < D || (mode != 0 && mode != 1)) return ORC_EINVAL;
  double* logdet = (double*)malloc(sizeof(double) * G);
  if (!logdet) return ORC_ENOMEM;
  for (int g = 0; g < G; ++g) logdet[g] = mode == 1 ? log_det_diag(dcovs + (size_t)g * D, D) : 0.0;
#pragma omp parallel for schedule(static) num_threads(NTHR)
  for (int64_t i = 0; i < N; ++i) {
    int arg = 0;
    double best = 0.0;
    for (int g = 0; g < G; ++g) {
      double v;
      if (mode == 0) {
        double s = 0.0;
        for (int d = 0; d < D; ++d) {
          double t = xval(S, i, d) - means[(size_t)g * D + d];
          s += t * t;
        }
        v = -s;
      } else {
        v = log(hefts[g]) + log_gauss_diag(S, i, means + (size_t)g * D,
                                           dcovs + (size_t)g * D, logdet[g], D);
      }
      if (g == 0 || v > best) {
        best = v;
        arg = g;
      }
    }
    out[i] = arg;
  }
  free(logdet);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Public entry points: FP32 samples (oracle_*) and FP64 samples             */
/* (oracle_*_f64), both D x N column-major with row stride ldx.              */
/* ------------------------------------------------------------------------ */

#define ORC_PAIR(NAME, PARAMS, ARGS)                                                   \
  int oracle_##NAME(const float* X, int64_t N, int D, int64_t ldx, PARAMS) {          \
    samples_t S = {X, NULL, ldx};                                                      \
    return NAME##_s(&S, N, D, ARGS);                                                   \
  }                                                                                    \
  int oracle_##NAME##_f64(const double* X, int64_t N, int D, int64_t ldx, PARAMS) {   \
    samples_t S = {NULL, X, ldx};                                                      \
    return NAME##_s(&S, N, D, ARGS);                                                   \
  }
#define P_(...) __VA_ARGS__

ORC_PAIR(loglik,
         P_(int G, int full, const double* hefts, const double* means, const double* covs,
            double* mean_loglik, double* per_sample),
         P_(G, full, hefts, means, covs, mean_loglik, per_sample))
ORC_PAIR(log_p_g, P_(int G, const double* means, const double* dcovs, int g, double* out),
         P_(G, means, dcovs, g, out))
ORC_PAIR(seed_spread,
         P_(int G, const double* lam, int64_t first, int64_t* idx_out, double* means_out),
         P_(G, lam, first, idx_out, means_out))
ORC_PAIR(responsibilities,
         P_(int G, int full, const double* hefts, const double* means, const double* covs,
            double* out),
         P_(G, full, hefts, means, covs, out))
ORC_PAIR(em_iter,
         P_(int G, int full, const double* hefts, const double* means, const double* covs,
            double var_floor, double* hefts_out, double* means_out, double* covs_out,
            double* mean_loglik, double* L_out),
         P_(G, full, hefts, means, covs, var_floor, hefts_out, means_out, covs_out, mean_loglik,
            L_out))
ORC_PAIR(global_stats, P_(double* mean, double* var), P_(mean, var))
ORC_PAIR(kmeans_iter,
         P_(int G, const double* lam, const double* means, double var_floor, double* means_out,
            double* dcovs_out, double* hefts_out, int64_t* counts_out, int32_t* assign_out,
            double* inertia, double* gap),
         P_(G, lam, means, var_floor, means_out, dcovs_out, hefts_out, counts_out, assign_out,
            inertia, gap))
ORC_PAIR(kmeans_dists, P_(int G, const double* lam, const double* means, double* out),
         P_(G, lam, means, out))
ORC_PAIR(assign,
         P_(int G, int mode, const double* hefts, const double* means, const double* dcovs,
            int32_t* out),
         P_(G, mode, hefts, means, dcovs, out))
