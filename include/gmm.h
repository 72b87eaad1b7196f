/*
 * gmm.h -- C ABI of the MI355X (gfx950) Gaussian-mixture training library.
 *
 * The operations follow Sanderson & Curtin, arXiv:1707.09094:
 *   gmm_global_stats   global diagonal covariance for the Mahalanobis k-means
 *                      distance (Sec. 3.1, Eq. 20)
 *   gmm_kmeans_iter    one k-means iteration: hard assignment (Sec. 3, Eq. 19),
 *                      new means, dead-mean resurrection (Sec. 3.1), and the
 *                      hand-off weights/variances (Sec. 3, Eqs. 5-7 with hard l)
 *   gmm_em_iter        one EM iteration: E-step in the log domain (Sec. 2.2,
 *                      Eqs. 15-18), responsibilities (Sec. 2, Eq. 3), M-step
 *                      (Sec. 2, Eqs. 4-7; accumulator split of Sec. 2.1,
 *                      Eqs. 8-14) and the variance floor (Sec. 2.2)
 *   gmm_loglik         per-sample and mean log-likelihood (Sec. 4 API:
 *                      log_p(X), avg_log_p(X))
 *   gmm_seed_means     initial means: subset or maximally spread subset of
 *                      the samples (Sec. 4 API seed_mode)
 *   gmm_log_p_gaussian per-sample and mean log-density under one Gaussian
 *                      (Sec. 4 API: log_p(X, g), avg_log_p(X, g))
 *   gmm_assign         closest Gaussian per sample and its histogram
 *                      (Sec. 4 API: assign, raw_hist)
 *   gmm_*_batched      the same operations for many independent models per
 *                      launch
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every array argument is a DEVICE pointer owned by the caller; the
 * library keeps no pointer after the call returns and allocates no device
 * memory: scratch space comes from the caller's workspace `ws` of `ws_bytes`
 * bytes (size it with gmm_workspace_bytes; 256-byte aligned).  All work is
 * enqueued on `stream` (a hipStream_t; NULL = the null stream) and nothing
 * synchronises with the host, so a sequence of calls can be captured into a
 * graph.  Calls that share a workspace must be ordered on one stream.
 *
 * Layouts (one sample per column, Sec. 4 API).  X is D x N column-major FP32:
 * element d of sample i is X[i*ldx + d], ldx >= D.  Parameters are FP32:
 *   hefts[g]                       weights, g < G
 *   means[g*D + d]                 column g = mean of Gaussian g
 *   covs[g*D + d]                  diagonal covariances (cov = GMM_COV_DIAG)
 *   covs[g*D*D + e*D + d]          full covariance of Gaussian g, column-major,
 *                                  symmetric (cov = GMM_COV_FULL)
 *
 * Errors.  Argument errors (null required pointer, N < 1, D < 1, G < 1,
 * ldx < D, unknown enum value, workspace too small, a shape outside the
 * supported range) are detected on the host before anything is enqueued:
 * the call returns GMM_EINVAL and writes nothing.  A failed launch returns
 * GMM_EHIP.  Numerical failures are detected on the device and OR-ed into
 * *dev_status (GMM_DEV_* bits; the call sets it to 0 first), which the caller
 * reads after synchronising: a non-finite log-likelihood or parameter
 * (GMM_DEV_NONFINITE: NaN/Inf in the data, or a covariance <= 0 on input --
 * the failure mode named at the end of Sec. 2.2) and, for full covariances, a
 * matrix that is not positive definite (GMM_DEV_NOTPD); GMM_DEV_BADDESC marks
 * a device-side index or descriptor out of range.  Outputs are then
 * unspecified.
 */
#ifndef GMM_H
#define GMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* host return codes */
#define GMM_OK 0
#define GMM_EINVAL (-1)
#define GMM_EHIP (-2)

/* device status bits */
#define GMM_DEV_OK 0
#define GMM_DEV_NONFINITE 1
#define GMM_DEV_NOTPD 2
#define GMM_DEV_BADDESC 4   /* batched: descriptor disagrees with Ns/Gs, model skipped;
                               gmm_seed_means: a subset index outside [0, N) */

/* covariance type (Sec. 4: diagonal covariances; full as in Eq. 2) */
#define GMM_COV_DIAG 0
#define GMM_COV_FULL 1

/* k-means distance (Sec. 3.1 / learn() dist_mode) */
#define GMM_DIST_EUCL 0
#define GMM_DIST_MAHA 1

/* seeding of gmm_seed_means (Sec. 4 API seed_mode) */
#define GMM_SEED_SUBSET 0   /* static_subset / random_subset */
#define GMM_SEED_SPREAD 1   /* static_spread / random_spread */

/* assignment distance of gmm_assign (Sec. 4 API: eucl_dist / prob_dist) */
#define GMM_ASSIGN_EUCL 0
#define GMM_ASSIGN_PROB 1

/* arithmetic of the log-density / distance contraction of the one-pass
 * kernels (diagonal covariances, D <= 128 and G <= 128) and, for EM and the
 * log-likelihood, of the sliced kernels (diagonal, D <= 128, G > 128, prec
 * BF16X3); gmm_em_path and gmm_kmeans_path report which family a shape runs.
 * Other shapes compute their log-densities exactly in FP64 (matrix cores for
 * D <= 128) or screen in FP32 with an FP64 recompute, and ignore prec.
 * GMM_PREC_FP32:   direct (x - mu)^2 form in FP32 on the vector ALUs.
 * GMM_PREC_BF16X3: the expanded form x^2 * Lambda - 2 x * (Lambda mu) + const
 *                  as a GEMM on the matrix cores with each FP32 operand split
 *                  into two BF16 parts (hi*hi + hi*lo + lo*hi, FP32 accumulate);
 *                  every sample's leading components (those within a fixed gap
 *                  of the best, see gmm_em_iter) are recomputed exactly, so the
 *                  result carries FP32-path accuracy. */
#define GMM_PREC_FP32 0
#define GMM_PREC_BF16X3 1

typedef void* gmm_stream_t; /* hipStream_t */

/* Library version, (major << 16) | minor. */
int gmm_version(void);

/* Human-readable name of a host return code. */
const char* gmm_status_string(int code);

/* Bytes of workspace that every entry point below needs for a problem of N
 * samples, D dimensions and G Gaussians with covariance type `cov` and
 * precision `prec` (one size serves them all).  Returns 0 for arguments out of
 * range. */
size_t gmm_workspace_bytes(int64_t N, int32_t D, int32_t G, int32_t cov, int32_t prec);

/* Global per-dimension mean and population variance (divide by N) of X, in
 * FP64: the global diagonal covariance of the Mahalanobis k-means distance
 * (Sec. 3.1, Eq. 20).  mean_out[D], var_out[D]: device FP64 outputs. */
int gmm_global_stats(const float* X, int64_t N, int32_t D, int64_t ldx, double* mean_out,
                     double* var_out, void* ws, size_t ws_bytes, gmm_stream_t stream);

/* One k-means iteration (Sec. 3; Eq. 19 with Eq. 20's distance).
 *   dist        GMM_DIST_EUCL: sum_d (x_d - mu_gd)^2;
 *               GMM_DIST_MAHA: sum_d (x_d - mu_gd)^2 / max(gvar_d, var_floor).
 *   gvar[D]     FP64 global variances (gmm_global_stats), required for MAHA,
 *               ignored (may be NULL) for EUCL.
 *   means[D*G]  in: current means; out: new means (average of the assigned
 *               samples; dead means resurrected, see below).
 *   dcovs[D*G]  out: max(mean squared deviation of the assigned samples about
 *               the new mean, var_floor); 1 for a cluster with no samples.
 *   hefts[G]    out: count_g / N.
 *   counts[G]   out: int64 number of samples assigned to each mean.
 *   assign[N]   out (may be NULL): index of the nearest input mean; the lowest
 *               index wins exact ties.
 *   inertia[1]  out: FP64 sum over samples of the distance to the nearest
 *               INPUT mean.
 *   n_recomputed[1]  out (may be NULL): samples whose two best FP32 (or BF16x3)
 *               distances were closer than the arithmetic's error bound and
 *               were re-decided in FP64.
 * Dead means (Sec. 3.1): clusters with no samples, taken in increasing index,
 * become a sample of the cluster with the largest remaining count (lowest
 * index on ties; it needs at least 2), the k-th donation from a cluster taking
 * its k-th lowest-index sample; each donation lowers the donor's remaining
 * count by one.  A dead mean with no eligible donor is kept.
 * prec: GMM_PREC_FP32 or GMM_PREC_BF16X3 (distance contraction). */
int gmm_kmeans_iter(const float* X, int64_t N, int32_t D, int64_t ldx, int32_t G, int32_t dist,
                    const double* gvar, float var_floor, float* means, float* dcovs,
                    float* hefts, int64_t* counts, int32_t* assign, double* inertia,
                    int32_t prec, int64_t* n_recomputed, int32_t* dev_status, void* ws,
                    size_t ws_bytes, gmm_stream_t stream);

/* One EM iteration (Sec. 2, Eqs. 3-7), parameters updated in place.
 *   hefts[G], means[D*G], covs (D*G diag or D*D*G full): in/out.
 *   var_floor   lower bound applied to every (diagonal) variance after the
 *               update (Sec. 2.2); the input parameters are used as given.
 *   mean_loglik[1]  out: FP64 mean log-likelihood of the INPUT parameters
 *               (the E-step's by-product; EM makes successive values
 *               non-decreasing).
 *   n_recomputed[1] out (may be NULL): diagonal models with D, G <= 128 (the
 *               one-pass kernels, either arithmetic form) or D <= 128 with
 *               prec BF16X3 (the sliced kernels): number of (sample, Gaussian)
 *               log-densities recomputed exactly, i.e. every pair whose
 *               screened value, widened by its rounding-error bound, comes
 *               within 30 nats of the sample's best; 0 for other shapes
 *               (their log-densities are exact FP64 or recomputed in FP64
 *               without being counted).
 * A Gaussian whose responsibilities sum to exactly 0 gets weight 0 and keeps
 * its mean and covariance.  Responsibilities (normalised per sample) below
 * exp(-40) are treated as 0.
 * Full covariances (cov = GMM_COV_FULL): Cholesky factors and log-determinants
 * in FP64; a factorisation that fails sets GMM_DEV_NOTPD. */
int gmm_em_iter(const float* X, int64_t N, int32_t D, int64_t ldx, int32_t G, int32_t cov,
                float* hefts, float* means, float* covs, float var_floor, int32_t prec,
                double* mean_loglik, int64_t* n_recomputed, int32_t* dev_status, void* ws,
                size_t ws_bytes, gmm_stream_t stream);

/* gmm_em_iter for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, validation, kernels and results, without `ws`/`ws_bytes`.
 * Its scratch space is a static device array of GMM_NOALLOC_SCRATCH_BYTES
 * (128 MiB) per GPU, held by the library from the first load of its code on
 * that GPU until the process ends; a shape whose gmm_workspace_bytes exceeds
 * it (e.g. D = 64, G = 512 at any N) returns GMM_EINVAL and writes nothing.
 * The call allocates nothing: no hipMalloc/hipFree, no events (profiling is
 * skipped for it).  Every call on one GPU shares that GPU's array, which keeps
 * the last call's contents (every call rewrites what it reads first): calls
 * ordered on one stream are safe, calls that may overlap in time on one GPU
 * (several streams or host threads) race and give undefined results. */
#define GMM_NOALLOC_SCRATCH_BYTES (128ull << 20)
int gmm_em_iter_noalloc(const float* X, int64_t N, int32_t D, int64_t ldx, int32_t G,
                        int32_t cov, float* hefts, float* means, float* covs, float var_floor,
                        int32_t prec, double* mean_loglik, int64_t* n_recomputed,
                        int32_t* dev_status, gmm_stream_t stream);

/* Log-likelihood of X under the given parameters (Sec. 4 API).
 *   mean_loglik[1]  out: FP64 average of log p(x_i | lambda)   (avg_log_p(X))
 *   per_sample[N]   out (may be NULL): FP32 log p(x_i | lambda) (log_p(X)) */
int gmm_loglik(const float* X, int64_t N, int32_t D, int64_t ldx, int32_t G, int32_t cov,
               const float* hefts, const float* means, const float* covs, int32_t prec,
               double* mean_loglik, float* per_sample, int32_t* dev_status, void* ws,
               size_t ws_bytes, gmm_stream_t stream);

/* Initial means (Sec. 4 API seed_mode), written to means[G*D].
 *   GMM_SEED_SUBSET  means[g] = sample idx[g] (idx: device int64[G], indices
 *                    the caller drew: random_subset), or, with idx = NULL,
 *                    sample floor(g N / G) (static_subset).  An index outside
 *                    [0, N) sets GMM_DEV_BADDESC and leaves that row as it was.
 *   GMM_SEED_SPREAD  farthest-first traversal ("maximally spread"): means[0] =
 *                    sample `first` (0: static_spread; a caller-drawn index:
 *                    random_spread); means[k+1] = the sample whose distance to
 *                    its nearest chosen seed is largest, lowest index on ties;
 *                    distance sum_d lam_d (x_d - y_d)^2 in FP64, lam_d = 1
 *                    (gvar = NULL) or 1 / max(gvar_d, var_floor) (the k-means
 *                    Mahalanobis weights; gvar from gmm_global_stats).  One pass
 *                    over X per seed.
 * The workspace is sized as for the same (N, D, G) with GMM_COV_DIAG. */
int gmm_seed_means(const float* X, int64_t N, int32_t D, int64_t ldx, int32_t G, int32_t mode,
                   const double* gvar, float var_floor, int64_t first, const int64_t* idx,
                   float* means, int32_t* dev_status, void* ws, size_t ws_bytes,
                   gmm_stream_t stream);

/* Log-density of X under ONE Gaussian g of a diagonal model, without its
 * weight (Sec. 4 API log_p(X, g), avg_log_p(X, g)):
 *   log N(x | mu_g, Sigma_g) = -1/2 (D log 2 pi + sum_d log sigma2_gd
 *                                    + sum_d (x_d - mu_gd)^2 / sigma2_gd),
 * computed in FP64 per sample.
 *   g           0 <= g < G; means[D*G], dcovs[D*G] as for gmm_em_iter (only
 *               row g is read).
 *   mean_out[1]     out (may be NULL): FP64 average over the N samples.
 *   per_sample[N]   out (may be NULL): FP32 value per sample.
 * At least one of the two outputs must be given (GMM_EINVAL otherwise).  A
 * non-finite value (e.g. a variance <= 0) sets GMM_DEV_NONFINITE.  The
 * workspace is sized as for the same (N, D, G) with GMM_COV_DIAG. */
int gmm_log_p_gaussian(const float* X, int64_t N, int32_t D, int64_t ldx, int32_t G, int32_t g,
                       const float* means, const float* dcovs, double* mean_out,
                       float* per_sample, int32_t* dev_status, void* ws, size_t ws_bytes,
                       gmm_stream_t stream);

/* Closest Gaussian per sample (Sec. 4 API assign / raw_hist), diagonal model.
 *   mode        GMM_ASSIGN_EUCL: nearest mean in Euclidean distance;
 *               GMM_ASSIGN_PROB: largest weighted log-likelihood
 *               log w_g + log N(x | mu_g, Sigma_g).
 *   assign[N]   out: int32 index (lowest index on exact ties).
 *   hist[G]     out (may be NULL): int64 count of samples per Gaussian. */
int gmm_assign(const float* X, int64_t N, int32_t D, int64_t ldx, int32_t G, int32_t mode,
               const float* hefts, const float* means, const float* dcovs, int32_t* assign,
               int64_t* hist, int32_t* dev_status, void* ws, size_t ws_bytes,
               gmm_stream_t stream);

/* ---- FP64 data (the paper's gmm_diag<double>, Sec. 4; the precision of its
 * speed-up experiment, Sec. 5.1) ---------------------------------------------
 * The same operations on FP64 samples with FP64 parameters, diagonal
 * covariances.  Layouts, conventions and semantics are those of the FP32
 * calls above, with double in place of float for X, hefts, means, dcovs,
 * per_sample and var_floor.  Supported shapes: D <= 128 and G up to what the
 * 32-sample tile of FP64 log-densities holds in LDS (about 480 components at
 * D = 128, 540 at D = 64); gmm_workspace_bytes_f64 returns 0 and the calls
 * return GMM_EINVAL beyond that.  Arithmetic: FP64 throughout.  The E-step
 * computes every log-density on the FP64 matrix cores (expanded form) and
 * then recomputes, in the FP64 direct form, every pair within 41 nats of the
 * sample's largest value, so every responsibility above exp(-40) and every
 * log-likelihood is as exact as FP64 rounding of the plain definition
 * (responsibilities below exp(-80), not exp(-40), are treated as 0); the
 * k-means assignment is the FP64 argmin (re-decided in the direct form when
 * the two smallest matrix-core distances are within their rounding bound). */
size_t gmm_workspace_bytes_f64(int64_t N, int32_t D, int32_t G);
int gmm_global_stats_f64(const double* X, int64_t N, int32_t D, int64_t ldx, double* mean_out,
                         double* var_out, void* ws, size_t ws_bytes, gmm_stream_t stream);
int gmm_kmeans_iter_f64(const double* X, int64_t N, int32_t D, int64_t ldx, int32_t G,
                        int32_t dist, const double* gvar, double var_floor, double* means,
                        double* dcovs, double* hefts, int64_t* counts, int32_t* assign,
                        double* inertia, int64_t* n_recomputed, int32_t* dev_status, void* ws,
                        size_t ws_bytes, gmm_stream_t stream);
int gmm_em_iter_f64(const double* X, int64_t N, int32_t D, int64_t ldx, int32_t G,
                    double* hefts, double* means, double* dcovs, double var_floor,
                    double* mean_loglik, int32_t* dev_status, void* ws, size_t ws_bytes,
                    gmm_stream_t stream);
int gmm_loglik_f64(const double* X, int64_t N, int32_t D, int64_t ldx, int32_t G,
                   const double* hefts, const double* means, const double* dcovs,
                   double* mean_loglik, double* per_sample, int32_t* dev_status, void* ws,
                   size_t ws_bytes, gmm_stream_t stream);

/* ---- kernel selection ----------------------------------------------------
 * Which kernel family gmm_em_iter / gmm_loglik (gmm_em_path) and
 * gmm_kmeans_iter (gmm_kmeans_path) run for a shape and arithmetic form.
 * Pure host functions with no side effect, for tests and tools; they return
 * GMM_EINVAL for arguments the calls would reject.
 *   GMM_PATH_ONEPASS_BF16X3  diagonal, D <= 128, G <= 128, prec BF16X3: the
 *                            one-pass kernel with the split-BF16 contraction
 *                            on the matrix cores and the exact recompute of
 *                            each sample's leading components
 *   GMM_PATH_ONEPASS_FP32    the same shapes, prec FP32 (or a shape whose
 *                            matrix-core fragments do not fit): the one-pass
 *                            kernel with the FP32 direct form
 *   GMM_PATH_WIDE_FP64       diagonal, D <= 128, G > 128, prec FP32 (and
 *                            k-means with either prec): every log-density
 *                            (distance) in FP64 on the matrix cores
 *   GMM_PATH_SLICED_BF16X3   EM / log-likelihood, diagonal, D <= 128, G > 128,
 *                            prec BF16X3: the one-pass kernel's split-BF16
 *                            screening over slices of at most 128 Gaussians,
 *                            in three passes (slice maxima; near pairs
 *                            recomputed in FP64 and slice sums; responsibilities
 *                            and the map step)
 *   GMM_PATH_GENERIC         diagonal, D > 128: FP32 direct-form screening with
 *                            an FP64 recompute of the near set (prec ignored)
 *   GMM_PATH_FULL_FP64       full covariances, D <= 64: FP64 matrix cores
 *   GMM_PATH_FULL_GENERIC    full covariances, 64 < D <= 128: FP32 screening,
 *                            FP64 near set */
#define GMM_PATH_ONEPASS_BF16X3 1
#define GMM_PATH_ONEPASS_FP32 2
#define GMM_PATH_WIDE_FP64 3
#define GMM_PATH_GENERIC 4
#define GMM_PATH_FULL_FP64 5
#define GMM_PATH_FULL_GENERIC 6
#define GMM_PATH_SLICED_BF16X3 7

int gmm_em_path(int32_t D, int32_t G, int32_t cov, int32_t prec);
int gmm_kmeans_path(int32_t D, int32_t G, int32_t prec);

/* ---- many independent diagonal models in one launch sequence --------------
 * The batch is described by an array of n_models descriptors in DEVICE
 * memory.  All models share D (<= 128) and the arithmetic form; each has its
 * own N >= 1 and 1 <= G <= 128.  The host arrays Ns[n_models] and
 * Gs[n_models] must repeat the descriptors' N and G: the host uses them to
 * size the launch and the workspace, the device uses the descriptors.
 * Per model the arithmetic is that of the single-model call (gmm_em_iter /
 * gmm_loglik / gmm_kmeans_iter with ldx = D); only the cut of the samples
 * into partial sums differs, so k-means assignments and counts are identical
 * and the floating-point results agree to rounding.  The calls below
 * enqueue a fixed number of kernels whatever n_models is and copy nothing
 * from the host, so a sequence of them can be captured into a graph.
 * `chunk` is the number of samples per work item (a positive multiple of
 * 32, typically from gmm_batched_autotune); every model's samples are cut
 * into consecutive items and a persistent grid processes all items of all
 * models in one launch. */
typedef struct {
  const float* X;       /* D x N column-major (ld = D) */
  int64_t N;
  int32_t G;
  int32_t reserved;     /* 0 */
  float* hefts;         /* [G] EM: in/out; k-means: out */
  float* means;         /* [D*G] in/out */
  float* covs;          /* [D*G] EM: diagonal covariances in/out; k-means: hand-off dcovs out */
  int64_t* counts;      /* [G] k-means: out (required) */
  int32_t* assign;      /* [N] k-means: out (required) */
  double* loglik;       /* [1] EM / loglik: mean log-likelihood of the input parameters, or NULL */
  double* inertia;      /* [1] k-means: inertia under the input means, or NULL */
  const double* gvar;   /* [D] k-means with GMM_DIST_MAHA: global variances (required) */
  int32_t* dev_status;  /* [1] out (required) */
} gmm_model_desc;

/* Workspace bytes for a batch (any of the batched calls, any chunk >= `chunk`). */
size_t gmm_batched_workspace_bytes(int32_t n_models, const int64_t* Ns, const int32_t* Gs,
                                   int32_t D, int32_t chunk);

/* One EM iteration of every model (gmm_em_iter semantics, diagonal). */
int gmm_em_iter_batched(const gmm_model_desc* models, int32_t n_models, const int64_t* Ns,
                        const int32_t* Gs, int32_t D, float var_floor, int32_t prec,
                        int32_t chunk, void* ws, size_t ws_bytes, gmm_stream_t stream);

/* Mean log-likelihood of every model (gmm_loglik semantics, diagonal). */
int gmm_loglik_batched(const gmm_model_desc* models, int32_t n_models, const int64_t* Ns,
                       const int32_t* Gs, int32_t D, int32_t prec, int32_t chunk, void* ws,
                       size_t ws_bytes, gmm_stream_t stream);

/* One k-means iteration of every model (gmm_kmeans_iter semantics). */
int gmm_kmeans_iter_batched(const gmm_model_desc* models, int32_t n_models, const int64_t* Ns,
                            const int32_t* Gs, int32_t D, int32_t dist, float var_floor,
                            int32_t chunk, void* ws, size_t ws_bytes, gmm_stream_t stream);

/* Per-model global mean and population variance (gmm_global_stats of each
 * model's X): mean_out and var_out are DEVICE arrays [n_models][D]. */
int gmm_global_stats_batched(const gmm_model_desc* models, int32_t n_models, int32_t D,
                             double* mean_out, double* var_out, gmm_stream_t stream);

/* Chooses `chunk` for a batch: times gmm_loglik_batched (which leaves the
 * models unchanged) for each candidate chunk in {1024, 2048, 4096, 8192,
 * 16384} (those the workspace can hold) and writes the fastest to *best_chunk.
 * The pass costs what the models' current parameters make it cost (how many
 * near pairs each sample has), so call it once they hold a fitted state, for
 * example after the k-means seeding, not on zeroed parameters.
 * Synchronises with the host; not for use under graph capture. */
int gmm_batched_autotune(const gmm_model_desc* models, int32_t n_models, const int64_t* Ns,
                         const int32_t* Gs, int32_t D, int32_t prec, void* ws, size_t ws_bytes,
                         gmm_stream_t stream, int32_t* best_chunk);

/* The autotune cache.  gmm_batched_autotune keeps each choice in a
 * per-process table keyed by (GPU architecture, D, largest G, floor(log2) of
 * the batch's total N, floor(log2) of the model count, arithmetic form,
 * covariance type) and returns a cached choice (one the workspace can hold)
 * without timing or launching anything.  When the environment variable
 * GMM_AUTOTUNE_CACHE names a file, the table is filled from it (lines "key
 * chunk") at the first call after a clear, and every new choice is appended
 * to it.  The table is guarded by a mutex.
 * Number of entries in the table: */
int gmm_autotune_cache_size(void);
/* Empties the table (the file is left as it is; it is read again at the next
 * gmm_batched_autotune). */
int gmm_autotune_cache_clear(void);

/* ---- instrumentation -----------------------------------------------------
 * When enabled, every launch of a data-pass kernel (one that reads all of X)
 * is bracketed by a pair of HIP events recorded on the caller's stream, and
 * the elapsed times are accumulated per kind.  For eager benchmarking only:
 * keep it disabled while a stream is being captured into a graph. */
#define GMM_PROF_EM 0        /* fused E-step + M-step map pass of gmm_em_iter */
#define GMM_PROF_KM_ASSIGN 1 /* k-means assignment pass */
#define GMM_PROF_KM_ACCUM 2  /* k-means accumulation pass */
#define GMM_PROF_LOGLIK 3    /* gmm_loglik pass */
#define GMM_PROF_STATS 4     /* gmm_global_stats passes */
#define GMM_PROF_BATCHED 5   /* batched data passes */

/* Enable (on != 0) or disable recording; either way the totals are reset. */
int gmm_profile_enable(int on);

/* Total milliseconds and number of launches recorded for `kind` since the last
 * gmm_profile_enable; waits for the recorded events. */
int gmm_profile_read(int32_t kind, double* ms_total, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* GMM_H */
