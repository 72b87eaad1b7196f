// gmm_api.hip -- the extern "C" entry points declared in include/gmm.h:
// host-side argument validation (everything is checked before the first
// enqueue, so a rejected call writes nothing), workspace carving, dispatch.
#include <hip/hip_runtime.h>

#include "gmm_internal.hpp"

using namespace gmm;

namespace {

constexpr int kMaxD = 4096;
constexpr int kMaxG = 4096;  // the per-sample near-set bitmask covers 64 x 64 components
constexpr int kMaxDFull = 128;

bool shape_ok(int64_t N, int32_t D, int64_t ldx, int32_t G) {
  return N >= 1 && D >= 1 && D <= kMaxD && G >= 1 && G <= kMaxG && ldx >= D &&
         N <= ((int64_t)1 << 40);
}

int status_of(hipError_t e) { return e == hipSuccess ? GMM_OK : GMM_EHIP; }

bool ws_ok(void* ws, size_t ws_bytes, int64_t N, int D, int G, int cov, Workspace* w) {
  if (!ws) return false;
  if (((uintptr_t)ws) % 256 != 0) return false;
  return carve(ws, ws_bytes, N, D, G, cov, w);
}

}  // namespace

extern "C" {

int gmm_version(void) { return (0 << 16) | 1; }

const char* gmm_status_string(int code) {
  switch (code) {
    case GMM_OK:
      return "ok";
    case GMM_EINVAL:
      return "invalid argument";
    case GMM_EHIP:
      return "HIP launch error";
    default:
      return "unknown status";
  }
}

size_t gmm_workspace_bytes(int64_t N, int32_t D, int32_t G, int32_t cov, int32_t prec) {
  if (!shape_ok(N, D, D, G)) return 0;
  if (cov != GMM_COV_DIAG && cov != GMM_COV_FULL) return 0;
  if (prec != GMM_PREC_FP32 && prec != GMM_PREC_BF16X3) return 0;
  if (cov == GMM_COV_FULL && D > kMaxDFull) return 0;
  Workspace w;
  carve(nullptr, 0, N, D, G, cov, &w);
  return w.bytes;
}

int gmm_global_stats(const float* X, int64_t N, int32_t D, int64_t ldx, double* mean_out,
                     double* var_out, void* ws, size_t ws_bytes, gmm_stream_t stream) {
  if (!X || !mean_out || !var_out || !shape_ok(N, D, ldx, 1)) return GMM_EINVAL;
  Workspace w;
  if (!ws_ok(ws, ws_bytes, N, D, 1, GMM_COV_DIAG, &w)) return GMM_EINVAL;
  return status_of(launch_global_stats(X, N, D, ldx, mean_out, var_out, w, (hipStream_t)stream));
}

int gmm_kmeans_iter(const float* X, int64_t N, int32_t D, int64_t ldx, int32_t G, int32_t dist,
                    const double* gvar, float var_floor, float* means, float* dcovs,
                    float* hefts, int64_t* counts, int32_t* assign, double* inertia,
                    int32_t prec, int64_t* n_recomputed, int32_t* dev_status, void* ws,
                    size_t ws_bytes, gmm_stream_t stream) {
  if (!X || !means || !dcovs || !hefts || !counts || !inertia || !dev_status) return GMM_EINVAL;
  if (!shape_ok(N, D, ldx, G)) return GMM_EINVAL;
  if (dist != GMM_DIST_EUCL && dist != GMM_DIST_MAHA) return GMM_EINVAL;
  if (dist == GMM_DIST_MAHA && !gvar) return GMM_EINVAL;
  if (prec != GMM_PREC_FP32 && prec != GMM_PREC_BF16X3) return GMM_EINVAL;
  if (!(var_floor >= 0.0f)) return GMM_EINVAL;
  Workspace w;
  if (!ws_ok(ws, ws_bytes, N, D, G, GMM_COV_DIAG, &w)) return GMM_EINVAL;
  return status_of(launch_kmeans(X, N, D, ldx, G, dist, gvar, var_floor, means, dcovs, hefts,
                                 counts, assign, inertia, prec, n_recomputed, dev_status, w,
                                 (hipStream_t)stream));
}

int gmm_em_iter(const float* X, int64_t N, int32_t D, int64_t ldx, int32_t G, int32_t cov,
                float* hefts, float* means, float* covs, float var_floor, int32_t prec,
                double* mean_loglik, int64_t* n_recomputed, int32_t* dev_status, void* ws,
                size_t ws_bytes, gmm_stream_t stream) {
  if (!X || !hefts || !means || !covs || !mean_loglik || !dev_status) return GMM_EINVAL;
  if (!shape_ok(N, D, ldx, G)) return GMM_EINVAL;
  if (cov != GMM_COV_DIAG && cov != GMM_COV_FULL) return GMM_EINVAL;
  if (prec != GMM_PREC_FP32 && prec != GMM_PREC_BF16X3) return GMM_EINVAL;
  if (cov == GMM_COV_FULL && D > kMaxDFull) return GMM_EINVAL;
  if (!(var_floor >= 0.0f)) return GMM_EINVAL;
  Workspace w;
  if (!ws_ok(ws, ws_bytes, N, D, G, cov, &w)) return GMM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (cov == GMM_COV_FULL)
    return status_of(launch_em_full(X, N, D, ldx, G, hefts, means, covs, var_floor, mean_loglik,
                                    n_recomputed, dev_status, w, st));
  return status_of(launch_em_diag(X, N, D, ldx, G, hefts, means, covs, var_floor, prec,
                                  mean_loglik, n_recomputed, dev_status, w, st));
}

int gmm_loglik(const float* X, int64_t N, int32_t D, int64_t ldx, int32_t G, int32_t cov,
               const float* hefts, const float* means, const float* covs, int32_t prec,
               double* mean_loglik, float* per_sample, int32_t* dev_status, void* ws,
               size_t ws_bytes, gmm_stream_t stream) {
  if (!X || !hefts || !means || !covs || !mean_loglik || !dev_status) return GMM_EINVAL;
  if (!shape_ok(N, D, ldx, G)) return GMM_EINVAL;
  if (cov != GMM_COV_DIAG && cov != GMM_COV_FULL) return GMM_EINVAL;
  if (prec != GMM_PREC_FP32 && prec != GMM_PREC_BF16X3) return GMM_EINVAL;
  if (cov == GMM_COV_FULL && D > kMaxDFull) return GMM_EINVAL;
  Workspace w;
  if (!ws_ok(ws, ws_bytes, N, D, G, cov, &w)) return GMM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (cov == GMM_COV_FULL)
    return status_of(launch_loglik_full(X, N, D, ldx, G, hefts, means, covs, mean_loglik,
                                        per_sample, dev_status, w, st));
  return status_of(launch_loglik_diag(X, N, D, ldx, G, hefts, means, covs, prec, mean_loglik,
                                      per_sample, dev_status, w, st));
}

int gmm_assign(const float* X, int64_t N, int32_t D, int64_t ldx, int32_t G, int32_t mode,
               const float* hefts, const float* means, const float* dcovs, int32_t* assign,
               int64_t* hist, int32_t* dev_status, void* ws, size_t ws_bytes,
               gmm_stream_t stream) {
  if (!X || !means || !assign || !dev_status) return GMM_EINVAL;
  if (!shape_ok(N, D, ldx, G)) return GMM_EINVAL;
  if (mode != GMM_ASSIGN_EUCL && mode != GMM_ASSIGN_PROB) return GMM_EINVAL;
  if (mode == GMM_ASSIGN_PROB && (!hefts || !dcovs)) return GMM_EINVAL;
  Workspace w;
  if (!ws_ok(ws, ws_bytes, N, D, G, GMM_COV_DIAG, &w)) return GMM_EINVAL;
  return status_of(launch_assign(X, N, D, ldx, G, mode, hefts, means, dcovs, assign, hist,
                                 dev_status, w, (hipStream_t)stream));
}

}  // extern "C"
