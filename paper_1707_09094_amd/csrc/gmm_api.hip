// gmm_api.hip -- the extern "C" entry points declared in include/gmm.h:
// host-side argument validation (everything is checked before the first
// enqueue, so a rejected call writes nothing), workspace carving, dispatch.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

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

// ---- autotune cache: key -> chosen work-item size ---------------------------
// Keyed by (GPU architecture, D, largest G, log2 of the batch's total N, log2
// of the model count, arithmetic form, covariance type).  Loaded from the file
// named by GMM_AUTOTUNE_CACHE at first use after a clear; new entries are
// appended to it as "key chunk" lines.
std::mutex g_tune_mu;
std::map<std::string, int32_t> g_tune;
bool g_tune_loaded = false;

int ilog2_floor(int64_t v) {
  int r = 0;
  while (v > 1) {
    v >>= 1;
    ++r;
  }
  return r;
}

bool tune_key(int32_t n_models, const int64_t* Ns, const int32_t* Gs, int32_t D, int32_t prec,
              std::string* key) {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return false;
  int64_t sumN = 0;
  int32_t gmax = 0;
  for (int m = 0; m < n_models; ++m) {
    sumN += Ns[m];
    gmax = Gs[m] > gmax ? Gs[m] : gmax;
  }
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s|D%d|G%d|N%d|M%d|p%d|diag", prop.gcnArchName, (int)D,
                (int)gmax, ilog2_floor(sumN), ilog2_floor(n_models), (int)prec);
  for (char* c = buf; *c; ++c)
    if (*c == ' ') *c = '_';
  *key = buf;
  return true;
}

// with g_tune_mu held
void tune_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("GMM_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char k[256];
  int v = 0;
  while (std::fscanf(f, "%255s %d", k, &v) == 2)
    if (v > 0) g_tune[k] = v;
  std::fclose(f);
}

void tune_store(const std::string& key, int32_t chunk) {
  g_tune[key] = chunk;
  const char* path = std::getenv("GMM_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d\n", key.c_str(), (int)chunk);
  std::fclose(f);
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

int gmm_seed_means(const float* X, int64_t N, int32_t D, int64_t ldx, int32_t G, int32_t mode,
                   const double* gvar, float var_floor, int64_t first, const int64_t* idx,
                   float* means, int32_t* dev_status, void* ws, size_t ws_bytes,
                   gmm_stream_t stream) {
  if (!X || !means || !dev_status) return GMM_EINVAL;
  if (!shape_ok(N, D, ldx, G)) return GMM_EINVAL;
  if (mode != GMM_SEED_SUBSET && mode != GMM_SEED_SPREAD) return GMM_EINVAL;
  if (mode == GMM_SEED_SPREAD && (first < 0 || first >= N)) return GMM_EINVAL;
  if (!(var_floor >= 0.0f)) return GMM_EINVAL;
  Workspace w;
  if (!ws_ok(ws, ws_bytes, N, D, G, GMM_COV_DIAG, &w)) return GMM_EINVAL;
  return status_of(launch_seed_means(X, N, D, ldx, G, mode, gvar, var_floor, first, idx, means,
                                     dev_status, w, (hipStream_t)stream));
}

int gmm_log_p_gaussian(const float* X, int64_t N, int32_t D, int64_t ldx, int32_t G, int32_t g,
                       const float* means, const float* dcovs, double* mean_out,
                       float* per_sample, int32_t* dev_status, void* ws, size_t ws_bytes,
                       gmm_stream_t stream) {
  if (!X || !means || !dcovs || !dev_status || (!mean_out && !per_sample)) return GMM_EINVAL;
  if (!shape_ok(N, D, ldx, G) || g < 0 || g >= G) return GMM_EINVAL;
  Workspace w;
  if (!ws_ok(ws, ws_bytes, N, D, G, GMM_COV_DIAG, &w)) return GMM_EINVAL;
  return status_of(launch_log_p_gaussian(X, N, D, ldx, g, means, dcovs, mean_out, per_sample,
                                         dev_status, w, (hipStream_t)stream));
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

// ---- FP64 data ---------------------------------------------------------------

size_t gmm_workspace_bytes_f64(int64_t N, int32_t D, int32_t G) {
  if (!shape_ok(N, D, D, G) || !em_f64_supported(D, G)) return 0;
  Workspace w;
  carve(nullptr, 0, N, D, G, GMM_COV_DIAG, &w);
  return w.bytes;
}

int gmm_global_stats_f64(const double* X, int64_t N, int32_t D, int64_t ldx, double* mean_out,
                         double* var_out, void* ws, size_t ws_bytes, gmm_stream_t stream) {
  if (!X || !mean_out || !var_out || !shape_ok(N, D, ldx, 1)) return GMM_EINVAL;
  Workspace w;
  if (!ws_ok(ws, ws_bytes, N, D, 1, GMM_COV_DIAG, &w)) return GMM_EINVAL;
  return status_of(
      launch_global_stats_f64(X, N, D, ldx, mean_out, var_out, w, (hipStream_t)stream));
}

int gmm_kmeans_iter_f64(const double* X, int64_t N, int32_t D, int64_t ldx, int32_t G,
                        int32_t dist, const double* gvar, double var_floor, double* means,
                        double* dcovs, double* hefts, int64_t* counts, int32_t* assign,
                        double* inertia, int64_t* n_recomputed, int32_t* dev_status, void* ws,
                        size_t ws_bytes, gmm_stream_t stream) {
  if (!X || !means || !dcovs || !hefts || !counts || !inertia || !dev_status) return GMM_EINVAL;
  if (!shape_ok(N, D, ldx, G) || !em_f64_supported(D, G)) return GMM_EINVAL;
  if (dist != GMM_DIST_EUCL && dist != GMM_DIST_MAHA) return GMM_EINVAL;
  if (dist == GMM_DIST_MAHA && !gvar) return GMM_EINVAL;
  if (!(var_floor >= 0.0)) return GMM_EINVAL;
  Workspace w;
  if (!ws_ok(ws, ws_bytes, N, D, G, GMM_COV_DIAG, &w)) return GMM_EINVAL;
  return status_of(launch_kmeans_f64(X, N, D, ldx, G, dist, gvar, var_floor, means, dcovs, hefts,
                                     counts, assign, inertia, n_recomputed, dev_status, w,
                                     (hipStream_t)stream));
}

int gmm_em_iter_f64(const double* X, int64_t N, int32_t D, int64_t ldx, int32_t G,
                    double* hefts, double* means, double* dcovs, double var_floor,
                    double* mean_loglik, int32_t* dev_status, void* ws, size_t ws_bytes,
                    gmm_stream_t stream) {
  if (!X || !hefts || !means || !dcovs || !mean_loglik || !dev_status) return GMM_EINVAL;
  if (!shape_ok(N, D, ldx, G) || !em_f64_supported(D, G)) return GMM_EINVAL;
  if (!(var_floor >= 0.0)) return GMM_EINVAL;
  Workspace w;
  if (!ws_ok(ws, ws_bytes, N, D, G, GMM_COV_DIAG, &w)) return GMM_EINVAL;
  return status_of(launch_em_diag_f64(X, N, D, ldx, G, hefts, means, dcovs, var_floor,
                                      mean_loglik, dev_status, w, (hipStream_t)stream));
}

int gmm_loglik_f64(const double* X, int64_t N, int32_t D, int64_t ldx, int32_t G,
                   const double* hefts, const double* means, const double* dcovs,
                   double* mean_loglik, double* per_sample, int32_t* dev_status, void* ws,
                   size_t ws_bytes, gmm_stream_t stream) {
  if (!X || !hefts || !means || !dcovs || !mean_loglik || !dev_status) return GMM_EINVAL;
  if (!shape_ok(N, D, ldx, G) || !em_f64_supported(D, G)) return GMM_EINVAL;
  Workspace w;
  if (!ws_ok(ws, ws_bytes, N, D, G, GMM_COV_DIAG, &w)) return GMM_EINVAL;
  return status_of(launch_loglik_diag_f64(X, N, D, ldx, G, hefts, means, dcovs, mean_loglik,
                                          per_sample, dev_status, w, (hipStream_t)stream));
}

int gmm_em_path(int32_t D, int32_t G, int32_t cov, int32_t prec) {
  if (!shape_ok(1, D, D, G)) return GMM_EINVAL;
  if (prec != GMM_PREC_FP32 && prec != GMM_PREC_BF16X3) return GMM_EINVAL;
  if (cov == GMM_COV_FULL)
    return D > kMaxDFull ? GMM_EINVAL : (D <= 64 ? GMM_PATH_FULL_FP64 : GMM_PATH_FULL_GENERIC);
  if (cov != GMM_COV_DIAG) return GMM_EINVAL;
  return em_diag_path(D, G, prec);
}

int gmm_kmeans_path(int32_t D, int32_t G, int32_t prec) {
  if (!shape_ok(1, D, D, G)) return GMM_EINVAL;
  if (prec != GMM_PREC_FP32 && prec != GMM_PREC_BF16X3) return GMM_EINVAL;
  return kmeans_path(D, G, prec);
}

// ---- many models -----------------------------------------------------------

}  // extern "C"

static_assert(sizeof(gmm_model_desc) == 96, "gmm_model_desc layout is part of the ABI");

namespace {

bool batch_shape_ok(const gmm_model_desc* models, int32_t n_models, const int64_t* Ns,
                    const int32_t* Gs, int32_t D, int32_t chunk, int* Gmax) {
  if (!models || !Ns || !Gs || n_models < 1 || D < 1 || D > kBatchMaxD) return false;
  if (chunk < 32 || chunk % 32 != 0) return false;
  int gm = 0;
  for (int m = 0; m < n_models; ++m) {
    if (Ns[m] < 1 || Ns[m] > ((int64_t)1 << 40) || Gs[m] < 1 || Gs[m] > kBatchMaxG) return false;
    gm = Gs[m] > gm ? Gs[m] : gm;
  }
  *Gmax = gm;
  return true;
}

bool batch_ws(void* ws, size_t ws_bytes, int32_t n_models, const int64_t* Ns, int D, int Gmax,
              int32_t chunk, BatchWorkspace* bw, int* n_items) {
  if (!ws || ((uintptr_t)ws) % 256 != 0) return false;
  const int cap = batch_item_count(n_models, Ns, chunk);
  if (cap < 1) return false;
  *n_items = cap;
  return carve_batched(ws, ws_bytes, n_models, D, Gmax, cap, bw);
}

}  // namespace

extern "C" {

size_t gmm_batched_workspace_bytes(int32_t n_models, const int64_t* Ns, const int32_t* Gs,
                                   int32_t D, int32_t chunk) {
  int Gmax = 0;
  if (!batch_shape_ok((const gmm_model_desc*)1, n_models, Ns, Gs, D, chunk, &Gmax)) return 0;
  const int cap = batch_item_count(n_models, Ns, chunk);
  if (cap < 1) return 0;
  BatchWorkspace bw;
  carve_batched(nullptr, 0, n_models, D, Gmax, cap, &bw);
  return bw.bytes;
}

static int em_batched_common(const gmm_model_desc* models, int32_t n_models, const int64_t* Ns,
                             const int32_t* Gs, int32_t D, float var_floor, int32_t prec,
                             int32_t chunk, void* ws, size_t ws_bytes, gmm_stream_t stream,
                             bool mstep) {
  int Gmax = 0, n_items = 0;
  if (!batch_shape_ok(models, n_models, Ns, Gs, D, chunk, &Gmax)) return GMM_EINVAL;
  if (prec != GMM_PREC_FP32 && prec != GMM_PREC_BF16X3) return GMM_EINVAL;
  if (!(var_floor >= 0.0f)) return GMM_EINVAL;
  if (!em_fast_supported(D, Gmax, prec)) return GMM_EINVAL;
  BatchWorkspace bw;
  if (!batch_ws(ws, ws_bytes, n_models, Ns, D, Gmax, chunk, &bw, &n_items)) return GMM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = launch_batch_plan(models, n_models, chunk, bw, st);
  if (e == hipSuccess)
    e = launch_em_batched(models, n_models, n_items, D, var_floor, prec, mstep, bw, st);
  return status_of(e);
}

int gmm_em_iter_batched(const gmm_model_desc* models, int32_t n_models, const int64_t* Ns,
                        const int32_t* Gs, int32_t D, float var_floor, int32_t prec,
                        int32_t chunk, void* ws, size_t ws_bytes, gmm_stream_t stream) {
  return em_batched_common(models, n_models, Ns, Gs, D, var_floor, prec, chunk, ws, ws_bytes,
                           stream, true);
}

int gmm_loglik_batched(const gmm_model_desc* models, int32_t n_models, const int64_t* Ns,
                       const int32_t* Gs, int32_t D, int32_t prec, int32_t chunk, void* ws,
                       size_t ws_bytes, gmm_stream_t stream) {
  return em_batched_common(models, n_models, Ns, Gs, D, 0.0f, prec, chunk, ws, ws_bytes, stream,
                           false);
}

int gmm_kmeans_iter_batched(const gmm_model_desc* models, int32_t n_models, const int64_t* Ns,
                            const int32_t* Gs, int32_t D, int32_t dist, float var_floor,
                            int32_t chunk, void* ws, size_t ws_bytes, gmm_stream_t stream) {
  int Gmax = 0, n_items = 0;
  if (!batch_shape_ok(models, n_models, Ns, Gs, D, chunk, &Gmax)) return GMM_EINVAL;
  if (dist != GMM_DIST_EUCL && dist != GMM_DIST_MAHA) return GMM_EINVAL;
  if (!(var_floor >= 0.0f)) return GMM_EINVAL;
  if (!km_fast_supported(D, Gmax)) return GMM_EINVAL;
  BatchWorkspace bw;
  if (!batch_ws(ws, ws_bytes, n_models, Ns, D, Gmax, chunk, &bw, &n_items)) return GMM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = launch_batch_plan(models, n_models, chunk, bw, st);
  if (e == hipSuccess)
    e = launch_kmeans_batched(models, n_models, n_items, D, dist, var_floor, bw, st);
  return status_of(e);
}

int gmm_global_stats_batched(const gmm_model_desc* models, int32_t n_models, int32_t D,
                             double* mean_out, double* var_out, gmm_stream_t stream) {
  if (!models || n_models < 1 || D < 1 || D > kBatchMaxD || !mean_out || !var_out)
    return GMM_EINVAL;
  return status_of(
      launch_global_stats_batched(models, n_models, D, mean_out, var_out, (hipStream_t)stream));
}

int gmm_batched_autotune(const gmm_model_desc* models, int32_t n_models, const int64_t* Ns,
                         const int32_t* Gs, int32_t D, int32_t prec, void* ws, size_t ws_bytes,
                         gmm_stream_t stream, int32_t* best_chunk) {
  if (!best_chunk || !Ns || !Gs || n_models < 1) return GMM_EINVAL;
  static const int32_t cand[] = {1024, 2048, 4096, 8192, 16384};
  std::string key;
  if (!tune_key(n_models, Ns, Gs, D, prec, &key)) return GMM_EHIP;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load();
    auto it = g_tune.find(key);
    if (it != g_tune.end() && ws_bytes >= gmm_batched_workspace_bytes(n_models, Ns, Gs, D,
                                                                       it->second)) {
      *best_chunk = it->second;
      return GMM_OK;
    }
  }
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return GMM_EHIP;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return GMM_EHIP;
  }
  float best = 0.0f;
  int32_t pick = 0;
  int rc = GMM_OK;
  for (int32_t c : cand) {
    if (ws_bytes < gmm_batched_workspace_bytes(n_models, Ns, Gs, D, c)) continue;
    rc = gmm_loglik_batched(models, n_models, Ns, Gs, D, prec, c, ws, ws_bytes, stream);
    if (rc != GMM_OK) break;
    float ms = 0.0f;
    if (hipEventRecord(a, st) != hipSuccess) { rc = GMM_EHIP; break; }
    for (int r = 0; r < 2 && rc == GMM_OK; ++r)
      rc = gmm_loglik_batched(models, n_models, Ns, Gs, D, prec, c, ws, ws_bytes, stream);
    if (rc != GMM_OK) break;
    if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
        hipEventElapsedTime(&ms, a, b) != hipSuccess) {
      rc = GMM_EHIP;
      break;
    }
    if (pick == 0 || ms < best) {
      best = ms;
      pick = c;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc != GMM_OK) return rc;
  if (pick == 0) return GMM_EINVAL;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_store(key, pick);
  }
  *best_chunk = pick;
  return GMM_OK;
}

int gmm_autotune_cache_size(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return (int)g_tune.size();
}

int gmm_autotune_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  g_tune_loaded = false;
  return GMM_OK;
}

}  // extern "C"
