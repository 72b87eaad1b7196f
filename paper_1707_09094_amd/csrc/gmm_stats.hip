// gmm_stats.hip -- global per-dimension mean and population variance in FP64,
// the global diagonal covariance of the Mahalanobis k-means distance
// (Sec. 3.1, Eq. 20).  Two passes over the data (mean, then centred squares),
// each reduced through fixed-order per-block FP64 partials.
#include "gmm_internal.hpp"

namespace gmm {

namespace {

constexpr int kNT = 256;

// Block b owns the contiguous sample range [b*chunk, min(N, (b+1)*chunk)).
// Thread t owns dimensions t, t+256, ...; it walks the block's samples in
// order, so every partial is a sequential FP64 sum.  When `mean` is non-null
// the pass sums squared deviations from it.
__global__ void __launch_bounds__(kNT) k_colsum(const float* __restrict__ X, int64_t N, int D,
                                                int64_t ldx, int64_t chunk,
                                                const double* __restrict__ mean,
                                                double* __restrict__ part) {
  const int b = blockIdx.x;
  const int64_t i0 = (int64_t)b * chunk;
  const int64_t i1 = min(N, i0 + chunk);
  for (int d = threadIdx.x; d < D; d += kNT) {
    double acc = 0.0;
    const double mu = mean ? mean[d] : 0.0;
    for (int64_t i = i0; i < i1; ++i) {
      double v = (double)X[i * ldx + d];
      if (mean) {
        v -= mu;
        acc += v * v;
      } else {
        acc += v;
      }
    }
    part[(size_t)b * D + d] = acc;
  }
}

// out[d] = (sum over blocks in order) / N.
__global__ void __launch_bounds__(kNT) k_colfinish(const double* __restrict__ part, int nb, int D,
                                                   int64_t N, double* __restrict__ out) {
  for (int d = blockIdx.x * kNT + threadIdx.x; d < D; d += gridDim.x * kNT) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(size_t)b * D + d];
    out[d] = s / (double)N;
  }
}

}  // namespace

hipError_t launch_global_stats(const float* X, int64_t N, int D, int64_t ldx, double* mean,
                               double* var, const Workspace& w, hipStream_t st) {
  const int nb = partial_blocks(N, 256);
  const int64_t chunk = (N + nb - 1) / nb;
  const int fb = (D + kNT - 1) / kNT;
  hipLaunchKernelGGL(k_colsum, dim3(nb), dim3(kNT), 0, st, X, N, D, ldx, chunk, nullptr,
                     w.partials);
  hipLaunchKernelGGL(k_colfinish, dim3(fb), dim3(kNT), 0, st, w.partials, nb, D, N, mean);
  hipLaunchKernelGGL(k_colsum, dim3(nb), dim3(kNT), 0, st, X, N, D, ldx, chunk, mean,
                     w.partials);
  hipLaunchKernelGGL(k_colfinish, dim3(fb), dim3(kNT), 0, st, w.partials, nb, D, N, var);
  return hipGetLastError();
}

}  // namespace gmm
