// gmm_stats.hip -- global per-dimension mean and population variance in FP64,
// the global diagonal covariance of the Mahalanobis k-means distance
// (Sec. 3.1, Eq. 20), in one pass over the data.
//
// Every value is taken relative to a per-dimension shift s_d (sample 0's
// value): S1_d = sum_i (x_id - s_d), S2_d = sum_i (x_id - s_d)^2 in FP64, then
// mean = s + S1/N and var = S2/N - (S1/N)^2.  The subtraction loses about
// log10(1 + (mean - s)^2 / var) digits of FP64's sixteen (one digit for a
// sample three standard deviations out), so the result matches the two-pass
// definition to far below the FP32 data's own resolution.
//
// Workgroups own contiguous sample ranges.  Inside one, the threads form a
// grid of R rows x C column groups of VEC consecutive dimensions (float4 loads
// when rows are 16-byte aligned): thread (r, c) takes samples r, r + R, ... of
// the range, eight loads in flight, so every thread reads while the whole row
// of D values is covered (at D = 100: 20 rows x 25 groups of four, 500 of 512
// threads).  Rows are combined in a fixed order, then workgroups in a fixed
// order by k_gstats_finish: results are bitwise repeatable.
#include "gmm_internal.hpp"

namespace gmm {

namespace {

constexpr int kNT = 512;  // threads of k_gstats (two workgroups per CU)
constexpr int kUnroll = 8;  // loads in flight per thread

// XT: float (VEC 4 or 1) or double (VEC 2 or 1) samples; VEC values per load.
template <typename XT, int VEC>
__global__ void __launch_bounds__(kNT) k_gstats(const XT* __restrict__ X, int64_t N, int D,
                                                int64_t ldx, int64_t chunk,
                                                double* __restrict__ part) {
  __shared__ double sh[2 * VEC * kNT];  // [row][group][VEC][S1, S2]
  const int C = (D + VEC - 1) / VEC;    // column groups of the whole row
  const int c0 = blockIdx.y * kNT;      // this workgroup's first group
  const int Cb = min(kNT, C - c0);
  const int R = kNT / Cb;
  const int tid = threadIdx.x;
  const int r = tid / Cb, c = tid - (tid / Cb) * Cb;
  const int d0 = (c0 + c) * VEC;
  const int b = blockIdx.x;
  const int64_t i0 = (int64_t)b * chunk;
  const int64_t i1 = min(N, i0 + chunk);
  double s1[VEC], s2[VEC];
#pragma unroll
  for (int k = 0; k < VEC; ++k) s1[k] = s2[k] = 0.0;
  if (r < R) {
    XT sh0[VEC];
#pragma unroll
    for (int k = 0; k < VEC; ++k) sh0[k] = X[min(d0 + k, D - 1)];
    auto add = [&](const XT* v) {
#pragma unroll
      for (int k = 0; k < VEC; ++k) {
        const double t = (double)v[k] - (double)sh0[k];
        s1[k] += t;
        s2[k] = fma(t, t, s2[k]);
      }
    };
    auto load = [&](int64_t i, XT* v) {
      const XT* p = X + i * ldx + d0;
      if constexpr (VEC == 4) {
        const float4 q = *(const float4*)p;
        v[0] = q.x;
        v[1] = q.y;
        v[2] = q.z;
        v[3] = q.w;
      } else if constexpr (VEC == 2) {
        const double2 q = *(const double2*)p;
        v[0] = q.x;
        v[1] = q.y;
      } else {
        v[0] = *p;
      }
    };
    int64_t i = i0 + r;
    for (; i + (kUnroll - 1) * (int64_t)R < i1; i += kUnroll * (int64_t)R) {
      XT v[kUnroll][VEC];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) load(i + u * (int64_t)R, v[u]);
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) add(v[u]);
    }
    for (; i < i1; i += R) {
      XT v[VEC];
      load(i, v);
      add(v);
    }
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      sh[((r * Cb + c) * VEC + k) * 2] = s1[k];
      sh[((r * Cb + c) * VEC + k) * 2 + 1] = s2[k];
    }
  }
  __syncthreads();
  for (int q = tid; q < Cb * VEC; q += kNT) {
    const int cc = q / VEC, k = q - cc * VEC;
    const int d = c0 * VEC + q;
    if (d >= D) continue;
    double a = 0.0, e = 0.0;
    for (int rr = 0; rr < R; ++rr) {
      a += sh[((rr * Cb + cc) * VEC + k) * 2];
      e += sh[((rr * Cb + cc) * VEC + k) * 2 + 1];
    }
    part[(size_t)b * 2 * D + d] = a;
    part[(size_t)b * 2 * D + D + d] = e;
  }
}

// mean_d = s_d + S1_d / N, var_d = S2_d / N - (S1_d / N)^2, the workgroups'
// partials summed in order.  One workgroup per dimension: its threads load the
// nb partials into LDS together, then one thread adds them in order (the
// arithmetic of a plain sequential loop, without its chain of dependent
// loads).
constexpr int kFT = 256;
template <typename XT>
__global__ void __launch_bounds__(kFT) k_gstats_finish(const XT* __restrict__ X,
                                                       const double* __restrict__ part, int nb,
                                                       int D, int64_t N,
                                                       double* __restrict__ mean,
                                                       double* __restrict__ var) {
  __shared__ double s1[kMaxBlocks], s2[kMaxBlocks];
  const int d = blockIdx.x;
  for (int b = threadIdx.x; b < nb; b += kFT) {
    s1[b] = part[(size_t)b * 2 * D + d];
    s2[b] = part[(size_t)b * 2 * D + D + d];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, e = 0.0;
    for (int b = 0; b < nb; ++b) {
      a += s1[b];
      e += s2[b];
    }
    const double m1 = a / (double)N;
    const double v = e / (double)N - m1 * m1;
    mean[d] = (double)X[d] + m1;
    var[d] = v > 0.0 ? v : 0.0;
  }
}

template <typename XT>
hipError_t global_stats_t(const XT* X, int64_t N, int D, int64_t ldx, double* mean, double* var,
                          const Workspace& w, hipStream_t st) {
  // the partial region holds kMaxBlocks x (2D + 1) doubles
  const int nb = partial_blocks(N, 1024);
  const int64_t chunk = (N + nb - 1) / nb;
  constexpr int V = sizeof(XT) == 4 ? 4 : 2;  // 16-byte loads
  const bool vec = D % V == 0 && ldx % V == 0 && ((uintptr_t)X) % 16 == 0;
  const int C = vec ? D / V : D;
  const dim3 grid(nb, (C + kNT - 1) / kNT);
  ProfScope ps(kProfStats, st);
  if (vec)
    hipLaunchKernelGGL((k_gstats<XT, V>), grid, dim3(kNT), 0, st, X, N, D, ldx, chunk,
                       w.partials);
  else
    hipLaunchKernelGGL((k_gstats<XT, 1>), grid, dim3(kNT), 0, st, X, N, D, ldx, chunk,
                       w.partials);
  hipLaunchKernelGGL(k_gstats_finish<XT>, dim3(D), dim3(kFT), 0, st, X,
                     (const double*)w.partials, nb, D, N, mean, var);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_global_stats(const float* X, int64_t N, int D, int64_t ldx, double* mean,
                               double* var, const Workspace& w, hipStream_t st) {
  return global_stats_t<float>(X, N, D, ldx, mean, var, w, st);
}

hipError_t launch_global_stats_f64(const double* X, int64_t N, int D, int64_t ldx, double* mean,
                                   double* var, const Workspace& w, hipStream_t st) {
  return global_stats_t<double>(X, N, D, ldx, mean, var, w, st);
}

}  // namespace gmm
