// gmm_full.hip -- EM iteration and log-likelihood for full covariances
// (Eq. 2 with a general Sigma; Eq. 7 / Eq. 8 for the update).
//
//   k_pre_full     one workgroup per component: Cholesky Sigma_g = L L^T in
//                  FP64, log|Sigma_g| = 2 sum_d log L_dd, the inverse factor
//                  W_g = L^-1 by forward substitution in FP64 (stored rounded to
//                  FP32) and c_g = log w_g - 1/2 (D log 2pi + log|Sigma_g|)
//                  (hi/lo FP32).  A non-positive pivot sets GMM_DEV_NOTPD.
//   k_estep_full   a_gi = c_g - 1/2 ||W_g (x_i - mu_g)||^2, log-sum-exp,
//                  responsibilities, and per-block FP64 partials of
//                  L, sum l*y, sum l*y y^T (lower triangle, packed) with
//                  y = x - mu_old.
//   k_fin_full     fixed-order reduce, mu = mu_old + S1/L,
//                  Sigma = S2/L - dmu dmu^T, floor on the diagonal.
#include "gmm_internal.hpp"

namespace gmm {

namespace {

constexpr int kNT = 256;

__global__ void k_init_full(int32_t* dev_status, int64_t* n_recomputed) {
  if (threadIdx.x == 0) {
    *dev_status = 0;
    if (n_recomputed) *n_recomputed = 0;
  }
}

// scratch: FP64 [G][D][D] factor L (column-major, L[e*D + d] = L_{d,e})
// followed by FP64 [G][D][D] inverse (row-major, Wi[r*D + c] = W_{r,c}).
__global__ void __launch_bounds__(kNT) k_pre_full(const float* __restrict__ hefts,
                                                  const float* __restrict__ covs, int D, int G,
                                                  double* __restrict__ scratch,
                                                  float* __restrict__ W_out,
                                                  double* __restrict__ W64_out,
                                                  float* __restrict__ c_out,
                                                  double* __restrict__ c64_out,
                                                  int32_t* __restrict__ dev_status) {
  __shared__ double diag;
  __shared__ int notpd;
  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const size_t DD = (size_t)D * D;
  const float* S = covs + DD * g;
  double* L = scratch + DD * g;
  double* Wi = scratch + DD * ((size_t)G + g);
  if (tid == 0) notpd = 0;
  for (size_t p = tid; p < DD; p += kNT) L[p] = 0.0;
  __syncthreads();
  for (int j = 0; j < D; ++j) {
    if (tid == 0) {
      double s = (double)S[(size_t)j * D + j];
      for (int k = 0; k < j; ++k) s -= L[(size_t)k * D + j] * L[(size_t)k * D + j];
      if (!(s > 0.0)) {
        notpd = 1;
        s = 1.0;  // keep going; the outputs are flagged invalid
      }
      diag = sqrt(s);
      L[(size_t)j * D + j] = diag;
    }
    __syncthreads();
    const double ljj = diag;
    for (int i = j + 1 + tid; i < D; i += kNT) {
      double t = (double)S[(size_t)j * D + i];
      for (int k = 0; k < j; ++k) t -= L[(size_t)k * D + i] * L[(size_t)k * D + j];
      L[(size_t)j * D + i] = t / ljj;
    }
    __syncthreads();
  }
  // Column c of W = L^-1 solves L w = e_c: w_r = 0 (r < c), then forward
  // substitution.  Thread c owns column c of Wi.
  for (int c = tid; c < D; c += kNT) {
    for (int r = 0; r < c; ++r) Wi[(size_t)r * D + c] = 0.0;
    for (int r = c; r < D; ++r) {
      double t = (r == c) ? 1.0 : 0.0;
      for (int k = c; k < r; ++k) t -= L[(size_t)k * D + r] * Wi[(size_t)k * D + c];
      Wi[(size_t)r * D + c] = t / L[(size_t)r * D + r];
    }
  }
  __syncthreads();
  float* Wg = W_out + DD * g;
  double* Wg64 = W64_out + DD * g;
  for (size_t p = tid; p < DD; p += kNT) {
    Wg[p] = (float)Wi[p];
    Wg64[p] = Wi[p];
  }
  if (tid == 0) {
    double ld = 0.0;
    for (int d = 0; d < D; ++d) ld += log(L[(size_t)d * D + d]);
    const double c = log((double)hefts[g]) - 0.5 * ((double)D * kLog2Pi + 2.0 * ld);
    const float hi = (float)c;
    c_out[g] = hi;
    c_out[G + g] = isfinite(c) ? (float)(c - (double)hi) : 0.0f;
    c64_out[g] = c;
    if (notpd) atomicOr(dev_status, GMM_DEV_NOTPD);
  }
}

// Packed lower-triangle index of (d, e), d >= e: column e starts at
// e*D - e*(e-1)/2.
__device__ __forceinline__ int tri_index(int d, int e, int D) { return e * D - (e * (e - 1)) / 2 + (d - e); }

template <bool MSTEP>
__global__ void __launch_bounds__(kNT) k_estep_full(
    const float* __restrict__ X, int64_t N, int D, int64_t ldx, int G, int T, int64_t chunk,
    const float* __restrict__ W, const float* __restrict__ cc, const double* __restrict__ W64,
    const double* __restrict__ c64, const float* __restrict__ means,
    double* __restrict__ part, double* __restrict__ ll_part, float* __restrict__ per_sample,
    int32_t* __restrict__ dev_status) {
  extern __shared__ float lds[];
  const int DS = D + 1;             // padded row stride (conflict-free column reads)
  float* xs = lds;                  // [T][D+1]
  float* as = xs + (size_t)T * DS;  // [T][G]
  double* lse = (double*)(as + (size_t)T * G + ((T * G) & 1));  // [T]
  uint32_t* gbits = (uint32_t*)(lse + T);  // [G/32]: component has a non-zero r in the tile
  const int NGB = (G + 31) / 32;
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wid = tid / kWave;
  const int nw = kNT / kWave;
  const int b = blockIdx.x;
  const int64_t i0 = (int64_t)b * chunk;
  const int64_t i1 = min(N, i0 + chunk);
  const int NT2 = D * (D + 1) / 2;
  const int P = 1 + D + NT2;
  double* pb = part + (size_t)b * G * P;
  if (tid == 0) bad = 0;
  if (MSTEP)
    for (int p = tid; p < G * P; p += kNT) pb[p] = 0.0;
  double llacc = 0.0;
  __syncthreads();
  for (int64_t t0 = i0; t0 < i1; t0 += T) {
    const int nt = (int)min((int64_t)T, i1 - t0);
    for (int p = tid; p < nt * D; p += kNT) {
      const int t = p / D, d = p - t * D;
      xs[(size_t)t * DS + d] = X[(t0 + t) * ldx + d];
    }
    for (int p = tid; p < NGB; p += kNT) gbits[p] = 0u;
    __syncthreads();
    // a_gi: wave per component (W_g and mu_g read uniformly), lane per sample
    for (int g = __builtin_amdgcn_readfirstlane(wid); g < G; g += nw) {
      const float* mu = means + (size_t)g * D;
      const float* Wg = W + (size_t)g * D * D;
      const float cg = cc[g], cl = cc[G + g];
      for (int t = lane; t < nt; t += kWave) {
        const float* x = xs + (size_t)t * DS;
        float acc = 0.0f;
        for (int r = 0; r < D; ++r) {
          float z = 0.0f;
          for (int c = 0; c <= r; ++c) z = fmaf(Wg[(size_t)r * D + c], x[c] - mu[c], z);
          acc = fmaf(z, z, acc);
        }
        as[(size_t)t * G + g] = (cg - 0.5f * acc) + cl;
      }
    }
    __syncthreads();
    // Screening in FP32, FP64 recompute of the near set (see the diagonal
    // kernel): a64 = c_g - 1/2 ||W_g (x - mu_g)||^2 with W_g = L_g^-1 in FP64;
    // lanes own rows r of the triangular product.
    for (int t = wid; t < nt; t += nw) {
      float* a = as + (size_t)t * G;
      const float* x = xs + (size_t)t * DS;
      float mx = -INFINITY;
      for (int g = lane; g < G; g += kWave) mx = fmaxf(mx, a[g]);
      mx = wave_max(mx);
      const double M = (double)mx;
      unsigned long long nearbits = 0;
      for (int c = 0, g0 = 0; g0 < G; ++c, g0 += kWave) {
        const int g = g0 + lane;
        const bool near = g < G && a[g] >= mx - kNearGap;
        if (near) nearbits |= 1ull << c;
        unsigned long long msk = __ballot(near);
        while (msk) {
          const int j = __ffsll((long long)msk) - 1;
          msk &= msk - 1;
          const int gg = g0 + j;
          const double* Wg = W64 + (size_t)gg * D * D;
          const float* mu = means + (size_t)gg * D;
          double q = 0.0;
          for (int r = lane; r < D; r += kWave) {
            double z = 0.0;
            for (int cc2 = 0; cc2 <= r; ++cc2)
              z += Wg[(size_t)r * D + cc2] * ((double)x[cc2] - (double)mu[cc2]);
            q += z * z;
          }
          q = wave_sum_d(q);
          if (lane == j) a[gg] = (float)(c64[gg] - 0.5 * q - M);
        }
      }
      double sm = 0.0;
      for (int c = 0, g0 = 0; g0 < G; ++c, g0 += kWave) {
        const int g = g0 + lane;
        if (g < G) sm += (double)__expf(((nearbits >> c) & 1ull) ? a[g] : a[g] - mx);
      }
      sm = wave_sum_d(sm);
      const double l = M + log(sm);
      if (MSTEP) {
        const float dl = (float)(l - M);
        for (int c = 0, g0 = 0; g0 < G; ++c, g0 += kWave) {
          const int g = g0 + lane;
          if (g < G) {
            const float z = (((nearbits >> c) & 1ull) ? a[g] : a[g] - mx) - dl;
            const float r = z >= -kRespCut ? __expf(z) : 0.0f;
            a[g] = r;
            if (r != 0.0f) atomicOr(&gbits[g >> 5], 1u << (g & 31));
          }
        }
      }
      if (lane == 0) {
        lse[t] = l;
        if (!isfinite(l)) bad = 1;
        if (per_sample) per_sample[t0 + t] = (float)l;
      }
    }
    __syncthreads();
    if (tid == 0)
      for (int t = 0; t < nt; ++t) llacc += lse[t];
    if (MSTEP) {
      // entry k of component g: 0 -> L, 1..D -> sum r y_d, then the packed
      // lower triangle sum r y_d y_e (d >= e, column e after column e-1).
      // Wave per component with a non-zero responsibility in the tile, lanes
      // over entries; the tile's contributions are added to the partials once.
      for (int g = wid; g < G; g += nw) {
        if (!((gbits[g >> 5] >> (g & 31)) & 1u)) continue;
        double* q = pb + (size_t)g * P;
        for (int k = lane; k < P; k += kWave) {
          int d = 0, e = 0;
          if (k >= 1 && k <= D) {
            d = k - 1;
          } else if (k > D) {
            int qq = k - 1 - D;
            while (qq >= D - e) {
              qq -= D - e;
              ++e;
            }
            d = e + qq;
          }
          const float mud = means[(size_t)g * D + d];
          const float mue = means[(size_t)g * D + e];
          double s = 0.0;
          for (int t = 0; t < nt; ++t) {
            const float r = as[(size_t)t * G + g];
            if (r != 0.0f) {
              if (k == 0) {
                s += (double)r;
              } else if (k <= D) {
                s += (double)r * (double)(xs[(size_t)t * DS + d] - mud);
              } else {
                s += (double)r * (double)(xs[(size_t)t * DS + d] - mud) *
                     (double)(xs[(size_t)t * DS + e] - mue);
              }
            }
          }
          q[k] += s;
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    ll_part[b] = llacc;
    if (bad) atomicOr(dev_status, GMM_DEV_NONFINITE);
  }
}

__global__ void __launch_bounds__(kNT) k_fin_full(const double* __restrict__ part, int nb, int64_t N,
                                                  int D, int G, float var_floor,
                                                  float* __restrict__ hefts,
                                                  float* __restrict__ means,
                                                  float* __restrict__ covs,
                                                  const double* __restrict__ ll_part,
                                                  double* __restrict__ mean_loglik,
                                                  int32_t* __restrict__ dev_status) {
  extern __shared__ double tot[];  // [P]
  __shared__ int bad;
  const int g = blockIdx.x;
  const int P = 1 + D + D * (D + 1) / 2;
  if (threadIdx.x == 0) bad = 0;
  for (int j = threadIdx.x; j < P; j += kNT) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[((size_t)b * G + g) * P + j];
    tot[j] = s;
  }
  __syncthreads();
  const double L = tot[0];
  if (threadIdx.x == 0) {
    hefts[g] = (float)(L / (double)N);
    if (!isfinite(L)) bad = 1;
  }
  if (L > 0.0) {
    float* C = covs + (size_t)g * D * D;
    const float* mo = means + (size_t)g * D;
    for (int p = threadIdx.x; p < D * D; p += kNT) {
      const int e = p / D, d = p - e * D;  // element (d, e), column-major
      const int hi = d > e ? d : e, lo = d > e ? e : d;
      const double dmh = tot[1 + hi] / L, dml = tot[1 + lo] / L;
      double v = tot[1 + D + tri_index(hi, lo, D)] / L - dmh * dml;
      if (d == e) {
        v = v > 0.0 ? v : 0.0;
        v = v > (double)var_floor ? v : (double)var_floor;
      }
      C[p] = (float)v;
      if (!isfinite(v)) bad = 1;
    }
    __syncthreads();  // every thread has read the old means through tot only
    for (int d = threadIdx.x; d < D; d += kNT) {
      const double mu = (double)mo[d] + tot[1 + d] / L;
      means[(size_t)g * D + d] = (float)mu;
      if (!isfinite(mu)) bad = 1;
    }
  }
  if (g == 0 && threadIdx.x == 0 && mean_loglik) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += ll_part[b];
    *mean_loglik = s / (double)N;
    if (!isfinite(s)) bad = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0 && bad) atomicOr(dev_status, GMM_DEV_NONFINITE);
}

__global__ void k_ll_finish_full(const double* __restrict__ ll_part, int nb, int64_t N,
                                 double* __restrict__ mean_loglik,
                                 int32_t* __restrict__ dev_status) {
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += ll_part[b];
    *mean_loglik = s / (double)N;
    if (!isfinite(s)) atomicOr(dev_status, GMM_DEV_NONFINITE);
  }
}

int tile_rows_full(int D, int G) {
  int T = 64;
  while (T > 1 && (size_t)T * (D + G + 3) * sizeof(float) + (size_t)(G / 8 + 8) > 60 * 1024)
    T >>= 1;
  return T;
}

}  // namespace

hipError_t launch_em_full(const float* X, int64_t N, int D, int64_t ldx, int G, float* hefts,
                          float* means, float* covs, float var_floor, double* mean_loglik,
                          int64_t* n_recomputed, int32_t* dev_status, const Workspace& w,
                          hipStream_t st) {
  const int T = tile_rows_full(D, G);
  const int nb = partial_blocks(N, 4 * T);
  const int64_t chunk = (N + nb - 1) / nb;
  const int P = 1 + D + D * (D + 1) / 2;
  const size_t lds = sizeof(float) * ((size_t)T * (D + 1 + G) + 1) + sizeof(double) * T +
                     sizeof(uint32_t) * ((G + 31) / 32);
  hipLaunchKernelGGL(k_init_full, dim3(1), dim3(64), 0, st, dev_status, n_recomputed);
  hipLaunchKernelGGL(k_pre_full, dim3(G), dim3(kNT), 0, st, hefts, covs, D, G, w.partials, w.W,
                     w.W64, w.c, w.c64, dev_status);
  {
    ProfScope ps(kProfEM, st);
    hipLaunchKernelGGL(k_estep_full<true>, dim3(nb), dim3(kNT), lds, st, X, N, D, ldx, G, T,
                       chunk, w.W, w.c, w.W64, w.c64, means, w.partials, w.scalars, nullptr,
                       dev_status);
  }
  hipLaunchKernelGGL(k_fin_full, dim3(G), dim3(kNT), sizeof(double) * P, st, w.partials, nb, N, D,
                     G, var_floor, hefts, means, covs, w.scalars, mean_loglik, dev_status);
  return hipGetLastError();
}

hipError_t launch_loglik_full(const float* X, int64_t N, int D, int64_t ldx, int G,
                              const float* hefts, const float* means, const float* covs,
                              double* mean_loglik, float* per_sample, int32_t* dev_status,
                              const Workspace& w, hipStream_t st) {
  const int T = tile_rows_full(D, G);
  const int nb = partial_blocks(N, 4 * T);
  const int64_t chunk = (N + nb - 1) / nb;
  const size_t lds = sizeof(float) * ((size_t)T * (D + 1 + G) + 1) + sizeof(double) * T +
                     sizeof(uint32_t) * ((G + 31) / 32);
  hipLaunchKernelGGL(k_init_full, dim3(1), dim3(64), 0, st, dev_status, nullptr);
  hipLaunchKernelGGL(k_pre_full, dim3(G), dim3(kNT), 0, st, hefts, covs, D, G, w.partials, w.W,
                     w.W64, w.c, w.c64, dev_status);
  {
    ProfScope ps(kProfLoglik, st);
    hipLaunchKernelGGL(k_estep_full<false>, dim3(nb), dim3(kNT), lds, st, X, N, D, ldx, G, T,
                       chunk, w.W, w.c, w.W64, w.c64, means, w.partials, w.scalars, per_sample,
                       dev_status);
  }
  hipLaunchKernelGGL(k_ll_finish_full, dim3(1), dim3(64), 0, st, w.scalars, nb, N, mean_loglik,
                     dev_status);
  return hipGetLastError();
}

}  // namespace gmm
