// gmm_kmeans.hip -- one k-means iteration (Sec. 3) and the assign() query of
// the Sec. 4 API, generic kernels for every accepted shape.
//
// Launch sequence of gmm_kmeans_iter:
//   k_km_pre        per-dimension distance weights lam_d: 1 (Euclidean) or
//                   1/max(global variance, floor) (Mahalanobis, Sec. 3.1
//                   Eq. 20), in FP64 and rounded to FP32
//   k_km_assign     hard assignment (Sec. 3, Eq. 19): FP32 direct-form
//                   distances, lowest index on ties; when the two best FP32
//                   distances are within twice their rounding-error bound the
//                   sample is re-decided in FP64, so the result is the FP64
//                   argmin.  (k_km_assign_f64, more than 128 components:
//                   FP64 matrix-core distances with the same gap test.)
//   k_km_accum      map step of Sec. 2.1 with hard l (Eqs. 9-11): per-block
//                   FP64 count, sum (x - mu_old), sum (x - mu_old)^2
//                   (k_km_accum_grp: components in LDS-sized groups)
//   k_km_fin        reduce step (Eqs. 12-14): new means, hand-off variances and
//                   weights (Sec. 3, Eqs. 5-7 with hard l), counts, and each
//                   component's inertia term sum_d lam_d sum (x - mu_old)^2
//   k_km_inertia    inertia = sum of those terms in component order
//   k_km_resurrect  dead-mean resurrection (Sec. 3.1), a single workgroup that
//                   does nothing unless some cluster is empty
#include <algorithm>

#include "gmm_internal.hpp"

namespace gmm {

namespace {

constexpr int kNT = 256;
constexpr int kRT = 1024;  // resurrection workgroup
constexpr float kU32 = 5.9604645e-08f;  // 2^-24

__global__ void k_km_init(int32_t* dev_status, int64_t* n_recomputed) {
  if (threadIdx.x == 0) {
    *dev_status = 0;
    if (n_recomputed) *n_recomputed = 0;
  }
}

__global__ void k_km_pre(const double* __restrict__ gvar, int D, float var_floor, int dist,
                         double* __restrict__ lam64, float* __restrict__ lam32) {
  for (int d = threadIdx.x + blockIdx.x * blockDim.x; d < D; d += blockDim.x * gridDim.x) {
    double l = 1.0;
    if (dist == GMM_DIST_MAHA) {
      double v = gvar[d];
      v = v > (double)var_floor ? v : (double)var_floor;
      l = 1.0 / v;
    }
    lam64[d] = l;
    lam32[d] = (float)l;
  }
}

// FP64 distance sum_d lam_d (x_d - mu_d)^2 of one sample to one mean.
__device__ __forceinline__ double dist64(const float* __restrict__ x, const float* __restrict__ mu,
                                         const double* __restrict__ lam, int D) {
  double s = 0.0;
  for (int d = 0; d < D; ++d) {
    const double t = (double)x[d] - (double)mu[d];
    s += lam[d] * t * t;
  }
  return s;
}

// One thread per sample (strided over the block's contiguous range).
// The FP32 sum of D non-negative terms, each with relative error <= 3u
// (difference, product, lam rounding), is within gamma = (D + 4) u of the
// exact value; the computed argmin is then provably the exact one when
// d2 - d1 > gamma (d1 + d2).  Twice that margin triggers the FP64 re-decision.
__global__ void __launch_bounds__(kNT) k_km_assign(
    const float* __restrict__ X, int64_t N, int D, int64_t ldx, int G, int64_t chunk,
    const float* __restrict__ means, const float* __restrict__ lam32,
    const double* __restrict__ lam64, int32_t* __restrict__ assign,
    int64_t* __restrict__ n_recomputed) {
  const int b = blockIdx.x;
  const int64_t i0 = (int64_t)b * chunk;
  const int64_t i1 = min(N, i0 + chunk);
  const float gamma = 2.0f * (float)(D + 4) * kU32;
  long long nrec = 0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kNT) {
    const float* x = X + i * ldx;
    float d1 = INFINITY, d2 = INFINITY;
    int arg = 0;
    for (int g = 0; g < G; ++g) {
      const float* mu = means + (size_t)g * D;
      float s = 0.0f;
      for (int d = 0; d < D; ++d) {
        const float t = x[d] - mu[d];
        s = fmaf(lam32[d] * t, t, s);
      }
      if (s < d1) {
        d2 = d1;
        d1 = s;
        arg = g;
      } else if (s < d2) {
        d2 = s;
      }
    }
    if (G > 1 && !(d2 - d1 > gamma * (d1 + d2))) {
      // near tie (or non-finite): decide in FP64, first minimum wins
      ++nrec;
      double best = INFINITY;
      arg = 0;
      for (int g = 0; g < G; ++g) {
        const double s = dist64(x, means + (size_t)g * D, lam64, D);
        if (s < best) {
          best = s;
          arg = g;
        }
      }
    }
    assign[i] = arg;
  }
  if (nrec) atomicAdd((unsigned long long*)n_recomputed, (unsigned long long)nrec);
}

// Per-block FP64 partials [G][2D+1]: count, sum y, sum y^2 with y = x - mu_old.
// Thread t owns dimensions t, t+256, ...; samples are visited in order.
__global__ void __launch_bounds__(kNT) k_km_accum(const float* __restrict__ X, int64_t N, int D,
                                                  int64_t ldx, int G, int64_t chunk,
                                                  const float* __restrict__ means,
                                                  const int32_t* __restrict__ assign,
                                                  double* __restrict__ part) {
  const int b = blockIdx.x;
  const int P = 2 * D + 1;
  double* pb = part + (size_t)b * G * P;
  for (int p = threadIdx.x; p < G * P; p += kNT) pb[p] = 0.0;
  __syncthreads();
  const int64_t i0 = (int64_t)b * chunk;
  const int64_t i1 = min(N, i0 + chunk);
  for (int64_t i = i0; i < i1; ++i) {
    const int g = assign[i];
    double* q = pb + (size_t)g * P;
    if (threadIdx.x == 0) q[0] += 1.0;
    for (int d = threadIdx.x; d < D; d += kNT) {
      const double y = (double)X[i * ldx + d] - (double)means[(size_t)g * D + d];
      q[1 + d] += y;
      q[1 + D + d] += y * y;
    }
  }
}

// Reduce step, one workgroup per component.  The inertia term of the
// component, sum_d lam_d sum_i (x_id - mu_gd)^2 about the input mean, comes
// from the same partials and is left in ig[g] for k_km_inertia.
template <typename XT>
__global__ void __launch_bounds__(kNT) k_km_fin(const double* __restrict__ part, int nb, int64_t N,
                                                int D, int G, double var_floor,
                                                const double* __restrict__ lam64,
                                                XT* __restrict__ means,
                                                XT* __restrict__ dcovs,
                                                XT* __restrict__ hefts,
                                                int64_t* __restrict__ counts,
                                                double* __restrict__ ig) {
  extern __shared__ double tot[];
  __shared__ double sh[kNT];
  const int g = blockIdx.x;
  const int P = 2 * D + 1;
  for (int j = threadIdx.x; j < P; j += kNT) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[((size_t)b * G + g) * P + j];
    tot[j] = s;
  }
  __syncthreads();
  const double c = tot[0];
  if (threadIdx.x == 0) {
    counts[g] = (int64_t)c;
    hefts[g] = (XT)(c / (double)N);
  }
  double in = 0.0;
  for (int d = threadIdx.x; d < D; d += kNT) {
    in += lam64[d] * tot[1 + D + d];
    if (c > 0.0) {
      const double dm = tot[1 + d] / c;
      double v = tot[1 + D + d] / c - dm * dm;
      v = v > 0.0 ? v : 0.0;
      v = v > var_floor ? v : var_floor;
      means[(size_t)g * D + d] = (XT)((double)means[(size_t)g * D + d] + dm);
      dcovs[(size_t)g * D + d] = (XT)v;
    } else {
      dcovs[(size_t)g * D + d] = (XT)1;
    }
  }
  in = block_sum_d<kNT>(in, sh);
  if (threadIdx.x == 0) ig[g] = in;
}

// Inertia = sum over components in index order.
__global__ void k_km_inertia(const double* __restrict__ ig, int G, double* __restrict__ inertia,
                             int32_t* __restrict__ dev_status) {
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += ig[g];
    *inertia = s;
    if (!isfinite(s)) atomicOr(dev_status, GMM_DEV_NONFINITE);
  }
}

// Dead-mean resurrection (Sec. 3.1), one workgroup.  rem/taken live in the
// (now free) partials area.
template <typename XT>
__global__ void __launch_bounds__(kRT) k_km_resurrect(const XT* __restrict__ X, int64_t N,
                                                      int D, int64_t ldx, int G,
                                                      const int64_t* __restrict__ counts,
                                                      const int32_t* __restrict__ assign,
                                                      XT* __restrict__ means,
                                                      int64_t* __restrict__ scratch) {
  __shared__ int any_dead;
  __shared__ long long s_val[kRT];
  __shared__ int s_idx[kRT];
  __shared__ long long s_cnt[kRT];
  __shared__ long long s_pick;
  const int tid = threadIdx.x;
  if (tid == 0) any_dead = 0;
  __syncthreads();
  for (int g = tid; g < G; g += kRT)
    if (counts[g] == 0) any_dead = 1;
  __syncthreads();
  if (!any_dead) return;
  int64_t* rem = scratch;
  int64_t* taken = scratch + G;
  for (int g = tid; g < G; g += kRT) {
    rem[g] = counts[g];
    taken[g] = 0;
  }
  __syncthreads();
  const int64_t slice = (N + kRT - 1) / kRT;
  for (int g = 0; g < G; ++g) {
    if (counts[g] != 0) continue;  // uniform across the workgroup
    // donor: largest remaining count, lowest index on ties
    long long bv = -1;
    int bi = 0;
    for (int k = tid; k < G; k += kRT)
      if ((long long)rem[k] > bv) {
        bv = rem[k];
        bi = k;
      }
    s_val[tid] = bv;
    s_idx[tid] = bi;
    __syncthreads();
    for (int s = kRT / 2; s > 0; s >>= 1) {
      if (tid < s) {
        const long long ov = s_val[tid + s];
        const int oi = s_idx[tid + s];
        if (ov > s_val[tid] || (ov == s_val[tid] && oi < s_idx[tid])) {
          s_val[tid] = ov;
          s_idx[tid] = oi;
        }
      }
      __syncthreads();
    }
    const long long rq = s_val[0];
    const int q = s_idx[0];
    __syncthreads();
    if (rq < 2) continue;
    const long long want = taken[q];
    // the want-th (0-based) sample assigned to q, in index order
    const int64_t a0 = (int64_t)tid * slice, a1 = min(N, a0 + slice);
    long long cnt = 0;
    for (int64_t i = a0; i < a1; ++i) cnt += (assign[i] == q);
    s_cnt[tid] = cnt;
    if (tid == 0) s_pick = -1;
    __syncthreads();
    if (tid == 0) {
      long long run = 0;
      for (int t = 0; t < kRT; ++t) {
        if (want < run + s_cnt[t]) {
          s_cnt[0] = t;          // owner thread
          s_val[0] = want - run;  // rank inside its slice
          break;
        }
        run += s_cnt[t];
      }
    }
    __syncthreads();
    const int owner = (int)s_cnt[0];
    if (tid == owner) {
      long long k = s_val[0];
      for (int64_t i = a0; i < a1; ++i)
        if (assign[i] == q) {
          if (k == 0) {
            s_pick = i;
            break;
          }
          --k;
        }
    }
    __syncthreads();
    const long long pick = s_pick;
    if (pick >= 0) {
      for (int d = tid; d < D; d += kRT) means[(size_t)g * D + d] = X[pick * ldx + d];
      if (tid == 0) {
        taken[q] += 1;
        rem[q] -= 1;
      }
    }
    __syncthreads();
  }
}

// ---- assign() query (Sec. 4 API) ------------------------------------------

// Euclidean: same FP32 + FP64 re-decision scheme as k_km_assign with lam = 1.
// Probabilistic: a_g = c_g - 1/2 sum_d (x s - m)^2 from the EM constants, with
// an FP64 re-decision when the best two are within a conservative bound.
__global__ void __launch_bounds__(kNT) k_assign(const float* __restrict__ X, int64_t N, int D,
                                                int64_t ldx, int G, int mode,
                                                const float* __restrict__ hefts,
                                                const float* __restrict__ means,
                                                const float* __restrict__ dcovs,
                                                const float* __restrict__ sT,
                                                const float* __restrict__ mT,
                                                const float* __restrict__ cc,
                                                int32_t* __restrict__ assign,
                                                unsigned long long* __restrict__ hist,
                                                int32_t* __restrict__ dev_status) {
  const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (i >= N) return;
  const float* x = X + i * ldx;
  int arg = 0;
  if (mode == GMM_ASSIGN_EUCL) {
    const float gamma = 2.0f * (float)(D + 4) * kU32;
    float d1 = INFINITY, d2 = INFINITY;
    for (int g = 0; g < G; ++g) {
      float s = 0.0f;
      for (int d = 0; d < D; ++d) {
        const float t = x[d] - means[(size_t)g * D + d];
        s = fmaf(t, t, s);
      }
      if (s < d1) {
        d2 = d1;
        d1 = s;
        arg = g;
      } else if (s < d2) {
        d2 = s;
      }
    }
    if (G > 1 && !(d2 - d1 > gamma * (d1 + d2))) {
      double best = INFINITY;
      arg = 0;
      for (int g = 0; g < G; ++g) {
        double s = 0.0;
        for (int d = 0; d < D; ++d) {
          const double t = (double)x[d] - (double)means[(size_t)g * D + d];
          s += t * t;
        }
        if (s < best) {
          best = s;
          arg = g;
        }
      }
      if (!isfinite(best)) atomicOr(dev_status, GMM_DEV_NONFINITE);
    }
  } else {
    float a1 = -INFINITY, a2 = -INFINITY, mag = 0.0f;
    for (int g = 0; g < G; ++g) {
      float acc = 0.0f;
      for (int d = 0; d < D; ++d) {
        const float u = fmaf(x[d], sT[(size_t)d * G + g], -mT[(size_t)d * G + g]);
        acc = fmaf(u, u, acc);
      }
      const float a = (cc[g] - 0.5f * acc) + cc[G + g];
      if (a > a1) {
        a2 = a1;
        a1 = a;
        arg = g;
      } else if (a > a2) {
        a2 = a;
      }
      mag = fmaxf(mag, fabsf(cc[g]) + 0.5f * acc);
    }
    // |error| of each FP32 a_g is below ~ (D + 8) u (|c_g| + sum u^2 / 2)
    // plus the rounding of m_gd (|m| u per term); 8x that bound re-decides.
    const float tol = 8.0f * (float)(D + 8) * kU32 * (mag + 1.0f);
    if (G > 1 && !(a1 - a2 > tol)) {
      double best = -INFINITY;
      arg = 0;
      for (int g = 0; g < G; ++g) {
        double ld = 0.0, q = 0.0;
        for (int d = 0; d < D; ++d) {
          const double v = (double)dcovs[(size_t)g * D + d];
          const double t = (double)x[d] - (double)means[(size_t)g * D + d];
          ld += log(v);
          q += t * t / v;
        }
        const double a = log((double)hefts[g]) - 0.5 * ((double)D * kLog2Pi + ld) - 0.5 * q;
        if (a > best) {
          best = a;
          arg = g;
        }
      }
      if (!isfinite(best)) atomicOr(dev_status, GMM_DEV_NONFINITE);
    }
  }
  assign[i] = arg;
  if (hist) atomicAdd(hist + arg, 1ull);
}

// ---- many components (G > 128, D <= 128): assignment on the matrix cores ----
// The nearest mean minimises s_g(x) = Q_g - 2 sum_d lam_d mu_gd x_d with Q_g =
// sum_d lam_d mu_gd^2 (the distance is sum_d lam_d x_d^2 + s_g).  s is computed
// in FP64 by v_mfma_f64_16x16x4f64 (the samples as the A operand, 16 per row
// block; B = -2 lam mu in its operand layout, [block of 16 means][k-step][64
// lanes]); its rounding error is at most (D + 8) 2^-52 (Q + 2 sqrt(Q X2)) with
// X2 = sum_d lam_d x_d^2, since sum_d |lam mu x| <= sqrt(Q X2).

// Fragments and Q_g; block 16 cb + n writes mean g = 16 cb + n (zero past G).
template <typename XT>
__global__ void __launch_bounds__(kNT) k_km_pre_f64(const double* __restrict__ lam64,
                                                    const XT* __restrict__ means, int D, int G,
                                                    double* __restrict__ Bk,
                                                    double* __restrict__ Qg) {
  __shared__ double sh[kNT];
  const int g = blockIdx.x;
  const int KQ = dpad4(D) / 4;
  const int cb = g >> 4, n = g & 15;
  double q = 0.0;
  for (int k = threadIdx.x; k < 4 * KQ; k += kNT) {
    double v = 0.0;
    if (g < G && k < D) {
      const double l = lam64[k];
      const double mu = (double)means[(size_t)g * D + k];
      v = -2.0 * l * mu;
      q += l * mu * mu;
    }
    Bk[((size_t)cb * KQ + (k >> 2)) * 64 + n + 16 * (k & 3)] = v;
  }
  q = block_sum_d<kNT>(q, sh);
  if (g < G && threadIdx.x == 0) Qg[g] = q;
}

// merge of (smallest value, its index, second smallest) pairs; ties go to the
// lower index, so the result is the first minimum whatever the order
__device__ __forceinline__ void km_merge(double& v1, int& g1, double& v2, double o1, int og,
                                         double o2) {
  if (o1 < v1 || (o1 == v1 && og < g1)) {
    v2 = fmin(v1, o2);
    v1 = o1;
    g1 = og;
  } else {
    v2 = fmin(v2, o1);
  }
}
template <int CTRL>
__device__ __forceinline__ void km_merge_dpp(double& v1, int& g1, double& v2) {
  const double o1 = dpp_d<CTRL>(v1), o2 = dpp_d<CTRL>(v2);
  const int og = __builtin_amdgcn_update_dpp(0, g1, CTRL, 0xF, 0xF, false);
  km_merge(v1, g1, v2, o1, og, o2);
}

// Hard assignment (Eq. 19) over tiles of 32 samples: wave per block of 16
// means, every sample's two smallest s and the first minimum's index (lanes,
// then the 16 lanes of a row, then the waves through LDS); a sample whose gap
// v2 - v1 exceeds twice the bound is decided, the others are re-decided over
// all means in the FP64 direct form, first minimum wins.
template <int KQM, typename XT>
__global__ void __launch_bounds__(kWNT) k_km_assign_f64(
    const XT* __restrict__ X, int64_t N, int D, int64_t ldx, int G, int64_t chunk,
    const double* __restrict__ Bk, const double* __restrict__ Qg,
    const XT* __restrict__ means, const double* __restrict__ lam64,
    int32_t* __restrict__ assign, int64_t* __restrict__ n_recomputed) {
  constexpr int NW = kWNT / kWave;
  __shared__ XT xs[kWT * 129];
  __shared__ double l64[128];
  __shared__ double wv1[NW][kWT], wv2[NW][kWT];
  __shared__ int wg1[NW][kWT];
  __shared__ double wq[NW];
  __shared__ int wrec[NW];
  const int XS = dpad4(D);
  const int KQ = XS / 4;
  const int NCB = (G + 15) / 16;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wid = tid / kWave;
  const int m = lane & 15, kb = lane >> 4;
  const int b = blockIdx.x;
  const int64_t i0 = (int64_t)b * chunk;
  const int64_t i1 = min(N, i0 + chunk);
  double qm = 0.0;
  for (int g = tid; g < G; g += kWNT) qm = fmax(qm, Qg[g]);
  for (int d = tid; d < D; d += kWNT) l64[d] = lam64[d];
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) qm = fmax(qm, __shfl_xor(qm, off));
  if (lane == 0) wq[wid] = qm;
  __syncthreads();
  double Qmax = wq[0];
  for (int w = 1; w < NW; ++w) Qmax = fmax(Qmax, wq[w]);
  int nrec = 0;
  for (int64_t t0 = i0; t0 < i1; t0 += kWT) {
    const int nt = (int)min((int64_t)kWT, i1 - t0);
    for (int p = tid; p < nt * XS; p += kWNT) {
      const int t = p / XS, d = p - t * XS;
      xs[p] = d < D ? X[(t0 + t) * ldx + d] : (XT)0;
    }
    __syncthreads();
    double xa[2][KQM];
    const int ta0 = min(m, nt - 1), ta1 = min(16 + m, nt - 1);
#pragma unroll
    for (int ks = 0; ks < KQM; ++ks) {
      const int d = min(4 * ks + kb, XS - 1);
      xa[0][ks] = ks < KQ ? (double)xs[ta0 * XS + d] : 0.0;
      xa[1][ks] = ks < KQ ? (double)xs[ta1 * XS + d] : 0.0;
    }
    double v1[2][4], v2[2][4];
    int g1[2][4];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v1[rb][j] = INFINITY;
        v2[rb][j] = INFINITY;
        g1[rb][j] = G;
      }
    for (int cb = __builtin_amdgcn_readfirstlane(wid); cb < NCB; cb += NW) {
      f64x4 c0 = {0.0, 0.0, 0.0, 0.0}, c1 = {0.0, 0.0, 0.0, 0.0};
      const double* fb = Bk + (size_t)cb * KQ * 64 + lane;
#pragma unroll
      for (int k0 = 0; k0 < KQM; k0 += 8) {
        double bb[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) bb[i] = k0 + i < KQ ? fb[(size_t)(k0 + i) * 64] : 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          if (k0 + i >= KQ) break;
          c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[0][k0 + i], bb[i], c0, 0, 0, 0);
          c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[1][k0 + i], bb[i], c1, 0, 0, 0);
        }
      }
      const int g = 16 * cb + m;
      const double Q = g < G ? Qg[g] : INFINITY;  // padding means never win
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double s0 = Q + c0[j], s1 = Q + c1[j];
        km_merge(v1[0][j], g1[0][j], v2[0][j], s0, g, INFINITY);
        km_merge(v1[1][j], g1[1][j], v2[1][j], s1, g, INFINITY);
      }
    }
    // lane (m, kb) holds samples 16 rb + 4 j + kb over means m + 16 cb: reduce
    // over the 16 lanes of the row, then across the waves
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        km_merge_dpp<0x121>(v1[rb][j], g1[rb][j], v2[rb][j]);
        km_merge_dpp<0x122>(v1[rb][j], g1[rb][j], v2[rb][j]);
        km_merge_dpp<0x124>(v1[rb][j], g1[rb][j], v2[rb][j]);
        km_merge_dpp<0x128>(v1[rb][j], g1[rb][j], v2[rb][j]);
        const int t = 16 * rb + 4 * j + kb;
        if (m == 0) {
          wv1[wid][t] = v1[rb][j];
          wv2[wid][t] = v2[rb][j];
          wg1[wid][t] = g1[rb][j];
        }
      }
    __syncthreads();
    if (tid < nt) {
      const int t = tid;
      double V1 = wv1[0][t], V2 = wv2[0][t];
      int G1 = wg1[0][t];
      for (int w = 1; w < NW; ++w) km_merge(V1, G1, V2, wv1[w][t], wg1[w][t], wv2[w][t]);
      const XT* x = xs + t * XS;
      double X2 = 0.0;
      for (int d = 0; d < D; ++d) X2 += l64[d] * (double)x[d] * (double)x[d];
      const double e = 1.01 * (D + 8.0) * 0x1p-52 * (Qmax + 2.0 * sqrt(Qmax * X2));
      int arg = G1;
      if (!(V2 - V1 > 2.0 * e) || G1 >= G) {
        // FP64 direct form over all means, first minimum wins
        double best = INFINITY;
        arg = 0;
        for (int g = 0; g < G; ++g) {
          const XT* mu = means + (size_t)g * D;
          double q = 0.0;
          for (int d = 0; d < D; ++d) {
            const double u = (double)x[d] - (double)mu[d];
            q += l64[d] * u * u;
          }
          if (q < best) {
            best = q;
            arg = g;
          }
        }
        ++nrec;
      }
      assign[t0 + t] = arg;
    }
    __syncthreads();  // xs and the merge slots are rewritten by the next tile
  }
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) nrec += __shfl_xor(nrec, off);
  if (lane == 0) wrec[wid] = nrec;
  __syncthreads();
  if (tid == 0) {
    long long nr = 0;
    for (int w = 0; w < NW; ++w) nr += wrec[w];
    if (nr) atomicAdd((unsigned long long*)n_recomputed, (unsigned long long)nr);
  }
}

// Map step of the hard assignment (Eqs. 9-11) with the components split in
// groups that fit in LDS: block (r, k) visits the samples of range r and
// accumulates, for the components of group k, the FP64 count, sum (x - mu_old)
// and sum (x - mu_old)^2 in LDS.  Component g is owned by wave (g - g0) % 16,
// which collects its members of each 1024-sample slice in sample order (lane p
// holds the p-th) and adds their rows lane-parallel over d with LDS FP64
// atomics; one wave per address, in program order, so the sums are
// deterministic.  Output: partials [range][G][2D+1] as the generic kernel.
constexpr int kAT = 1024;   // threads of the grouped accumulation
constexpr int kASL = 1024;  // assignments staged per slice
template <int DPL, typename XT>
__global__ void __launch_bounds__(kAT) k_km_accum_grp(const XT* __restrict__ X, int64_t N,
                                                      int D, int64_t ldx, int G, int GG,
                                                      int64_t chunk,
                                                      const XT* __restrict__ means,
                                                      const int32_t* __restrict__ assign,
                                                      double* __restrict__ part) {
  extern __shared__ double lacc[];
  const int r = blockIdx.x;
  const int g0 = blockIdx.y * GG;
  const int gn = min(GG, G - g0);
  const int P = 2 * D + 1;
  XT* mu = (XT*)(lacc + (size_t)GG * P);  // [GG][D]
  int* sa = (int*)(mu + (size_t)GG * D);         // [kASL] group-relative component or -1
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wid = tid / kWave;
  constexpr int NWV = kAT / kWave;
  for (int p = tid; p < gn * P; p += kAT) lacc[p] = 0.0;
  for (int p = tid; p < gn * D; p += kAT) mu[p] = means[(size_t)g0 * D + p];
  const int64_t i0 = (int64_t)r * chunk;
  const int64_t i1 = min(N, i0 + chunk);
  for (int64_t s0 = i0; s0 < i1; s0 += kASL) {
    const int ns = (int)min((int64_t)kASL, i1 - s0);
    __syncthreads();  // previous slice consumed (and, first time, LDS set up)
    for (int p = tid; p < kASL; p += kAT) {
      int rel = -1;
      if (p < ns) {
        rel = assign[s0 + p] - g0;
        if (rel < 0 || rel >= gn) rel = -1;
      }
      sa[p] = rel;
    }
    __syncthreads();
    int cnt = 0;    // members collected (wave-uniform)
    int midx = 0;   // lane p: slice offset of the p-th member
    int mrel = 0;   // lane p: its group-relative component
    auto flush = [&]() {
      for (int k0 = 0; k0 < cnt; k0 += 8) {
        XT xv[8][DPL];
        int rr[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int k = min(k0 + u, cnt - 1);
          const int off = __builtin_amdgcn_readlane(midx, k);
          rr[u] = __builtin_amdgcn_readlane(mrel, k);
          const XT* xr = X + (s0 + off) * ldx;
#pragma unroll
          for (int j = 0; j < DPL; ++j) {
            const int d = lane + kWave * j;
            xv[u][j] = d < D ? xr[d] : (XT)0;
          }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (k0 + u >= cnt) break;
          double* q = lacc + (size_t)rr[u] * P;
          const XT* m = mu + (size_t)rr[u] * D;
#pragma unroll
          for (int j = 0; j < DPL; ++j) {
            const int d = lane + kWave * j;
            if (d < D) {
              const double y = (double)xv[u][j] - (double)m[d];
              atomicAdd(q + 1 + d, y);
              atomicAdd(q + 1 + D + d, y * y);
            }
          }
          if (lane == 0) atomicAdd(q, 1.0);
        }
      }
      cnt = 0;
    };
    for (int sub = 0; sub < kASL / kWave; ++sub) {
      const int rel = sa[sub * kWave + lane];
      const bool mine = rel >= 0 && (rel % NWV) == wid;
      const uint64_t bal = __ballot(mine);
      if (!bal) continue;
      const int pc = __popcll(bal);
      if (cnt + pc > kWave) flush();
      // lane p in [cnt, cnt + pc) takes the (p - cnt)-th set bit of bal
      const int k = lane - cnt;
      if (k >= 0 && k < pc) {
        int kk = k, pos = 0;
        uint64_t m = bal;
        int c = __popc((uint32_t)m);
        if (kk >= c) { kk -= c; pos += 32; m >>= 32; }
        c = __popc((uint32_t)m & 0xFFFFu);
        if (kk >= c) { kk -= c; pos += 16; m >>= 16; }
        c = __popc((uint32_t)m & 0xFFu);
        if (kk >= c) { kk -= c; pos += 8; m >>= 8; }
        c = __popc((uint32_t)m & 0xFu);
        if (kk >= c) { kk -= c; pos += 4; m >>= 4; }
        c = __popc((uint32_t)m & 0x3u);
        if (kk >= c) { kk -= c; pos += 2; m >>= 2; }
        c = (int)(m & 1u);
        if (kk >= c) pos += 1;
        midx = sub * kWave + pos;
        mrel = sa[midx];
      }
      cnt += pc;
    }
    flush();
  }
  __syncthreads();
  double* pb = part + ((size_t)r * G + g0) * P;
  for (int p = tid; p < gn * P; p += kAT) pb[p] = lacc[p];
}

size_t km_accum_grp_lds(int D, int GG, size_t esz = sizeof(float)) {
  return sizeof(double) * (size_t)GG * (2 * D + 1) + esz * (size_t)GG * D + sizeof(int) * kASL;
}

__global__ void k_zero_i64(int64_t* p, int n, int32_t* dev_status) {
  for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < n; i += blockDim.x * gridDim.x) p[i] = 0;
  if (dev_status && blockIdx.x == 0 && threadIdx.x == 0) *dev_status = 0;
}

// The matrix-core assignment kernel takes D <= 128 and more components than the
// one-pass kernel takes.
bool km_use_wide(int D, int G) { return D <= 128 && G > 128; }

// Largest component group of the grouped map step that fits in LDS (0: none).
int km_accum_group_max(int D, size_t esz = sizeof(float)) {
  const size_t per = sizeof(double) * (2 * (size_t)D + 1) + esz * (size_t)D;
  const size_t avail = 160 * 1024 - sizeof(int) * kASL;
  return (int)(avail / per);
}

// Dynamic LDS above the 64 KB default needs the kernel's limit raised; the
// limit plus the kernel's static LDS must stay within the 160 KB of a CU, so
// it is raised to exactly what the launch asks for.
void set_max_lds(const void* kern, size_t bytes) {
  if (bytes > 64 * 1024)
    (void)hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

int kmeans_path(int D, int G, int prec) {
  if (km_fast_supported(D, G))
    return prec == GMM_PREC_BF16X3 && km2_supported(D, G) ? GMM_PATH_ONEPASS_BF16X3
                                                          : GMM_PATH_ONEPASS_FP32;
  return km_use_wide(D, G) ? GMM_PATH_WIDE_FP64 : GMM_PATH_GENERIC;
}

namespace {

// The tile kernels of one k-means iteration: assignment (FP64 matrix cores when
// wide, the only form for FP64 data; else the FP32 direct form with its FP64
// re-decision), the map step, the reduce step, inertia and resurrection.
template <typename XT>
hipError_t kmeans_tiles(const XT* X, int64_t N, int D, int64_t ldx, int G, int dist,
                        const double* gvar, double var_floor, XT* means, XT* dcovs, XT* hefts,
                        int64_t* counts, int32_t* asg, double* inertia, bool wide,
                        int64_t* n_recomputed, int32_t* dev_status, const Workspace& w,
                        hipStream_t st) {
  const int nb = partial_blocks(N, 256);
  const int64_t chunk = (N + nb - 1) / nb;
  int64_t* nrec = n_recomputed ? n_recomputed : w.counters;
  hipLaunchKernelGGL(k_km_init, dim3(1), dim3(64), 0, st, dev_status, n_recomputed);
  hipLaunchKernelGGL(k_km_pre, dim3((D + 255) / 256), dim3(256), 0, st, gvar, D, (float)var_floor,
                     dist, w.lam64, w.lam32);
  if (wide) {
    hipLaunchKernelGGL(k_km_pre_f64<XT>, dim3(16 * ((G + 15) / 16)), dim3(kNT), 0, st,
                       (const double*)w.lam64, (const XT*)means, D, G, w.Bx64, w.cq64);
    ProfScope ps(kProfKmAssign, st);
    if (D <= 64)
      hipLaunchKernelGGL((k_km_assign_f64<16, XT>), dim3(nb), dim3(kWNT), 0, st, X, N, D, ldx, G,
                         chunk, (const double*)w.Bx64, (const double*)w.cq64, (const XT*)means,
                         (const double*)w.lam64, asg, nrec);
    else
      hipLaunchKernelGGL((k_km_assign_f64<32, XT>), dim3(nb), dim3(kWNT), 0, st, X, N, D, ldx, G,
                         chunk, (const double*)w.Bx64, (const double*)w.cq64, (const XT*)means,
                         (const double*)w.lam64, asg, nrec);
  } else if constexpr (sizeof(XT) == 4) {
    ProfScope ps(kProfKmAssign, st);
    hipLaunchKernelGGL(k_km_assign, dim3(nb), dim3(kNT), 0, st, X, N, D, ldx, G, chunk, means,
                       w.lam32, w.lam64, asg, nrec);
  }
  int nba = nb;  // partial sets of the map step
  {
    ProfScope ps(kProfKmAccum, st);
    const int GGmax = D <= 4 * kWave ? km_accum_group_max(D, sizeof(XT)) : 0;
    if (GGmax >= 1) {
      const int ngrp = (G + GGmax - 1) / GGmax;
      const int GG = (G + ngrp - 1) / ngrp;
      // about 2048 blocks in all, at least 64 sample ranges (fewer when N is small)
      const int want = std::max(64, (2048 + ngrp - 1) / ngrp);
      nba = std::min(partial_blocks(N, 2048), want);
      const int64_t ach = (N + nba - 1) / nba;
      const size_t lds = km_accum_grp_lds(D, GG, sizeof(XT));
      if (D <= kWave) {
        set_max_lds((const void*)k_km_accum_grp<1, XT>, lds);
        hipLaunchKernelGGL((k_km_accum_grp<1, XT>), dim3(nba, ngrp), dim3(kAT), lds, st, X, N, D,
                           ldx, G, GG, ach, (const XT*)means, (const int32_t*)asg, w.partials);
      } else if (D <= 2 * kWave) {
        set_max_lds((const void*)k_km_accum_grp<2, XT>, lds);
        hipLaunchKernelGGL((k_km_accum_grp<2, XT>), dim3(nba, ngrp), dim3(kAT), lds, st, X, N, D,
                           ldx, G, GG, ach, (const XT*)means, (const int32_t*)asg, w.partials);
      } else {
        set_max_lds((const void*)k_km_accum_grp<4, XT>, lds);
        hipLaunchKernelGGL((k_km_accum_grp<4, XT>), dim3(nba, ngrp), dim3(kAT), lds, st, X, N, D,
                           ldx, G, GG, ach, (const XT*)means, (const int32_t*)asg, w.partials);
      }
    } else if constexpr (sizeof(XT) == 4) {
      hipLaunchKernelGGL(k_km_accum, dim3(nb), dim3(kNT), 0, st, X, N, D, ldx, G, chunk, means,
                         asg, w.partials);
    }
  }
  // per-component inertia terms in c64 (unused by k-means)
  hipLaunchKernelGGL(k_km_fin<XT>, dim3(G), dim3(kNT), sizeof(double) * (2 * D + 1), st,
                     w.partials, nba, N, D, G, var_floor, (const double*)w.lam64, means, dcovs,
                     hefts, counts, w.c64);
  hipLaunchKernelGGL(k_km_inertia, dim3(1), dim3(64), 0, st, w.c64, G, inertia, dev_status);
  hipLaunchKernelGGL(k_km_resurrect<XT>, dim3(1), dim3(kRT), 0, st, X, N, D, ldx, G,
                     (const int64_t*)counts, (const int32_t*)asg, means, (int64_t*)w.partials);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_kmeans(const float* X, int64_t N, int D, int64_t ldx, int G, int dist,
                         const double* gvar, float var_floor, float* means, float* dcovs,
                         float* hefts, int64_t* counts, int32_t* assign, double* inertia,
                         int prec, int64_t* n_recomputed, int32_t* dev_status, const Workspace& w,
                         hipStream_t st) {
  // prec selects the screening form of the one-pass kernel (FP32 direct, or
  // BF16x3 on the matrix cores); the decisions are exact either way
  int32_t* asg = assign ? assign : w.assign;
  if (km_fast_supported(D, G)) {
    hipLaunchKernelGGL(k_km_init, dim3(1), dim3(64), 0, st, dev_status, n_recomputed);
    hipError_t e = launch_kmeans_fast(X, N, D, ldx, G, dist, gvar, var_floor, means, dcovs, hefts,
                                      counts, asg, inertia,
                                      n_recomputed ? n_recomputed : w.counters, dev_status, w, st,
                                      prec);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_km_resurrect<float>, dim3(1), dim3(kRT), 0, st, X, N, D, ldx, G,
                       (const int64_t*)counts, (const int32_t*)asg, means, (int64_t*)w.partials);
    return hipGetLastError();
  }
  return kmeans_tiles<float>(X, N, D, ldx, G, dist, gvar, (double)var_floor, means, dcovs, hefts,
                             counts, asg, inertia, km_use_wide(D, G), n_recomputed, dev_status,
                             w, st);
}

bool kmeans_f64_supported(int D) { return D >= 1 && D <= 128; }

hipError_t launch_kmeans_f64(const double* X, int64_t N, int D, int64_t ldx, int G, int dist,
                             const double* gvar, double var_floor, double* means, double* dcovs,
                             double* hefts, int64_t* counts, int32_t* assign, double* inertia,
                             int64_t* n_recomputed, int32_t* dev_status, const Workspace& w,
                             hipStream_t st) {
  return kmeans_tiles<double>(X, N, D, ldx, G, dist, gvar, var_floor, means, dcovs, hefts, counts,
                              assign ? assign : w.assign, inertia, true, n_recomputed, dev_status,
                              w, st);
}

namespace {

// ---- seeding of the initial means (Sec. 4 API seed modes) ------------------

__global__ void k_seed_init(int64_t* cur, int64_t first, int32_t* dev_status) {
  if (threadIdx.x == 0) {
    *cur = first;
    *dev_status = 0;
  }
}

// Subset modes: block g copies sample idx[g] (caller-drawn indices: random
// subset) or floor(g N / G) (static subset) into means[g]; an index outside
// [0, N) sets GMM_DEV_BADDESC and leaves the row unchanged.
__global__ void __launch_bounds__(256) k_seed_subset(const float* __restrict__ X, int64_t N,
                                                     int D, int64_t ldx, int G,
                                                     const int64_t* __restrict__ idx,
                                                     float* __restrict__ means,
                                                     int32_t* __restrict__ dev_status) {
  const int g = blockIdx.x;
  const int64_t q = N / G, r = N % G;
  const int64_t s = idx ? idx[g] : (int64_t)g * q + ((int64_t)g * r) / G;
  if (s < 0 || s >= N) {
    if (threadIdx.x == 0) atomicOr(dev_status, GMM_DEV_BADDESC);
    return;
  }
  for (int d = threadIdx.x; d < D; d += 256) means[(size_t)g * D + d] = X[s * ldx + d];
}

// Spread mode (farthest-first traversal), pass k: seed k is sample *cur; its
// row goes to means[k] and every sample's distance to its nearest seed so far,
// dmin[i] = min(dmin[i], sum_d lam_d (x_id - y_d)^2), is updated (k = 0: set).
// Each term lam_d * (u * u) is rounded on its own (an empty asm statement
// keeps the compiler from fusing it into the add) and added in the order
// d = 0..D-1, so the values, and hence the choice of the next seed, are those
// of the plain sequential definition.  Samples
// pass through LDS in tiles of kST, kSD dimensions at a time.  Each workgroup
// leaves its largest dmin and the lowest sample index holding it in
// pval/pidx[b].
constexpr int kST = 256;
constexpr int kSD = 32;
__global__ void __launch_bounds__(kST) k_spread_pass(const float* __restrict__ X, int64_t N,
                                                     int D, int64_t ldx, int64_t chunk,
                                                     const double* __restrict__ lam, int k,
                                                     const int64_t* __restrict__ cur,
                                                     float* __restrict__ means,
                                                     double* __restrict__ dmin,
                                                     double* __restrict__ pval,
                                                     double* __restrict__ pidx,
                                                     int32_t* __restrict__ dev_status) {
  __shared__ float xs[kST][kSD + 1];
  __shared__ double ys[kSD], ls[kSD];
  __shared__ double bv[kST];
  __shared__ int64_t bi[kST];
  const int tid = threadIdx.x;
  const int64_t s = *cur;
  const float* y = X + s * ldx;
  if (blockIdx.x == 0)
    for (int d = tid; d < D; d += kST) means[(size_t)k * D + d] = y[d];
  const int64_t i0 = (int64_t)blockIdx.x * chunk;
  const int64_t i1 = min(N, i0 + chunk);
  double best = -1.0;
  int64_t besti = INT64_MAX;
  bool bad = false;
  for (int64_t t0 = i0; t0 < i1; t0 += kST) {
    const int nt = (int)min((int64_t)kST, i1 - t0);
    double q = 0.0;
    for (int d0 = 0; d0 < D; d0 += kSD) {
      const int nd = min(kSD, D - d0);
      __syncthreads();
      for (int p = tid; p < nt * nd; p += kST) {
        const int t = p / nd, c = p - t * nd;
        xs[t][c] = X[(t0 + t) * ldx + d0 + c];
      }
      if (tid < nd) {
        ys[tid] = (double)y[d0 + tid];
        ls[tid] = lam ? lam[d0 + tid] : 1.0;
      }
      __syncthreads();
      if (tid < nt)
        for (int c = 0; c < nd; ++c) {
          const double u = (double)xs[tid][c] - ys[c];
          double term = ls[c] * (u * u);
          asm volatile("" : "+v"(term));  // rounded on its own: no fused add
          q = q + term;
        }
    }
    if (tid < nt) {
      const int64_t i = t0 + tid;
      const double dm = (k == 0 || q < dmin[i]) ? q : dmin[i];
      dmin[i] = dm;
      if (!isfinite(q)) bad = true;
      if (dm > best) {  // a thread's samples come in increasing order
        best = dm;
        besti = i;
      }
    }
  }
  bv[tid] = best;
  bi[tid] = besti;
  __syncthreads();
  for (int h = kST / 2; h > 0; h >>= 1) {
    if (tid < h) {
      const double v2 = bv[tid + h];
      const int64_t i2 = bi[tid + h];
      if (v2 > bv[tid] || (v2 == bv[tid] && i2 < bi[tid])) {
        bv[tid] = v2;
        bi[tid] = i2;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    pval[blockIdx.x] = bv[0];
    pidx[blockIdx.x] = (double)bi[0];
  }
  if (bad) atomicOr(dev_status, GMM_DEV_NONFINITE);
}

// The next seed: the largest of the workgroups' maxima, the earliest workgroup
// (lowest sample index) on ties.
__global__ void k_spread_pick(const double* __restrict__ pval, const double* __restrict__ pidx,
                              int nb, int64_t* __restrict__ cur) {
  if (threadIdx.x == 0) {
    double best = -1.0;
    double bi = 0.0;
    for (int b = 0; b < nb; ++b)
      if (pval[b] > best) {
        best = pval[b];
        bi = pidx[b];
      }
    *cur = (int64_t)bi;
  }
}

// Mahalanobis weights of the seeding distance: 1 / max(global variance, floor)
// in FP64 (Sec. 3.1, Eq. 20).
__global__ void k_seed_lambda(const double* __restrict__ gvar, int D, float var_floor,
                              double* __restrict__ lam) {
  for (int d = threadIdx.x; d < D; d += blockDim.x) {
    const double v = gvar[d] > (double)var_floor ? gvar[d] : (double)var_floor;
    lam[d] = 1.0 / v;
  }
}

}  // namespace

hipError_t launch_seed_means(const float* X, int64_t N, int D, int64_t ldx, int G, int mode,
                             const double* gvar, float var_floor, int64_t first,
                             const int64_t* idx, float* means, int32_t* dev_status,
                             const Workspace& w, hipStream_t st) {
  int64_t* cur = w.counters;
  hipLaunchKernelGGL(k_seed_init, dim3(1), dim3(64), 0, st, cur, first, dev_status);
  if (mode == GMM_SEED_SUBSET) {
    hipLaunchKernelGGL(k_seed_subset, dim3(G), dim3(256), 0, st, X, N, D, ldx, G, idx, means,
                       dev_status);
    return hipGetLastError();
  }
  const double* lam = nullptr;
  if (gvar) {
    hipLaunchKernelGGL(k_seed_lambda, dim3(1), dim3(256), 0, st, gvar, D, var_floor, w.lam64);
    lam = w.lam64;
  }
  const int nb = partial_blocks(N, 4 * kST);
  const int64_t chunk = (N + nb - 1) / nb;
  double* pval = w.scalars;
  double* pidx = w.scalars + kMaxBlocks;
  for (int k = 0; k < G; ++k) {
    hipLaunchKernelGGL(k_spread_pass, dim3(nb), dim3(kST), 0, st, X, N, D, ldx, chunk, lam, k,
                       (const int64_t*)cur, means, w.dmin, pval, pidx, dev_status);
    if (k + 1 < G)
      hipLaunchKernelGGL(k_spread_pick, dim3(1), dim3(64), 0, st, pval, pidx, nb, cur);
  }
  return hipGetLastError();
}

hipError_t launch_assign(const float* X, int64_t N, int D, int64_t ldx, int G, int mode,
                         const float* hefts, const float* means, const float* dcovs,
                         int32_t* assign, int64_t* hist, int32_t* dev_status, const Workspace& w,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(256), 0, st, hist ? hist : w.counters,
                     hist ? G : 8, dev_status);
  if (mode == GMM_ASSIGN_PROB) {
    hipError_t e = launch_pre_diag(hefts, means, dcovs, D, G, w, st);
    if (e != hipSuccess) return e;
  }
  const int64_t nblk = (N + kNT - 1) / kNT;
  hipLaunchKernelGGL(k_assign, dim3((unsigned)nblk), dim3(kNT), 0, st, X, N, D, ldx, G, mode,
                     hefts, means, dcovs, w.s, w.m, w.c, assign, (unsigned long long*)hist,
                     dev_status);
  return hipGetLastError();
}

}  // namespace gmm
