// gmm_em.hip -- EM iteration and log-likelihood for diagonal covariances,
// generic kernels valid for every shape the API accepts.
//
// One EM iteration (Sec. 2, Eqs. 3-7) is three or four launches on one stream:
//   k_pre_diag      per-component constants in FP64 (Sec. 2.2, Eq. 15):
//                   s_gd = 1/sigma_gd, m_gd = mu_gd/sigma_gd (rounded to FP32)
//                   and c_g = log w_g - 1/2 (D log 2pi + sum_d log sigma2_gd)
//                   (kept as an FP32 hi/lo pair)
//   k_frag_diag64   (G > 128, D <= 128) the expanded form's coefficients
//                   [-lam/2, lam mu] in the FP64 MFMA operand layout
//   k_estep_diag    sample tiles: log-densities a_gi (G > 128, D <= 128: exact
//                   FP64 on the matrix cores, logdens_diag_f64; otherwise the
//                   FP32 direct form c_g - 1/2 sum_d (x_di s_gd - m_gd)^2 with
//                   an FP64 recompute of the near set), max-shifted
//                   log-sum-exp per sample (Eqs. 16-18), responsibilities
//                   (Eq. 3), and the map step of Sec. 2.1 (Eqs. 9-11) into
//                   per-block FP64 partials.  The moments are accumulated about
//                   the component's current mean (y = x - mu_old): L, sum l*y,
//                   sum l*y^2, which makes the one-pass covariance of Eq. 8
//                   free of cancellation.
//   k_fin_diag      reduce step (Eqs. 12-14) over the block partials in a fixed
//                   order, Eq. 5 weights, Eq. 6 means, Eq. 7 variances about the
//                   new mean, the variance floor, and the mean log-likelihood.
#include "gmm_internal.hpp"

namespace gmm {

namespace {

constexpr int kNT = 256;

__global__ void k_init(int32_t* dev_status, int64_t* n_recomputed, int64_t* counters) {
  if (threadIdx.x == 0) {
    if (dev_status) *dev_status = 0;
    if (n_recomputed) *n_recomputed = 0;
  }
  if (threadIdx.x < 8) counters[threadIdx.x] = 0;
}

// One workgroup per component g.  XT: the parameters' type (FP32, or FP64 for
// FP64 data).
template <typename XT>
__global__ void __launch_bounds__(kNT) k_pre_diag(const XT* __restrict__ hefts,
                                                  const XT* __restrict__ means,
                                                  const XT* __restrict__ covs, int D, int G,
                                                  float* __restrict__ s_out,
                                                  float* __restrict__ m_out,
                                                  float* __restrict__ c_out,
                                                  double* __restrict__ c64_out,
                                                  double* __restrict__ lam64_out) {
  __shared__ double sh[kNT];
  const int g = blockIdx.x;
  double ld = 0.0, qm = 0.0;
  for (int d = threadIdx.x; d < D; d += kNT) {
    const double v = (double)covs[(size_t)g * D + d];
    const double mu = (double)means[(size_t)g * D + d];
    const double lam = 1.0 / v;
    const double s = sqrt(lam);
    s_out[(size_t)d * G + g] = (float)s;
    m_out[(size_t)d * G + g] = (float)(mu * s);
    lam64_out[(size_t)g * D + d] = lam;
    ld += log(v);
    qm += lam * mu * mu;
  }
  const double logdet = block_sum_d<kNT>(ld, sh);
  const double quad = block_sum_d<kNT>(qm, sh);
  if (threadIdx.x == 0) {
    c_out[2 * G + g] = isfinite(quad) ? (float)(1.0001 * quad) : INFINITY;  // Q_g, error bounds
    const double c = log((double)hefts[g]) - 0.5 * ((double)D * kLog2Pi + logdet);
    const float hi = (float)c;
    c_out[g] = hi;  // -inf for a zero weight: that component gets l = 0
    c_out[G + g] = isfinite(c) ? (float)(c - (double)hi) : 0.0f;
    c64_out[g] = c;
  }
}

// Expanded-form operands of the FP64 matrix-core E-step (D <= 128): block
// 16 cb + n (n < 16) writes component g's B fragments, feature k = 4 ks + kr
// (kr = lane / 16) holding -lam_gk / 2 for k < dpad4(D) (x_k^2) and
// lam mu for k - dpad4(D) (x); zero for padding components and dimensions.
// Also c0_g = c_g - Q_g / 2 and Q_g = sum_d lam mu^2 in FP64.
template <typename XT>
__global__ void __launch_bounds__(kNT) k_frag_diag64(const XT* __restrict__ means,
                                                     const double* __restrict__ lam64,
                                                     const double* __restrict__ c64, int D, int G,
                                                     double* __restrict__ Bx64,
                                                     double* __restrict__ cq64) {
  __shared__ double sh[kNT];
  const int g = blockIdx.x;
  const int DP4 = dpad4(D), KQ = DP4 / 2;
  const int cb = g >> 4, n = g & 15;
  double* f = Bx64 + (size_t)cb * KQ * 64;
  double q = 0.0;
  for (int k = threadIdx.x; k < 2 * DP4; k += kNT) {
    const int ks = k >> 2, kr = k & 3;
    double v = 0.0;
    if (g < G) {
      const int d = k < DP4 ? k : k - DP4;
      if (d < D) {
        const double lam = lam64[(size_t)g * D + d];
        const double mu = (double)means[(size_t)g * D + d];
        v = k < DP4 ? -0.5 * lam : lam * mu;
        if (k >= DP4) q += lam * mu * mu;
      }
    }
    f[(size_t)ks * 64 + n + 16 * kr] = v;
  }
  q = block_sum_d<kNT>(q, sh);
  if (g < G && threadIdx.x == 0) {
    cq64[g] = c64[g] - 0.5 * q;
    cq64[G + g] = q;
  }
}

// The FP64 matrix-core E-step over a tile of up to 32 samples (D <= 128):
// a_g(x) = c0_g + sum_k A_k B_gk with A = [x_d^2, x_d] (the samples, 16 per row
// block, as the A operand of v_mfma_f64_16x16x4f64) and B the expanded
// coefficients [-lam/2, lam mu] (k_frag_diag64), the x^2 and x halves
// accumulated apart.  Output lane l, register j of row block rb is (sample
// 16 rb + 4 j + l/16, component 16 cb + l%16).  The rounding error of the sum is
// at most (2 dpad4(D) + 8) 2^-52 (T1 + sqrt(2 T1 Q) + Q + |c0|) with T1 =
// sum lam x^2 / 2 (the x^2 half) and Q = sum lam mu^2, since sum |lam mu x| <=
// sqrt(Q 2 T1); a pair whose bound exceeds 1e-9 nats is recomputed in the FP64
// direct form.  Each (sample, block of 16 components) gets its own reference,
// R = the block's largest value rounded to FP32, stored in rcb[t][cb]; as[t][g]
// receives a - R in FP32.  For every pair that can carry a responsibility above
// e^-40, a lies within 40 nats of the sample's maximum, which bounds R from
// above, so |a - R| <= 40 and the FP32 entry is accurate to 40 2^-24 nats.
// Wave per block of 16 components.
// XH > 0 (dpad4(D) <= 4 XH): the A operand's x values of the tile's two row
// blocks are held in registers for all component blocks, and both halves of
// the expanded form run side by side (x^2 times -lam/2, x times lam mu: four
// independent accumulator chains).  XH = 0: any D <= 128, the operand is
// rebuilt from LDS per component block.
template <int XH, typename XT>
__device__ __forceinline__ void logdens_diag_f64(const XT* __restrict__ xs, int XS, int nt, int D, int G,
                                 const double* __restrict__ Bx64,
                                 const double* __restrict__ cq64,
                                 const double* __restrict__ c64,
                                 const double* __restrict__ lam64,
                                 const XT* __restrict__ means, XT* __restrict__ as,
                                 int AS, float* __restrict__ rcb, int RS, int wid, int nw,
                                 int lane) {
  const int DP4 = XS;           // dimensions padded to 4 (zeros in xs)
  const int KQ = DP4 / 2;       // k-steps of 4 features
  const int KQ1 = DP4 / 4;      // of which the x^2 half
  const int NCB = (G + 15) / 16;
  const int m = lane & 15, kb = lane >> 4;
  const int ta0 = min(m, nt - 1), ta1 = min(16 + m, nt - 1);  // A rows (past nt: dropped)
  const double ek = (2.0 * DP4 + 8.0) * 0x1p-52;
  double xh[2][XH > 0 ? XH : 1];
  if (XH > 0) {
#pragma unroll
    for (int i = 0; i < XH; ++i) {
      const int d = min(4 * i + kb, DP4 - 1);
      xh[0][i] = i < KQ1 ? (double)xs[(size_t)ta0 * XS + d] : 0.0;
      xh[1][i] = i < KQ1 ? (double)xs[(size_t)ta1 * XS + d] : 0.0;
    }
  }
  for (int cb = __builtin_amdgcn_readfirstlane(wid); cb < NCB; cb += nw) {
    f64x4 c1[2], c2[2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      c1[rb] = f64x4{0.0, 0.0, 0.0, 0.0};
      c2[rb] = f64x4{0.0, 0.0, 0.0, 0.0};
    }
    const double* fb = Bx64 + (size_t)cb * KQ * 64 + lane;
    if (XH > 0) {
#pragma unroll
      for (int i0 = 0; i0 < XH; i0 += 8) {
        double bs[8], bx[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int ks = min(i0 + i, KQ1 - 1);
          bs[i] = fb[(size_t)ks * 64];
          bx[i] = fb[(size_t)(KQ1 + ks) * 64];
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          if (i0 + i >= KQ1) break;
          const double x0 = xh[0][i0 + i], x1 = xh[1][i0 + i];
          c1[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0 * x0, bs[i], c1[0], 0, 0, 0);
          c1[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1 * x1, bs[i], c1[1], 0, 0, 0);
          c2[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, bx[i], c2[0], 0, 0, 0);
          c2[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, bx[i], c2[1], 0, 0, 0);
        }
      }
    } else {
      for (int k0 = 0; k0 < KQ; k0 += 8) {
        double bb[8], a0[8], a1[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int ks = min(k0 + i, KQ - 1);
          const int k = 4 * ks + kb;
          const bool sq = ks < KQ1;
          const int d = sq ? k : k - DP4;
          bb[i] = fb[(size_t)ks * 64];
          const double x0 = (double)xs[(size_t)ta0 * XS + d];
          const double x1 = (double)xs[(size_t)ta1 * XS + d];
          a0[i] = sq ? x0 * x0 : x0;
          a1[i] = sq ? x1 * x1 : x1;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int ks = k0 + i;
          if (ks >= KQ) break;
          if (ks < KQ1) {
            c1[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[i], bb[i], c1[0], 0, 0, 0);
            c1[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[i], bb[i], c1[1], 0, 0, 0);
          } else {
            c2[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[i], bb[i], c2[0], 0, 0, 0);
            c2[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[i], bb[i], c2[1], 0, 0, 0);
          }
        }
      }
    }
    const int g = 16 * cb + m;
    const bool gv = g < G;
    const double c0 = gv ? cq64[g] : 0.0, Q = gv ? cq64[G + g] : 0.0;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int t = 16 * rb + 4 * j + kb;
        double a = -INFINITY;
        if (gv && t < nt) {
          a = c0 + (c1[rb][j] + c2[rb][j]);
          // the bound, first with sqrt(2 T1 Q) <= T1 + Q/2 (no square root)
          const double T1 = fmax(-c1[rb][j], 0.0);
          const double base = T1 + Q + fabs(c0);
          if (!(ek * (base + (T1 + 0.5 * Q)) <= 1e-9) &&
              !(ek * (base + sqrt(2.0 * T1 * Q)) <= 1e-9)) {
            // extreme data (or non-finite): FP64 direct form
            const XT* x = xs + (size_t)t * XS;
            double q = 0.0;
            for (int d = 0; d < D; ++d) {
              const double u = (double)x[d] - (double)means[(size_t)g * D + d];
              q += u * u * lam64[(size_t)g * D + d];
            }
            a = c64[g] - 0.5 * q;
          }
        }
        // the block's largest value over the 16 lanes of the row (all lanes),
        // in FP32: the largest of the rounded values is the rounded largest
        float v = (float)a;
        v = fmaxf(v, dpp_f<0x121>(v));
        v = fmaxf(v, dpp_f<0x122>(v));
        v = fmaxf(v, dpp_f<0x124>(v));
        v = fmaxf(v, dpp_f<0x128>(v));
        if (t < nt) {
          if (gv) as[(size_t)t * AS + g] = v > -INFINITY ? (XT)(a - (double)v) : -INFINITY;
          if (m == 0) rcb[(size_t)t * RS + cb] = v;
        }
      }
  }
}

// E-step (+ optional M-step map) over the block's contiguous sample range.
// LDS: xs[T][D] samples (WIDE: rows padded to dpad4(D) with zeros),
// as[T][G] log-densities (WIDE: relative to the references rcb) then
// responsibilities, lse[T], the tile's component mask (WIDE: then rcb[T][NCB],
// a reference per sample and block of 16 components).  T is chosen on the host
// so the tile fits in LDS.
// XT: the type of the samples and parameters.  FP32 data as above.  FP64 data
// (WIDE only): xs and as hold FP64 values, and in the log-sum-exp every pair
// within kExactGap nats of the sample's largest matrix-core value is computed
// again in the FP64 direct form before the responsibilities are taken, so
// every responsibility above exp(-40) comes from a log-density good to FP64
// rounding (the matrix-core values alone carry up to their rounding bound,
// 1e-9 nats, which moves a responsibility below exp(-41) by a relative 1e-9).
// Responsibilities below exp(-80) are set to 0 (FP32 data: exp(-40)): at the
// FP64 bar a component made of one sample has a variance that far samples'
// tiny responsibilities still move at 1e-11 with the FP32 cut.
constexpr double kExactGap = 41.0;
constexpr double kRespCut64 = 80.0;
template <bool MSTEP, bool WIDE, typename XT>
__global__ void __launch_bounds__(kNT, 2) k_estep_diag(
    const XT* __restrict__ X, int64_t N, int D, int64_t ldx, int G, int T, int64_t chunk,
    const float* __restrict__ sT, const float* __restrict__ mT, const float* __restrict__ cc,
    const double* __restrict__ c64, const double* __restrict__ lam64,
    const double* __restrict__ Bx64, const double* __restrict__ cq64,
    const XT* __restrict__ means, double* __restrict__ part, double* __restrict__ ll_part,
    XT* __restrict__ per_sample, int32_t* __restrict__ dev_status) {
  static_assert(WIDE || sizeof(XT) == 4, "FP64 data takes the matrix-core form");
  constexpr bool F64 = sizeof(XT) == 8;
  extern __shared__ double lds_d[];
  const int XS = WIDE ? ((D + 3) & ~3) : D;  // row stride of xs
  const int AS = WIDE ? G + 8 : G;            // row stride of as
  XT* xs = (XT*)lds_d;                // [T][XS]
  XT* as = xs + (size_t)T * XS;       // [T][AS]
  double* lse = (double*)(as + (size_t)T * AS + ((T * AS) & 1));  // [T]
  uint32_t* gbits = (uint32_t*)(lse + T);  // [G/32]: component has a non-zero r in the tile
  const int RS = (G + 15) / 16;  // WIDE: row stride of rcb
  float* rcb = (float*)(gbits + ((G + 31) / 32 + 3) / 4 * 4);  // WIDE: [T][RS] references
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wid = tid / kWave;
  const int nw = kNT / kWave;
  const int b = blockIdx.x;
  const int64_t i0 = (int64_t)b * chunk;
  const int64_t i1 = min(N, i0 + chunk);
  const int P = 2 * D + 1;
  const int NGB = (G + 31) / 32;
  double* pb = part + (size_t)b * G * P;
  if (tid == 0) bad = 0;
  if (MSTEP) {
    for (int p = tid; p < G * P; p += kNT) pb[p] = 0.0;
    __threadfence();  // the zeros land before any atomic update of the partials
  }
  double llacc = 0.0;  // thread 0 only
  __syncthreads();

  for (int64_t t0 = i0; t0 < i1; t0 += T) {
    const int nt = (int)min((int64_t)T, i1 - t0);
    for (int p = tid; p < nt * XS; p += kNT) {
      const int t = p / XS, d = p - t * XS;
      xs[p] = d < D ? X[(t0 + t) * ldx + d] : (XT)0;
    }
    for (int p = tid; p < NGB; p += kNT) gbits[p] = 0u;
    __syncthreads();
    if constexpr (!WIDE) {
      // a_gi: one (sample, component) pair per thread iteration.
      for (int p = tid; p < nt * G; p += kNT) {
        const int t = p / G, g = p - t * G;
        const float* x = xs + (size_t)t * XS;
        float acc = 0.0f;
        for (int d = 0; d < D; ++d) {
          const float u = fmaf(x[d], sT[(size_t)d * G + g], -mT[(size_t)d * G + g]);
          acc = fmaf(u, u, acc);
        }
        as[p] = (cc[g] - 0.5f * acc) + cc[G + g];
      }
    } else {
      // exact log-densities on the matrix cores, relative to per-block references
      if (XS <= 64)
        logdens_diag_f64<16>(xs, XS, nt, D, G, Bx64, cq64, c64, lam64, means, as, AS, rcb, RS,
                             wid, nw, lane);
      else
        logdens_diag_f64<0>(xs, XS, nt, D, G, Bx64, cq64, c64, lam64, means, as, AS, rcb, RS,
                            wid, nw, lane);
    }
    __syncthreads();
    if constexpr (WIDE && F64) {
      // FP64 data: log-sum-exp (Eqs. 16-18) about M = max_cb R_cb from the
      // values (R_cb - M) + (a - R_cb), after the pairs within kExactGap nats of
      // the largest are recomputed in the FP64 direct form; kKL threads per
      // sample
      const int ts = tid / kKL, j = tid % kKL;
      if (ts < nt) {  // uniform over the kKL threads of a sample
        XT* a = as + (size_t)ts * AS;
        const float* rr = rcb + (size_t)ts * RS;
        float Mf = -INFINITY;
        for (int c = j; c < RS; c += kKL) Mf = fmaxf(Mf, rr[c]);
#pragma unroll
        for (int off = 1; off < kKL; off <<= 1) Mf = fmaxf(Mf, __shfl_xor(Mf, off));
        const double M = Mf > -INFINITY ? (double)Mf : 0.0;
        double dn = -INFINITY;
        for (int g = j; g < G; g += kKL) {
          const double v = ((double)rr[g >> 4] - M) + (double)a[g];
          a[g] = v;
          dn = fmax(dn, v);
        }
#pragma unroll
        for (int off = 1; off < kKL; off <<= 1) dn = fmax(dn, __shfl_xor(dn, off));
        const XT* x = xs + (size_t)ts * XS;
        double dx = -INFINITY;
        for (int g = j; g < G; g += kKL)
          if (a[g] >= dn - kExactGap) {
            double q = 0.0;
            for (int d = 0; d < D; ++d) {
              const double u = (double)x[d] - (double)means[(size_t)g * D + d];
              q += u * u * lam64[(size_t)g * D + d];
            }
            a[g] = (c64[g] - 0.5 * q) - M;
            dx = fmax(dx, (double)a[g]);
          }
#pragma unroll
        for (int off = 1; off < kKL; off <<= 1) dx = fmax(dx, __shfl_xor(dx, off));
        dx = dx > -INFINITY ? dx : 0.0;
        double sm = 0.0;
        for (int g = j; g < G; g += kKL) sm += exp((double)a[g] - dx);
#pragma unroll
        for (int off = 1; off < kKL; off <<= 1) sm += __shfl_xor(sm, off);
        const double ls = log(sm);
        const double l = (M + dx) + ls;
        if (MSTEP) {
          for (int g = j; g < G; g += kKL) {
            const double z = ((double)a[g] - dx) - ls;
            const double r = z >= -kRespCut64 ? exp(z) : 0.0;
            a[g] = r;
            if (r != 0.0) atomicOr(&gbits[g >> 5], 1u << (g & 31));
          }
        }
        if (j == 0) {
          lse[ts] = l;
          if (!isfinite(l)) bad = 1;
          if (per_sample) per_sample[t0 + ts] = (XT)l;
        }
      }
    } else if constexpr (WIDE) {
      // log-sum-exp (Eqs. 16-18) about M = max_cb R_cb, each value taken as
      // (R_cb - M) + (a - R_cb) in FP64, and responsibilities; kKL threads per
      // sample
      const int ts = tid / kKL, j = tid % kKL;
      if (ts < nt) {  // uniform over the kKL threads of a sample
        float* a = as + (size_t)ts * AS;
        const float* rr = rcb + (size_t)ts * RS;
        float M = -INFINITY;
        for (int c = j; c < RS; c += kKL) M = fmaxf(M, rr[c]);
#pragma unroll
        for (int off = 1; off < kKL; off <<= 1) M = fmaxf(M, __shfl_xor(M, off));
        M = M > -INFINITY ? M : 0.0f;
        // the value relative to M, computed once and kept in place of a - R_cb
        float dn = -INFINITY;
        for (int g = j; g < G; g += kKL) {
          const float v = (float)(((double)rr[g >> 4] - (double)M) + (double)a[g]);
          a[g] = v;
          dn = fmaxf(dn, v);
        }
#pragma unroll
        for (int off = 1; off < kKL; off <<= 1) dn = fmaxf(dn, __shfl_xor(dn, off));
        dn = dn > -INFINITY ? dn : 0.0f;
        double sm = 0.0;
        for (int g = j; g < G; g += kKL) sm += (double)__expf(a[g] - dn);
#pragma unroll
        for (int off = 1; off < kKL; off <<= 1) sm += __shfl_xor(sm, off);
        const double l = ((double)M + (double)dn) + log(sm);
        if (MSTEP) {
          const float dl = (float)log(sm);
          for (int g = j; g < G; g += kKL) {
            const float z = (a[g] - dn) - dl;
            const float r = z >= -kRespCut ? __expf(z) : 0.0f;
            a[g] = r;
            if (r != 0.0f) atomicOr(&gbits[g >> 5], 1u << (g & 31));
          }
        }
        if (j == 0) {
          lse[ts] = l;
          if (!isfinite(l)) bad = 1;
          if (per_sample) per_sample[t0 + ts] = (float)l;
        }
      }
    } else
    // One wave per sample: the FP32 values screen the components; every one
    // that, widened by its rounding-error bound, could come within kNearGap
    // nats of the best is recomputed in FP64 (a_g = c_g - 1/2 sum_d (x_d -
    // mu_gd)^2 / sigma2_gd, Eq. 15), and the sample's log-sum-exp (Eqs. 16-18)
    // is assembled in FP64 from those plus the FP32 values of the rest.  mx
    // is max_g (a_g - err_g), a lower bound of the exact maximum.
    for (int t = wid; t < nt; t += nw) {
      float* a = as + (size_t)t * G;
      const float* x = xs + (size_t)t * XS;
      float mx = -INFINITY;
      for (int g = lane; g < G; g += kWave)
        mx = fmaxf(mx, a[g] - err_direct(2.0f * (cc[g] - a[g]), cc[2 * G + g], cc[g], D));
      mx = wave_max(mx);
      const double M = (double)mx;
      // bit c of nearbits: component c*64 + lane is in the near set; its
      // entry of a[] then holds (a64 - M) instead of the FP32 value
      unsigned long long nearbits = 0;
      for (int c = 0, g0 = 0; g0 < G; ++c, g0 += kWave) {
        const int g = g0 + lane;
        const bool near =
            g < G &&
            a[g] + err_direct(2.0f * (cc[g] - a[g]), cc[2 * G + g], cc[g], D) >= mx - kNearGap;
        if (near) nearbits |= 1ull << c;
        unsigned long long msk = __ballot(near);
        while (msk) {
          const int j = __ffsll((long long)msk) - 1;
          msk &= msk - 1;
          const int gg = g0 + j;
          double q = 0.0;
          for (int d = lane; d < D; d += kWave) {
            const double u = (double)x[d] - (double)means[(size_t)gg * D + d];
            q += u * u * lam64[(size_t)gg * D + d];
          }
          q = wave_sum_d(q);
          if (lane == j) a[gg] = (float)(c64[gg] - 0.5 * q - M);
        }
      }
      // reference: M + dn, dn the largest recomputed (a64 - M)
      float dn = -INFINITY;
      for (int c = 0, g0 = 0; g0 < G; ++c, g0 += kWave) {
        const int g = g0 + lane;
        if (g < G && ((nearbits >> c) & 1ull)) dn = fmaxf(dn, a[g]);
      }
      dn = wave_max(dn);
      dn = dn > -INFINITY ? dn : 0.0f;
      double sm = 0.0;
      for (int c = 0, g0 = 0; g0 < G; ++c, g0 += kWave) {
        const int g = g0 + lane;
        if (g < G) {
          const float v = ((nearbits >> c) & 1ull) ? a[g] - dn : (a[g] - mx) - dn;
          sm += (double)__expf(v);
        }
      }
      sm = wave_sum_d(sm);
      const double l = (M + (double)dn) + log(sm);
      if (MSTEP) {
        const float dl = (float)log(sm);
        for (int c = 0, g0 = 0; g0 < G; ++c, g0 += kWave) {
          const int g = g0 + lane;
          if (g < G) {
            const float z = (((nearbits >> c) & 1ull) ? a[g] - dn : (a[g] - mx) - dn) - dl;
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
      // map step (Eqs. 9-11) about the current mean: the tile's components
      // with a non-zero responsibility, four at a time per wave, lanes over
      // dimensions; the tile's contributions are added to the block's FP64
      // partials once, by atomic adds whose result is not waited for.
      // Component g always goes to wave g % 4 and dimension d to lane d % 64,
      // so every partial is updated by one lane only, in tile order: the sums
      // are those of plain read-modify-write updates.
      static_assert(kNT / kWave == 4, "component ownership assumes four waves");
      const uint32_t own = 0x11111111u << wid;  // bits g % 4 == wid of a word
      int wi = 0;
      uint32_t bits = __builtin_amdgcn_readfirstlane(gbits[0] & own);
      for (;;) {
        int gq[4] = {0, 0, 0, 0};
        int nq = 0;
        while (nq < 4) {
          while (bits == 0u && ++wi < NGB)
            bits = __builtin_amdgcn_readfirstlane(gbits[wi] & own);
          if (bits == 0u) break;
          const int g = 32 * wi + __builtin_ctz(bits);
          bits &= bits - 1u;
#pragma unroll
          for (int k = 0; k < 4; ++k) gq[k] = nq == k ? g : gq[k];
          ++nq;
        }
        if (nq == 0) break;
        // the tile's samples with a non-zero responsibility for each (T <= 64)
        unsigned long long mk[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
          mk[k] = k < nq ? __ballot(lane < nt && as[(size_t)lane * AS + gq[k]] != (XT)0) : 0ull;
        double cnt[4] = {0.0, 0.0, 0.0, 0.0};
        for (int d = lane; d < D; d += kWave) {
          XT mu[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) mu[k] = k < nq ? means[(size_t)gq[k] * D + d] : (XT)0;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            if (k >= nq) break;
            double s1 = 0.0, s2 = 0.0, l = 0.0;
            for (unsigned long long mm = mk[k]; mm; mm &= mm - 1) {
              const int t = __ffsll((long long)mm) - 1;
              const XT r = as[(size_t)t * AS + gq[k]];
              // FP32 data: the difference of two FP32 values; FP64 data: FP64
              const double y = (double)(xs[(size_t)t * XS + d] - mu[k]);
              const double ry = (double)r * y;
              s1 += ry;
              s2 += ry * y;
              l += (double)r;
            }
            double* q = pb + (size_t)gq[k] * P;
            unsafeAtomicAdd(q + 1 + d, s1);
            unsafeAtomicAdd(q + 1 + D + d, s2);
            cnt[k] = l;
          }
        }
        if (lane == 0) {
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (k < nq) unsafeAtomicAdd(pb + (size_t)gq[k] * P, cnt[k]);
        }
        if (nq < 4) break;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    ll_part[b] = llacc;
    if (bad) atomicOr(dev_status, GMM_DEV_NONFINITE);
  }
}

// Reduce step: one workgroup per component.  Thread j sums column j of the
// partials over blocks 0..nb-1 in order.
template <typename XT>
__global__ void __launch_bounds__(kNT) k_fin_diag(const double* __restrict__ part, int nb, int64_t N,
                                                  int D, int G, double var_floor,
                                                  XT* __restrict__ hefts,
                                                  XT* __restrict__ means,
                                                  XT* __restrict__ covs,
                                                  const double* __restrict__ ll_part,
                                                  double* __restrict__ mean_loglik,
                                                  int32_t* __restrict__ dev_status) {
  extern __shared__ double tot[];  // [P]
  __shared__ int bad;
  const int g = blockIdx.x;
  const int P = 2 * D + 1;
  if (threadIdx.x == 0) bad = 0;
  for (int j = threadIdx.x; j < P; j += kNT) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[((size_t)b * G + g) * P + j];
    tot[j] = s;
  }
  __syncthreads();
  const double L = tot[0];
  if (threadIdx.x == 0) {
    const XT w = (XT)(L / (double)N);  // Eq. 5
    hefts[g] = w;
    if (!isfinite(w)) bad = 1;
  }
  if (L > 0.0) {
    for (int d = threadIdx.x; d < D; d += kNT) {
      const double dm = tot[1 + d] / L;                  // Eq. 6, relative to mu_old
      const double mu = (double)means[(size_t)g * D + d] + dm;
      double v = tot[1 + D + d] / L - dm * dm;           // Eq. 7 about the new mean
      v = v > 0.0 ? v : 0.0;
      v = v > var_floor ? v : var_floor;  // floor, Sec. 2.2
      means[(size_t)g * D + d] = (XT)mu;
      covs[(size_t)g * D + d] = (XT)v;
      if (!isfinite(mu) || !isfinite(v)) bad = 1;
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

__global__ void k_ll_finish(const double* __restrict__ ll_part, int nb, int64_t N,
                            double* __restrict__ mean_loglik, int32_t* __restrict__ dev_status) {
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += ll_part[b];
    *mean_loglik = s / (double)N;
    if (!isfinite(s)) atomicOr(dev_status, GMM_DEV_NONFINITE);
  }
}

// Per-Gaussian log-density (Sec. 4 API log_p(X, g), avg_log_p(X, g)) of a
// diagonal model, without the weight: log N(x | mu_g, Sigma_g) =
// -1/2 (D log 2 pi + sum_d log sigma2_gd + sum_d (x_d - mu_gd)^2 / sigma2_gd),
// in FP64 per sample.  Tiles of kLT samples pass through LDS kLD dimensions at
// a time (coalesced row segments); thread t of the workgroup owns sample t of
// each tile and keeps its running sum of values; the workgroup's total, in a
// fixed order, goes to part[b].
constexpr int kLT = 256;
constexpr int kLD = 32;
__global__ void __launch_bounds__(kLT) k_log_p_g(const float* __restrict__ X, int64_t N, int D,
                                                 int64_t ldx, int g,
                                                 const float* __restrict__ means,
                                                 const float* __restrict__ dcovs, int64_t chunk,
                                                 float* __restrict__ per_sample,
                                                 double* __restrict__ part,
                                                 int32_t* __restrict__ dev_status) {
  __shared__ float xs[kLT][kLD + 1];
  __shared__ double lam[kLD], mu[kLD];
  __shared__ double sh[kLT];
  const int tid = threadIdx.x;
  const int b = blockIdx.x;
  const int64_t i0 = (int64_t)b * chunk;
  const int64_t i1 = min(N, i0 + chunk);
  const float* mg = means + (size_t)g * D;
  const float* vg = dcovs + (size_t)g * D;
  // c = -1/2 (D log 2 pi + sum_d log sigma2_d), summed in a fixed order
  double ld = 0.0;
  for (int d = tid; d < D; d += kLT) ld += log((double)vg[d]);
  ld = block_sum_d<kLT>(ld, sh);
  const double c = -0.5 * ((double)D * 1.8378770664093454836 + ld);  // log 2 pi
  double acc = 0.0;
  bool bad = false;
  for (int64_t t0 = i0; t0 < i1; t0 += kLT) {
    const int nt = (int)min((int64_t)kLT, i1 - t0);
    double q = 0.0;
    for (int d0 = 0; d0 < D; d0 += kLD) {
      const int nd = min(kLD, D - d0);
      __syncthreads();  // the previous chunk's readers are done
      for (int p = tid; p < nt * nd; p += kLT) {
        const int t = p / nd, k = p - t * nd;
        xs[t][k] = X[(t0 + t) * ldx + d0 + k];
      }
      if (tid < nd) {
        lam[tid] = 1.0 / (double)vg[d0 + tid];
        mu[tid] = (double)mg[d0 + tid];
      }
      __syncthreads();
      if (tid < nt)
        for (int k = 0; k < nd; ++k) {
          const double u = (double)xs[tid][k] - mu[k];
          q += u * u * lam[k];
        }
    }
    if (tid < nt) {
      const double a = c - 0.5 * q;
      if (per_sample) per_sample[t0 + tid] = (float)a;
      if (!isfinite(a)) bad = true;
      acc += a;
    }
  }
  acc = block_sum_d<kLT>(acc, sh);
  if (tid == 0) part[b] = acc;
  if (bad) atomicOr(dev_status, GMM_DEV_NONFINITE);
}

// LDS bytes of k_estep_diag for tile rows T (WIDE: rows of xs padded to 4,
// rows of as padded by 8, and the per-block references rcb); esz: bytes of a
// sample value (4, or 8 for FP64 data).
size_t estep_lds(int D, int G, int T, bool wide, size_t esz = sizeof(float)) {
  const size_t XS = wide ? (size_t)((D + 3) & ~3) : (size_t)D;
  const size_t AS = wide ? (size_t)G + 8 : (size_t)G;
  size_t b = esz * ((size_t)T * (XS + AS) + 1) + sizeof(double) * T;
  b += sizeof(uint32_t) * (((size_t)(G + 31) / 32 + 3) / 4 * 4);
  if (wide) b += sizeof(float) * (size_t)T * ((G + 15) / 16);
  return b;
}

// The WIDE form (exact FP64 log-densities on the matrix cores) is used for
// D <= 128 and more components than the one-pass kernels take, when its tile
// fits in LDS.
bool use_wide(int D, int G) {
  return D <= 128 && G > 128 && estep_lds(D, G, kWT, true) <= 159 * 1024;  // + static LDS
}

template <bool MSTEP, bool WIDE, typename XT, typename... Args>
void launch_estep_diag(int nb, size_t lds, hipStream_t st, Args... args) {
  auto kern = k_estep_diag<MSTEP, WIDE, XT>;
  // dynamic LDS above the 64 KB default: raise the kernel's limit to exactly
  // this launch's size (limit plus static LDS must fit the CU's 160 KB)
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  hipLaunchKernelGGL(kern, dim3(nb), dim3(kNT), lds, st, args...);
}

int tile_rows(int D, int G) {
  int T = 64;
  while (T > 1 && (size_t)T * (D + G + 2) * sizeof(float) + (size_t)(G / 8 + 8) > 60 * 1024)
    T >>= 1;
  return T;
}

// EM iteration (mstep) or log-likelihood of the tile kernels: WIDE (FP64
// matrix cores, the only form for FP64 data) or the FP32 direct form.
template <typename XT>
hipError_t em_tiles(const XT* X, int64_t N, int D, int64_t ldx, int G, const XT* hefts_in,
                    XT* hefts, XT* means, XT* covs, double var_floor, bool wide, bool mstep,
                    double* mean_loglik, XT* per_sample, int64_t* n_recomputed,
                    int32_t* dev_status, const Workspace& w, hipStream_t st) {
  const int T = wide ? kWT : tile_rows(D, G);
  const int nb = partial_blocks(N, 4 * T);
  int64_t chunk = (N + nb - 1) / nb;
  const size_t lds = estep_lds(D, G, T, wide, sizeof(XT));
  hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, st, dev_status, n_recomputed, w.counters);
  hipLaunchKernelGGL(k_pre_diag<XT>, dim3(G), dim3(kNT), 0, st, hefts_in, (const XT*)means,
                     (const XT*)covs, D, G, w.s, w.m, w.c, w.c64, w.lamg64);
  if (wide)
    hipLaunchKernelGGL(k_frag_diag64<XT>, dim3(16 * ((G + 15) / 16)), dim3(kNT), 0, st,
                       (const XT*)means, (const double*)w.lamg64, (const double*)w.c64, D, G,
                       w.Bx64, w.cq64);
  {
    ProfScope ps(mstep ? kProfEM : kProfLoglik, st);
#define GMM_ESTEP_ARGS                                                                      \
  nb, lds, st, X, N, D, ldx, G, T, chunk, (const float*)w.s, (const float*)w.m,             \
      (const float*)w.c, (const double*)w.c64, (const double*)w.lamg64,                     \
      (const double*)w.Bx64, (const double*)w.cq64, (const XT*)means, w.partials, w.scalars, \
      per_sample, dev_status
    if constexpr (sizeof(XT) == 8) {
      if (mstep) launch_estep_diag<true, true, XT>(GMM_ESTEP_ARGS);
      else launch_estep_diag<false, true, XT>(GMM_ESTEP_ARGS);
    } else {
      if (wide && mstep) launch_estep_diag<true, true, XT>(GMM_ESTEP_ARGS);
      else if (wide) launch_estep_diag<false, true, XT>(GMM_ESTEP_ARGS);
      else if (mstep) launch_estep_diag<true, false, XT>(GMM_ESTEP_ARGS);
      else launch_estep_diag<false, false, XT>(GMM_ESTEP_ARGS);
    }
#undef GMM_ESTEP_ARGS
  }
  if (!mstep) {
    hipLaunchKernelGGL(k_ll_finish, dim3(1), dim3(64), 0, st, w.scalars, nb, N, mean_loglik,
                       dev_status);
    return hipGetLastError();
  }
  // [2D + 1] FP64 totals: above the 64 KB default for D > 4095
  const size_t fin_lds = sizeof(double) * (2 * D + 1);
  if (fin_lds > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)k_fin_diag<XT>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)fin_lds);
  hipLaunchKernelGGL(k_fin_diag<XT>, dim3(G), dim3(kNT), fin_lds, st, w.partials, nb, N, D, G,
                     var_floor, hefts, means, covs, w.scalars, mean_loglik, dev_status);
  return hipGetLastError();
}

}  // namespace

int em_diag_path(int D, int G, int prec) {
  if (em_fast_supported(D, G, prec))
    return prec == GMM_PREC_BF16X3 ? GMM_PATH_ONEPASS_BF16X3 : GMM_PATH_ONEPASS_FP32;
  if (prec == GMM_PREC_BF16X3 && G > 128 && em2s_supported(D, G)) return GMM_PATH_SLICED_BF16X3;
  return use_wide(D, G) ? GMM_PATH_WIDE_FP64 : GMM_PATH_GENERIC;
}

bool em_f64_supported(int D, int G) {
  return D >= 1 && D <= 128 && G >= 1 &&
         estep_lds(D, G, kWT, true, sizeof(double)) <= 159 * 1024;
}

hipError_t launch_pre_diag(const float* hefts, const float* means, const float* covs, int D,
                           int G, const Workspace& w, hipStream_t st) {
  hipLaunchKernelGGL(k_pre_diag<float>, dim3(G), dim3(kNT), 0, st, hefts, means, covs, D, G, w.s,
                     w.m, w.c, w.c64, w.lamg64);
  return hipGetLastError();
}

hipError_t launch_em_diag(const float* X, int64_t N, int D, int64_t ldx, int G, float* hefts,
                          float* means, float* covs, float var_floor, int prec,
                          double* mean_loglik, int64_t* n_recomputed, int32_t* dev_status,
                          const Workspace& w, hipStream_t st) {
  const int path = em_diag_path(D, G, prec);
  if (path == GMM_PATH_ONEPASS_BF16X3 || path == GMM_PATH_ONEPASS_FP32) {
    int nb = 0;
    // k_pre_fast clears the status word and the counters
    hipError_t e = launch_em_fast(X, N, D, ldx, G, hefts, means, covs, prec, true, n_recomputed,
                                  nullptr, dev_status, w, st, &nb);
    if (e != hipSuccess) return e;
    return launch_fin_welford(nb, N, D, G, var_floor, hefts, means, covs, mean_loglik,
                              dev_status, w, st);
  }
  if (path == GMM_PATH_SLICED_BF16X3) {
    int nb = 0;
    hipError_t e = launch_em_sliced(X, N, D, ldx, G, hefts, means, covs, true, n_recomputed,
                                    nullptr, dev_status, w, st, &nb);
    if (e != hipSuccess) return e;
    return launch_fin_welford(nb, N, D, G, var_floor, hefts, means, covs, mean_loglik,
                              dev_status, w, st);
  }
  return em_tiles<float>(X, N, D, ldx, G, hefts, hefts, means, covs, (double)var_floor,
                         path == GMM_PATH_WIDE_FP64, true, mean_loglik, nullptr, n_recomputed,
                         dev_status, w, st);
}

hipError_t launch_em_diag_f64(const double* X, int64_t N, int D, int64_t ldx, int G,
                              double* hefts, double* means, double* covs, double var_floor,
                              double* mean_loglik, int32_t* dev_status, const Workspace& w,
                              hipStream_t st) {
  return em_tiles<double>(X, N, D, ldx, G, hefts, hefts, means, covs, var_floor, true, true,
                          mean_loglik, nullptr, nullptr, dev_status, w, st);
}

hipError_t launch_loglik_diag_f64(const double* X, int64_t N, int D, int64_t ldx, int G,
                                  const double* hefts, const double* means, const double* covs,
                                  double* mean_loglik, double* per_sample, int32_t* dev_status,
                                  const Workspace& w, hipStream_t st) {
  return em_tiles<double>(X, N, D, ldx, G, hefts, nullptr, (double*)means, (double*)covs, 0.0,
                          true, false, mean_loglik, per_sample, nullptr, dev_status, w, st);
}

hipError_t launch_log_p_gaussian(const float* X, int64_t N, int D, int64_t ldx, int g,
                                 const float* means, const float* dcovs, double* mean_out,
                                 float* per_sample, int32_t* dev_status, const Workspace& w,
                                 hipStream_t st) {
  const int nb = partial_blocks(N, 4 * kLT);
  const int64_t chunk = (N + nb - 1) / nb;
  hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, st, dev_status, nullptr, w.counters);
  hipLaunchKernelGGL(k_log_p_g, dim3(nb), dim3(kLT), 0, st, X, N, D, ldx, g, means, dcovs, chunk,
                     per_sample, w.scalars, dev_status);
  if (mean_out)
    hipLaunchKernelGGL(k_ll_finish, dim3(1), dim3(64), 0, st, w.scalars, nb, N, mean_out,
                       dev_status);
  return hipGetLastError();
}

hipError_t launch_loglik_diag(const float* X, int64_t N, int D, int64_t ldx, int G,
                              const float* hefts, const float* means, const float* covs, int prec,
                              double* mean_loglik, float* per_sample, int32_t* dev_status,
                              const Workspace& w, hipStream_t st) {
  const int path = em_diag_path(D, G, prec);
  if (path == GMM_PATH_ONEPASS_BF16X3 || path == GMM_PATH_ONEPASS_FP32) {
    int nb = 0;
    // k_pre_fast clears the status word and the counters
    hipError_t e = launch_em_fast(X, N, D, ldx, G, hefts, means, covs, prec, false, nullptr,
                                  per_sample, dev_status, w, st, &nb);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ll_finish, dim3(1), dim3(64), 0, st, w.scalars, nb, N, mean_loglik,
                       dev_status);
    return hipGetLastError();
  }
  if (path == GMM_PATH_SLICED_BF16X3) {
    int nb = 0;
    hipError_t e = launch_em_sliced(X, N, D, ldx, G, hefts, means, covs, false, nullptr,
                                    per_sample, dev_status, w, st, &nb);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ll_finish, dim3(1), dim3(64), 0, st, w.scalars, nb, N, mean_loglik,
                       dev_status);
    return hipGetLastError();
  }
  return em_tiles<float>(X, N, D, ldx, G, hefts, nullptr, (float*)means, (float*)covs, 0.0,
                         path == GMM_PATH_WIDE_FP64, false, mean_loglik, per_sample, nullptr,
                         dev_status, w, st);
}

}  // namespace gmm
