// gmm_em_fast.hip -- one-pass EM kernels for diagonal covariances with up to
// 128 Gaussians and 128 dimensions (the shapes of the D=100/G=100 and batched
// D=40 workloads).  Shapes outside that envelope use the generic kernels of
// gmm_em.hip.  Two arithmetic forms:
//   k_em2      the expanded form c'_g + sum_k A_gk B_kn (Sec. 2.2 Eq. 15
//              expanded, A_g = [Lambda_g mu_g ; -1/2 Lambda_g], B_n = [x_n ;
//              x_n^2]) on the matrix cores, v_mfma_f32_16x16x32_bf16 with both
//              operands split into BF16 hi + lo and the three products hi*hi,
//              hi*lo, lo*hi accumulated in FP32; described at its definition;
//   k_em_fast  the FP32 direct form on the vector ALUs, described here.
//
// k_em_fast: workgroup of 8 waves, persistent over a contiguous range of
// samples, tiles of T = 32 samples; the next tile is loaded into registers (all
// loads issued at once) while the current one is processed.  Per tile:
//   1. the tile's samples are staged in LDS (xf[n][d]);
//   2. screening: FP32 log-densities a_gn = c_g - 1/2 sum_d (x_d s_gd - m_gd)^2
//      of every (component, sample) pair (s = 1/sigma, m = mu/sigma, staged in
//      LDS);
//   3. per sample, M_n = max_g (a_gn - e_gn), a lower bound of the exact best
//      log-density, where e_gn bounds the rounding error of the screening value
//      (err_direct: from q = 2 (c_g - a_gn) and Q_g = sum_d lam_gd mu_gd^2),
//      and the near set {g: a_gn + e_gn >= M_n - 30}.
//      Near (sample, component) pairs are recomputed by 8-lane groups: in FP64
//      from the FP32 parameters when the sample has two or more near
//      components (their relative values decide shared responsibilities), else
//      in the FP32 direct form when its bound is below 1e-3 nats (FP64
//      otherwise): that value sets the sample's log-likelihood.  A component
//      with a tiny variance (a floored one-sample cluster) has a huge e_gn, so
//      its pairs join the near set wherever its exact value could matter;
//   4. log-sum-exp per sample (Eqs. 16-18) about M_n + max(recomputed - M_n),
//      summed in FP64; responsibilities (Eq. 3); those below exp(-40) are 0;
//   5. the map step of Sec. 2.1 (Eqs. 9-11) in a weighted Welford form (West's
//      update) on the deviations y = x - mu_old from the current mean: wave w
//      owns components g = w, w+8, ...; lane owns dimensions d = lane, lane+64
//      (the old means sit in LDS);
//      for every sample with a non-zero responsibility r, in sample order,
//        L' = L + r, delta = y - m, m += delta r / L', Q += delta^2 r L / L'
//      except that a sample carrying more than half of L' sets
//      m = y - delta L / L' (rounded relative to its own y, not to a mean
//      that earlier, far-off samples of tiny weight have set; the first
//      sample sets m = y exactly).  m is the block's weighted mean of
//      y and Q its weighted sum of squared deviations from it; neither update
//      subtracts two large accumulated sums, so the one-pass covariance of
//      Eq. 8 loses nothing to cancellation (one sample gives Q = 0 exactly).
//      Blocks are combined in fixed order by the pairwise update of (L, m, Q)
//      in FP64 (k_fin_welford).
#include "gmm_internal.hpp"

namespace gmm {

namespace {

constexpr int kNW = 8;            // waves per workgroup
constexpr int kThreads = kNW * kWave;
constexpr int kT = 32;            // samples per tile
constexpr int kPF = 8;            // prefetch registers per thread: kT * 128 / kThreads


struct FastArgs {
  const float* X;
  int64_t N;
  int64_t ldx;
  int64_t chunk;
  int D, G, KS;             // KS: number of 32-deep k-steps of the expanded form
  const float* prm;         // [2][G][D+1]: s then m
  const float* cc;          // [2][G] direct-form constant, hi/lo
  const float* cexp;        // [2][G] expanded-form constant, hi/lo
  const bf16x8* Whi;        // [RB][KS][64] fragments of A (hi)
  const bf16x8* Wlo;        // same, lo part
  const double* c64;        // [G]
  const double* lam64;      // [G][D]
  const float* means;       // [G][D] current means (centre of the moments)
  double* part;             // [nb][G][2D+1]
  double* ll_part;          // [nb]
  float* per_sample;        // [N] or null
  int32_t* dev_status;
  int64_t* n_rec;           // or null
  // component slices (sliced passes only): the pass works on components
  // g0 .. g0 + G - 1 of Gt; per-sample, per-slice arrays [S][NS]
  int g0, Gt, Gs, sl, S;
  int64_t NS;
  float* wM;                // bounded maximum of the slice's values
  float* wD;                // reference of the slice's sum: largest exact near value - M
  float* wS;                // sum over the slice of exp(value - M - wD)
  float* wR;                // [S][NG][kCapR] exact near values of MODE 2 (value - M), read by MODE 3
  int64_t NG;               // 16-sample groups: ceil(N / 16)
};

// LDS layout of k_em_fast: the direct-form parameters are staged (ps, pm); the
// moment accumulators live in registers.
struct Lds {
  float* ps;        // [G][D+1]
  float* pm;        // [G][D+1]
  float* xf;        // [T][D]
  float* as;        // [G][T]
  float* mu;        // [G][D] current means
  float* pmax;      // [NW][T]
  double* psum;     // [NW][T]
  uint32_t* nbits;  // [T][4]
  int* ncnt;        // [T]
  int* pcount;      // [1]
  uint16_t* plist;  // [T*G]
  float* cq;        // [3][G] c_g (hi), Q_g = sum_d lam mu^2, c lo
  int* dmax;        // [T] max over the near set of (a - M_lo), order-mapped
};

template <typename F>
__host__ __device__ inline size_t lds_walk(int D, int G, F&& at) {
  size_t w = 0;
  auto put = [&](int which, size_t words, size_t align_words) {
    w = (w + align_words - 1) / align_words * align_words;
    at(which, w);
    w += words;
  };
  put(0, (size_t)G * (D + 1), 1);
  put(1, (size_t)G * (D + 1), 1);
  put(2, (size_t)kT * D, 4);
  put(3, (size_t)G * kT, 1);
  put(7, kNW * kT, 1);
  put(8, 2 * kNW * kT, 2);
  put(9, kT * 4, 1);
  put(10, kT, 1);
  put(11, 1, 1);
  put(12, ((size_t)kT * G + 1) / 2, 1);
  put(13, (size_t)G * D, 1);
  put(14, (size_t)3 * G, 1);
  put(15, kT, 1);
  return w;
}

__host__ __device__ inline size_t fast_lds_bytes(int D, int G) {
  return lds_walk(D, G, [](int, size_t) {}) * 4 + 64;
}

__device__ inline Lds carve_lds(char* base, int D, int G) {
  Lds L;
  float* f = (float*)base;
  lds_walk(D, G, [&](int which, size_t off) {
    switch (which) {
      case 0: L.ps = f + off; break;
      case 1: L.pm = f + off; break;
      case 2: L.xf = f + off; break;
      case 3: L.as = f + off; break;
      case 7: L.pmax = f + off; break;
      case 8: L.psum = (double*)(f + off); break;
      case 9: L.nbits = (uint32_t*)(f + off); break;
      case 10: L.ncnt = (int*)(f + off); break;
      case 11: L.pcount = (int*)(f + off); break;
      case 12: L.plist = (uint16_t*)(f + off); break;
      case 13: L.mu = f + off; break;
      case 14: L.cq = f + off; break;
      default: L.dmax = (int*)(f + off); break;
    }
  });
  return L;
}

__device__ __forceinline__ double group8_sum_d(double v) {
  v += __shfl_xor(v, 1, kWave);
  v += __shfl_xor(v, 2, kWave);
  v += __shfl_xor(v, 4, kWave);
  return v;
}

// Global -> register load of one tile: element p = tid + 512 i of the tile's
// nt x D block (row-major); every load of the tile is issued before any use.
__device__ __forceinline__ void tile_prefetch(const FastArgs& a, int64_t t0, int nt, int tid,
                                              float (&pf)[kPF]) {
  const int D = a.D;
  const int tot = nt * D;
  if (a.ldx == D) {
    const float* src = a.X + t0 * D;
#pragma unroll
    for (int i = 0; i < kPF; ++i) {
      const int p = tid + kThreads * i;
      pf[i] = p < tot ? src[p] : 0.0f;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kPF; ++i) {
      const int p = tid + kThreads * i;
      float v = 0.0f;
      if (p < tot) {
        const int n = p / D, d = p - n * D;
        v = a.X[(t0 + n) * a.ldx + d];
      }
      pf[i] = v;
    }
  }
}

// The tile loop over samples [i0, i1) of one model; partials go to slot b.
template <int CPW, int DPL, bool MSTEP>
__device__ __forceinline__ void em_range(const FastArgs& a, int64_t i0, int64_t i1, int b,
                                         char* lds_raw) {
  const int D = a.D, G = a.G;
  const int DP = D + 1;
  const Lds L = carve_lds(lds_raw, D, G);
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int w = tid / kWave;

  const int P = 2 * D + 1;
  for (int g = tid; g < G; g += kThreads) {
    const float c = a.cc[g];
    // Q_g from the two forms' constants: c - cexp = Q_g / 2
    const float Q = 2.0f * ((c + a.cc[G + g]) - (a.cexp[g] + a.cexp[G + g]));
    L.cq[g] = c;
    L.cq[G + g] = isfinite(Q) ? 1.0001f * fmaxf(Q, 0.0f) : 0.0f;
    L.cq[2 * G + g] = a.cc[G + g];
  }
  // rounding-error bound (nats) of a screening value v of component g
  auto scr_err = [&](float v, int g) -> float {
    const float c = L.cq[g], Q = L.cq[G + g];
    return err_direct(2.0f * (c - v), Q, c, D);
  };
  // stage the direct-form parameters and the current means
  for (int p = tid; p < G * DP; p += kThreads) {
    L.ps[p] = a.prm[p];
    L.pm[p] = a.prm[(size_t)G * DP + p];
  }
  if (MSTEP)
    for (int p = tid; p < G * D; p += kThreads) L.mu[p] = a.means[p];

  // Welford accumulators of component g = w + 8c, dimension d = lane + 64j
  float S1[CPW][DPL], S2[CPW][DPL], Lc[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    Lc[c] = 0.0f;
#pragma unroll
    for (int j = 0; j < DPL; ++j) {
      S1[c][j] = 0.0f;
      S2[c][j] = 0.0f;
    }
  }
  double llacc = 0.0;  // lanes < kT of wave 0: samples n = lane of every tile
  int bad = 0;
  long long nrec = 0;

  float pf[kPF];
  if (i0 < i1) tile_prefetch(a, i0, (int)min((int64_t)kT, i1 - i0), tid, pf);

  for (int64_t t0 = i0; t0 < i1; t0 += kT) {
    const int nt = (int)min((int64_t)kT, i1 - t0);
    // 1. samples loaded last iteration -> LDS (zeros past the tail); the next
    // tile's loads are issued right after
#pragma unroll
    for (int i = 0; i < kPF; ++i) {
      const int p = tid + kThreads * i;
      if (p < kT * D) L.xf[p] = pf[i];
    }
    if (t0 + kT < i1) tile_prefetch(a, t0 + kT, (int)min((int64_t)kT, i1 - t0 - kT), tid, pf);
    if (tid < kT) {
      L.ncnt[tid] = 0;
      L.dmax[tid] = f2ord(-INFINITY);
      L.nbits[tid * 4 + 0] = L.nbits[tid * 4 + 1] = L.nbits[tid * 4 + 2] = L.nbits[tid * 4 + 3] = 0u;
    }
    if (tid == 0) *L.pcount = 0;
    __syncthreads();

    // 2. screening
    {
      // direct form: thread owns component g = lane + 64 (w & 1) and samples
      // n = 8 (w >> 1) .. + 7
      const int g = lane + kWave * (w & 1);
      const int n0 = 8 * (w >> 1);
      if (g < G) {
        float acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = 0.0f;
        const float* sg = L.ps + g * DP;
        const float* mg = L.pm + g * DP;
        for (int d = 0; d < D; ++d) {
          const float s = sg[d], m = mg[d];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const float u = fmaf(L.xf[(n0 + q) * D + d], s, -m);
            acc[q] = fmaf(u, u, acc[q]);
          }
        }
        const float chi = L.cq[g], clo = L.cq[2 * G + g];
#pragma unroll
        for (int q = 0; q < 8; ++q) L.as[g * kT + n0 + q] = (chi - 0.5f * acc[q]) + clo;
      }
    }
    __syncthreads();

    // 3a. per-sample M_lo = max_g (v_g - err_g), a lower bound of the exact
    // maximum: wave w scans components g = w + 8c; lane n = lane%32, half =
    // lane/32 takes every other one
    const int n = lane & (kT - 1);
    const int half = lane >> 5;
    {
      float mx = -INFINITY;
      for (int g = w + kNW * half; g < G; g += 2 * kNW) {
        const float v = L.as[g * kT + n];
        mx = fmaxf(mx, v - scr_err(v, g));
      }
      mx = fmaxf(mx, __shfl_xor(mx, 32, kWave));
      if (half == 0) L.pmax[w * kT + n] = mx;
    }
    __syncthreads();
    float M = -INFINITY;
#pragma unroll
    for (int q = 0; q < kNW; ++q) M = fmaxf(M, L.pmax[q * kT + n]);
    // 3b. near pairs: those whose value could come within kNearGap of the maximum
    if (n < nt) {
      for (int g = w + kNW * half; g < G; g += 2 * kNW) {
        const float v = L.as[g * kT + n];
        if (v + scr_err(v, g) >= M - kNearGap) {
          const int slot = atomicAdd(L.pcount, 1);
          L.plist[slot] = (uint16_t)((n << 8) | g);
          atomicAdd(&L.ncnt[n], 1);
          atomicOr(&L.nbits[n * 4 + (g >> 5)], 1u << (g & 31));
        }
      }
    }
    __syncthreads();
    // 3c. recompute near pairs, one 8-lane group per pair: FP64 when the sample
    // has two or more, else the FP32 direct form if its bound is below
    // kExactTol (FP64 otherwise).  Entries then hold a - M_lo; dmax[n] gets
    // their maximum.
    {
      const int np = *L.pcount;
      const int grp = tid >> 3, gl = tid & 7;
      for (int p = grp; p < np; p += kThreads / 8) {
        const int code = L.plist[p];
        const int pn = code >> 8, g = code & 255;
        const float* x = L.xf + pn * D;
        float Mp = -INFINITY;
#pragma unroll
        for (int q = 0; q < kNW; ++q) Mp = fmaxf(Mp, L.pmax[q * kT + pn]);
        bool exact64 = L.ncnt[pn] >= 2;
        double val = 0.0;
        if (!exact64) {
          // the screening value is already the direct form
          const float v = L.as[g * kT + pn];
          val = (double)v;
          exact64 = !(err_direct(2.0f * (L.cq[g] - v), L.cq[G + g], L.cq[g], D) <= kExactTol);
        }
        if (exact64) {
          const float* mu_g = a.means + (size_t)g * D;
          const double* lg = a.lam64 + (size_t)g * D;
          double q = 0.0;
          for (int d = gl; d < D; d += 8) {
            const double u = (double)x[d] - (double)mu_g[d];
            q += u * u * lg[d];
          }
          q = group8_sum_d(q);
          val = a.c64[g] - 0.5 * q;
        }
        if (gl == 0) {
          const float rel = (float)(val - (double)Mp);
          L.as[g * kT + pn] = rel;
          atomicMax(&L.dmax[pn], f2ord(rel));
          if (exact64) ++nrec;
        }
      }
    }
    __syncthreads();
    // 4. log-sum-exp about M_lo + dmax: entries of near pairs hold a - M_lo,
    // the rest the screening value (each at least kNearGap below the maximum)
    float Dn = ord2f(L.dmax[n]);
    Dn = Dn > -INFINITY ? Dn : 0.0f;  // padding samples have no near pair
    {
      double s = 0.0;
      for (int g = w + kNW * half; g < G; g += 2 * kNW) {
        const bool near = (L.nbits[n * 4 + (g >> 5)] >> (g & 31)) & 1u;
        const float v = L.as[g * kT + n];
        s += (double)__expf(near ? v - Dn : (v - M) - Dn);
      }
      s += __shfl_xor(s, 32, kWave);
      if (half == 0) L.psum[w * kT + n] = s;
    }
    __syncthreads();
    double tot = 0.0;
#pragma unroll
    for (int q = 0; q < kNW; ++q) tot += L.psum[q * kT + n];
    const double lse = ((double)M + (double)Dn) + log(tot);
    if (w == 0 && half == 0 && n < nt) {
      llacc += lse;
      if (!isfinite(lse)) bad = 1;
      if (a.per_sample) a.per_sample[t0 + n] = (float)lse;
    }
    if (MSTEP) {
      const float dl = (float)log(tot);
      for (int g = w + kNW * half; g < G; g += 2 * kNW) {
        const bool near = (L.nbits[n * 4 + (g >> 5)] >> (g & 31)) & 1u;
        const float v = L.as[g * kT + n];
        const float z = (near ? v - Dn : (v - M) - Dn) - dl;
        L.as[g * kT + n] = (n < nt && z >= -kRespCut) ? __expf(z) : 0.0f;
      }
      // 5. moments of this wave's components (written above by this wave only)
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const int g = w + kNW * c;
        if (g < G) {
          const float r_l = lane < kT ? L.as[g * kT + lane] : 0.0f;
          unsigned long long msk = __ballot(r_l != 0.0f);
          while (msk) {
            const int nn = __ffsll((long long)msk) - 1;
            msk &= msk - 1;
            const float r = L.as[g * kT + nn];
            const float Lo = Lc[c];
            const float Ln = Lo + r;
            const float inv = r / Ln;
            const float wo = Lo / Ln;
            const float w2 = inv * Lo;
            const bool dom = inv > 0.5f;  // the sample outweighs the run so far
            Lc[c] = Ln;
#pragma unroll
            for (int j = 0; j < DPL; ++j) {
              const int d = lane + kWave * j;
              if (d < D) {
                const float y = L.xf[nn * D + d] - L.mu[g * D + d];
                if (Lo == 0.0f) {
                  S1[c][j] = y;
                } else {
                  const float dl = y - S1[c][j];
                  S1[c][j] = dom ? fmaf(-wo, dl, y) : fmaf(inv, dl, S1[c][j]);
                  S2[c][j] = fmaf(w2 * dl, dl, S2[c][j]);
                }
              }
            }
          }
        }
      }
    }
    __syncthreads();
  }

  // block partials in FP64
  if (MSTEP) {
    double* pb = a.part + (size_t)b * G * P;
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int g = w + kNW * c;
      if (g < G) {
        if (lane == 0) pb[(size_t)g * P] = (double)Lc[c];
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
          const int d = lane + kWave * j;
          if (d < D) {
            pb[(size_t)g * P + 1 + d] = (double)S1[c][j];
            pb[(size_t)g * P + 1 + D + d] = (double)S2[c][j];
          }
        }
      }
    }
  }
  // log-likelihood: lanes 0..31 of wave 0, fixed-order tree
  if (w == 0) {
    double v = lane < kT ? llacc : 0.0;
    v = wave_sum_d(v);
    if (lane == 0) a.ll_part[b] = v;
  }
  if (bad) atomicOr(a.dev_status, GMM_DEV_NONFINITE);
  if (a.n_rec) {
    long long v = nrec;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    if (lane == 0 && v) atomicAdd((unsigned long long*)a.n_rec, (unsigned long long)v);
  }
}

template <int CPW, int DPL, bool MSTEP>
__global__ void __launch_bounds__(kThreads) k_em_fast(FastArgs a) {
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  const int b = blockIdx.x;
  const int64_t i0 = (int64_t)b * a.chunk;
  const int64_t i1 = min(a.N, i0 + a.chunk);
  em_range<CPW, DPL, MSTEP>(a, i0, i1, b, lds_raw);
}

// ---- many models ----------------------------------------------------------

// Per-model constants live at model * stride in each of these regions.
struct BatchConst {
  float* prm;      // stride 2 * Gmax * (D+1)
  float* cc;       // stride 2 * Gmax
  float* cexp;     // stride 2 * Gmax
  bf16x8* Whi;     // stride RBmax * KS * 64
  bf16x8* Wlo;
  double* c64;     // stride Gmax
  double* lam64;   // stride Gmax * D
  int Gmax, RBmax, KS;
};

template <int CPW, int DPL, bool MSTEP>
__global__ void __launch_bounds__(kThreads) k_em_fast_batched(FastArgs base,
                                                              const gmm_model_desc* models,
                                                              const BatchItemDev* items,
                                                              const int* n_items, BatchConst bc) {
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  const int ni = *n_items;
  const int D = base.D;
  const int P = 2 * D + 1;
  for (int it = blockIdx.x; it < ni; it += gridDim.x) {
    const BatchItemDev item = items[it];
    const gmm_model_desc& m = models[item.model];
    FastArgs a = base;
    const size_t mi = (size_t)item.model;
    a.X = m.X;
    a.N = m.N;
    a.ldx = D;
    a.G = m.G;
    a.prm = bc.prm + mi * 2 * bc.Gmax * (D + 1);
    a.cc = bc.cc + mi * 2 * bc.Gmax;
    a.cexp = bc.cexp + mi * 2 * bc.Gmax;
    a.Whi = bc.Whi + mi * bc.RBmax * bc.KS * 64;
    a.Wlo = bc.Wlo + mi * bc.RBmax * bc.KS * 64;
    a.c64 = bc.c64 + mi * bc.Gmax;
    a.lam64 = bc.lam64 + mi * bc.Gmax * D;
    a.means = m.means;
    a.part = base.part + (size_t)it * bc.Gmax * P;
    a.ll_part = base.ll_part + it;
    a.per_sample = nullptr;
    a.dev_status = m.dev_status;
    a.n_rec = nullptr;
    em_range<CPW, DPL, MSTEP>(a, item.i0, item.i1, 0, lds_raw);
    __syncthreads();
  }
}

// Per-component constants of the fast kernel for component g (one workgroup).
__device__ void pre_component(const float* __restrict__ hefts, const float* __restrict__ means,
                              const float* __restrict__ covs, int D, int G, int KS, int g,
                              float* __restrict__ prm, float* __restrict__ cc,
                              float* __restrict__ cexp, bf16x8* __restrict__ Whi,
                              bf16x8* __restrict__ Wlo, double* __restrict__ c64,
                              double* __restrict__ lam64) {
  __shared__ double sh[256];
  const int DP = D + 1;
  double ld = 0.0, q = 0.0;
  for (int d = threadIdx.x; d < D; d += 256) {
    const double v = (double)covs[(size_t)g * D + d];
    const double mu = (double)means[(size_t)g * D + d];
    const double lam = 1.0 / v;
    const double s = sqrt(lam);
    prm[(size_t)g * DP + d] = (float)s;
    prm[(size_t)G * DP + (size_t)g * DP + d] = (float)(mu * s);
    lam64[(size_t)g * D + d] = lam;
    ld += log(v);
    q += lam * mu * mu;
  }
  if (threadIdx.x == 0) {
    prm[(size_t)g * DP + D] = 0.0f;
    prm[(size_t)G * DP + (size_t)g * DP + D] = 0.0f;
  }
  const double logdet = block_sum_d<256>(ld, sh);
  const double quad = block_sum_d<256>(q, sh);
  if (threadIdx.x == 0) {
    const double c = log((double)hefts[g]) - 0.5 * ((double)D * kLog2Pi + logdet);
    const float hi = (float)c;
    cc[g] = hi;
    cc[G + g] = isfinite(c) ? (float)(c - (double)hi) : 0.0f;
    c64[g] = c;
    const double ce = c - 0.5 * quad;
    const float ehi = (float)ce;
    cexp[g] = ehi;
    cexp[G + g] = isfinite(ce) ? (float)(ce - (double)ehi) : 0.0f;
  }
  // MFMA fragments of component g's row: the coefficient A_gk of feature k is
  // lam mu for the feature x_d and -lam/2 for x_d^2, 0 beyond, interleaved:
  // k = 2d for x_d, k = 2d + 1 for x_d^2.  The fragment of (row block, k-step
  // ks, lane l) holds features 32 ks + 8 (l/16) + i, i = 0..7, of component
  // 16 rb + l%16.
  const int rb = g >> 4, row = g & 15;
  for (int e = threadIdx.x; e < KS * 4 * 8; e += 256) {
    const int ks = e / 32, r = e - ks * 32, lq = r >> 3, i = r & 7;
    const int k = 32 * ks + 8 * lq + i;
    const int d = k >> 1;
    const bool sq = k & 1;
    float v = 0.0f;
    if (d < D && k < 2 * D) {
      const double lam = 1.0 / (double)covs[(size_t)g * D + d];
      v = sq ? (float)(-0.5 * lam) : (float)(lam * (double)means[(size_t)g * D + d]);
    }
    const __bf16 h = (__bf16)v;
    const __bf16 l = (__bf16)(v - (float)h);
    const int lanei = 16 * lq + row;
    const size_t idx = ((size_t)rb * KS + ks) * 64 + lanei;
    ((__bf16*)(Whi + idx))[i] = h;
    ((__bf16*)(Wlo + idx))[i] = l;
  }
}

// Zero A fragments for row g (a padding row of the last row block).
__device__ void zero_component_rows(bf16x8* Whi, bf16x8* Wlo, int KS, int g) {
  const int rb = g >> 4, row = g & 15;
  for (int e = threadIdx.x; e < KS * 4; e += 256) {
    const int ks = e / 4, lq = e & 3;
    const size_t idx = ((size_t)rb * KS + ks) * 64 + 16 * lq + row;
    bf16x8 z;
#pragma unroll
    for (int i = 0; i < 8; ++i) z[i] = (__bf16)0.0f;
    Whi[idx] = z;
    Wlo[idx] = z;
  }
}

// grid 16 * ceil(G / 16): block g < G computes component g, the others zero
// the padding rows of the last row block; block 0 also clears the status word,
// the recompute counter and the workspace counters of the call.
__global__ void __launch_bounds__(256) k_pre_fast(const float* __restrict__ hefts,
                                                  const float* __restrict__ means,
                                                  const float* __restrict__ covs, int D, int G,
                                                  int KS, float* __restrict__ prm,
                                                  float* __restrict__ cc,
                                                  float* __restrict__ cexp,
                                                  bf16x8* __restrict__ Whi,
                                                  bf16x8* __restrict__ Wlo,
                                                  double* __restrict__ c64,
                                                  double* __restrict__ lam64,
                                                  int32_t* __restrict__ dev_status,
                                                  int64_t* __restrict__ n_recomputed,
                                                  int64_t* __restrict__ counters) {
  const int g = blockIdx.x;
  if (g == 0) {
    if (threadIdx.x == 0) {
      *dev_status = 0;
      if (n_recomputed) *n_recomputed = 0;
    }
    if (threadIdx.x < 8) counters[threadIdx.x] = 0;
  }
  if (g >= G) {
    zero_component_rows(Whi, Wlo, KS, g);
    return;
  }
  pre_component(hefts, means, covs, D, G, KS, g, prm, cc, cexp, Whi, Wlo, c64, lam64);
}

// grid (16 * RBmax, n_models): component g of model blockIdx.y.
__global__ void __launch_bounds__(256) k_pre_fast_batched(const gmm_model_desc* models, int D,
                                                          BatchConst bc) {
  const int mi = blockIdx.y;
  const gmm_model_desc& m = models[mi];
  if (!batch_desc_ok(m, bc.Gmax)) return;
  const int G = m.G;
  const int g = blockIdx.x;
  bf16x8* Whi = bc.Whi + (size_t)mi * bc.RBmax * bc.KS * 64;
  bf16x8* Wlo = bc.Wlo + (size_t)mi * bc.RBmax * bc.KS * 64;
  if (g >= G) {
    if (g < 16 * ((G + 15) / 16)) zero_component_rows(Whi, Wlo, bc.KS, g);
    return;
  }
  pre_component(m.hefts, m.means, m.covs, D, G, bc.KS, g, bc.prm + (size_t)mi * 2 * bc.Gmax * (D + 1),
                bc.cc + (size_t)mi * 2 * bc.Gmax, bc.cexp + (size_t)mi * 2 * bc.Gmax, Whi, Wlo,
                bc.c64 + (size_t)mi * bc.Gmax, bc.lam64 + (size_t)mi * bc.Gmax * D);
}

// Reduce step for the Welford partials [nb][G][1 + 2D] = (L, m, Q), m being
// the weighted mean of x - mu_old: one workgroup per component (D <= 128),
// thread per dimension, blocks (or the segments k_welford_seg combined, every
// seg-th block) combined in order by L = La + Lb,
// m = ma + (mb - ma) Lb / L, Q = Qa + Qb + (mb - ma)^2 La Lb / L
// (welford_combine).
// Then Eq. 5 (w = L/N), Eq. 6 (mu = mu_old + m), Eq. 7 (sigma2 = Q/L) and the
// floor.
__global__ void __launch_bounds__(256) k_fin_welford(const double* __restrict__ part, int nb,
                                                     int seg,
                                                     int64_t N, int D, int G, float var_floor,
                                                     float* __restrict__ hefts,
                                                     float* __restrict__ means,
                                                     float* __restrict__ covs,
                                                     const double* __restrict__ ll_part,
                                                     double* __restrict__ mean_loglik,
                                                     int32_t* __restrict__ dev_status) {
  __shared__ int bad;
  __shared__ WelfordLds S;
  const int g = blockIdx.x;
  const int P = 2 * D + 1;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  double m, Q;
  const double Ltot = welford_combine<256, 32>(part + (size_t)g * P, (size_t)seg * G * P,
                                               (nb + seg - 1) / seg, D, S, m, Q);
  const int d = threadIdx.x;
  if (d < D && Ltot > 0.0) {
    double v = Q / Ltot;
    v = v > 0.0 ? v : 0.0;
    v = v > (double)var_floor ? v : (double)var_floor;
    means[(size_t)g * D + d] = (float)((double)means[(size_t)g * D + d] + m);
    covs[(size_t)g * D + d] = (float)v;
    if (!isfinite(m) || !isfinite(v)) bad = 1;
  }
  if (threadIdx.x == 0) {
    const float w = (float)(Ltot / (double)N);
    hefts[g] = w;
    if (!isfinite(w)) bad = 1;
  }
  if (g == 0 && mean_loglik) {
    const double s = ordered_sum<256>(ll_part, nb, S.lb);
    if (threadIdx.x == 0) {
      *mean_loglik = s / (double)N;
      if (!isfinite(s)) bad = 1;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && bad) atomicOr(dev_status, GMM_DEV_NONFINITE);
}

// Reduce step of the batched form: grid (Gmax, n_models); block (g, m)
// combines model m's items in order (same arithmetic as k_fin_welford).
__global__ void __launch_bounds__(256) k_fin_welford_batched(const gmm_model_desc* models,
                                                             const int2* mitems, int D, int Gmax,
                                                             float var_floor,
                                                             const double* __restrict__ part,
                                                             const double* __restrict__ ll_part,
                                                             int mstep) {
  __shared__ int bad;
  __shared__ WelfordLds S;
  const int mi = blockIdx.y;
  const gmm_model_desc& m = models[mi];
  const int g = blockIdx.x;
  const int first = mitems[mi].x, cnt = mitems[mi].y;
  if (cnt == 0 || g >= m.G) return;
  const int P = 2 * D + 1;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  if (mstep) {
    double mu, Q;
    const double Ltot = welford_combine<256, 8>(part + ((size_t)first * Gmax + g) * P,
                                             (size_t)Gmax * P, cnt, D, S, mu, Q);
    const int d = threadIdx.x;
    if (d < D && Ltot > 0.0) {
      double v = Q / Ltot;
      v = v > 0.0 ? v : 0.0;
      v = v > (double)var_floor ? v : (double)var_floor;
      const double mn = (double)m.means[(size_t)g * D + d] + mu;
      m.means[(size_t)g * D + d] = (float)mn;
      m.covs[(size_t)g * D + d] = (float)v;
      if (!isfinite(mn) || !isfinite(v)) bad = 1;
    }
    if (threadIdx.x == 0) {
      const float w = (float)(Ltot / (double)m.N);
      m.hefts[g] = w;
      if (!isfinite(w)) bad = 1;
    }
  }
  if (g == 0 && threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < cnt; ++k) s += ll_part[first + k];
    if (m.loglik) *m.loglik = s / (double)m.N;
    if (!isfinite(s)) bad = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0 && bad) atomicOr(m.dev_status, GMM_DEV_NONFINITE);
}

// ---- sample-major BF16X3 kernel ----------------------------------------------
//
// Each wave owns groups of 16 consecutive samples and runs their E-step in
// registers.  The MFMA A operand holds the samples' features, interleaved as
// [x_d, x_d^2] and split into BF16 hi + lo; the B operand holds the
// components' coefficients [lam mu, -lam/2] (hi + lo, staged in LDS once per
// work range).  Output lane l, register j is (sample 4 (l/16) + j, component
// 16 cb + l%16), so every per-sample reduction (bounded maximum, near count,
// log-sum-exp) is a butterfly over the 16 lanes of a lane row.  Near pairs are
// recomputed exactly, in FP64 from the FP32 parameters, two pairs per 16-lane
// row at a time (all loads of both issued first).  The map step of component g
// is done by wave g % 8 (its "owner"), which keeps (L, m, Q) of its components
// in registers; every 128 samples the waves pass their non-zero
// responsibilities to the owners through LDS lists, in a fixed order, with one
// barrier per 128 samples when the lists fit.  Where LDS has room (D <= 64, few
// components) the staged form also keeps each round's samples and the
// components' FP64 constants in LDS, so the recompute and the map step read no
// global memory.

constexpr int kGS = 16;             // samples per wave group
constexpr int kRoundN = kNW * kGS;  // samples per block round
constexpr int kCapM = 16;           // pairs per (source, owner) list per pass
constexpr int kCapR = 64;           // near pairs recomputed per chunk per wave

struct Lds2 {
  bf16x8* wh;    // [RB][KS][64] B fragments (hi)
  bf16x8* wl;    // lo
  float* cq;     // [G][8]: c hi, Q, c lo, cexp hi, cexp lo, -, -, -
  float* mw;     // [NW][16] per-sample bounded maximum
  int* cw;       // [NW][16] per-sample near count
  int* rcode;    // [NW][kCapR] near pair: sample | component << 8
  float* rval;   // [NW][kCapR] exact value - maximum bound
  int2* sub;     // [2][NW source][NW owner][kCapM] (sample | component << 8, r), by round parity
  int* subn;     // [2][NW source][NW owner] pairs of the round
  int* need;     // [2] largest list of the round
  double* llw;   // [NW]
  int2* osort;   // [NW][64] an owner's pairs ordered by component slot
};

template <typename F>
__host__ __device__ inline size_t lds2_walk(int G, int KS, F&& at) {
  size_t w = 0;
  auto put = [&](int which, size_t words, size_t align_words) {
    w = (w + align_words - 1) / align_words * align_words;
    at(which, w);
    w += words;
  };
  const size_t RB = ((size_t)G + 15) / 16;
  put(0, RB * KS * 64 * 4, 4);
  put(1, RB * KS * 64 * 4, 4);
  put(2, 8 * 16 * RB, 4);  // padded to whole row blocks
  put(3, kNW * 16, 1);
  put(4, kNW * 16, 1);
  put(5, kNW * kCapR, 1);
  put(6, kNW * kCapR, 1);
  put(7, 2 * (size_t)kNW * kNW * kCapM * 2, 2);
  put(8, 2 * kNW * kNW, 1);
  put(9, 2, 1);
  put(10, 2 * kNW, 2);
  put(11, kNW * 64 * 2, 2);
  return w;
}

__host__ __device__ inline size_t em2_lds_bytes(int G, int KS) {
  return lds2_walk(G, KS, [](int, size_t) {}) * 4 + 64;
}

// k-steps of the sample-major fragment layout (compile-time in the kernel)
__host__ __device__ inline int em2_ks(int D) { return D <= 64 ? 4 : 8; }

// Staged form (D <= 64): after the layout above, each round's samples
// [2 by round parity][128][D] (floats), the precisions lam [G][D] (doubles),
// the constants c [G] (doubles) and the means [G][D] (floats), so the near-pair
// recompute and the map step read LDS only.  With G <= 16 the same bytes
// later hold the 8 waves' map-step states [8][G][2D + 1] (floats).
__host__ __device__ inline size_t em2_stage_off(int G, int KS) {
  return (em2_lds_bytes(G, KS) + 15) / 16 * 16;
}
__host__ __device__ inline size_t em2_stage_lds_bytes(int D, int G) {
  const size_t st = (size_t)4 * 2 * kRoundN * D + (size_t)8 * G * D + (size_t)8 * G +
                    (size_t)4 * G * D;
  const size_t mg = G <= 16 ? (size_t)4 * kNW * G * (2 * D + 1) : 0;
  return em2_stage_off(G, 4) + (st > mg ? st : mg);
}
// LDS of the staged form for models of up to G components (a batch item
// with G' <= G components uses its own, smaller layout, whose map-step states
// for G' <= 16 must fit as well)
inline size_t em2_stage_lds_max(int D, int G) {
  const size_t a = em2_stage_lds_bytes(D, G), b = em2_stage_lds_bytes(D, G < 16 ? G : 16);
  return a > b ? a : b;
}
inline bool em2_stage_fits(int D, int G) {
  return D <= 64 && em2_stage_lds_max(D, G) <= 160 * 1024;
}

__device__ inline Lds2 carve_lds2(char* base, int G, int KS) {
  Lds2 L;
  float* f = (float*)base;
  lds2_walk(G, KS, [&](int which, size_t off) {
    switch (which) {
      case 0: L.wh = (bf16x8*)(f + off); break;
      case 1: L.wl = (bf16x8*)(f + off); break;
      case 2: L.cq = f + off; break;
      case 3: L.mw = f + off; break;
      case 4: L.cw = (int*)(f + off); break;
      case 5: L.rcode = (int*)(f + off); break;
      case 6: L.rval = f + off; break;
      case 7: L.sub = (int2*)(f + off); break;
      case 8: L.subn = (int*)(f + off); break;
      case 9: L.need = (int*)(f + off); break;
      case 10: L.llw = (double*)(f + off); break;
      default: L.osort = (int2*)(f + off); break;
    }
  });
  return L;
}

// A sample's log-sum-exp less M from its per-slice references D_q and sums
// S_q: D* = max_q D_q (returned) and log(sum over slices of S_q exp(D_q - D*))
// (in ls); the total is D* + ls.  The rescaling and the logarithm are taken in
// FP32, as the one-pass kernel takes its logarithm (about 1e-7 nats).
__device__ __forceinline__ float slice_lse(const float* pd, const float* ps, int S, int64_t NS,
                                           double& ls) {
  float dstar = -INFINITY;
  for (int q = 0; q < S; ++q) dstar = fmaxf(dstar, pd[(size_t)q * NS]);
  double tot = 0.0;
  for (int q = 0; q < S; ++q)
    tot += (double)(ps[(size_t)q * NS] * __expf(pd[(size_t)q * NS] - dstar));
  ls = (double)__logf((float)tot);
  return dstar;
}

// Fragments are laid out for KST = 4 DPL k-steps (16 dimensions each, zero
// past D), so every LDS offset below is a compile-time immediate.
//
// MODE 0: one pass over all G components (G <= 128).  With more components
// than one workgroup's LDS holds, three passes over slices of them, each
// workgroup (b, slice) screening its slice for its sample range:
//   MODE 1  the slice's bounded maximum per sample -> wM[slice][n];
//   MODE 2  the global bound M = max over slices (k_wmax, run between
//           MODES 1 and 2, leaves it in slot 0 of wM), the slice's near pairs
//           recomputed exactly, their largest value less M (0 without near
//           pairs) -> wD[slice][n] and the slice's sum of
//           exp(value - M - wD) -> wS[slice][n];
//   MODE 3  log-sum-exp M + D* + log(sum over slices of
//           wS exp(wD - D*)), D* = max over slices of wD (Eqs. 16-18; the
//           log-likelihood pass k_wll, run between MODES 2 and 3, leaves M,
//           D* and the logarithm of each sample in slot 0 of wM, wD, wS),
//           the responsibilities and the map step of the slice's components.
// Near pairs are the same in MODES 2 and 3 (same bound, same M, same order)
// and always taken in FP64: MODE 2 stores the first kCapR exact values of
// each 16-sample group and slice (wR), MODE 3 reads them and recomputes only
// beyond kCapR.
template <int CPW, int DPL, bool MSTEP, int MODE = 0, bool STG = false>
__device__ __forceinline__ void em2_range(const FastArgs& a, int64_t i0, int64_t i1, int b,
                                          char* lds_raw) {
  static_assert(!STG || (MODE == 0 && DPL == 1), "staged form: one pass, D <= 64");
  constexpr int RBT = (CPW + 1) / 2;  // row blocks of 16 components
  constexpr int KST = 4 * DPL;        // k-steps of 16 dimensions
  const int D = a.D, G = a.G;
  const int g0 = MODE ? a.g0 : 0;   // first component of the slice
  const int Gt = MODE ? a.Gt : G;   // components of the model
  const int P = 2 * D + 1;
  const int RB = (G + 15) / 16;
  const Lds2 L = carve_lds2(lds_raw, G, KST);
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int w = tid / kWave;
  const int KSr = (2 * D + 31) / 32;  // k-steps holding data
  const float ecoef = err_expanded_coef(KSr);
  const float B2 = 2.0f * ecoef;

  {
    const bf16x8* const whs = a.Whi + (size_t)(g0 / 16) * KST * 64;
    const bf16x8* const wls = a.Wlo + (size_t)(g0 / 16) * KST * 64;
    for (int p = tid; p < RB * KST * 64; p += kThreads) {
      L.wh[p] = whs[p];
      L.wl[p] = wls[p];
    }
  }
  for (int g = tid; g < 16 * RB; g += kThreads) {
    float* q = L.cq + 8 * g;
    if (g < G) {
      const int gg = g0 + g;
      const float c = a.cc[gg];
      const float Q = 2.0f * ((c + a.cc[Gt + gg]) - (a.cexp[gg] + a.cexp[Gt + gg]));
      const float Qb = isfinite(Q) ? 1.0001f * fmaxf(Q, 0.0f) : 0.0f;
      q[0] = c;
      q[1] = Qb;
      q[2] = a.cc[Gt + gg];
      q[3] = a.cexp[gg];
      q[4] = a.cexp[Gt + gg];
      // err_expanded(2 (c - v), Q, c) = coef (2 max(c - v, 0) + Q) + K is
      // E0 - 2 coef min(v, c) with E0 = coef (2c + Q) + K; the slack covers
      // the FP32 evaluation of E0 and of that product
      const float K = 1.01f * 0x1p-23f * (fabsf(c) + 0.5f * Qb);
      const float e0 = ecoef * (2.0f * c + Qb) + K;
      q[5] = isfinite(e0) ? e0 + 0x1p-20f * (2.0f * ecoef * fabsf(c) + ecoef * Qb + K) : 0.0f;
    } else {  // padding component: value -inf
      q[0] = 0.0f;
      q[1] = 0.0f;
      q[2] = 0.0f;
      q[3] = -INFINITY;
      q[4] = 0.0f;
      q[5] = 0.0f;
    }
  }


  // staged form: the FP64 constants and the means of all G components (one
  // pass, so g0 = 0) and each round's samples in LDS
  float* const xs = STG ? (float*)(lds_raw + em2_stage_off(G, KST)) : nullptr;
  double* const slam = STG ? (double*)(xs + 2 * kRoundN * D) : nullptr;
  double* const sc64 = STG ? slam + G * D : nullptr;
  float* const smu = STG ? (float*)(sc64 + G) : nullptr;
  if constexpr (STG) {
    for (int i = tid; i < G * D; i += kThreads) {
      slam[i] = a.lam64[i];
      smu[i] = a.means[i];
    }
    for (int g = tid; g < G; g += kThreads) sc64[g] = a.c64[g];
  }

  // the owner's old means in registers when they take few (they are read by
  // every map-step chunk); otherwise reloaded per chunk
  // private map step (staged form, G <= 16): every wave keeps (L, m, Q) of
  // all G components for its own samples, so no list passes between waves and
  // a round takes no barrier; the 8 states are combined at the end of the
  // range.  Otherwise each component has one owner wave.
  constexpr bool kPriv = MSTEP && STG && CPW <= 2;
  constexpr int kPG = kPriv ? 16 : 1;
  float Lp[kPG], P1[kPG], P2[kPG], mup[kPG];
#pragma unroll
  for (int g = 0; g < kPG; ++g) {
    Lp[g] = 0.0f;
    P1[g] = 0.0f;
    P2[g] = 0.0f;
    mup[g] = kPriv && g < G ? a.means[(size_t)g * D + min(lane, D - 1)] : 0.0f;
  }
  constexpr bool kMuReg = MSTEP && !kPriv && CPW * DPL <= 8;
  float mur[kMuReg ? CPW : 1][DPL];
#pragma unroll
  for (int c = 0; c < (kMuReg ? CPW : 1); ++c)
#pragma unroll
    for (int jd = 0; jd < DPL; ++jd) {
      const int g = w + kNW * c;
      mur[c][jd] = kMuReg && g < G ? a.means[(size_t)(g0 + g) * D + min(lane + kWave * jd, D - 1)]
                                   : 0.0f;
    }
  // owner accumulators: component g = w + 8 c, dimension d = lane + 64 j
  float Lc[CPW], S1[CPW][DPL], S2[CPW][DPL];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    Lc[c] = 0.0f;
#pragma unroll
    for (int j = 0; j < DPL; ++j) {
      S1[c][j] = 0.0f;
      S2[c][j] = 0.0f;
    }
  }
  double llacc = 0.0;
  int bad = 0;
  long long nrec = 0;
  __syncthreads();

  const int rowq = lane >> 4;  // output rows: samples 4 rowq + j
  const int colc = lane & 15;  // output column: component 16 cb + colc
  const int kg = lane >> 4;    // A operand: dimensions 16 ks + 4 kg + 0..3
  const int na = lane & 15;    // A operand: sample na
  const unsigned long long lt = (1ull << lane) - 1ull;
  const unsigned long long cls = 0x0101010101010101ull << (lane & 7);
  float* const mw = L.mw + w * 16;
  int* const cw = L.cw + w * 16;
  int* const rcode = L.rcode + w * kCapR;
  float* const rval = L.rval + w * kCapR;
  const bf16x8* const whl = L.wh + lane;
  const bf16x8* const wll = L.wl + lane;
  const float* const cql = L.cq + 8 * colc;

  // staged form: the next round's rows of this wave, one row per register
  // (lane d holds dimension d), loaded a round ahead
  float pf[STG ? kGS : 1];
  if constexpr (STG) {
    const int64_t s0n = i0 + (int64_t)kGS * w;
#pragma unroll
    for (int n = 0; n < kGS; ++n)
      pf[n] = (lane < D && s0n + n < i1) ? a.X[(s0n + n) * a.ldx + lane] : 0.0f;
  }

  int round = 0;
  for (int64_t base = i0; base < i1; base += kRoundN, ++round) {
    const int64_t s0 = base + (int64_t)kGS * w;
    // staged form: this wave's 16 rows of the round (loaded into registers
    // during the previous round, zero past i1) go to LDS.  Buffers alternate
    // by round parity: an owner reads them until its map step ends, before
    // the next round's barrier, and this wave refills a buffer only two rounds
    // later, after that barrier.
    float* const xsr = STG ? xs + (size_t)(round & 1) * kRoundN * D : nullptr;
    if constexpr (STG) {
      float* const dst = xsr + (size_t)kGS * w * D;
#pragma unroll
      for (int n = 0; n < kGS; ++n)
        if (lane < D) dst[n * D + lane] = pf[n];
      wave_lds_sync();
    }

    // 1-2. screening on the matrix cores.  A fragments: the group's samples,
    // features [x_d, x_d^2] interleaved, split into BF16 hi + lo; each block
    // of 16 components accumulates in FP32 and lands in the scalar array
    // acc[cb][j] (sample 4 rowq + j, component 16 cb + colc).
    float acc[RBT][4];
    {
      const int64_t ia = s0 + na;
      // the staged rows are zero past i1
      const bool va = STG || ia < i1;
      const float* xr = STG ? xsr + (kGS * w + na) * D + 4 * kg : a.X + (va ? ia : i0) * a.ldx + 4 * kg;
      int dl = D - 4 * kg;  // this lane's dimensions are 16 ks + q < dl
      // opaque per round, so the bound tests are not hoisted out of the round
      // loop (they would stay live in registers for the whole kernel)
      asm volatile("" : "+v"(dl));
      if constexpr (MODE != 1) {
      // every load of the group's samples first; then k-step by k-step, the
      // step's split operands built and multiplied into all component blocks
      // (one independent accumulator per block, each summed in k order)
      float xv[KST][4];
#pragma unroll
      for (int ks = 0; ks < KST; ++ks)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          xv[ks][q] = (va && 16 * ks + q < dl) ? xr[16 * ks + q] : 0.0f;
      f32x4 c[RBT];
#pragma unroll
      for (int cb = 0; cb < RBT; ++cb) c[cb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      // an opaque zero per round: the fragment loads below are loop-invariant
      // where the round stores nothing to LDS, and hoisted they would hold
      // every fragment in registers
      int kof = 0;
      asm volatile("" : "+v"(kof));
#pragma unroll
      for (int ks = 0; ks < KST; ++ks) {
        bf16x8 ah, al;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float x = xv[ks][i >> 1];
          const float v = (i & 1) ? x * x : x;
          const __bf16 h = (__bf16)v;
          ah[i] = h;
          al[i] = (__bf16)(v - (float)h);
        }
#pragma unroll
        for (int cb = 0; cb < RBT; ++cb) {
          if (cb < RB) {
            const bf16x8 bh = whl[kof + (cb * KST + ks) * 64];
            const bf16x8 bl = wll[kof + (cb * KST + ks) * 64];
            c[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c[cb], 0, 0, 0);
            c[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c[cb], 0, 0, 0);
            c[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c[cb], 0, 0, 0);
          }
        }
        // one k-step's operand loads in flight at a time (unbounded, the
        // scheduler hoists them all and the registers spill)
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int cb = 0; cb < RBT; ++cb)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[cb][j] = c[cb][j];
      } else {
      // the slice-maximum pass: all split operands first, then block by
      // block (in this short round the k-outer order above is compiled into
      // spilling branchy code); the same products in the same order
      bf16x8 ah[KST], al[KST];
#pragma unroll
      for (int ks = 0; ks < KST; ++ks) {
        float xv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) xv[q] = (va && 16 * ks + q < dl) ? xr[16 * ks + q] : 0.0f;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float x = xv[i >> 1];
          const float v = (i & 1) ? x * x : x;
          const __bf16 h = (__bf16)v;
          ah[ks][i] = h;
          al[ks][i] = (__bf16)(v - (float)h);
        }
      }
#pragma unroll
      for (int cb = 0; cb < RBT; ++cb) {
        f32x4 c = {0.0f, 0.0f, 0.0f, 0.0f};
        if (cb < RB) {
#pragma unroll
          for (int ks = 0; ks < KST; ++ks) {
            const bf16x8 bh = whl[(cb * KST + ks) * 64];
            const bf16x8 bl = wll[(cb * KST + ks) * 64];
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[ks], bh, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[ks], bl, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[ks], bh, c, 0, 0, 0);
          }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[cb][j] = c[j];
      }
      }
    }

    if constexpr (STG) {
      // the next round's rows, in flight during the rest of this round
      const int64_t s0n = s0 + kRoundN;
#pragma unroll
      for (int n = 0; n < kGS; ++n)
        pf[n] = (lane < D && s0n + n < i1) ? a.X[(s0n + n) * a.ldx + lane] : 0.0f;
    }
    // 3. values, their error bounds, per-sample bounded maximum M and near set
    bool vj[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) vj[j] = s0 + 4 * rowq + j < i1;
    float M[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
#pragma unroll
    for (int cb = 0; cb < RBT; ++cb) {
      const float* q = cql + 8 * 16 * cb;
      const bool vg = cb < RB;
      const float ch = vg ? q[0] : 0.0f, E0 = vg ? q[5] : 0.0f;
      const float eh = vg ? q[3] : -INFINITY, el = vg ? q[4] : 0.0f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float v = vj[j] ? (acc[cb][j] + eh) + el : -INFINITY;
        acc[cb][j] = v;
        if (MODE < 2) M[j] = fmaxf(M[j], v - fmaf(-B2, fminf(v, ch), E0));
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (MODE < 2) {
#pragma unroll
      for (int j = 0; j < 4; ++j) M[j] = row16_max(M[j]);
    } else {
      // MODES 2 and 3: the bound over all slices, combined into slot 0 (by
      // k_wmax after MODE 1; k_wll keeps it there)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (vj[j]) M[j] = a.wM[s0 + 4 * rowq + j];
    }
    if constexpr (MODE == 1) {
      if (colc == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (vj[j]) a.wM[(size_t)a.sl * a.NS + s0 + 4 * rowq + j] = M[j];
      }
      continue;
    }
    uint32_t nearb = 0;  // bit 4 cb + j
#pragma unroll
    for (int cb = 0; cb < RBT; ++cb) {
      const float* q = cql + 8 * 16 * cb;
      const bool vg = cb < RB;
      const float ch = vg ? q[0] : 0.0f, E0 = vg ? q[5] : 0.0f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float v = acc[cb][j];
        if (v > -INFINITY && v + fmaf(-B2, fminf(v, ch), E0) >= M[j] - kNearGap)
          nearb |= 1u << (4 * cb + j);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // near pairs in lane-major order: lane l's pairs (block-major) follow
    // those of lanes < l; per-sample counts packed one byte per row sample
    int np = 0;
    const int mybase = wave_prefix_small(__popc(nearb), lt, ~0ull, &np);
    {
      int pk = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) pk += __popc(nearb & (0x11111111u << j)) << (8 * j);
      pk = row16_sum_i(pk);
      if (colc == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          mw[4 * rowq + j] = M[j];
          cw[4 * rowq + j] = (pk >> (8 * j)) & 0xFF;
        }
      }
    }
    if (MODE != 2) nrec += np;

    // 4. exact values of the near pairs, kCapR at a time
    float* const wrg =
        MODE >= 2 ? a.wR + ((size_t)a.sl * a.NG + (size_t)(s0 / kGS)) * kCapR : nullptr;
    for (int c0 = 0; c0 < np; c0 += kCapR) {
      if (MODE == 3 && c0 == 0) {
        // the near-pair pass's values, in the same order
        int k = mybase;
#pragma unroll
        for (int cb = 0; cb < RBT; ++cb)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if ((nearb >> (4 * cb + j)) & 1u) {
              if (k < kCapR) acc[cb][j] = wrg[k];
              ++k;
            }
        continue;
      }
      int k = mybase - c0;
#pragma unroll
      for (int cb = 0; cb < RBT; ++cb)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if ((nearb >> (4 * cb + j)) & 1u) {
            if (k >= 0 && k < kCapR) rcode[k] = (4 * rowq + j) | ((16 * cb + colc) << 8);
            ++k;
          }
      wave_lds_sync();
      {
        // PU pairs per 16-lane row at a time (p, p + 4, ...); lane l16 of the
        // row takes dimensions l16 + 16 i, and every load of those pairs is
        // issued before any use.  The value is c - q/2 in FP64 from the FP32
        // sample and parameters (q summed over the row in FP64).  Two pairs
        // in flight where D <= 64; one where 128 dimensions per row would
        // take twice the registers.
        constexpr int NE = 4 * DPL;  // dimensions per lane (D <= 64 NE)
        constexpr int PU = DPL == 1 ? 2 : 1;
        const int rid = lane >> 4, l16 = lane & 15;
        const int nc = min(kCapR, np - c0);
        for (int p = rid; p < nc; p += 4 * PU) {
          int n[PU], g[PU];
          bool has[PU];
          float xv[PU][NE], mv[PU][NE];
          double lv[PU][NE], cg[PU];
#pragma unroll
          for (int h = 0; h < PU; ++h) {
            has[h] = p + 4 * h < nc;
            const int code = rcode[has[h] ? p + 4 * h : p];
            n[h] = code & 15;
            g[h] = code >> 8;
            const int gg = g0 + g[h];
            const float* xr = STG ? xsr + (kGS * w + n[h]) * D : a.X + (s0 + n[h]) * a.ldx;
            const float* mu_g = STG ? smu + g[h] * D : a.means + (size_t)gg * D;
            const double* lg = STG ? slam + g[h] * D : a.lam64 + (size_t)gg * D;
#pragma unroll
            for (int i = 0; i < NE; ++i) {
              const int dc = min(l16 + 16 * i, D - 1);
              xv[h][i] = xr[dc];
              mv[h][i] = mu_g[dc];
              lv[h][i] = lg[dc];
            }
            cg[h] = STG ? sc64[g[h]] : a.c64[gg];
          }
          double q[PU];
#pragma unroll
          for (int h = 0; h < PU; ++h) {
            q[h] = 0.0;
#pragma unroll
            for (int i = 0; i < NE; ++i) {
              const double u = (double)xv[h][i] - (double)mv[h][i];
              q[h] = l16 + 16 * i < D ? q[h] + u * u * lv[h][i] : q[h];
            }
          }
#pragma unroll
          for (int h = 0; h < PU; ++h) q[h] = row16_sum(q[h]);
          if (l16 == 0) {
#pragma unroll
            for (int h = 0; h < PU; ++h)
              if (has[h]) {
                const double val = cg[h] - 0.5 * q[h];
                const float rv = (float)(val - (double)mw[n[h]]);
                rval[p + 4 * h] = rv;
                if (MODE == 2 && c0 == 0) wrg[p + 4 * h] = rv;
              }
          }
        }
      }
      wave_lds_sync();
      k = mybase - c0;
#pragma unroll
      for (int cb = 0; cb < RBT; ++cb)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if ((nearb >> (4 * cb + j)) & 1u) {
            if (k >= 0 && k < kCapR) acc[cb][j] = rval[k];
            ++k;
          }
      wave_lds_sync();
    }

    // 5. log-sum-exp about M + max(near - M) (Eqs. 16-18) and responsibilities
    if constexpr (MODE == 2) {
      // the slice's sum about its largest exact near value (an exact value
      // can lie far above M when its screening bound is wide)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float dm = -INFINITY;
#pragma unroll
        for (int cb = 0; cb < RBT; ++cb)
          if ((nearb >> (4 * cb + j)) & 1u) dm = fmaxf(dm, acc[cb][j]);
        dm = row16_max(dm);
        const float dn = dm > -INFINITY ? dm : 0.0f;
        float sf = 0.0f;  // this lane's few terms in FP32, the row's total in FP64
#pragma unroll
        for (int cb = 0; cb < RBT; ++cb) {
          const bool nr = (nearb >> (4 * cb + j)) & 1u;
          sf += __expf((nr ? acc[cb][j] : acc[cb][j] - M[j]) - dn);
        }
        const double sm = row16_sum((double)sf);
        if (vj[j] && colc == 0) {
          const size_t o = (size_t)a.sl * a.NS + s0 + 4 * rowq + j;
          a.wD[o] = dn;
          a.wS[o] = (float)sm;
        }
      }
      continue;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if constexpr (MODE == 3) {
        // lse = M + D* + log(sum over slices in slice order): D* and the
        // logarithm combined by k_wll into slot 0 (which also took the
        // log-likelihood)
        float dstar = 0.0f, ls = 0.0f;
        if (vj[j]) {
          dstar = a.wD[s0 + 4 * rowq + j];
          ls = a.wS[s0 + 4 * rowq + j];
        }
#pragma unroll
        for (int cb = 0; cb < RBT; ++cb) {
          const bool nr = (nearb >> (4 * cb + j)) & 1u;
          const float z = ((nr ? acc[cb][j] : acc[cb][j] - M[j]) - dstar) - ls;
          acc[cb][j] = (vj[j] && z >= -kRespCut) ? __expf(z) : 0.0f;
        }
        __builtin_amdgcn_sched_barrier(0);
        continue;
      }
      float dm = -INFINITY;
#pragma unroll
      for (int cb = 0; cb < RBT; ++cb)
        if ((nearb >> (4 * cb + j)) & 1u) dm = fmaxf(dm, acc[cb][j]);
      dm = row16_max(dm);
      const float dn = dm > -INFINITY ? dm : 0.0f;
      float sf = 0.0f;  // this lane's few terms in FP32, the row's total in FP64
#pragma unroll
      for (int cb = 0; cb < RBT; ++cb) {
        const bool nr = (nearb >> (4 * cb + j)) & 1u;
        const float t = nr ? acc[cb][j] - dn : (acc[cb][j] - M[j]) - dn;
        sf += __expf(t);
      }
      const double sm = row16_sum((double)sf);
      const float ls = __logf((float)sm);
      const double lse = ((double)M[j] + (double)dn) + (double)ls;
      if (vj[j] && colc == 0) {
        llacc += lse;
        if (!isfinite(lse)) bad = 1;
        if (a.per_sample) a.per_sample[s0 + 4 * rowq + j] = (float)lse;
      }
      if (MSTEP) {
#pragma unroll
        for (int cb = 0; cb < RBT; ++cb) {
          const bool nr = (nearb >> (4 * cb + j)) & 1u;
          const float z = (nr ? acc[cb][j] - dn : (acc[cb][j] - M[j]) - dn) - ls;
          acc[cb][j] = (vj[j] && z >= -kRespCut) ? __expf(z) : 0.0f;
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }

    if constexpr (kPriv) {
      // 6'. the wave's own samples in order, each sample's components in
      // order.  Sample 4 q + j's responsibility of component g sits in lane
      // 16 q + g of acc[0][j]; four ballots mark the non-zero ones.
      unsigned long long nzm[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) nzm[j] = __ballot(acc[0][j] != 0.0f);
      for (int q = 0; q < 4; ++q) {
        float xv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) xv[j] = xsr[(kGS * w + 4 * q + j) * D + min(lane, D - 1)];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const unsigned m16 = (unsigned)(nzm[j] >> (16 * q)) & 0xFFFFu;
          if (m16 == 0u) continue;
#pragma unroll
          for (int g = 0; g < 16; ++g) {
            if ((m16 >> g) & 1u) {
              const float r = __int_as_float(
                  __builtin_amdgcn_readlane(__float_as_int(acc[0][j]), 16 * q + g));
              const float y = xv[j] - mup[g];
              const float Lo = Lp[g];
              const float Ln = Lo + r;
              const float rc = __builtin_amdgcn_rcpf(Ln);
              const float inv = r * rc;
              const float wo = Lo * rc;
              const float w2 = inv * Lo;
              // the owner form's update (a dominant sample sets the mean
              // from its own side)
              const bool dom = inv > 0.5f;
              Lp[g] = Ln;
              const float dl = y - P1[g];
              P1[g] = dom ? fmaf(-wo, dl, y) : fmaf(inv, dl, P1[g]);
              P2[g] = fmaf(w2 * dl, dl, P2[g]);
            }
          }
        }
      }
    } else if (MSTEP) {
      // 6. hand the non-zero responsibilities to their owners (the owner of
      // component 16 cb + colc is wave colc % 8 = lane % 8)
      // non-zero responsibilities, lane-major within each owner class (lanes
      // l with l % 8 = owner)
      uint32_t nzb = 0;
#pragma unroll
      for (int cb = 0; cb < RBT; ++cb)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (acc[cb][j] != 0.0f) nzb |= 1u << (4 * cb + j);
      int mine = 0;
      const int cbase = wave_prefix_small(__popc(nzb), lt, cls, &mine);
      // lists and counts alternate between two buffers by round parity: a
      // wave writes round r + 2's lists only after the barrier of round r + 1,
      // which every owner reaches after its map step of round r, so a round
      // whose lists fit kCapM takes one barrier
      int2* const subb = L.sub + (size_t)(round & 1) * kNW * kNW * kCapM;
      int* const subnb = L.subn + (round & 1) * kNW * kNW;
      if (lane < kNW) subnb[w * kNW + lane] = mine;
      int need = 0;  // longest list of the round (known after the first barrier)
      for (int pass = 0;; ++pass) {
        int2* const dst = subb + (size_t)(w * kNW + (lane & 7)) * kCapM;
        int k = cbase - pass * kCapM;
#pragma unroll
        for (int cb = 0; cb < RBT; ++cb)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if ((nzb >> (4 * cb + j)) & 1u) {
              if (k >= 0 && k < kCapM)
                dst[k] = make_int2((4 * rowq + j) | ((16 * cb + colc) << 8),
                                   __float_as_int(acc[cb][j]));
              ++k;
            }
        __syncthreads();
        if (pass == 0) {
          need = subnb[lane];  // the 64 counts, one per lane
          need = max(need, __shfl_xor(need, 1));
          need = max(need, __shfl_xor(need, 2));
          need = max(need, __shfl_xor(need, 4));
          need = max(need, __shfl_xor(need, 8));
          need = max(need, __shfl_xor(need, 16));
          need = max(need, __shfl_xor(need, 32));
        }
        // owner w: the map step (Eqs. 9-11) in West's weighted Welford form on
        // y = x - mu_old, lists taken in source-wave order
        int pre[kNW + 1];
        pre[0] = 0;
#pragma unroll
        for (int src = 0; src < kNW; ++src)
          pre[src + 1] = pre[src] + max(0, min(kCapM, subnb[src * kNW + w] - pass * kCapM));
        const int tot = pre[kNW];
        int2* const os = L.osort + w * 64;
        for (int k0 = 0; k0 < tot; k0 += 64) {
          // stable partition of up to 64 of this owner's pairs by component
          // slot c = g / 8 (source order kept within a slot)
          const int k = k0 + lane;
          const bool ok = k < tot;
          int src = 0;
#pragma unroll
          for (int t = 1; t < kNW; ++t) src = k >= pre[t] ? t : src;
          const int2 e = ok ? subb[(size_t)(src * kNW + w) * kCapM + (k - pre[src])]
                            : make_int2(0, 0);
          const int cs = ok ? (e.x >> 11) : -1;
          int cnt[CPW];
          int off = 0, mypos = 0;
#pragma unroll
          for (int c = 0; c < CPW; ++c) {
            const unsigned long long m = __ballot(cs == c);
            if (cs == c) mypos = off + __popcll(m & lt);
            cnt[c] = __popcll(m);
            off += cnt[c];
          }
          // row of the sample within the round | component << 8
          if (ok) os[mypos] = make_int2((kGS * src + (e.x & 15)) | (e.x & ~0xFF), e.y);
          wave_lds_sync();
          // the map step (Eqs. 9-11) in West's weighted Welford form on
          // y = x - mu_old, slot by slot, pairs in the order above
          int o = 0;
          // opaque per chunk, so the per-slot row addresses below are not
          // hoisted out of the round loop
          int wo = w;
          asm volatile("" : "+v"(wo));
          // D <= 64, rows in global memory: the deviation row of every
          // slot's first pair is fetched before any update, so those loads
          // share one round trip (the rest of a slot's pairs follow as below)
          constexpr bool kFirst = !STG && DPL == 1;
          float yf[kFirst ? CPW : 1];
          if constexpr (kFirst) {
            int rowf[CPW];
            int of = 0;
#pragma unroll
            for (int c = 0; c < CPW; ++c) {
              // an empty slot reads the round's first sample (in range)
              rowf[c] = cnt[c] > 0 ? (os[min(of, 63)].x & 0xFF) : 0;
              of += cnt[c];
            }
#pragma unroll
            for (int c = 0; c < CPW; ++c) {
              const int g = g0 + wo + kNW * c;
              const float m0 = kMuReg ? mur[kMuReg ? c : 0][0]
                                      : a.means[(size_t)min(g, Gt - 1) * D + min(lane, D - 1)];
              yf[c] = a.X[(base + rowf[c]) * a.ldx + min(lane, D - 1)] - m0;
            }
          }
#pragma unroll
          for (int c = 0; c < CPW; ++c) {
            const int cc = cnt[c];
            if (cc > 0) {
              const int g = g0 + wo + kNW * c;
              float mu[DPL];
#pragma unroll
              for (int jd = 0; jd < DPL; ++jd)
                mu[jd] = kMuReg ? mur[kMuReg ? c : 0][jd]
                         : STG  ? smu[g * D + min(lane + kWave * jd, D - 1)]
                                : a.means[(size_t)g * D + min(lane + kWave * jd, D - 1)];
              if constexpr (kFirst) {
                const float r = __int_as_float(os[o].y);
                if (r != 0.0f) {
                  const float Lo = Lc[c];
                  const float Ln = Lo + r;
                  const float rc = __builtin_amdgcn_rcpf(Ln);
                  const float inv = r * rc;
                  const float wo = Lo * rc;
                  const float w2 = inv * Lo;
                  const bool dom = inv > 0.5f;
                  Lc[c] = Ln;
                  const float dl = yf[c] - S1[c][0];
                  S1[c][0] = dom ? fmaf(-wo, dl, yf[c]) : fmaf(inv, dl, S1[c][0]);
                  S2[c][0] = fmaf(w2 * dl, dl, S2[c][0]);
                }
              }
              for (int q0 = kFirst ? 1 : 0; q0 < cc; q0 += 4) {
                float rq[4], y[4][DPL];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  const int2 e2 = os[o + min(q0 + i, cc - 1)];
                  rq[i] = q0 + i < cc ? __int_as_float(e2.y) : 0.0f;
                  const float* xr = STG ? xsr + (e2.x & 0xFF) * D
                                        : a.X + (base + (e2.x & 0xFF)) * a.ldx;
#pragma unroll
                  for (int jd = 0; jd < DPL; ++jd)
                    y[i][jd] = xr[min(lane + kWave * jd, D - 1)] - mu[jd];
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  const float r = rq[i];
                  if (r != 0.0f) {
                    const float Lo = Lc[c];
                    const float Ln = Lo + r;
                    const float rc = __builtin_amdgcn_rcpf(Ln);
                    const float inv = r * rc;
                    const float wo = Lo * rc;
                    const float w2 = inv * Lo;
                    // a sample outweighing the run so far takes the mean from
                    // its own side (the first sample sets it exactly: wo = 0)
                    const bool dom = inv > 0.5f;
                    Lc[c] = Ln;
#pragma unroll
                    for (int jd = 0; jd < DPL; ++jd) {
                      const float dl = y[i][jd] - S1[c][jd];
                      S1[c][jd] = dom ? fmaf(-wo, dl, y[i][jd]) : fmaf(inv, dl, S1[c][jd]);
                      S2[c][jd] = fmaf(w2 * dl, dl, S2[c][jd]);
                    }
                  }
                }
              }
              o += cc;
            }
          }
          wave_lds_sync();
        }
        if ((pass + 1) * kCapM >= need) break;
        __syncthreads();  // this buffer is refilled by the next pass
      }
    }
  }

  if constexpr (MODE == 1 || MODE == 2) return;
  if constexpr (kPriv) {
    // the 8 waves' states of each component, combined in wave order by the
    // pairwise update of (L, m, Q) in FP64 (as across work ranges); the
    // round buffers and the FP64 constants are free here
    __syncthreads();
    float* const mb = xs;  // [8][G][2D + 1]
#pragma unroll
    for (int g = 0; g < 16; ++g)
      if (g < G) {
        float* const o = mb + (size_t)(w * G + g) * P;
        if (lane == 0) o[0] = Lp[g];
        if (lane < D) {
          o[1 + lane] = P1[g];
          o[1 + D + lane] = P2[g];
        }
      }
    __syncthreads();
    double* pb = a.part + (size_t)b * Gt * P;
    for (int g = w; g < G; g += kNW) {
      double Lt = 0.0, mt = 0.0, Qt = 0.0;
      for (int q = 0; q < kNW; ++q) {
        const float* const o = mb + (size_t)(q * G + g) * P;
        const double Lb = (double)o[0];
        if (Lb == 0.0) continue;
        const double mbq = lane < D ? (double)o[1 + lane] : 0.0;
        const double Qb = lane < D ? (double)o[1 + D + lane] : 0.0;
        const double Ln = Lt + Lb;
        const double dl = mbq - mt;
        mt += dl * (Lb / Ln);
        Qt += Qb + dl * dl * (Lt * Lb / Ln);
        Lt = Ln;
      }
      if (lane == 0) pb[(size_t)g * P] = Lt;
      if (lane < D) {
        pb[(size_t)g * P + 1 + lane] = mt;
        pb[(size_t)g * P + 1 + D + lane] = Qt;
      }
    }
  } else if (MSTEP) {
    double* pb = a.part + (size_t)b * Gt * P + (size_t)g0 * P;
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int g = w + kNW * c;
      if (g < G) {
        if (lane == 0) pb[(size_t)g * P] = (double)Lc[c];
#pragma unroll
        for (int jd = 0; jd < DPL; ++jd) {
          const int d = lane + kWave * jd;
          if (d < D) {
            pb[(size_t)g * P + 1 + d] = (double)S1[c][jd];
            pb[(size_t)g * P + 1 + D + d] = (double)S2[c][jd];
          }
        }
      }
    }
  }
  if (a.n_rec && lane == 0 && nrec)
    atomicAdd((unsigned long long*)a.n_rec, (unsigned long long)nrec);
  if (MODE == 3) return;  // k_wll took the log-likelihood
  {
    const double v = wave_sum_d(llacc);
    if (lane == 0) L.llw[w] = v;
  }
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kNW; ++q) s += L.llw[q];
    a.ll_part[b] = s;
  }
  if (bad) atomicOr(a.dev_status, GMM_DEV_NONFINITE);
}

template <int CPW, int DPL, bool MSTEP, bool STG>
__global__ void __launch_bounds__(kThreads) k_em2(FastArgs a) {
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  const int b = blockIdx.x;
  const int64_t i0 = (int64_t)b * a.chunk;
  const int64_t i1 = min(a.N, i0 + a.chunk);
  em2_range<CPW, DPL, MSTEP, 0, STG>(a, i0, i1, b, lds_raw);
}

// One sliced pass (MODE 1, 2 or 3): grid (work ranges, slices); slice s holds
// components Gs s .. min(Gs (s + 1), Gt) - 1.
template <int DPL, int MODE>
__global__ void __launch_bounds__(kThreads) k_em2s(FastArgs a) {
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  const int b = blockIdx.x;
  FastArgs s = a;
  s.sl = blockIdx.y;
  s.g0 = s.sl * s.Gs;
  s.G = min(s.Gs, s.Gt - s.g0);
  const int64_t i0 = (int64_t)b * a.chunk;
  const int64_t i1 = min(a.N, i0 + a.chunk);
  em2_range<16, DPL, MODE == 3, MODE>(s, i0, i1, b, lds_raw);
}

// The bound over all slices of each sample into slot 0 of wM (in place: the
// maximum is unchanged by it, so later passes may take it again).
__global__ void __launch_bounds__(256) k_wmax(float* __restrict__ wM, int S, int64_t NS,
                                              int64_t N) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  float m = wM[n];
  for (int q = 1; q < S; ++q) m = fmaxf(m, wM[(size_t)q * NS + n]);
  wM[n] = m;
}

// Log-likelihood of the sliced passes: per sample lse = M + slice_lse, the
// workgroup's samples summed per thread and the threads in order.  With comb
// set it also leaves, in slot 0 of each array, what the map pass needs of the
// sample: M (wM), D* (wD) and log(sum over slices of S_q exp(D_q - D*)) (wS),
// each thread reading all slots of its sample before it writes them.
constexpr int kWllT = 256;
__global__ void __launch_bounds__(kWllT) k_wll(float* __restrict__ wM, float* __restrict__ wD,
                                               float* __restrict__ wS, int S, int64_t NS,
                                               int64_t N, int64_t chunk,
                                               float* __restrict__ per_sample,
                                               double* __restrict__ ll_part,
                                               int32_t* __restrict__ dev_status, int comb) {
  __shared__ double sh[kWllT];
  const int b = blockIdx.x;
  const int64_t i0 = (int64_t)b * chunk;
  const int64_t i1 = min(N, i0 + chunk);
  double acc = 0.0;
  int bad = 0;
  for (int64_t n = i0 + threadIdx.x; n < i1; n += kWllT) {
    float m = -INFINITY;
    for (int q = 0; q < S; ++q) m = fmaxf(m, wM[(size_t)q * NS + n]);
    double ls;
    const float dstar = slice_lse(wD + n, wS + n, S, NS, ls);
    const double lse = ((double)m + (double)dstar) + ls;
    acc += lse;
    if (!isfinite(lse)) bad = 1;
    if (per_sample) per_sample[n] = (float)lse;
    if (comb) {
      wM[n] = m;
      wD[n] = dstar;
      wS[n] = (float)ls;  // a float widened: exact
    }
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < kWllT; ++i) t += sh[i];
    ll_part[b] = t;
  }
  if (bad) atomicOr(dev_status, GMM_DEV_NONFINITE);
}

template <int CPW, int DPL, bool MSTEP, bool STG>
__global__ void __launch_bounds__(kThreads) k_em2_batched(FastArgs base,
                                                          const gmm_model_desc* models,
                                                          const BatchItemDev* items,
                                                          const int* n_items, BatchConst bc) {
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  const int ni = *n_items;
  const int D = base.D;
  const int P = 2 * D + 1;
  for (int it = blockIdx.x; it < ni; it += gridDim.x) {
    const BatchItemDev item = items[it];
    const gmm_model_desc& m = models[item.model];
    FastArgs a = base;
    const size_t mi = (size_t)item.model;
    a.X = m.X;
    a.N = m.N;
    a.ldx = D;
    a.G = m.G;
    a.prm = bc.prm + mi * 2 * bc.Gmax * (D + 1);
    a.cc = bc.cc + mi * 2 * bc.Gmax;
    a.cexp = bc.cexp + mi * 2 * bc.Gmax;
    a.Whi = bc.Whi + mi * bc.RBmax * bc.KS * 64;
    a.Wlo = bc.Wlo + mi * bc.RBmax * bc.KS * 64;
    a.c64 = bc.c64 + mi * bc.Gmax;
    a.lam64 = bc.lam64 + mi * bc.Gmax * D;
    a.means = m.means;
    a.part = base.part + (size_t)it * bc.Gmax * P;
    a.ll_part = base.ll_part + it;
    a.per_sample = nullptr;
    a.dev_status = m.dev_status;
    a.n_rec = nullptr;
    // the smallest component-block template that holds the model's G
    if (CPW > 2 && a.G <= 16)
      em2_range<(CPW > 2 ? 2 : CPW), DPL, MSTEP, 0, STG>(a, item.i0, item.i1, 0, lds_raw);
    else if (CPW > 4 && a.G <= 32)
      em2_range<(CPW > 4 ? 4 : CPW), DPL, MSTEP, 0, STG>(a, item.i0, item.i1, 0, lds_raw);
    else if (CPW > 8 && a.G <= 64)
      em2_range<(CPW > 8 ? 8 : CPW), DPL, MSTEP, 0, STG>(a, item.i0, item.i1, 0, lds_raw);
    else em2_range<CPW, DPL, MSTEP, 0, STG>(a, item.i0, item.i1, 0, lds_raw);
    __syncthreads();
  }
}

template <int CPW, int DPL, bool MSTEP>
void launch_one(const FastArgs& a, int nb, size_t lds, hipStream_t st) {
  auto kern = k_em_fast<CPW, DPL, MSTEP>;
  static bool attr_set = false;  // benign race: setting the attribute twice is harmless
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    attr_set = true;
  }
  hipLaunchKernelGGL(kern, dim3(nb), dim3(kThreads), lds, st, a);
}

template <bool MSTEP>
void dispatch_cpw(const FastArgs& a, int nb, size_t lds, hipStream_t st) {
  {
  const int cpw = (a.G + kNW - 1) / kNW;
  const int dpl = (a.D + kWave - 1) / kWave;
  if (dpl == 1) {
    if (cpw <= 2) launch_one<2, 1, MSTEP>(a, nb, lds, st);
    else if (cpw <= 4) launch_one<4, 1, MSTEP>(a, nb, lds, st);
    else if (cpw <= 8) launch_one<8, 1, MSTEP>(a, nb, lds, st);
    else if (cpw <= 13) launch_one<13, 1, MSTEP>(a, nb, lds, st);
    else launch_one<16, 1, MSTEP>(a, nb, lds, st);
  } else {
    if (cpw <= 2) launch_one<2, 2, MSTEP>(a, nb, lds, st);
    else if (cpw <= 4) launch_one<4, 2, MSTEP>(a, nb, lds, st);
    else if (cpw <= 8) launch_one<8, 2, MSTEP>(a, nb, lds, st);
    else if (cpw <= 13) launch_one<13, 2, MSTEP>(a, nb, lds, st);
    else launch_one<16, 2, MSTEP>(a, nb, lds, st);
  }
  }
}

template <int CPW, int DPL, bool MSTEP, bool STG = false>
void launch_em2_one(const FastArgs& a, int nb, size_t lds, hipStream_t st) {
  auto kern = k_em2<CPW, DPL, MSTEP, STG>;
  static bool attr_set = false;  // benign race: setting the attribute twice is harmless
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    attr_set = true;
  }
  hipLaunchKernelGGL(kern, dim3(nb), dim3(kThreads), lds, st, a);
}

template <bool MSTEP>
void dispatch_em2(const FastArgs& a, int nb, size_t lds, hipStream_t st, bool stg) {
  const int cpw = (a.G + kNW - 1) / kNW;
  if (stg) {
    if (cpw <= 2) launch_em2_one<2, 1, MSTEP, true>(a, nb, lds, st);
    else if (cpw <= 4) launch_em2_one<4, 1, MSTEP, true>(a, nb, lds, st);
    else if (cpw <= 8) launch_em2_one<8, 1, MSTEP, true>(a, nb, lds, st);
    else if (cpw <= 13) launch_em2_one<13, 1, MSTEP, true>(a, nb, lds, st);
    else launch_em2_one<16, 1, MSTEP, true>(a, nb, lds, st);
  } else if (a.D <= 64) {
    if (cpw <= 2) launch_em2_one<2, 1, MSTEP>(a, nb, lds, st);
    else if (cpw <= 4) launch_em2_one<4, 1, MSTEP>(a, nb, lds, st);
    else if (cpw <= 8) launch_em2_one<8, 1, MSTEP>(a, nb, lds, st);
    else if (cpw <= 13) launch_em2_one<13, 1, MSTEP>(a, nb, lds, st);
    else launch_em2_one<16, 1, MSTEP>(a, nb, lds, st);
  } else {
    if (cpw <= 2) launch_em2_one<2, 2, MSTEP>(a, nb, lds, st);
    else if (cpw <= 4) launch_em2_one<4, 2, MSTEP>(a, nb, lds, st);
    else if (cpw <= 8) launch_em2_one<8, 2, MSTEP>(a, nb, lds, st);
    else if (cpw <= 13) launch_em2_one<13, 2, MSTEP>(a, nb, lds, st);
    else launch_em2_one<16, 2, MSTEP>(a, nb, lds, st);
  }
}

// LDS of the sliced passes: MODE 1 uses the fragments and constants, MODE 2
// also the near-pair buffers, MODE 3 all of it.
size_t em2s_lds_bytes(int Gs, int KS, int mode) {
  const int upto = mode == 1 ? 3 : (mode == 2 ? 7 : -1);
  if (upto < 0) return em2_lds_bytes(Gs, KS);
  size_t r = 0;
  lds2_walk(Gs, KS, [&](int which, size_t off) {
    if (which == upto) r = off;
  });
  return r * 4 + 64;
}

template <int DPL, int MODE>
void launch_em2s_one(const FastArgs& a, int nb, hipStream_t st) {
  auto kern = k_em2s<DPL, MODE>;
  static bool attr_set = false;  // benign race: setting the attribute twice is harmless
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    attr_set = true;
  }
  hipLaunchKernelGGL(kern, dim3(nb, a.S), dim3(kThreads), em2s_lds_bytes(a.Gs, a.KS, MODE), st,
                     a);
}

}  // namespace

int em_fast_blocks(int64_t N) {
  int64_t b = (N + kT * 4 - 1) / (kT * 4);
  if (b < 1) b = 1;
  if (b > 256) b = 256;
  return (int)b;
}

// components per slice: the largest multiple of 16 (at most 128) whose LDS
// fits one CU, then evened out over the slices
int em2s_slice_max(int D) {
  if (D < 1 || D > 128) return 0;
  for (int gs = 128; gs >= 16; gs -= 16)
    if (em2_lds_bytes(gs, em2_ks(D)) <= 160 * 1024) return gs;
  return 0;
}

bool em2s_supported(int D, int G) { return G >= 1 && em2s_slice_max(D) > 0; }

int em2s_slices(int D, int G) {
  const int gm = em2s_slice_max(D);
  return gm > 0 && G >= 1 ? (G + gm - 1) / gm : 0;
}

hipError_t launch_em_sliced(const float* X, int64_t N, int D, int64_t ldx, int G,
                            const float* hefts, const float* means, const float* covs, bool mstep,
                            int64_t* n_recomputed, float* per_sample, int32_t* dev_status,
                            const Workspace& w, hipStream_t st, int* nb_out) {
  const int KS = em2_ks(D);
  const int S = em2s_slices(D, G);
  if (S < 1 || !w.wM || !w.wD || !w.wS || !w.wR) return hipErrorInvalidValue;
  const int Gs = 16 * (((G + S - 1) / S + 15) / 16);
  const int nb0 = em_fast_blocks(N);
  FastArgs a;
  a.X = X;
  a.N = N;
  a.ldx = ldx;
  a.chunk = ((N + nb0 - 1) / nb0 + kRoundN - 1) / kRoundN * kRoundN;
  const int nb = (int)((N + a.chunk - 1) / a.chunk);
  a.D = D;
  a.G = Gs;
  a.KS = KS;
  a.prm = w.prm;
  a.cc = w.c;
  a.cexp = w.cexp;
  a.Whi = (const bf16x8*)w.Bhi;
  a.Wlo = (const bf16x8*)w.Blo;
  a.c64 = w.c64;
  a.lam64 = w.lamg64;
  a.means = means;
  a.part = w.partials;
  a.ll_part = w.scalars;
  a.per_sample = per_sample;
  a.dev_status = dev_status;
  a.n_rec = n_recomputed;
  a.g0 = 0;
  a.Gt = G;
  a.Gs = Gs;
  a.sl = 0;
  a.S = S;
  a.NS = N;
  a.wM = w.wM;
  a.wD = w.wD;
  a.wS = w.wS;
  a.wR = w.wR;
  a.NG = (N + kGS - 1) / kGS;
  hipLaunchKernelGGL(k_pre_fast, dim3(16 * ((G + 15) / 16)), dim3(256), 0, st, hefts, means,
                     covs, D, G, KS, w.prm, w.c, w.cexp, (bf16x8*)w.Bhi, (bf16x8*)w.Blo, w.c64,
                     w.lamg64, dev_status, n_recomputed, w.counters);
  {
    ProfScope ps(mstep ? kProfEM : kProfLoglik, st);
    // bounds, near pairs and slice sums; the log-likelihood (and, before a
    // map pass, each sample's combination of its slices); the map pass
    if (D <= 64) launch_em2s_one<1, 1>(a, nb, st);
    else launch_em2s_one<2, 1>(a, nb, st);
    hipLaunchKernelGGL(k_wmax, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, w.wM, S, N,
                       N);
    if (D <= 64) launch_em2s_one<1, 2>(a, nb, st);
    else launch_em2s_one<2, 2>(a, nb, st);
    hipLaunchKernelGGL(k_wll, dim3(nb), dim3(kWllT), 0, st, w.wM, w.wD, w.wS, S, N, N, a.chunk,
                       per_sample, w.scalars, dev_status, mstep ? 1 : 0);
    if (mstep) {
      if (D <= 64) launch_em2s_one<1, 3>(a, nb, st);
      else launch_em2s_one<2, 3>(a, nb, st);
    }
  }
  *nb_out = nb;
  return hipGetLastError();
}

bool em_fast_supported(int D, int G, int prec) {
  if (D < 1 || D > 128 || G < 1 || G > 128) return false;
  if (prec == GMM_PREC_BF16X3) return em2_lds_bytes(G, em2_ks(D)) <= 160 * 1024;
  return fast_lds_bytes(D, G) <= 160 * 1024;
}

hipError_t launch_em_fast(const float* X, int64_t N, int D, int64_t ldx, int G, const float* hefts,
                          const float* means, const float* covs, int prec, bool mstep,
                          int64_t* n_recomputed, float* per_sample, int32_t* dev_status,
                          const Workspace& w, hipStream_t st, int* nb_out) {
  const int KS = em2_ks(D);  // k-steps of the expanded form's fragments
  const int nb = em_fast_blocks(N);
  FastArgs a;
  a.X = X;
  a.N = N;
  a.ldx = ldx;
  a.chunk = ((N + nb - 1) / nb + kT - 1) / kT * kT;
  a.D = D;
  a.G = G;
  a.KS = KS;
  a.prm = w.prm;
  a.cc = w.c;
  a.cexp = w.cexp;
  a.Whi = (const bf16x8*)w.Bhi;
  a.Wlo = (const bf16x8*)w.Blo;
  a.c64 = w.c64;
  a.lam64 = w.lamg64;
  a.means = means;
  a.part = w.partials;
  a.ll_part = w.scalars;
  a.per_sample = per_sample;
  a.dev_status = dev_status;
  a.n_rec = n_recomputed;
  hipLaunchKernelGGL(k_pre_fast, dim3(16 * ((G + 15) / 16)), dim3(256), 0, st, hefts, means,
                     covs, D, G, KS, w.prm, w.c, w.cexp, (bf16x8*)w.Bhi, (bf16x8*)w.Blo, w.c64,
                     w.lamg64, dev_status, n_recomputed, w.counters);
  {
    ProfScope ps(mstep ? kProfEM : kProfLoglik, st);
    if (prec == GMM_PREC_BF16X3) {
      // sample-major kernel: work ranges in whole 128-sample rounds
      const int64_t ch = ((N + nb - 1) / nb + kRoundN - 1) / kRoundN * kRoundN;
      a.chunk = ch;
      const int nb2 = (int)((N + ch - 1) / ch);
      const bool stg = em2_stage_fits(D, G);
      const size_t lds = stg ? em2_stage_lds_max(D, G) : em2_lds_bytes(G, KS);
      if (mstep) dispatch_em2<true>(a, nb2, lds, st, stg);
      else dispatch_em2<false>(a, nb2, lds, st, stg);
      *nb_out = nb2;
      return hipGetLastError();
    }
    const size_t lds = fast_lds_bytes(D, G);
    if (mstep) dispatch_cpw<true>(a, nb, lds, st);
    else dispatch_cpw<false>(a, nb, lds, st);
  }
  *nb_out = nb;
  return hipGetLastError();
}

hipError_t launch_fin_welford(int nb, int64_t N, int D, int G, float var_floor, float* hefts,
                              float* means, float* covs, double* mean_loglik, int32_t* dev_status,
                              const Workspace& w, hipStream_t st) {
  // more than 64 blocks: segments of 32 first (G x segments workgroups), so
  // that the G final chains are short
  const int seg = nb > 64 ? 32 : 1;
  if (seg > 1)
    hipLaunchKernelGGL(k_welford_seg, dim3(G, (nb + seg - 1) / seg), dim3(256), 0, st, w.partials,
                       nb, seg, D, G);
  hipLaunchKernelGGL(k_fin_welford, dim3(G), dim3(256), 0, st, w.partials, nb, seg, N, D, G,
                     var_floor, hefts, means, covs, w.scalars, mean_loglik, dev_status);
  return hipGetLastError();
}

namespace {

template <bool MSTEP, int CPW, int DPL>
void launch_batched_one(const FastArgs& base, const gmm_model_desc* models, const BatchWorkspace& bw,
                        const BatchConst& bc, int grid, size_t lds, hipStream_t st) {
  auto kern = k_em_fast_batched<CPW, DPL, MSTEP>;
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    attr_set = true;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, st, base, models, bw.items,
                     bw.n_items, bc);
}

template <bool MSTEP, int CPW, int DPL, bool STG = false>
void launch_em2_batched_one(const FastArgs& base, const gmm_model_desc* models,
                            const BatchWorkspace& bw, const BatchConst& bc, int grid, size_t lds,
                            hipStream_t st) {
  auto kern = k_em2_batched<CPW, DPL, MSTEP, STG>;
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    attr_set = true;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, st, base, models, bw.items,
                     bw.n_items, bc);
}

template <bool MSTEP>
void dispatch_em2_batched(const FastArgs& base, const gmm_model_desc* models,
                          const BatchWorkspace& bw, const BatchConst& bc, int grid, size_t lds,
                          hipStream_t st, bool stg) {
  const int cpw = (bw.Gmax + kNW - 1) / kNW;
  if (stg) {
    if (cpw <= 2) launch_em2_batched_one<MSTEP, 2, 1, true>(base, models, bw, bc, grid, lds, st);
    else if (cpw <= 4) launch_em2_batched_one<MSTEP, 4, 1, true>(base, models, bw, bc, grid, lds, st);
    else if (cpw <= 8) launch_em2_batched_one<MSTEP, 8, 1, true>(base, models, bw, bc, grid, lds, st);
    else launch_em2_batched_one<MSTEP, 16, 1, true>(base, models, bw, bc, grid, lds, st);
  } else if (bw.D <= 64) {
    if (cpw <= 2) launch_em2_batched_one<MSTEP, 2, 1>(base, models, bw, bc, grid, lds, st);
    else if (cpw <= 4) launch_em2_batched_one<MSTEP, 4, 1>(base, models, bw, bc, grid, lds, st);
    else if (cpw <= 8) launch_em2_batched_one<MSTEP, 8, 1>(base, models, bw, bc, grid, lds, st);
    else launch_em2_batched_one<MSTEP, 16, 1>(base, models, bw, bc, grid, lds, st);
  } else {
    if (cpw <= 2) launch_em2_batched_one<MSTEP, 2, 2>(base, models, bw, bc, grid, lds, st);
    else if (cpw <= 4) launch_em2_batched_one<MSTEP, 4, 2>(base, models, bw, bc, grid, lds, st);
    else if (cpw <= 8) launch_em2_batched_one<MSTEP, 8, 2>(base, models, bw, bc, grid, lds, st);
    else launch_em2_batched_one<MSTEP, 16, 2>(base, models, bw, bc, grid, lds, st);
  }
}

template <bool MSTEP>
void dispatch_batched(const FastArgs& base, const gmm_model_desc* models, const BatchWorkspace& bw,
                      const BatchConst& bc, int grid, size_t lds, hipStream_t st) {
  const int cpw = (bw.Gmax + kNW - 1) / kNW;
  if (bw.D <= 64) {
    if (cpw <= 2) launch_batched_one<MSTEP, 2, 1>(base, models, bw, bc, grid, lds, st);
    else if (cpw <= 4) launch_batched_one<MSTEP, 4, 1>(base, models, bw, bc, grid, lds, st);
    else if (cpw <= 8) launch_batched_one<MSTEP, 8, 1>(base, models, bw, bc, grid, lds, st);
    else launch_batched_one<MSTEP, 16, 1>(base, models, bw, bc, grid, lds, st);
  } else {
    if (cpw <= 2) launch_batched_one<MSTEP, 2, 2>(base, models, bw, bc, grid, lds, st);
    else if (cpw <= 4) launch_batched_one<MSTEP, 4, 2>(base, models, bw, bc, grid, lds, st);
    else if (cpw <= 8) launch_batched_one<MSTEP, 8, 2>(base, models, bw, bc, grid, lds, st);
    else launch_batched_one<MSTEP, 16, 2>(base, models, bw, bc, grid, lds, st);
  }
}

}  // namespace

bool em_batched_supported(int D, int Gmax, int prec) {
  return em_fast_supported(D, Gmax, prec);
}

hipError_t launch_em_batched(const gmm_model_desc* models, int n_models, int n_items_host, int D,
                             float var_floor, int prec, bool mstep, const BatchWorkspace& bw,
                             hipStream_t st) {
  BatchConst bc;
  bc.prm = bw.prm;
  bc.cc = bw.cc;
  bc.cexp = bw.cexp;
  bc.Whi = (bf16x8*)bw.Whi;
  bc.Wlo = (bf16x8*)bw.Wlo;
  bc.c64 = bw.c64;
  bc.lam64 = bw.lam64;
  bc.Gmax = bw.Gmax;
  bc.RBmax = bw.RBmax;
  bc.KS = bw.KS;
  FastArgs base{};
  base.D = D;
  base.KS = bw.KS;
  base.part = bw.partials;
  base.ll_part = bw.sparts;
  hipLaunchKernelGGL(k_pre_fast_batched, dim3(16 * bw.RBmax, n_models), dim3(256), 0, st, models,
                     D, bc);
  const bool stg = prec == GMM_PREC_BF16X3 && em2_stage_fits(D, bw.Gmax);
  const size_t lds = prec == GMM_PREC_BF16X3
                         ? (stg ? em2_stage_lds_max(D, bw.Gmax) : em2_lds_bytes(bw.Gmax, em2_ks(D)))
                         : fast_lds_bytes(D, bw.Gmax);
  const int grid = n_items_host < 256 ? (n_items_host < 1 ? 1 : n_items_host) : 256;
  {
    ProfScope ps(kProfBatched, st);
    if (prec == GMM_PREC_BF16X3) {
      if (mstep) dispatch_em2_batched<true>(base, models, bw, bc, grid, lds, st, stg);
      else dispatch_em2_batched<false>(base, models, bw, bc, grid, lds, st, stg);
    } else {
      if (mstep) dispatch_batched<true>(base, models, bw, bc, grid, lds, st);
      else dispatch_batched<false>(base, models, bw, bc, grid, lds, st);
    }
  }
  hipLaunchKernelGGL(k_fin_welford_batched, dim3(bw.Gmax, n_models), dim3(256), 0, st, models,
                     bw.mitems, D, bw.Gmax, var_floor, bw.partials, bw.sparts, mstep ? 1 : 0);
  return hipGetLastError();
}

}  // namespace gmm
