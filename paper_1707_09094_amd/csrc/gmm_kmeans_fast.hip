// gmm_kmeans_fast.hip -- one-pass k-means iteration for D <= 128 dimensions
// and G <= 128 means (larger shapes use the generic kernels of
// gmm_kmeans.hip).  Two screening forms: k_km2 (matrix cores, BF16x3; every
// batched call and the single-model call in that precision; described at its
// definition) and k_km_fast (FP32 direct form, the single-model FP32 call),
// described here.
//
// Workgroup of 8 waves, persistent over a contiguous sample range, tiles of 32
// samples (next tile prefetched into registers).  Per tile:
//   1. distances (Sec. 3 Eq. 19 with the Eq. 20 weights) in FP32:
//        d_gn = sum_d u^2,  u = fma(x_d, s_d, -m_gd),  s_d = sqrt(lam_d),
//        m_gd = mu_gd s_d
//      thread per (mean, 8 samples);
//   2. per sample the best and second-best distance (lowest index on ties).
//      With e = 2^-24, every FP32 distance is within
//        bound(d) = 2 e ((D + 6) d + 2 sqrt(d) max_g |m_g|)
//      of sum_d s_d^2 (x_d - mu_gd)^2, so when d2 - d1 <= bound(d1) +
//      bound(d2) the sample is re-decided in FP64 over all means (first
//      minimum wins); the counted samples are reported as n_recomputed;
//   3. FP64 distance of each sample to its chosen mean (inertia), 8 lanes per
//      sample;
//   4. map step of Sec. 2.1 with l in {0,1}: wave w owns means g = w, w+8, ...;
//      for its samples, in sample order, the weighted-Welford update (West) of
//      (count, mean of y, sum of squared deviations) with y = x - mu_old.
#include "gmm_internal.hpp"

namespace gmm {

namespace {

constexpr int kNW = 8;
constexpr int kThreads = kNW * kWave;
constexpr int kT = 32;
constexpr int kPF = 8;
constexpr float kE32 = 5.9604645e-08f;

struct KmArgs {
  const float* X;
  int64_t N;
  int64_t ldx;
  int64_t chunk;
  int D, G;
  const float* means;   // [G][D]
  const float* mprm;    // [G][D+1]: m_gd = mu_gd s_d
  const float* sd;      // [D]: s_d
  const double* lam64;  // [D]
  const float* mnorm;   // [1]: max_g |m_g|
  int32_t* assign;      // [N]
  double* part;         // [nb][G][2D+1]
  double* in_part;      // [nb]
  int64_t* n_rec;
  int32_t* dev_status;
};

template <typename F>
__host__ __device__ inline size_t km_lds_walk(int D, int G, F&& at) {
  size_t w = 0;
  auto put = [&](int which, size_t words, size_t align_words) {
    w = (w + align_words - 1) / align_words * align_words;
    at(which, w);
    w += words;
  };
  put(0, (size_t)G * D, 1);        // mu
  put(1, (size_t)G * (D + 1), 1);  // m
  put(2, D, 1);                    // s
  put(3, 2 * (size_t)D, 2);        // lam64
  put(4, (size_t)kT * D, 4);       // xf
  put(5, (size_t)G * kT, 1);       // dist
  put(6, kNW * kT, 1);             // pbest
  put(7, kNW * kT, 1);             // psec
  put(8, kNW * kT, 1);             // parg
  put(9, kT, 1);                   // arg
  put(10, 2 * kT, 2);              // dist64 of the chosen mean
  return w;
}

__host__ __device__ inline size_t km_lds_bytes(int D, int G) {
  return km_lds_walk(D, G, [](int, size_t) {}) * 4 + 64;
}

template <int CPW, int DPL>
__device__ __forceinline__ void km_range(const KmArgs& a, int64_t i0, int64_t i1, int b,
                                         char* lds_raw) {
  const int D = a.D, G = a.G;
  const int DP = D + 1;
  float *mu, *mm, *sv, *xf, *dist, *pbest, *psec;
  double *l64, *d64;
  int *parg, *arg;
  {
    float* f = (float*)lds_raw;
    km_lds_walk(D, G, [&](int which, size_t off) {
      switch (which) {
        case 0: mu = f + off; break;
        case 1: mm = f + off; break;
        case 2: sv = f + off; break;
        case 3: l64 = (double*)(f + off); break;
        case 4: xf = f + off; break;
        case 5: dist = f + off; break;
        case 6: pbest = f + off; break;
        case 7: psec = f + off; break;
        case 8: parg = (int*)(f + off); break;
        case 9: arg = (int*)(f + off); break;
        default: d64 = (double*)(f + off); break;
      }
    });
  }
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int w = tid / kWave;
  const int P = 2 * D + 1;

  for (int p = tid; p < G * D; p += kThreads) mu[p] = a.means[p];
  for (int p = tid; p < G * DP; p += kThreads) mm[p] = a.mprm[p];
  for (int p = tid; p < D; p += kThreads) {
    sv[p] = a.sd[p];
    l64[p] = a.lam64[p];
  }
  const float mnorm = *a.mnorm;

  float Lc[CPW], S1[CPW][DPL], S2[CPW][DPL];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    Lc[c] = 0.0f;
#pragma unroll
    for (int j = 0; j < DPL; ++j) S1[c][j] = S2[c][j] = 0.0f;
  }
  double inacc = 0.0;  // wave 0, lane n < kT: sample n of every tile
  int bad = 0;
  long long nrec = 0;

  float pf[kPF];
  auto prefetch = [&](int64_t t0, int nt) {
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
  };
  if (i0 < i1) prefetch(i0, (int)min((int64_t)kT, i1 - i0));
  __syncthreads();

  for (int64_t t0 = i0; t0 < i1; t0 += kT) {
    const int nt = (int)min((int64_t)kT, i1 - t0);
#pragma unroll
    for (int i = 0; i < kPF; ++i) {
      const int p = tid + kThreads * i;
      if (p < kT * D) xf[p] = pf[i];
    }
    if (t0 + kT < i1) prefetch(t0 + kT, (int)min((int64_t)kT, i1 - t0 - kT));
    __syncthreads();

    // 1. distances: thread owns mean g = lane + 64 (w & 1), samples 8 (w >> 1) + q
    {
      const int g = lane + kWave * (w & 1);
      const int n0 = 8 * (w >> 1);
      if (g < G) {
        float acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = 0.0f;
        const float* mg = mm + g * DP;
        for (int d = 0; d < D; ++d) {
          const float s = sv[d], m = mg[d];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const float u = fmaf(xf[(n0 + q) * D + d], s, -m);
            acc[q] = fmaf(u, u, acc[q]);
          }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) dist[g * kT + n0 + q] = acc[q];
      }
    }
    __syncthreads();

    // 2. best / second best; lanes 0..31 = samples, lanes 32..63 repeat them
    const int n = lane & (kT - 1);
    {
      float b1 = INFINITY, b2 = INFINITY;
      int ag = G;  // "none" sorts after every real index
      for (int g = w; g < G; g += kNW) {
        const float v = dist[g * kT + n];
        if (v < b1) {
          b2 = b1;
          b1 = v;
          ag = g;
        } else if (v < b2) {
          b2 = v;
        }
      }
      if (lane < kT) {
        pbest[w * kT + n] = b1;
        psec[w * kT + n] = b2;
        parg[w * kT + n] = ag;
      }
    }
    __syncthreads();
    if (w == 0 && lane < kT) {
      float d1 = INFINITY, d2 = INFINITY;
      int ag = G;
#pragma unroll
      for (int q = 0; q < kNW; ++q) {
        const float v = pbest[q * kT + n];
        const int gq = parg[q * kT + n];
        if (v < d1 || (v == d1 && gq < ag)) {
          d2 = fminf(d2, d1);
          d1 = v;
          ag = gq;
        } else {
          d2 = fminf(d2, v);
        }
        d2 = fminf(d2, psec[q * kT + n]);
      }
      if (n < nt) {
        const float bnd1 = 2.0f * kE32 * ((float)(D + 6) * d1 + 2.0f * sqrtf(d1) * mnorm);
        const float bnd2 = 2.0f * kE32 * ((float)(D + 6) * d2 + 2.0f * sqrtf(d2) * mnorm);
        if (G > 1 && !(d2 - d1 > 2.0f * (bnd1 + bnd2))) {
          // near tie or non-finite value: decide in FP64, first minimum wins
          ++nrec;
          const float* x = xf + n * D;
          double best = INFINITY;
          ag = 0;
          for (int g = 0; g < G; ++g) {
            double s = 0.0;
            for (int d = 0; d < D; ++d) {
              const double t = (double)x[d] - (double)mu[g * D + d];
              s += l64[d] * t * t;
            }
            if (s < best) {
              best = s;
              ag = g;
            }
          }
          if (!(best < INFINITY)) {
            bad = 1;
            ag = 0;
          }
        }
        a.assign[t0 + n] = ag;
      } else {
        ag = -1;
      }
      arg[n] = ag;
    }
    __syncthreads();

    // 3. FP64 distance to the chosen mean: 8 lanes per sample (waves 0..3)
    if (tid < kT * 8) {
      const int s = tid >> 3, gl = tid & 7;
      const int g = arg[s];
      double q = 0.0;
      if (g >= 0) {
        const float* x = xf + s * D;
        const float* m = mu + g * D;
        for (int d = gl; d < D; d += 8) {
          const double t = (double)x[d] - (double)m[d];
          q += l64[d] * t * t;
        }
      }
      q += __shfl_xor(q, 1, kWave);
      q += __shfl_xor(q, 2, kWave);
      q += __shfl_xor(q, 4, kWave);
      if (gl == 0) d64[s] = q;
    }
    __syncthreads();
    if (w == 0 && lane < nt) {
      inacc += d64[lane];
      if (!isfinite(d64[lane])) bad = 1;
    }

    // 4. map step, one-hot responsibilities
    {
      const int an = lane < kT ? arg[lane] : -1;
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const int g = w + kNW * c;
        if (g < G) {
          unsigned long long msk = __ballot(an == g);
          while (msk) {
            const int nn = __ffsll((long long)msk) - 1;
            msk &= msk - 1;
            const float Lo = Lc[c];
            const float Ln = Lo + 1.0f;
            const float inv = 1.0f / Ln;
            const float w2 = Lo * inv;
            Lc[c] = Ln;
#pragma unroll
            for (int j = 0; j < DPL; ++j) {
              const int d = lane + kWave * j;
              if (d < D) {
                const float y = xf[nn * D + d] - mu[g * D + d];
                if (Lo == 0.0f) {
                  S1[c][j] = y;
                } else {
                  const float dy = y - S1[c][j];
                  S1[c][j] = fmaf(inv, dy, S1[c][j]);
                  S2[c][j] = fmaf(w2 * dy, dy, S2[c][j]);
                }
              }
            }
          }
        }
      }
    }
    __syncthreads();
  }

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
  if (w == 0) {
    const double v = wave_sum_d(lane < kT ? inacc : 0.0);
    if (lane == 0) a.in_part[b] = v;
  }
  if (bad) atomicOr(a.dev_status, GMM_DEV_NONFINITE);
  if (w == 0 && a.n_rec) {
    long long v = nrec;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    if (lane == 0 && v) atomicAdd((unsigned long long*)a.n_rec, (unsigned long long)v);
  }
}

template <int CPW, int DPL>
__global__ void __launch_bounds__(kThreads) k_km_fast(KmArgs a) {
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  const int b = blockIdx.x;
  const int64_t i0 = (int64_t)b * a.chunk;
  const int64_t i1 = min(a.N, i0 + a.chunk);
  km_range<CPW, DPL>(a, i0, i1, b, lds_raw);
}

// lam_d, s_d = sqrt(lam_d), m_gd = mu_gd s_d and max_g |m_g| (one workgroup).
__device__ void km_pre(const double* __restrict__ gvar, int D, int G, float var_floor, int dist,
                       const float* __restrict__ means, double* __restrict__ lam64,
                       float* __restrict__ sd, float* __restrict__ mprm,
                       float* __restrict__ mnorm) {
  __shared__ float red[256];
  for (int d = threadIdx.x; d < D; d += 256) {
    double l = 1.0;
    if (dist == GMM_DIST_MAHA) {
      double v = gvar[d];
      v = v > (double)var_floor ? v : (double)var_floor;
      l = 1.0 / v;
    }
    lam64[d] = l;
    sd[d] = (float)sqrt(l);
  }
  __syncthreads();
  float mx = 0.0f;
  for (int g = threadIdx.x; g < G; g += 256) {
    double q = 0.0;
    for (int d = 0; d < D; ++d) {
      const float m = (float)((double)means[(size_t)g * D + d] * (double)sd[d]);
      mprm[(size_t)g * (D + 1) + d] = m;
      q += (double)m * (double)m;
    }
    mprm[(size_t)g * (D + 1) + D] = 0.0f;
    mx = fmaxf(mx, (float)sqrt(q) * 1.0000002f);
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *mnorm = red[0];
}

__global__ void __launch_bounds__(256) k_km_pre_fast(const double* __restrict__ gvar, int D,
                                                     int G, float var_floor, int dist,
                                                     const float* __restrict__ means,
                                                     double* __restrict__ lam64,
                                                     float* __restrict__ sd,
                                                     float* __restrict__ mprm,
                                                     float* __restrict__ mnorm) {
  km_pre(gvar, D, G, var_floor, dist, means, lam64, sd, mprm, mnorm);
}

// Reduce step of the k-means map: pairwise (count, mean, M2) combination in
// block order, new means, hand-off variances/weights, counts, inertia.
__global__ void __launch_bounds__(256) k_km_fin_fast(const double* __restrict__ part, int nb,
                                                     int seg, int64_t N, int D, int G,
                                                     float var_floor,
                                                     float* __restrict__ means,
                                                     float* __restrict__ dcovs,
                                                     float* __restrict__ hefts,
                                                     int64_t* __restrict__ counts,
                                                     const double* __restrict__ in_part,
                                                     double* __restrict__ inertia,
                                                     int32_t* __restrict__ dev_status) {
  __shared__ WelfordLds S;
  const int g = blockIdx.x;
  const int P = 2 * D + 1;
  double m, Q;
  // blocks, or every seg-th block holding its segment's combination
  const double Ltot = welford_combine<256, 32>(part + (size_t)g * P, (size_t)seg * G * P,
                                               (nb + seg - 1) / seg, D, S, m, Q);
  const int d = threadIdx.x;
  if (d < D) {
    if (Ltot > 0.0) {
      double v = Q / Ltot;
      v = v > 0.0 ? v : 0.0;
      v = v > (double)var_floor ? v : (double)var_floor;
      means[(size_t)g * D + d] = (float)((double)means[(size_t)g * D + d] + m);
      dcovs[(size_t)g * D + d] = (float)v;
    } else {
      dcovs[(size_t)g * D + d] = 1.0f;
    }
  }
  if (threadIdx.x == 0) {
    counts[g] = (int64_t)Ltot;
    hefts[g] = (float)(Ltot / (double)N);
  }
  if (g == 0) {
    const double s = ordered_sum<256>(in_part, nb, S.lb);
    if (threadIdx.x == 0) {
      *inertia = s;
      if (!isfinite(s)) atomicOr(dev_status, GMM_DEV_NONFINITE);
    }
  }
}

__global__ void __launch_bounds__(256) k_km_fin_batched(const gmm_model_desc* models,
                                                        const int2* mitems, int D, int Gmax,
                                                        float var_floor,
                                                        const double* __restrict__ part,
                                                        const double* __restrict__ in_part) {
  __shared__ WelfordLds S;
  const int mi = blockIdx.y;
  const gmm_model_desc& m = models[mi];
  const int g = blockIdx.x;
  const int first = mitems[mi].x, cnt = mitems[mi].y;
  if (cnt == 0 || g >= m.G) return;
  const int P = 2 * D + 1;
  double mu, Q;
  const double Ltot = welford_combine<256, 8>(part + ((size_t)first * Gmax + g) * P,
                                           (size_t)Gmax * P, cnt, D, S, mu, Q);
  const int d = threadIdx.x;
  if (d < D) {
    if (Ltot > 0.0) {
      double v = Q / Ltot;
      v = v > 0.0 ? v : 0.0;
      v = v > (double)var_floor ? v : (double)var_floor;
      m.means[(size_t)g * D + d] = (float)((double)m.means[(size_t)g * D + d] + mu);
      m.covs[(size_t)g * D + d] = (float)v;
    } else {
      m.covs[(size_t)g * D + d] = 1.0f;
    }
  }
  if (threadIdx.x == 0) {
    m.counts[g] = (int64_t)Ltot;
    m.hefts[g] = (float)(Ltot / (double)m.N);
  }
  if (g == 0 && threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < cnt; ++k) s += in_part[first + k];
    if (m.inertia) *m.inertia = s;
    if (!isfinite(s)) atomicOr(m.dev_status, GMM_DEV_NONFINITE);
  }
}

// Dead-mean resurrection per model (one workgroup of 256 per model; same rule
// as the single-model kernel of gmm_kmeans.hip).
__global__ void __launch_bounds__(256) k_km_resurrect_batched(const gmm_model_desc* models,
                                                              int D, int Gmax,
                                                              int64_t* scratch) {
  constexpr int NT = 256;
  __shared__ int any_dead;
  __shared__ long long s_val[NT];
  __shared__ int s_idx[NT];
  __shared__ long long s_cnt[NT];
  __shared__ long long s_pick;
  const int mi = blockIdx.x;
  const gmm_model_desc& m = models[mi];
  if (!batch_desc_ok(m, Gmax)) return;
  const int G = m.G;
  const int64_t N = m.N;
  const int tid = threadIdx.x;
  if (tid == 0) any_dead = 0;
  __syncthreads();
  for (int g = tid; g < G; g += NT)
    if (m.counts[g] == 0) any_dead = 1;
  __syncthreads();
  if (!any_dead) return;
  int64_t* rem = scratch + (size_t)mi * 2 * Gmax;
  int64_t* taken = rem + Gmax;
  for (int g = tid; g < G; g += NT) {
    rem[g] = m.counts[g];
    taken[g] = 0;
  }
  __syncthreads();
  const int64_t slice = (N + NT - 1) / NT;
  for (int g = 0; g < G; ++g) {
    if (m.counts[g] != 0) continue;
    long long bv = -1;
    int bi = 0;
    for (int k = tid; k < G; k += NT)
      if ((long long)rem[k] > bv) {
        bv = rem[k];
        bi = k;
      }
    s_val[tid] = bv;
    s_idx[tid] = bi;
    __syncthreads();
    for (int sft = NT / 2; sft > 0; sft >>= 1) {
      if (tid < sft) {
        const long long ov = s_val[tid + sft];
        const int oi = s_idx[tid + sft];
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
    const int64_t a0 = (int64_t)tid * slice, a1 = min(N, a0 + slice);
    long long cnt = 0;
    for (int64_t i = a0; i < a1; ++i) cnt += (m.assign[i] == q);
    s_cnt[tid] = cnt;
    if (tid == 0) s_pick = -1;
    __syncthreads();
    if (tid == 0) {
      long long run = 0;
      for (int t = 0; t < NT; ++t) {
        if (want < run + s_cnt[t]) {
          s_cnt[0] = t;
          s_val[0] = want - run;
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
        if (m.assign[i] == q) {
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
      for (int d = tid; d < D; d += NT) m.means[(size_t)g * D + d] = m.X[pick * D + d];
      if (tid == 0) {
        taken[q] += 1;
        rem[q] -= 1;
      }
    }
    __syncthreads();
  }
}

// Per-model global mean / population variance, two FP64 passes, one
// workgroup per model.  Thread t < S*D (S = 256 / D sample stripes) sums
// dimension t % D over samples i = t / D + S k with four interleaved FP64
// accumulators; stripes are then combined in stripe order, so the result
// is the same on every run.
__global__ void __launch_bounds__(256) k_gstats_batched(const gmm_model_desc* models, int D,
                                                        double* mean_out, double* var_out) {
  __shared__ double sh[256];
  __shared__ double mean_s[256];
  const int mi = blockIdx.x;
  const gmm_model_desc& m = models[mi];
  if (m.N < 1 || m.X == nullptr) {
    if (threadIdx.x == 0 && m.dev_status) *m.dev_status = GMM_DEV_BADDESC;
    return;
  }
  const int t = threadIdx.x;
  const int S = 256 / D;
  const bool act = t < S * D;
  const int d = act ? t % D : 0, stripe = act ? t / D : 0;
  const int64_t N = m.N;
  const float* X = m.X;
  for (int pass = 0; pass < 2; ++pass) {
    const double mu = pass ? mean_s[d] : 0.0;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (act) {
      int64_t i = stripe;
      const int64_t step = S;
      for (; i + 3 * step < N; i += 4 * step) {
        const double x0 = (double)X[i * D + d] - mu;
        const double x1 = (double)X[(i + step) * D + d] - mu;
        const double x2 = (double)X[(i + 2 * step) * D + d] - mu;
        const double x3 = (double)X[(i + 3 * step) * D + d] - mu;
        a0 += pass ? x0 * x0 : x0;
        a1 += pass ? x1 * x1 : x1;
        a2 += pass ? x2 * x2 : x2;
        a3 += pass ? x3 * x3 : x3;
      }
      for (; i < N; i += step) {
        const double x0 = (double)X[i * D + d] - mu;
        a0 += pass ? x0 * x0 : x0;
      }
    }
    sh[t] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (t < D) {
      double tot = 0.0;
      for (int q = 0; q < S; ++q) tot += sh[q * D + t];
      if (pass == 0) {
        mean_s[t] = tot / (double)N;
      } else {
        mean_out[(size_t)mi * D + t] = mean_s[t];
        var_out[(size_t)mi * D + t] = tot / (double)N;
      }
    }
    __syncthreads();
  }
}

__global__ void k_zero_status_batched(const gmm_model_desc* models, int n_models) {
  for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < n_models; m += gridDim.x * blockDim.x)
    *models[m].dev_status = 0;
}

// ---- sample-major k-means kernel ---------------------------------------------
//
// With u = sqrt(lam) x and m_g = sqrt(lam) mu_g, the weighted distance is
// d_g = |u|^2 - s_g with s_g = 2 m_g.u - |m_g|^2, so the nearest mean
// maximises s_g.  The matrix cores compute m_g.u (u and m_g split into BF16
// hi + lo, three products, FP32 accumulation) for 16 samples x 16 means per
// tile, samples as the A operand, so a lane row holds 4 samples x 16 means.
// Every s_g carries a rigorous error bound e_g (representation of u and m_g,
// the split, the accumulation, the final rounding); the candidates of a
// sample are the means with s_g + e_g >= max_h (s_h - e_h), which always
// include the exact nearest one.  A sample with one candidate is decided;
// otherwise the candidates' distances are recomputed in FP64 and the first
// minimum wins.  The FP64 distance to the chosen mean (from the features still
// in registers and the means in LDS) gives the inertia.  The map step
// (counts, means, variances of the assigned samples) is the owner-wave
// Welford of the EM kernel with r = 1.

constexpr int kKGS = 16;              // samples per wave group
constexpr int kKRound = kNW * kKGS;   // samples per block round
constexpr int kKCapM = 16;            // pairs per (source, owner) list per pass (= kKGS: one pass)
constexpr int kCandMax = 8;           // candidate list per sample (more: all means)

struct Km2Args {
  const float* X;
  int64_t N;
  int64_t ldx;
  int64_t chunk;
  int D, G;
  const bf16x8* Whi;    // [RB][KSK][64] fragments of m_g (hi)
  const bf16x8* Wlo;
  const float* cq;      // [16 RB][4]: |m_g|^2 hi, lo, bound of |m_g|, 0
  const float* means;   // [G][D] current means
  const double* lam64;  // [D]
  const float* sd;      // [D] sqrt(lam) in FP32
  int32_t* assign;      // [N] or null
  double* part;         // [nb][G][2D+1]
  double* in_part;      // [nb]
  int64_t* n_rec;
  int32_t* dev_status;
};

struct KLds {
  bf16x8* wh;
  bf16x8* wl;
  float* cq;     // [16 RB][4]
  float* mu;     // [G][D]
  double* lam;   // [D]
  float* sd;     // [D]
  float* un;     // [NW][16] |u| of each sample (bound)
  int* cand;     // [NW][16][kCandMax]
  int* ccnt;     // [NW][16]
  int2* sub;     // [2][NW][NW][kKCapM], by round parity
  int* subn;     // [2][NW][NW]
  int* need;     // [2]
  int2* osort;   // [NW][64]
  double* inw;   // [NW]
};

template <typename F>
__host__ __device__ inline size_t km2_lds_walk(int D, int G, int KSK, F&& at) {
  size_t w = 0;
  auto put = [&](int which, size_t words, size_t align_words) {
    w = (w + align_words - 1) / align_words * align_words;
    at(which, w);
    w += words;
  };
  const size_t RB = ((size_t)G + 15) / 16;
  put(0, RB * KSK * 64 * 4, 4);
  put(1, RB * KSK * 64 * 4, 4);
  put(2, 16 * RB * 4, 4);
  put(3, (size_t)G * D, 1);
  put(4, 2 * (size_t)D, 2);
  put(5, D, 1);
  put(6, kNW * 16, 1);
  put(7, kNW * 16 * kCandMax, 1);
  put(8, kNW * 16, 1);
  put(9, 2 * (size_t)kNW * kNW * kKCapM * 2, 2);
  put(10, 2 * kNW * kNW, 1);
  put(11, 2, 1);
  put(12, kNW * 64 * 2, 2);
  put(13, 2 * kNW, 2);
  return w;
}

__host__ __device__ inline size_t km2_lds_bytes(int D, int G, int KSK) {
  return km2_lds_walk(D, G, KSK, [](int, size_t) {}) * 4 + 64;
}

// k-steps (32 dimensions each) of the k-means fragment layout
__host__ __device__ inline int km2_ks(int D) { return D <= 64 ? 2 : 4; }

// Staged form (D <= 64): after the layout above, each round's samples
// [2 by round parity][128][D] (floats), written from the registers that
// already hold them, so the map step reads LDS; with G <= 16 the same bytes
// later hold the 8 waves' map-step states [8][G][2D + 1] (floats).
__host__ __device__ inline size_t km2_stage_off(int D, int G) {
  return (km2_lds_bytes(D, G, 2) + 15) / 16 * 16;
}
__host__ __device__ inline size_t km2_stage_lds_bytes(int D, int G) {
  const size_t st = (size_t)4 * 2 * kKRound * D;
  const size_t mg = G <= 16 ? (size_t)4 * kNW * G * (2 * D + 1) : 0;
  return km2_stage_off(D, G) + (st > mg ? st : mg);
}
// for models of up to G means (a batch item with fewer uses its own layout)
inline size_t km2_stage_lds_max(int D, int G) {
  const size_t a = km2_stage_lds_bytes(D, G), b = km2_stage_lds_bytes(D, G < 16 ? G : 16);
  return a > b ? a : b;
}
inline bool km2_stage_fits(int D, int G) {
  return D <= 64 && km2_stage_lds_max(D, G) <= 160 * 1024;
}

__device__ inline KLds carve_klds(char* base, int D, int G, int KSK) {
  KLds L;
  float* f = (float*)base;
  km2_lds_walk(D, G, KSK, [&](int which, size_t off) {
    switch (which) {
      case 0: L.wh = (bf16x8*)(f + off); break;
      case 1: L.wl = (bf16x8*)(f + off); break;
      case 2: L.cq = f + off; break;
      case 3: L.mu = f + off; break;
      case 4: L.lam = (double*)(f + off); break;
      case 5: L.sd = f + off; break;
      case 6: L.un = f + off; break;
      case 7: L.cand = (int*)(f + off); break;
      case 8: L.ccnt = (int*)(f + off); break;
      case 9: L.sub = (int2*)(f + off); break;
      case 10: L.subn = (int*)(f + off); break;
      case 11: L.need = (int*)(f + off); break;
      case 12: L.osort = (int2*)(f + off); break;
      default: L.inw = (double*)(f + off); break;
    }
  });
  return L;
}

template <int CPW, int DPL, bool STG = false>
__device__ __forceinline__ void km2_range(const Km2Args& a, int64_t i0, int64_t i1, int b,
                                          char* lds_raw) {
  static_assert(!STG || DPL == 1, "staged form: D <= 64");
  constexpr int RBT = (CPW + 1) / 2;  // row blocks of 16 means
  constexpr int KSK = 2 * DPL;        // k-steps of 32 dimensions
  const int D = a.D, G = a.G;
  const int P = 2 * D + 1;
  const int RB = (G + 15) / 16;
  const KLds L = carve_klds(lds_raw, D, G, KSK);
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int w = tid / kWave;
  // bound of |s_g error| / (|m_g| |u|): representation of u and m (2 x 2
  // roundings each), the BF16 split (3 x 2^-16), FP32 accumulation of
  // 3 x 32 x KSK products, times 2 for s = 2 m.u, plus 5 % margin
  const float kcoef =
      1.05f * 2.0f * (3.0f * 0x1p-16f + 96.0f * (float)KSK * 0x1p-24f + 4.0f * 0x1p-24f);

  for (int p = tid; p < RB * KSK * 64; p += kThreads) {
    L.wh[p] = a.Whi[p];
    L.wl[p] = a.Wlo[p];
  }
  for (int p = tid; p < 16 * RB * 4; p += kThreads) L.cq[p] = a.cq[p];
  for (int p = tid; p < G * D; p += kThreads) L.mu[p] = a.means[p];
  for (int d = tid; d < D; d += kThreads) {
    L.lam[d] = a.lam64[d];
    L.sd[d] = a.sd[d];
  }

  float* const xs = STG ? (float*)(lds_raw + km2_stage_off(D, G)) : nullptr;
  // private map step (staged form, G <= 16): every wave keeps (count, m, Q)
  // of all G means for its own samples, so no list passes between waves and
  // a round takes no barrier; the 8 states are combined at the end of the
  // range.  Otherwise each mean has one owner wave.
  constexpr bool kPriv = STG && CPW <= 2;
  constexpr int kPG = kPriv ? 16 : 1;
  float Lp[kPG], P1[kPG], P2[kPG], mup[kPG];
#pragma unroll
  for (int g = 0; g < kPG; ++g) {
    Lp[g] = 0.0f;
    P1[g] = 0.0f;
    P2[g] = 0.0f;
    mup[g] = kPriv && g < G ? a.means[(size_t)g * D + min(lane, D - 1)] : 0.0f;
  }
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
  double inacc = 0.0;
  long long nrec = 0;
  __syncthreads();

  const int rowq = lane >> 4, colc = lane & 15;  // output layout
  const int kg = lane >> 4, na = lane & 15;      // A operand layout
  const unsigned long long lt = (1ull << lane) - 1ull;
  float* const un = L.un + w * 16;
  int* const cand = L.cand + w * 16 * kCandMax;
  int* const ccnt = L.ccnt + w * 16;
  const bf16x8* const whl = L.wh + lane;
  const bf16x8* const wll = L.wl + lane;
  const float* const cql = L.cq + 4 * colc;

  int round = 0;
  for (int64_t base = i0; base < i1; base += kKRound, ++round) {
    const int64_t s0 = base + (int64_t)kKGS * w;
    const int64_t ia = s0 + na;
    const bool va = ia < i1;

    // 1. features (kept for the FP64 distances) and the A fragments of u
    float xv[KSK][8];
    float acc[RBT][4];
    {
      const float* xr = a.X + (va ? ia : i0) * a.ldx + 8 * kg;
      int dl = D - 8 * kg;  // this lane's dimensions are 32 ks + i < dl
      asm volatile("" : "+v"(dl));
#pragma unroll
      for (int ks = 0; ks < KSK; ++ks)
#pragma unroll
        for (int i = 0; i < 8; ++i) xv[ks][i] = (va && 32 * ks + i < dl) ? xr[32 * ks + i] : 0.0f;
      if constexpr (STG) {
        // the round's rows to LDS (zero past i1).  Buffers alternate by round
        // parity: an owner reads them until its map step ends, before the next
        // round's barrier, and this wave refills a buffer two rounds later.
        float* const dst = xs + (size_t)(round & 1) * kKRound * D + (size_t)(kKGS * w + na) * D;
#pragma unroll
        for (int ks = 0; ks < KSK; ++ks)
#pragma unroll
          for (int i = 0; i < 8; ++i)
            if (32 * ks + 8 * kg + i < D) dst[32 * ks + 8 * kg + i] = xv[ks][i];
      }
      bf16x8 ah[KSK], al[KSK];
      float usq = 0.0f;
#pragma unroll
      for (int ks = 0; ks < KSK; ++ks)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int d = 32 * ks + 8 * kg + i;
          const float u = d < D ? xv[ks][i] * L.sd[min(d, D - 1)] : 0.0f;
          usq = fmaf(u, u, usq);
          const __bf16 h = (__bf16)u;
          ah[ks][i] = h;
          al[ks][i] = (__bf16)(u - (float)h);
        }
      usq += __shfl_xor(usq, 16, kWave);
      usq += __shfl_xor(usq, 32, kWave);
      if (kg == 0) un[na] = sqrtf(usq) * 1.0001f + 1e-30f;
#pragma unroll
      for (int cb = 0; cb < RBT; ++cb) {
        f32x4 c = {0.0f, 0.0f, 0.0f, 0.0f};
        if (cb < RB) {
#pragma unroll
          for (int ks = 0; ks < KSK; ++ks) {
            const bf16x8 bh = whl[(cb * KSK + ks) * 64];
            const bf16x8 bl = wll[(cb * KSK + ks) * 64];
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[ks], bh, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[ks], bl, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[ks], bh, c, 0, 0, 0);
          }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[cb][j] = c[j];
      }
    }
    wave_lds_sync();

    // 2. s_g, bounds, candidates (per sample, in increasing mean index)
    bool vj[4];
    float unj[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      vj[j] = s0 + 4 * rowq + j < i1;
      unj[j] = un[4 * rowq + j];
    }
    float M[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
#pragma unroll
    for (int cb = 0; cb < RBT; ++cb) {
      const float* q = cql + 4 * 16 * cb;
      const bool vg = cb < RB;
      const float mh = vg ? q[0] : INFINITY, ml = vg ? q[1] : 0.0f, mn = vg ? q[2] : 0.0f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float sv = vj[j] ? (2.0f * acc[cb][j] - mh) - ml : -INFINITY;
        acc[cb][j] = sv;
        const float e = kcoef * mn * unj[j] + 0x1p-22f * (2.0f * mn * unj[j] + fabsf(mh));
        M[j] = fmaxf(M[j], sv - e);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) M[j] = row16_max(M[j]);
    uint32_t candb = 0;
#pragma unroll
    for (int cb = 0; cb < RBT; ++cb) {
      const float* q = cql + 4 * 16 * cb;
      const bool vg = cb < RB;
      const float mh = vg ? q[0] : INFINITY, mn = vg ? q[2] : 0.0f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float sv = acc[cb][j];
        const float e = kcoef * mn * unj[j] + 0x1p-22f * (2.0f * mn * unj[j] + fabsf(mh));
        if (sv > -INFINITY && sv + e >= M[j]) candb |= 1u << (4 * cb + j);
      }
    }
    {
      int cntj[4] = {0, 0, 0, 0};
      const unsigned int below = (1u << colc) - 1u;
#pragma unroll
      for (int cb = 0; cb < RBT; ++cb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bool cd = (candb >> (4 * cb + j)) & 1u;
          const unsigned int seg =
              (unsigned int)((__ballot(cd) >> (16 * rowq)) & 0xFFFFull);
          if (cd) {
            const int pos = cntj[j] + __popc(seg & below);
            if (pos < kCandMax) cand[(4 * rowq + j) * kCandMax + pos] = 16 * cb + colc;
          }
          cntj[j] += __popc(seg);
        }
      if (colc == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) ccnt[4 * rowq + j] = cntj[j];
      }
    }
    wave_lds_sync();

    // 3. decision and FP64 distance of the chosen mean (A layout: the 4 lanes
    // of sample na hold all its dimensions)
    int best = -1;
    double bestd = INFINITY;
    {
      const int cn = va ? ccnt[na] : 0;
      const int ncand = cn > kCandMax ? G : cn;
      int kmax = ncand;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) kmax = max(kmax, __shfl_xor(kmax, o, kWave));
      for (int k = 0; k < kmax; ++k) {
        if (k < ncand) {
          const int g = cn > kCandMax ? k : cand[na * kCandMax + k];
          const float* mug = L.mu + g * D;
          double d64 = 0.0;
#pragma unroll
          for (int ks = 0; ks < KSK; ++ks)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              const int d = 32 * ks + 8 * kg + i;
              const int dc = min(d, D - 1);
              const double t = (double)xv[ks][i] - (double)mug[dc];
              d64 = d < D ? fma(t * t, L.lam[dc], d64) : d64;
            }
          d64 += __shfl_xor(d64, 16, kWave);
          d64 += __shfl_xor(d64, 32, kWave);
          if (d64 < bestd) {
            bestd = d64;
            best = g;
          }
        }
      }
      if (kg == 0 && cn > 1) ++nrec;
      if (va && kg == 0) {
        if (a.assign) a.assign[ia] = best;
        inacc += bestd;
      }
    }

    const bool has = va && kg == 0 && best >= 0;
    if constexpr (kPriv) {
      // 4'. the wave's samples in order; sample n's chosen mean is in lane n
      const float* const xsr = xs + (size_t)(round & 1) * kKRound * D;
      for (int q = 0; q < 4; ++q) {
        float xq[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) xq[j] = xsr[(kKGS * w + 4 * q + j) * D + min(lane, D - 1)];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int g = __builtin_amdgcn_readlane(has ? best : -1, 4 * q + j);
          if (g < 0) continue;
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            if (g == k) {
              const float y = xq[j] - mup[k];
              const float Lo = Lp[k];
              const float Ln = Lo + 1.0f;
              const float inv = __builtin_amdgcn_rcpf(Ln);
              const float w2 = inv * Lo;
              Lp[k] = Ln;
              const float dlt = y - P1[k];
              P1[k] = Lo == 0.0f ? y : fmaf(inv, dlt, P1[k]);
              P2[k] = fmaf(w2 * dlt, dlt, P2[k]);
            }
          }
        }
      }
      continue;
    }
    // 4. hand (sample, chosen mean) to the mean's owner wave best % 8
    const int own = has ? (best & 7) : 0;
    int mypos = 0, mine = 0;
#pragma unroll
    for (int o = 0; o < kNW; ++o) {
      const unsigned long long m = __ballot(has && own == o);
      if (own == o) mypos = __popcll(m & lt);
      // every lane of class o (lane % 8 == o) holds owner o's count: the
      // row-rotation maximum below reads lanes 0-15
      if ((lane & 7) == o) mine = __popcll(m);
    }
    // lists and counts alternate between two buffers by round parity (a wave
    // writes round r + 2's lists only after the barrier of round r + 1, which
    // every owner reaches after its map step of round r): one barrier a round
    int2* const subb = L.sub + (size_t)(round & 1) * kNW * kNW * kKCapM;
    int* const subnb = L.subn + (round & 1) * kNW * kNW;
    if (lane < kNW) subnb[w * kNW + lane] = mine;
    int need = 0;  // longest list of the round (at most kKGS = kKCapM)
    for (int pass = 0;; ++pass) {
      const int k = mypos - pass * kKCapM;
      if (has && k >= 0 && k < kKCapM)
        subb[(size_t)(w * kNW + own) * kKCapM + k] = make_int2(na | (best << 8), 0);
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
      int pre[kNW + 1];
      pre[0] = 0;
#pragma unroll
      for (int src = 0; src < kNW; ++src)
        pre[src + 1] = pre[src] + max(0, min(kKCapM, subnb[src * kNW + w] - pass * kKCapM));
      const int tot = pre[kNW];
      int2* const os = L.osort + w * 64;
      for (int k0 = 0; k0 < tot; k0 += 64) {
        const int kk = k0 + lane;
        const bool ok = kk < tot;
        int src = 0;
#pragma unroll
        for (int t = 1; t < kNW; ++t) src = kk >= pre[t] ? t : src;
        const int2 e = ok ? subb[(size_t)(src * kNW + w) * kKCapM + (kk - pre[src])]
                          : make_int2(0, 0);
        const int cs = ok ? (e.x >> 11) : -1;
        int cnt[CPW];
        int off = 0, pos = 0;
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
          const unsigned long long m = __ballot(cs == c);
          if (cs == c) pos = off + __popcll(m & lt);
          cnt[c] = __popcll(m);
          off += cnt[c];
        }
        if (ok) os[pos] = make_int2((kKGS * src + (e.x & 15)) | (e.x & ~0xFF), 0);
        wave_lds_sync();
        // the map step with l in {0, 1}: West's Welford on y = x - mu_old,
        // slot by slot, samples in the order above
        int o = 0;
        int wo = w;
        asm volatile("" : "+v"(wo));
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
          const int cc = cnt[c];
          if (cc > 0) {
            const int g = wo + kNW * c;
            float mu[DPL];
#pragma unroll
            for (int jd = 0; jd < DPL; ++jd) mu[jd] = L.mu[g * D + min(lane + kWave * jd, D - 1)];
            for (int q0 = 0; q0 < cc; q0 += 4) {
              bool okq[4];
              float y[4][DPL];
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const int2 e2 = os[o + min(q0 + i, cc - 1)];
                okq[i] = q0 + i < cc;
                const float* xr = STG ? xs + (size_t)(round & 1) * kKRound * D + (e2.x & 0xFF) * D
                                      : a.X + (base + (e2.x & 0xFF)) * a.ldx;
#pragma unroll
                for (int jd = 0; jd < DPL; ++jd)
                  y[i][jd] = xr[min(lane + kWave * jd, D - 1)] - mu[jd];
              }
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                if (okq[i]) {
                  const float Lo = Lc[c];
                  const float Ln = Lo + 1.0f;
                  const float inv = __builtin_amdgcn_rcpf(Ln);
                  const float w2 = inv * Lo;
                  Lc[c] = Ln;
#pragma unroll
                  for (int jd = 0; jd < DPL; ++jd) {
                    const float dlt = y[i][jd] - S1[c][jd];
                    S1[c][jd] = Lo == 0.0f ? y[i][jd] : fmaf(inv, dlt, S1[c][jd]);
                    S2[c][jd] = fmaf(w2 * dlt, dlt, S2[c][jd]);
                  }
                }
              }
            }
            o += cc;
          }
        }
        wave_lds_sync();
      }
      if ((pass + 1) * kKCapM >= need) break;
      __syncthreads();  // this buffer is refilled by the next pass
    }
  }

  double* pb = a.part + (size_t)b * G * P;
  if constexpr (kPriv) {
    // the 8 waves' states of each mean, combined in wave order by the
    // pairwise update of (count, m, Q) in FP64 (as across work ranges)
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
  }
#pragma unroll
  for (int c = 0; c < (kPriv ? 0 : CPW); ++c) {
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
  {
    const double v = wave_sum_d(inacc);
    if (lane == 0) L.inw[w] = v;
  }
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kNW; ++q) s += L.inw[q];
    a.in_part[b] = s;
  }
  if (a.n_rec) {
    long long v = nrec;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    if (lane == 0 && v) atomicAdd((unsigned long long*)a.n_rec, (unsigned long long)v);
  }
}

template <int CPW, int DPL, bool STG>
__global__ void __launch_bounds__(kThreads) k_km2(Km2Args a) {
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  const int b = blockIdx.x;
  const int64_t i0 = (int64_t)b * a.chunk;
  const int64_t i1 = min(a.N, i0 + a.chunk);
  km2_range<CPW, DPL, STG>(a, i0, i1, b, lds_raw);
}

// Per-mean constants: block g < 16 RB.  lam and s = sqrt(lam) per dimension
// (block 0 stores them), m_g = mu_g s in FP32, its MFMA fragments (hi/lo;
// zero for padding means), |m_g|^2 in FP64 split hi/lo, and a bound of |m_g|.
__device__ void km2_pre_mean(const double* __restrict__ gvar, int D, int G, float var_floor,
                             int dist, const float* __restrict__ means, int KSK, int g,
                             double* __restrict__ lam64, float* __restrict__ sd,
                             bf16x8* __restrict__ Whi, bf16x8* __restrict__ Wlo,
                             float* __restrict__ cq) {
  __shared__ float sdl[128];
  __shared__ double sh[256];
  for (int d = threadIdx.x; d < D; d += 256) {
    double l = 1.0;
    if (dist == GMM_DIST_MAHA) {
      double v = gvar[d];
      v = v > (double)var_floor ? v : (double)var_floor;
      l = 1.0 / v;
    }
    const float s = (float)sqrt(l);
    sdl[d] = s;
    if (g == 0) {
      lam64[d] = l;
      sd[d] = s;
    }
  }
  __syncthreads();
  const int rb = g >> 4, row = g & 15;
  double q = 0.0;
  for (int e = threadIdx.x; e < KSK * 4 * 8; e += 256) {
    const int ks = e / 32, r = e - ks * 32, lq = r >> 3, i = r & 7;
    const int d = 32 * ks + 8 * lq + i;
    float v = 0.0f;
    if (g < G && d < D) v = (float)((double)means[(size_t)g * D + d] * (double)sdl[d]);
    q += (double)v * (double)v;
    const __bf16 h = (__bf16)v;
    const size_t idx = ((size_t)rb * KSK + ks) * 64 + 16 * lq + row;
    ((__bf16*)(Whi + idx))[i] = h;
    ((__bf16*)(Wlo + idx))[i] = (__bf16)(v - (float)h);
  }
  const double mm = block_sum_d<256>(q, sh);
  if (threadIdx.x == 0) {
    float* c = cq + 4 * g;
    if (g < G) {
      const float hi = (float)mm;
      c[0] = hi;
      c[1] = (float)(mm - (double)hi);
      c[2] = (float)sqrt(mm) * 1.0001f;
    } else {
      c[0] = INFINITY;  // padding mean: s = -inf
      c[1] = 0.0f;
      c[2] = 0.0f;
    }
    c[3] = 0.0f;
  }
}

__global__ void __launch_bounds__(256) k_km2_pre(const double* __restrict__ gvar, int D, int G,
                                                 float var_floor, int dist,
                                                 const float* __restrict__ means, int KSK,
                                                 double* __restrict__ lam64,
                                                 float* __restrict__ sd, bf16x8* __restrict__ Whi,
                                                 bf16x8* __restrict__ Wlo,
                                                 float* __restrict__ cq) {
  km2_pre_mean(gvar, D, G, var_floor, dist, means, KSK, blockIdx.x, lam64, sd, Whi, Wlo, cq);
}

// Per-model constants of the batched form: per-model strides of the fragment
// (RBmax * KSl * 64), table (kps), lam and s (D) regions.
struct Km2Batch {
  bf16x8* Whi;
  bf16x8* Wlo;
  float* cq;
  double* lam64;
  float* sd;
  int RBmax, KSl, Gmax;
  size_t kps;
};

// grid (16 RBmax, n_models)
__global__ void __launch_bounds__(256) k_km2_pre_batched(const gmm_model_desc* models, int D,
                                                         float var_floor, int dist, int KSK,
                                                         Km2Batch kb) {
  const int mi = blockIdx.y;
  const gmm_model_desc& m = models[mi];
  if (!batch_desc_ok(m, kb.Gmax)) return;
  if ((int)blockIdx.x >= 16 * ((m.G + 15) / 16)) return;
  const size_t fo = (size_t)mi * kb.RBmax * kb.KSl * 64;
  km2_pre_mean(m.gvar, D, m.G, var_floor, dist, m.means, KSK, blockIdx.x,
               kb.lam64 + (size_t)mi * D, kb.sd + (size_t)mi * D, kb.Whi + fo, kb.Wlo + fo,
               kb.cq + (size_t)mi * kb.kps);
}

template <int CPW, int DPL, bool STG>
__global__ void __launch_bounds__(kThreads) k_km2_batched(Km2Args base,
                                                          const gmm_model_desc* models,
                                                          const BatchItemDev* items,
                                                          const int* n_items, Km2Batch kb) {
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  const int ni = *n_items;
  const int D = base.D;
  const int P = 2 * D + 1;
  for (int it = blockIdx.x; it < ni; it += gridDim.x) {
    const BatchItemDev item = items[it];
    const gmm_model_desc& m = models[item.model];
    const size_t mi = (size_t)item.model;
    Km2Args a = base;
    a.X = m.X;
    a.N = m.N;
    a.ldx = D;
    a.G = m.G;
    const size_t fo = mi * kb.RBmax * kb.KSl * 64;
    a.Whi = kb.Whi + fo;
    a.Wlo = kb.Wlo + fo;
    a.cq = kb.cq + mi * kb.kps;
    a.means = m.means;
    a.lam64 = kb.lam64 + mi * D;
    a.sd = kb.sd + mi * D;
    a.assign = m.assign;
    a.part = base.part + (size_t)it * kb.Gmax * P;
    a.in_part = base.in_part + it;
    a.n_rec = nullptr;
    a.dev_status = m.dev_status;
    // the smallest component-block template that holds the model's G
    if (CPW > 2 && a.G <= 16)
      km2_range<(CPW > 2 ? 2 : CPW), DPL, STG>(a, item.i0, item.i1, 0, lds_raw);
    else if (CPW > 4 && a.G <= 32)
      km2_range<(CPW > 4 ? 4 : CPW), DPL, STG>(a, item.i0, item.i1, 0, lds_raw);
    else if (CPW > 8 && a.G <= 64)
      km2_range<(CPW > 8 ? 8 : CPW), DPL, STG>(a, item.i0, item.i1, 0, lds_raw);
    else km2_range<CPW, DPL, STG>(a, item.i0, item.i1, 0, lds_raw);
    __syncthreads();
  }
}

template <int CPW, int DPL>
void km_launch_one(const KmArgs& a, int nb, size_t lds, hipStream_t st) {
  auto kern = k_km_fast<CPW, DPL>;
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    attr_set = true;
  }
  hipLaunchKernelGGL(kern, dim3(nb), dim3(kThreads), lds, st, a);
}

template <int CPW, int DPL, bool STG = false>
void km2_launch_one(const Km2Args& a, int nb, size_t lds, hipStream_t st) {
  auto kern = k_km2<CPW, DPL, STG>;
  static bool attr_set = false;  // benign race: setting the attribute twice is harmless
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    attr_set = true;
  }
  hipLaunchKernelGGL(kern, dim3(nb), dim3(kThreads), lds, st, a);
}

void km2_dispatch(const Km2Args& a, int nb, size_t lds, hipStream_t st, bool stg) {
  const int cpw = (a.G + kNW - 1) / kNW;
  if (stg) {
    if (cpw <= 2) km2_launch_one<2, 1, true>(a, nb, lds, st);
    else if (cpw <= 4) km2_launch_one<4, 1, true>(a, nb, lds, st);
    else if (cpw <= 8) km2_launch_one<8, 1, true>(a, nb, lds, st);
    else if (cpw <= 13) km2_launch_one<13, 1, true>(a, nb, lds, st);
    else km2_launch_one<16, 1, true>(a, nb, lds, st);
  } else if (a.D <= 64) {
    if (cpw <= 2) km2_launch_one<2, 1>(a, nb, lds, st);
    else if (cpw <= 4) km2_launch_one<4, 1>(a, nb, lds, st);
    else if (cpw <= 8) km2_launch_one<8, 1>(a, nb, lds, st);
    else if (cpw <= 13) km2_launch_one<13, 1>(a, nb, lds, st);
    else km2_launch_one<16, 1>(a, nb, lds, st);
  } else {
    if (cpw <= 2) km2_launch_one<2, 2>(a, nb, lds, st);
    else if (cpw <= 4) km2_launch_one<4, 2>(a, nb, lds, st);
    else if (cpw <= 8) km2_launch_one<8, 2>(a, nb, lds, st);
    else if (cpw <= 13) km2_launch_one<13, 2>(a, nb, lds, st);
    else km2_launch_one<16, 2>(a, nb, lds, st);
  }
}

template <int CPW, int DPL, bool STG = false>
void km2_launch_batched_one(const Km2Args& base, const gmm_model_desc* models,
                            const BatchWorkspace& bw, const Km2Batch& kb, int grid, size_t lds,
                            hipStream_t st) {
  auto kern = k_km2_batched<CPW, DPL, STG>;
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    attr_set = true;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, st, base, models, bw.items,
                     bw.n_items, kb);
}

}  // namespace

bool km2_supported(int D, int G) {
  if (D < 1 || D > 128 || G < 1 || G > 128) return false;
  return km2_lds_bytes(D, G, km2_ks(D)) <= 160 * 1024;
}

bool km_fast_supported(int D, int G) {
  if (D < 1 || D > 128 || G < 1 || G > 128) return false;
  return km_lds_bytes(D, G) <= 160 * 1024;
}

// The k-means reduce; more than 64 blocks: segments of 32 first, so that the
// G final chains are short.
static void launch_km_fin(int nb, int64_t N, int D, int G, float var_floor, float* means,
                          float* dcovs, float* hefts, int64_t* counts, double* inertia,
                          int32_t* dev_status, const Workspace& w, hipStream_t st) {
  const int seg = nb > 64 ? 32 : 1;
  if (seg > 1)
    hipLaunchKernelGGL(k_welford_seg, dim3(G, (nb + seg - 1) / seg), dim3(256), 0, st, w.partials,
                       nb, seg, D, G);
  hipLaunchKernelGGL(k_km_fin_fast, dim3(G), dim3(256), 0, st, w.partials, nb, seg, N, D, G,
                     var_floor, means, dcovs, hefts, counts, w.scalars, inertia, dev_status);
}

hipError_t launch_kmeans_fast(const float* X, int64_t N, int D, int64_t ldx, int G, int dist,
                              const double* gvar, float var_floor, float* means, float* dcovs,
                              float* hefts, int64_t* counts, int32_t* assign, double* inertia,
                              int64_t* n_recomputed, int32_t* dev_status, const Workspace& w,
                              hipStream_t st, int prec) {
  if (prec == GMM_PREC_BF16X3 && km2_supported(D, G)) {
    const int KSK = km2_ks(D);
    const int RB = (G + 15) / 16;
    hipLaunchKernelGGL(k_km2_pre, dim3(16 * RB), dim3(256), 0, st, gvar, D, G, var_floor, dist,
                       means, KSK, w.lam64, w.lam32, (bf16x8*)w.Bhi, (bf16x8*)w.Blo, w.prm);
    int64_t nb64 = (N + kKRound - 1) / kKRound;
    if (nb64 < 1) nb64 = 1;
    if (nb64 > 256) nb64 = 256;
    const int64_t ch = ((N + nb64 - 1) / nb64 + kKRound - 1) / kKRound * kKRound;
    const int nb = (int)((N + ch - 1) / ch);
    Km2Args a;
    a.X = X;
    a.N = N;
    a.ldx = ldx;
    a.chunk = ch;
    a.D = D;
    a.G = G;
    a.Whi = (const bf16x8*)w.Bhi;
    a.Wlo = (const bf16x8*)w.Blo;
    a.cq = w.prm;
    a.means = means;
    a.lam64 = w.lam64;
    a.sd = w.lam32;
    a.assign = assign;
    a.part = w.partials;
    a.in_part = w.scalars;
    a.n_rec = n_recomputed;
    a.dev_status = dev_status;
    {
      ProfScope ps(kProfKmAssign, st);
      const bool stg = km2_stage_fits(D, G);
      km2_dispatch(a, nb, stg ? km2_stage_lds_max(D, G) : km2_lds_bytes(D, G, KSK), st, stg);
    }
    launch_km_fin(nb, N, D, G, var_floor, means, dcovs, hefts, counts, inertia, dev_status, w, st);
    return hipGetLastError();
  }
  int64_t nb64 = (N + 2 * kT - 1) / (2 * kT);
  if (nb64 < 1) nb64 = 1;
  if (nb64 > 256) nb64 = 256;
  const int nb = (int)nb64;
  KmArgs a;
  a.X = X;
  a.N = N;
  a.ldx = ldx;
  a.chunk = ((N + nb - 1) / nb + kT - 1) / kT * kT;
  a.D = D;
  a.G = G;
  a.means = means;
  a.mprm = w.prm;
  a.sd = w.lam32;
  a.lam64 = w.lam64;
  a.mnorm = w.c;
  a.assign = assign;
  a.part = w.partials;
  a.in_part = w.scalars;
  a.n_rec = n_recomputed;
  a.dev_status = dev_status;
  hipLaunchKernelGGL(k_km_pre_fast, dim3(1), dim3(256), 0, st, gvar, D, G, var_floor, dist, means,
                     w.lam64, w.lam32, w.prm, w.c);
  const size_t lds = km_lds_bytes(D, G);
  {
    ProfScope ps(kProfKmAssign, st);
    const int cpw = (G + kNW - 1) / kNW;
    if (D <= 64) {
      if (cpw <= 2) km_launch_one<2, 1>(a, nb, lds, st);
      else if (cpw <= 4) km_launch_one<4, 1>(a, nb, lds, st);
      else if (cpw <= 8) km_launch_one<8, 1>(a, nb, lds, st);
      else if (cpw <= 13) km_launch_one<13, 1>(a, nb, lds, st);
      else km_launch_one<16, 1>(a, nb, lds, st);
    } else {
      if (cpw <= 2) km_launch_one<2, 2>(a, nb, lds, st);
      else if (cpw <= 4) km_launch_one<4, 2>(a, nb, lds, st);
      else if (cpw <= 8) km_launch_one<8, 2>(a, nb, lds, st);
      else if (cpw <= 13) km_launch_one<13, 2>(a, nb, lds, st);
      else km_launch_one<16, 2>(a, nb, lds, st);
    }
  }
  launch_km_fin(nb, N, D, G, var_floor, means, dcovs, hefts, counts, inertia, dev_status, w, st);
  return hipGetLastError();
}

hipError_t launch_kmeans_batched(const gmm_model_desc* models, int n_models, int n_items_host,
                                 int D, int dist, float var_floor, const BatchWorkspace& bw,
                                 hipStream_t st) {
  // every model through the matrix-core screening kernel (decisions exact)
  const int KSK = km2_ks(D);
  Km2Batch kb;
  kb.Whi = (bf16x8*)bw.Whi;
  kb.Wlo = (bf16x8*)bw.Wlo;
  kb.cq = bw.kmprm;
  kb.lam64 = bw.klam64;
  kb.sd = bw.ksd;
  kb.RBmax = bw.RBmax;
  kb.KSl = bw.KS;
  kb.Gmax = bw.Gmax;
  kb.kps = bw.kpstride;
  hipLaunchKernelGGL(k_km2_pre_batched, dim3(16 * bw.RBmax, n_models), dim3(256), 0, st, models,
                     D, var_floor, dist, KSK, kb);
  Km2Args base{};
  base.D = D;
  base.part = bw.partials;
  base.in_part = bw.sparts;
  const bool stg = km2_stage_fits(D, bw.Gmax);
  const size_t lds = stg ? km2_stage_lds_max(D, bw.Gmax) : km2_lds_bytes(D, bw.Gmax, KSK);
  const int grid = n_items_host < 256 ? (n_items_host < 1 ? 1 : n_items_host) : 256;
  {
    ProfScope ps(kProfBatched, st);
    const int cpw = (bw.Gmax + kNW - 1) / kNW;
    if (stg) {
      if (cpw <= 2) km2_launch_batched_one<2, 1, true>(base, models, bw, kb, grid, lds, st);
      else if (cpw <= 4) km2_launch_batched_one<4, 1, true>(base, models, bw, kb, grid, lds, st);
      else if (cpw <= 8) km2_launch_batched_one<8, 1, true>(base, models, bw, kb, grid, lds, st);
      else km2_launch_batched_one<16, 1, true>(base, models, bw, kb, grid, lds, st);
    } else if (D <= 64) {
      if (cpw <= 2) km2_launch_batched_one<2, 1>(base, models, bw, kb, grid, lds, st);
      else if (cpw <= 4) km2_launch_batched_one<4, 1>(base, models, bw, kb, grid, lds, st);
      else if (cpw <= 8) km2_launch_batched_one<8, 1>(base, models, bw, kb, grid, lds, st);
      else km2_launch_batched_one<16, 1>(base, models, bw, kb, grid, lds, st);
    } else {
      if (cpw <= 2) km2_launch_batched_one<2, 2>(base, models, bw, kb, grid, lds, st);
      else if (cpw <= 4) km2_launch_batched_one<4, 2>(base, models, bw, kb, grid, lds, st);
      else if (cpw <= 8) km2_launch_batched_one<8, 2>(base, models, bw, kb, grid, lds, st);
      else km2_launch_batched_one<16, 2>(base, models, bw, kb, grid, lds, st);
    }
  }
  hipLaunchKernelGGL(k_km_fin_batched, dim3(bw.Gmax, n_models), dim3(256), 0, st, models,
                     bw.mitems, D, bw.Gmax, var_floor, bw.partials, bw.sparts);
  hipLaunchKernelGGL(k_km_resurrect_batched, dim3(n_models), dim3(256), 0, st, models, D, bw.Gmax,
                     bw.kscratch);
  return hipGetLastError();
}

hipError_t launch_global_stats_batched(const gmm_model_desc* models, int n_models, int D,
                                       double* mean_out, double* var_out, hipStream_t st) {
  hipLaunchKernelGGL(k_gstats_batched, dim3(n_models), dim3(256), 0, st, models, D, mean_out,
                     var_out);
  return hipGetLastError();
}

}  // namespace gmm
