// gmm_full.hip -- EM iteration and log-likelihood for full covariances
// (Eq. 2 with a general Sigma; Eq. 7 / Eq. 8 for the update).
//
//   k_pre_full     one workgroup per component: Cholesky Sigma_g = L L^T in
//                  FP64, log|Sigma_g| = 2 sum_d log L_dd, the inverse factor
//                  W_g = L^-1 by forward substitution in FP64 (also rounded to
//                  FP32), c_g = log w_g - 1/2 (D log 2pi + log|Sigma_g|) (FP64
//                  and hi/lo FP32) and, for D <= 64, W_g in the FP64 MFMA
//                  operand layout with b_g = W_g mu_g.  A non-positive pivot
//                  sets GMM_DEV_NOTPD.
//   k_estep_full   a_gi = c_g - 1/2 ||W_g (x_i - mu_g)||^2 (D <= 64: exact FP64
//                  on the matrix cores; larger D: FP32 screening with an FP64
//                  recompute of the 30-nat window), log-sum-exp,
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
                                                  const float* __restrict__ covs,
                                                  const float* __restrict__ means, int D, int G,
                                                  double* __restrict__ scratch,
                                                  float* __restrict__ W_out,
                                                  double* __restrict__ W64_out,
                                                  double* __restrict__ Wf64,
                                                  double* __restrict__ b64,
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
  if (D <= 64) {
    // B-operand fragments of W_g^T for v_mfma_f64_16x16x4f64: fragment (row
    // block cb, k-step ks, lane l) is W_g[16 cb + l%16][4 ks + l/16] (zero past
    // D); and b_g = W_g mu_g in FP64, zero-padded to whole row blocks.
    const int RBr = (D + 15) / 16, KQ = D <= 32 ? 8 : 16;
    double* f = Wf64 + (size_t)g * RBr * KQ * 64;
    for (int e = tid; e < RBr * KQ * 64; e += kNT) {
      const int l = e & 63, rest = e >> 6;
      const int ks = rest % KQ, cb = rest / KQ;
      const int r = 16 * cb + (l & 15), k = 4 * ks + (l >> 4);
      f[e] = (r < D && k < D) ? Wi[(size_t)r * D + k] : 0.0;
    }
    for (int r = tid; r < 16 * RBr; r += kNT) {
      double t = 0.0;
      if (r < D)
        for (int c = 0; c <= r; ++c) t += Wi[(size_t)r * D + c] * (double)means[(size_t)g * D + c];
      b64[(size_t)g * 16 * RBr + r] = t;
    }
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

// LDS of the near-set recompute: per wave, up to kWB FP64 entries of W_g's
// packed rows and up to kWR row offsets b_r = (W_g mu_g)_r.
constexpr int kWB = 1024;
constexpr int kWR = 64;

// Exact log-densities of a tile on the matrix cores (D <= 4 KQ): Z = X W_g^T -
// 1 b_g^T in FP64 (v_mfma_f64_16x16x4f64; the samples are the A operand, 16 per
// row block, W_g^T the B operand), then a_g = c_g - 1/2 sum_r Z_r^2 in FP64.
// Wave per component; output lane l, register j is (sample 4 j + l/16 of the row
// block, row 16 cb + l%16 of W_g), so the sum over rows is a 16-lane butterfly.
template <int KQ>
__device__ void logdens_full_f64(const float* __restrict__ xs, int DS, int nt, int D, int G,
                                 const double* __restrict__ Wf64,
                                 const double* __restrict__ b64,
                                 const double* __restrict__ c64, double* __restrict__ as64,
                                 int wid, int nw, int lane) {
  constexpr int RBM = KQ / 2;  // most row blocks of W_g (D <= 4 KQ)
  const int RBr = (D + 15) / 16;
  const int NRB = (nt + 15) / 16;  // row blocks of samples (nt <= 64)
  const int m = lane & 15, kb = lane >> 4;
  double xa[4][KQ];  // A operands: sample 16 rb + m, dimension 4 ks + kb
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const int t = min(16 * rb + m, nt - 1);  // rows past nt: a valid row, output dropped
#pragma unroll
    for (int ks = 0; ks < KQ; ++ks) {
      const int k = 4 * ks + kb;
      xa[rb][ks] = k < D ? (double)xs[(size_t)t * DS + k] : 0.0;
    }
  }
  const size_t fstride = (size_t)RBr * KQ * 64;
  for (int g = __builtin_amdgcn_readfirstlane(wid); g < G; g += nw) {
    double qp[4][4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int j = 0; j < 4; ++j) qp[rb][j] = 0.0;
#pragma unroll
    for (int cb = 0; cb < RBM; ++cb) {
      if (cb >= RBr) break;
      double wb[KQ];
#pragma unroll
      for (int ks = 0; ks < KQ; ++ks)
        wb[ks] = Wf64[(size_t)g * fstride + ((size_t)cb * KQ + ks) * 64 + lane];
      const double bv = b64[(size_t)g * 16 * RBr + 16 * cb + m];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        if (rb >= NRB) break;
        f64x4 c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < KQ; ++ks) {
          if (4 * ks >= D) break;
          c = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[rb][ks], wb[ks], c, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double z = c[j] - bv;  // rows past D: 0 - 0
          qp[rb][j] = fma(z, z, qp[rb][j]);
        }
      }
    }
    const double cg = c64[g];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      if (rb >= NRB) break;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double q = row16_sum(qp[rb][j]);
        const int t = 16 * rb + 4 * j + kb;
        if (m == 0 && t < nt) as64[(size_t)t * G + g] = cg - 0.5 * q;
      }
    }
  }
}

// Map step of one component over one tile on the matrix cores (FP64): with
// y' = [x - mu_g, 1] (D + 1 entries), C = sum_t r_t y'_t y'_t^T is the rank
// update v_mfma_f64_16x16x4f64 builds from A = (r y')^T and B = y' (4 samples
// per k-step); its lower triangle holds sum r y_d y_e, its last row sum r y_e
// and its corner sum r.  Lane l, register j of block (rb, cb) is entry
// (16 rb + 4 j + l/16, 16 cb + l%16).  The tile's sums are added to the
// component's FP64 partials q (count, first moments, packed lower triangle).
template <int RBYM, int KC>
__device__ void map_full_f64(const float* __restrict__ xs, int DS, int nm,
                             const int* __restrict__ mlist, int D, int G,
                             const float* __restrict__ as, const float* __restrict__ mu_g,
                             double* __restrict__ q, int g, int lane, double* __restrict__ stg) {
  constexpr int NB = RBYM * (RBYM + 1) / 2;  // lower-triangle blocks
  const int RBY = (D + 16) / 16;             // row blocks of y'
  const int m = lane & 15, kb = lane >> 4;
  float mue[RBYM];
#pragma unroll
  for (int cb = 0; cb < RBYM; ++cb) {
    const int e = 16 * cb + m;
    mue[cb] = e < D ? mu_g[e] : 0.0f;  // column D of the tile holds 1
  }
  f64x4 c[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) c[i] = f64x4{0.0, 0.0, 0.0, 0.0};
  // only the tile's samples with a non-zero responsibility (mlist[0..nm), in
  // increasing order) take part: 4 per k-step
  const int nks = (nm + 3) / 4;
  // k-steps (4 samples each) KC at a time: their fragments of y' are built,
  // then every block takes them
  for (int k0 = 0; k0 < nks; k0 += KC) {
    double yb[RBYM][KC], rr[KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const int j = 4 * (k0 + kk) + kb;
      const bool ok = j < nm;
      const int tt = ok ? mlist[j] : 0;
      rr[kk] = ok ? (double)as[(size_t)tt * G + g] : 0.0;
#pragma unroll
      for (int cb = 0; cb < RBYM; ++cb) {
        const int e = 16 * cb + m;
        yb[cb][kk] = (ok && e <= D) ? (double)(xs[(size_t)tt * DS + e] - mue[cb]) : 0.0;
      }
    }
#pragma unroll
    for (int rb = 0, i = 0; rb < RBYM; ++rb)
#pragma unroll
      for (int cb = 0; cb <= rb; ++cb, ++i) {
        if (rb >= RBY) continue;
#pragma unroll
        for (int kk = 0; kk < KC; ++kk)
          c[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(rr[kk] * yb[rb][kk], yb[cb][kk], c[i], 0,
                                                      0, 0);
      }
  }
#pragma unroll
  for (int rb = 0, i = 0; rb < RBYM; ++rb)
#pragma unroll
    for (int cb = 0; cb <= rb; ++cb, ++i) {
      if (rb >= RBY) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int d = 16 * rb + 4 * j + kb, e = 16 * cb + m;
        int k = -1;
        if (d == D && e == D) k = 0;
        else if (d == D && e < D) k = 1 + e;
        else if (d < D && e <= d) k = 1 + D + tri_index(d, e, D);
        // every entry has one (block, lane, register) of the one wave that
        // owns the component
        if (k >= 0) {
          if (stg) stg[k] = c[i][j];
          else unsafeAtomicAdd(q + k, c[i][j]);  // an ordered update (one lane)
        }
      }
    }
  if (stg) {
    // the staged entries go out in address order, entry k from lane k % 64:
    // whole cache lines per atomic instruction, still one updating lane
    wave_lds_sync();
    const int P = 1 + D + D * (D + 1) / 2;
    for (int k = lane; k < P; k += kWave) unsafeAtomicAdd(q + k, stg[k]);
  }
}

// FKS: k-steps of 4 of the FP64 matrix-core log-densities (8: D <= 32, 16:
// D <= 64), 0 for the vector-ALU screening with the FP64 near-set recompute.
template <bool MSTEP, int FKS>
__global__ void __launch_bounds__(kNT, 2) k_estep_full(
    const float* __restrict__ X, int64_t N, int D, int64_t ldx, int G, int T, int64_t chunk,
    const float* __restrict__ W, const double* __restrict__ Wf64, const double* __restrict__ b64,
    const float* __restrict__ cc, const double* __restrict__ W64,
    const double* __restrict__ c64, const float* __restrict__ means,
    double* __restrict__ part, double* __restrict__ ll_part, float* __restrict__ per_sample,
    int32_t* __restrict__ dev_status) {
  extern __shared__ double ldsd[];
  __shared__ int mlist_s[kNT / kWave][64];  // per wave: a component's member samples
  const int nw = kNT / kWave;
  constexpr bool F64 = FKS > 0;
  double* as64 = ldsd;                                      // F64: [T][G] log-densities
  double* wst = as64 + (F64 ? (size_t)T * G : 0);           // [nw][kWB] packed rows of W_g
  double* bst = wst + (F64 ? 0 : (size_t)nw * kWB);         // [nw][kWR] b_r
  double* lse = bst + (F64 ? 0 : (size_t)nw * kWR);         // [T]
  double* mst = lse + T;                                    // [nw][D] mu_g (near recompute)
  float* xs = (float*)(mst + (F64 ? 0 : (size_t)nw * D));   // [T][D+1]
  const int DS = D + 1;                        // padded row stride (conflict-free column reads)
  float* as = xs + (size_t)T * DS;             // [T][G]
  float* mxs = as + (size_t)T * G;             // [T] screened maximum
  uint32_t* gbits = (uint32_t*)(mxs + T);      // [G/32]: component has a non-zero r in the tile
  const int NGB = (G + 31) / 32;
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wid = tid / kWave;
  const int b = blockIdx.x;
  const int64_t i0 = (int64_t)b * chunk;
  const int64_t i1 = min(N, i0 + chunk);
  const int NT2 = D * (D + 1) / 2;
  const int P = 1 + D + NT2;
  double* pb = part + (size_t)b * G * P;
  double* wl = wst + (size_t)wid * kWB;
  double* bl = bst + (size_t)wid * kWR;
  double* ml = mst + (size_t)wid * D;
  if (tid == 0) bad = 0;
  if (MSTEP) {
    for (int p = tid; p < G * P; p += kNT) pb[p] = 0.0;
    __threadfence();  // the zeros land before any atomic update of the partials
  }
  double llacc = 0.0;
  __syncthreads();
  for (int64_t t0 = i0; t0 < i1; t0 += T) {
    const int nt = (int)min((int64_t)T, i1 - t0);
    for (int p = tid; p < nt * DS; p += kNT) {  // column D holds 1 (see the map step)
      const int t = p / DS, d = p - t * DS;
      xs[p] = d < D ? X[(t0 + t) * ldx + d] : 1.0f;
    }
    for (int p = tid; p < NGB; p += kNT) gbits[p] = 0u;
    __syncthreads();
    // a_gi: exact FP64 values on the matrix cores for D <= 64; otherwise FP32
    // screening (wave per component, W_g and mu_g read uniformly, lane per
    // sample) and the FP64 near-set recompute below
    if (F64)
      logdens_full_f64<(F64 ? FKS : 8)>(xs, DS, nt, D, G, Wf64, b64, c64, as64, wid, nw, lane);
    else
    for (int g = __builtin_amdgcn_readfirstlane(wid); g < G; g += nw) {
      const float* mu = means + (size_t)g * D;
      const float* Wg = W + (size_t)g * D * D;
      const float cg = cc[g], cl = cc[G + g];
      for (int t = lane; t < nt; t += kWave) {
        const float* x = xs + (size_t)t * DS;
        float acc = 0.0f;
        for (int r = 0; r < D; ++r) {
          const float* wr = Wg + (size_t)r * D;
          float z = 0.0f;
          int c = 0;
          for (; c + 8 <= r + 1; c += 8) {  // operands of 8 terms loaded together
            float wv[8], mv[8], xv[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              wv[i] = wr[c + i];
              mv[i] = mu[c + i];
              xv[i] = x[c + i];
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) z = fmaf(wv[i], xv[i] - mv[i], z);
          }
          for (; c <= r; ++c) z = fmaf(wr[c], x[c] - mu[c], z);
          acc = fmaf(z, z, acc);
        }
        as[(size_t)t * G + g] = (cg - 0.5f * acc) + cl;
      }
    }
    __syncthreads();
    // screened maximum per sample
    for (int t = wid; t < nt && !F64; t += nw) {
      const float* a = as + (size_t)t * G;
      float mx = -INFINITY;
      for (int g = lane; g < G; g += kWave) mx = fmaxf(mx, a[g]);
      mx = wave_max(mx);
      if (lane == 0) mxs[t] = mx;
    }
    __syncthreads();
    // Near set {g : a_g >= mx - kNearGap} recomputed in FP64 from the FP32
    // parameters: a64 = c_g - 1/2 ||z||^2, z = W_g x - W_g mu_g with W_g =
    // L_g^-1 in FP64.  Wave per component, lane per sample; the packed rows of
    // W_g are staged in LDS a chunk at a time and read by all near lanes.
    // Every value is moved to the frame of its sample's M = mx.
    for (int g = __builtin_amdgcn_readfirstlane(wid); g < G && !F64; g += nw) {
      float* ag = as + g;
      const int t = lane;
      const float mx = t < nt ? mxs[t] : 0.0f;
      const float v = t < nt ? ag[(size_t)t * G] : -INFINITY;
      const bool near = t < nt && v >= mx - kNearGap;
      const unsigned long long msk = __ballot(near);
      double q = 0.0;
      if (msk) {
        const double* Wg = W64 + (size_t)g * D * D;
        const float* x = xs + (size_t)(t < nt ? t : 0) * DS;
        for (int c = lane; c < D; c += kWave) ml[c] = (double)means[(size_t)g * D + c];
        for (int r0 = 0; r0 < D;) {
          // rows r0 .. r1-1: packed entries off(r) = r(r+1)/2 - off(r0)
          int r1 = r0, ne = 0;
          while (r1 < D && r1 - r0 < kWR && ne + r1 + 1 <= kWB) {
            ne += r1 + 1;
            ++r1;
          }
          const int base = r0 * (r0 + 1) / 2;
          for (int r = r0; r < r1; ++r)
            for (int c = lane; c <= r; c += kWave) wl[r * (r + 1) / 2 - base + c] = Wg[(size_t)r * D + c];
          wave_lds_sync();
          for (int r = r0 + lane; r < r1; r += kWave) {
            const double* wr = wl + r * (r + 1) / 2 - base;
            double s = 0.0;
            for (int c = 0; c <= r; ++c) s = fma(wr[c], ml[c], s);
            bl[r - r0] = s;
          }
          wave_lds_sync();
          if (near) {
            for (int r = r0; r < r1; ++r) {
              const double* wr = wl + r * (r + 1) / 2 - base;
              double z = -bl[r - r0];
              int c = 0;
              for (; c + 8 <= r + 1; c += 8) {
                double wv[8];
                float xv[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                  wv[i] = wr[c + i];
                  xv[i] = x[c + i];
                }
#pragma unroll
                for (int i = 0; i < 8; ++i) z = fma(wv[i], (double)xv[i], z);
              }
              for (; c <= r; ++c) z = fma(wr[c], (double)x[c], z);
              q = fma(z, z, q);
            }
          }
          wave_lds_sync();  // the next chunk overwrites the staging buffers
          r0 = r1;
        }
      }
      if (t < nt) {
        const double M = (double)mx;
        ag[(size_t)t * G] = near ? (float)(c64[g] - 0.5 * q - M) : v - mx;
      }
    }
    __syncthreads();
    // log-sum-exp about M + max (Eqs. 16-18) and responsibilities
    for (int t = wid; t < nt && F64; t += nw) {
      const double* a64 = as64 + (size_t)t * G;
      float* a = as + (size_t)t * G;
      double M = -INFINITY;
      for (int g = lane; g < G; g += kWave) M = fmax(M, a64[g]);
      for (int off = 1; off < kWave; off <<= 1) M = fmax(M, __shfl_xor(M, off));
      const double Mr = M > -INFINITY ? M : 0.0;
      double sm = 0.0;
      for (int g = lane; g < G; g += kWave) sm += (double)__expf((float)(a64[g] - Mr));
      sm = wave_sum_d(sm);
      const double l = Mr + log(sm);
      if (MSTEP) {
        for (int g = lane; g < G; g += kWave) {
          const float z = (float)(a64[g] - l);
          const float r = z >= -kRespCut ? __expf(z) : 0.0f;
          a[g] = r;
          if (r != 0.0f) atomicOr(&gbits[g >> 5], 1u << (g & 31));
        }
      }
      if (lane == 0) {
        lse[t] = l;
        if (!isfinite(l)) bad = 1;
        if (per_sample) per_sample[t0 + t] = (float)l;
      }
    }
    for (int t = wid; t < nt && !F64; t += nw) {
      float* a = as + (size_t)t * G;
      const double M = (double)mxs[t];
      float dn = -INFINITY;
      for (int g = lane; g < G; g += kWave) dn = fmaxf(dn, a[g]);
      dn = wave_max(dn);
      dn = dn > -INFINITY ? dn : 0.0f;
      double sm = 0.0;
      for (int g = lane; g < G; g += kWave) sm += (double)__expf(a[g] - dn);
      sm = wave_sum_d(sm);
      const double l = (M + (double)dn) + log(sm);
      if (MSTEP) {
        const float dl = (float)log(sm);
        for (int g = lane; g < G; g += kWave) {
          const float z = (a[g] - dn) - dl;
          const float r = z >= -kRespCut ? __expf(z) : 0.0f;
          a[g] = r;
          if (r != 0.0f) atomicOr(&gbits[g >> 5], 1u << (g & 31));
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
    constexpr bool MAP64 = FKS == 8;  // D <= 32: the map step on the matrix cores too
    if (MSTEP && MAP64) {
      // map step (Eqs. 9-11) on the matrix cores, wave per component with a
      // non-zero responsibility in the tile, over the list of its samples
      // with r != 0 (T <= 64: one lane per sample)
      int* ml = mlist_s[wid];
      const unsigned long long lt = (1ull << lane) - 1ull;
      // each wave stages a component's entries in the log-density buffer, free
      // once the responsibilities are taken, when it is large enough
      const int PS = (1 + D + D * (D + 1) / 2 + 1) & ~1;
      double* stg = (size_t)T * G >= (size_t)nw * PS ? as64 + (size_t)wid * PS : nullptr;
      for (int g = wid; g < G; g += nw) {
        if (!((gbits[g >> 5] >> (g & 31)) & 1u)) continue;
        const bool mine = lane < nt && as[(size_t)lane * G + g] != 0.0f;
        const unsigned long long mem = __ballot(mine);
        if (mine) ml[__popcll(mem & lt)] = lane;
        wave_lds_sync();
        map_full_f64<3, 4>(xs, DS, __popcll(mem), ml, D, G, as, means + (size_t)g * D,
                           pb + (size_t)g * P, g, lane, stg);
        wave_lds_sync();  // the list is rewritten for the next component
      }
    }
    if (MSTEP && !MAP64) {
      // entry k of component g: 0 -> L, 1..D -> sum r y_d, then the packed
      // lower triangle sum r y_d y_e (d >= e, column e after column e-1).
      // Wave per component with a non-zero responsibility in the tile, lanes
      // over entries (kSL per lane at a time, their (d, e) decoded once),
      // visiting only the tile's samples with r != 0 (a ballot mask, T <= 64).
      // Every entry is (r y_d) y_e: column D of the tile holds 1 and mu is taken
      // as 0 there, so y = 1 stands in for the missing factors of L and sum r y.
      // The tile's contributions are added to the partials once.
      constexpr int kSL = 9;
      for (int g = wid; g < G; g += nw) {
        if (!((gbits[g >> 5] >> (g & 31)) & 1u)) continue;
        const unsigned long long mem = __ballot(lane < nt && as[(size_t)lane * G + g] != 0.0f);
        double* q = pb + (size_t)g * P;
        const float* mug = means + (size_t)g * D;
        for (int k0 = 0; k0 < P; k0 += kWave * kSL) {
          int od[kSL], oe[kSL];
          float md[kSL], me[kSL];
#pragma unroll
          for (int i = 0; i < kSL; ++i) {
            const int k = k0 + lane + kWave * i;
            int d = D, e = D;  // k = 0 (and k >= P): both factors 1
            if (k >= 1 && k <= D) {
              d = k - 1;
            } else if (k > D && k < P) {
              int qq = k - 1 - D;
              e = 0;
              while (qq >= D - e) {
                qq -= D - e;
                ++e;
              }
              d = e + qq;
            }
            od[i] = d;
            oe[i] = e;
            md[i] = d < D ? mug[d] : 0.0f;
            me[i] = e < D ? mug[e] : 0.0f;
          }
          double sum[kSL];
#pragma unroll
          for (int i = 0; i < kSL; ++i) sum[i] = 0.0;
          for (unsigned long long m = mem; m; m &= m - 1) {
            const int t = __ffsll((long long)m) - 1;
            const double r = (double)as[(size_t)t * G + g];
            const float* xt = xs + (size_t)t * DS;
#pragma unroll
            for (int i = 0; i < kSL; ++i) {
              const double yd = (double)(xt[od[i]] - md[i]);
              const double ye = (double)(xt[oe[i]] - me[i]);
              sum[i] = fma(r * yd, ye, sum[i]);
            }
          }
#pragma unroll
          for (int i = 0; i < kSL; ++i) {
            const int k = k0 + lane + kWave * i;
            if (k < P) unsafeAtomicAdd(q + k, sum[i]);  // entry k: this lane only
          }
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

// LDS of k_estep_full for tile rows T.
// LDS of k_estep_full for tile rows T (f64: the FP64 matrix-core form).
size_t estep_full_lds(int D, int G, int T, bool f64) {
  const size_t dbl = f64 ? (size_t)T * G + T : (size_t)(kNT / kWave) * (kWB + kWR + D) + T;
  return sizeof(double) * dbl + sizeof(float) * ((size_t)T * (D + 1 + G) + T) +
         sizeof(uint32_t) * ((G + 31) / 32);
}

int tile_rows_full(int D, int G) {
  int T = 64;  // at most one wave of samples (ballot masks over the tile)
  while (T > 1 && estep_full_lds(D, G, T, D <= 64) > 62 * 1024) T >>= 1;  // default LDS limit
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
  const size_t lds = estep_full_lds(D, G, T, D <= 64);
  hipLaunchKernelGGL(k_init_full, dim3(1), dim3(64), 0, st, dev_status, n_recomputed);
  hipLaunchKernelGGL(k_pre_full, dim3(G), dim3(kNT), 0, st, hefts, covs, means, D, G, w.partials,
                     w.W, w.W64, w.Wf64, w.b64, w.c, w.c64, dev_status);
  {
    ProfScope ps(kProfEM, st);
    auto kern = D <= 32 ? k_estep_full<true, 8> : D <= 64 ? k_estep_full<true, 16>
                                                           : k_estep_full<true, 0>;
    hipLaunchKernelGGL(kern, dim3(nb), dim3(kNT), lds, st, X, N, D, ldx, G, T, chunk, w.W,
                       w.Wf64, w.b64, w.c, w.W64, w.c64, means, w.partials, w.scalars, nullptr,
                       dev_status);
  }
  // [P] FP64 totals: above the 64 KB default from D = 127 on (67 KB at D = 128)
  const size_t fin_lds = sizeof(double) * P;
  if (fin_lds > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)k_fin_full, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)fin_lds);
  hipLaunchKernelGGL(k_fin_full, dim3(G), dim3(kNT), fin_lds, st, w.partials, nb, N, D,
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
  const size_t lds = estep_full_lds(D, G, T, D <= 64);
  hipLaunchKernelGGL(k_init_full, dim3(1), dim3(64), 0, st, dev_status, nullptr);
  hipLaunchKernelGGL(k_pre_full, dim3(G), dim3(kNT), 0, st, hefts, covs, means, D, G, w.partials,
                     w.W, w.W64, w.Wf64, w.b64, w.c, w.c64, dev_status);
  {
    ProfScope ps(kProfLoglik, st);
    auto kern = D <= 32 ? k_estep_full<false, 8> : D <= 64 ? k_estep_full<false, 16>
                                                            : k_estep_full<false, 0>;
    hipLaunchKernelGGL(kern, dim3(nb), dim3(kNT), lds, st, X, N, D, ldx, G, T, chunk, w.W,
                       w.Wf64, w.b64, w.c, w.W64, w.c64, means, w.partials, w.scalars,
                       per_sample, dev_status);
  }
  hipLaunchKernelGGL(k_ll_finish_full, dim3(1), dim3(64), 0, st, w.scalars, nb, N, mean_loglik,
                     dev_status);
  return hipGetLastError();
}

}  // namespace gmm
