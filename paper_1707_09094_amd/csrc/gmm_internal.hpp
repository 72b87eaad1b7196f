// gmm_internal.hpp -- shared definitions of the gfx950 GMM library (not part of
// the public ABI; see include/gmm.h for that).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/gmm.h"

namespace gmm {

constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kMaxBlocks = 512;      // E/M grid: 2 workgroups per CU on 256 CUs
// Responsibilities (normalised per sample) below exp(-40) are set to 0: a
// component then loses at most N e^-40 ~ 4e-18 N of its mass L_g.
constexpr float kRespCut = 40.0f;
// Near set of a sample: every component whose screened log-density, widened by
// its rounding-error bound, comes within this many nats of the largest
// guaranteed lower bound.  Those are recomputed exactly (FP64 from the FP32
// parameters, or FP32 direct form where its bound is below kExactTol).
constexpr float kNearGap = 30.0f;
constexpr float kExactTol = 1e-3f;
constexpr double kLog2Pi = 1.8378770664093454835606594728112353;

// ---- rounding-error bounds of the FP32 screening values --------------------
// a_g(x) = c_g - q/2, q = sum_d lam_gd (x_d - mu_gd)^2, Q_g = sum_d lam_gd mu_gd^2.
// Direct form: u_d = fma(x_d, s_gd, -m_gd) with s = sqrt(lam), m = mu s each
// rounded once, so |du_d| <= 2^-24 (|u_d| + sqrt(lam_d)(|x_d| + |mu_d|)); with
// (|x|+|mu|)^2 <= 2 (x-mu)^2 + 8 mu^2, Cauchy-Schwarz and D sequential FMAs,
// |dq| <= 2^-24 ((2 + D) q + 2 sqrt(q (2q + 8Q))); adding c (hi + lo) and
// forming c - q/2 rounds twice more.  q is taken from the screened value, whose
// own error is covered by the 1% margin.
__device__ __forceinline__ float err_direct(float q, float Q, float c, int D) {
  q = fmaxf(q, 0.0f);
  const float t = 2.0f * sqrtf(q * (2.0f * q + 8.0f * Q));
  return 1.01f * (0x1p-25f * ((2.0f + (float)D) * q + t) + 0x1p-23f * (fabsf(c) + 0.5f * q));
}

// Expanded form in BF16x3 (A = [lam mu; -lam/2], B = [x; x^2], hi/lo split):
// each product is off by <= 3 2^-16 |A||B|, the FP32 accumulation of 3*32*KS
// terms by <= 96 KS 2^-24 sum|A||B|, and sum|A||B| <= (1 + sqrt 2)(q + Q);
// adding cexp = c - Q/2 (hi + lo) rounds twice more.
__device__ __forceinline__ float err_expanded_coef(int KS) {
  return 1.02f * 2.4142136f * (3.0f * 0x1p-16f + 96.0f * (float)KS * 0x1p-24f + 0x1p-23f);
}
__device__ __forceinline__ float err_expanded(float q, float Q, float c, float coef) {
  q = fmaxf(q, 0.0f);
  return coef * (q + Q) + 1.01f * 0x1p-23f * (fabsf(c) + 0.5f * Q);
}

// Order-preserving map float <-> int (for integer atomicMax in LDS).
__device__ __forceinline__ int f2ord(float f) {
  const int i = __float_as_int(f);
  return i >= 0 ? i : i ^ 0x7FFFFFFF;
}
__device__ __forceinline__ float ord2f(int i) { return __int_as_float(i >= 0 ? i : i ^ 0x7FFFFFFF); }

// ---- wave-level helpers of the sample-major kernels --------------------------
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double f64x4;

// Butterflies over the 16 lanes of a row by DPP row rotations (no address
// registers): after rotations by 1, 2, 4 and 8 every lane holds the reduction
// of all 16.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xFFFFFFFFll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float row16_max(float v) {
  v = fmaxf(v, dpp_f<0x121>(v));
  v = fmaxf(v, dpp_f<0x122>(v));
  v = fmaxf(v, dpp_f<0x124>(v));
  v = fmaxf(v, dpp_f<0x128>(v));
  return v;
}
__device__ __forceinline__ float row16_sum_f(float v) {
  v += dpp_f<0x121>(v);
  v += dpp_f<0x122>(v);
  v += dpp_f<0x124>(v);
  v += dpp_f<0x128>(v);
  return v;
}
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_d<0x121>(v);
  v += dpp_d<0x122>(v);
  v += dpp_d<0x124>(v);
  v += dpp_d<0x128>(v);
  return v;
}
// quad (4-lane) sums by DPP quad permutations
__device__ __forceinline__ float quad_sum(float v) {
  v += dpp_f<0xB1>(v);  // quad_perm [1,0,3,2]
  v += dpp_f<0x4E>(v);  // quad_perm [2,3,0,1]
  return v;
}
__device__ __forceinline__ double quad_sum_d(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  return v;
}

// Exclusive prefix over lanes (and wave total) of a per-lane count v < 64,
// by bit slices: 6 ballots instead of a scan.  With a lane mask `sel`, only
// lanes in sel are counted (prefix and total over them).
__device__ __forceinline__ int wave_prefix_small(int v, unsigned long long lt,
                                                 unsigned long long sel, int* total) {
  int pre = 0, tot = 0;
#pragma unroll
  for (int b = 0; b < 6; ++b) {
    const unsigned long long m = __ballot((v >> b) & 1) & sel;
    pre += __popcll(m & lt) << b;
    tot += __popcll(m) << b;
  }
  *total = tot;
  return pre;
}

// Row (16-lane) sum of an int by DPP rotations.
__device__ __forceinline__ int row16_sum_i(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x121, 0xF, 0xF, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x122, 0xF, 0xF, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x124, 0xF, 0xF, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false);
  return v;
}

// Orders this wave's LDS accesses across lanes (the LDS executes one wave's
// operations in issue order; this keeps the compiler from reordering them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


// ---- tiles of the kernels for D <= 128 and many components -----------------
constexpr int kWNT = 256;  // threads per workgroup
constexpr int kWT = 32;    // tile rows (two 16-row blocks of the matrix cores)
constexpr int kKL = 8;     // threads per sample in their per-sample passes

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Number of workgroups of the per-block-partial kernels (E/M, k-means
// accumulation, global statistics).  A function of N only, so a given problem
// always reduces in the same order.
inline int partial_blocks(int64_t N, int64_t per_block_min) {
  int64_t b = (N + per_block_min - 1) / per_block_min;
  if (b < 1) b = 1;
  if (b > kMaxBlocks) b = kMaxBlocks;
  return (int)b;
}

// Values stored per (block, component) in the FP64 partials.
inline int partial_width(int D, int cov) {
  return cov == GMM_COV_FULL ? 1 + D + D * (D + 1) / 2 : 2 * D + 1;
}

// Carving of the caller's workspace.  Every region is 256-byte aligned.
struct Workspace {
  // per-component constants of the E-step (see em precompute kernels)
  float* s;        // diag: [D][G] 1/sigma (d-major)      full: unused
  float* m;        // diag: [D][G] mu/sigma                full: unused
  float* c;        // [3][G] log w - 1/2 (D log 2pi + log|Sigma|), split hi/lo; Q_g
  float* W;        // full: [G][D][D] inverse Cholesky factor (row-major lower)
  float* prm;      // fast diag kernel: [2][G][D+1] 1/sigma then mu/sigma
  uint16_t* Bhi;   // BF16X3 expanded weights [G][K] hi part
  uint16_t* Blo;   // BF16X3 expanded weights [G][K] lo part
  float* cexp;     // BF16X3: [2][G] constant of the expanded form, hi/lo
  double* c64;     // [G] log w - 1/2 (D log 2pi + log|Sigma|) in FP64
  double* lamg64;  // diag: [G][D] 1/sigma2 in FP64
  double* W64;     // full: [G][D][D] inverse Cholesky factor in FP64 (row-major lower)
  double* Bx64;    // diag, D <= 128: FP64 MFMA fragments of the expanded form, see
                   // diag_frag_count
  double* cq64;    // D <= 128: [2][G] c_g - Q_g / 2 and Q_g = sum_d lam mu^2 (FP64); the
                   // k-means kernel keeps its Q_g in the first half
  double* Wf64;    // full, D <= 64: FP64 MFMA fragments of W, see full_frag_count
  double* b64;     // full, D <= 64: [G][16 * ceil(D/16)] b_g = W_g mu_g
  double* partials;   // [B][G][P]
  double* scalars;    // [4][B] per-block FP64 sums (log-likelihood / inertia)
  int32_t* assign;    // [N] k-means assignment scratch
  double* dmin;       // [N] spread seeding: distance to the nearest seed (same memory)
  double* lam64;      // [D] k-means distance weights (FP64)
  float* lam32;       // [D] the same rounded to FP32
  int64_t* counters;  // [8] device counters
  float* wM;          // sliced BF16x3 E-step: [S][N] per-slice bounded maxima
  float* wD;          // [S][N] per-slice references of the sums
  float* wS;          // [S][N] per-slice sums of exp(value - M - reference)
  float* wR;          // [S][ceil(N/16)][64] exact near values passed between the passes
  size_t bytes;
};

// component slices of the sliced BF16x3 E-step (0: the shape has no such path)
int em2s_slices(int D, int G);
bool em_fast_supported(int D, int G, int prec);

// expanded-form depth (features) of the MFMA fragments: 128 or 256 for the
// one-pass kernels (D <= 64 / D <= 128), padded to 32 beyond
inline int kexp_K(int D) { return D <= 64 ? 128 : (D <= 128 ? 256 : ((2 * D + 31) / 32) * 32); }

// Full covariances with D <= 64: the whitening W_g (x - mu_g) runs in FP64 on
// the matrix cores; per component ceil(D/16) row blocks x kq(D) k-steps of 4 x
// 64 lanes, one double each.
inline int full_kq(int D) { return D <= 32 ? 8 : 16; }
inline size_t full_frag_count(int D, int G) {
  return D <= 64 ? (size_t)G * ((D + 15) / 16) * full_kq(D) * 64 : 0;
}

// Diagonal covariances with D <= 128: the expanded form c_g - Q_g/2 +
// sum_d (-lam/2 x_d^2 + lam mu x_d) in FP64 on the matrix cores; per block of 16
// components dpad4(D)/2 k-steps of 4 features x 64 lanes, one double each.
__host__ __device__ inline int dpad4(int D) { return (D + 3) & ~3; }
inline size_t diag_frag_count(int D, int G) {
  return D <= 128 ? (size_t)((G + 15) / 16) * (dpad4(D) / 2) * 64 : 0;
}

inline bool carve(void* base, size_t avail, int64_t N, int D, int G, int cov, Workspace* w) {
  size_t off = 0;
  auto take = [&](size_t n) {
    size_t o = off;
    off = align_up(off + n);
    return o;
  };
  const int B = kMaxBlocks;
  const int P = partial_width(D, cov);
  const int K = kexp_K(D);
  size_t o_s = take(sizeof(float) * (size_t)D * G);
  size_t o_m = take(sizeof(float) * (size_t)D * G);
  size_t o_c = take(sizeof(float) * 3 * (size_t)G);
  size_t o_W = take(cov == GMM_COV_FULL ? sizeof(float) * (size_t)D * D * G : 0);
  const size_t GP = ((size_t)G + 15) / 16 * 16;
  // direct-form parameters [2][G][D+1]; also the k-means table [16 RB][4]
  const size_t n_prm = 2 * (size_t)G * (D + 1);
  size_t o_prm = take(sizeof(float) * (n_prm > 64 * GP / 16 ? n_prm : 64 * GP / 16));
  size_t o_bh = take(sizeof(uint16_t) * (size_t)K * GP);
  size_t o_bl = take(sizeof(uint16_t) * (size_t)K * GP);
  size_t o_ce = take(sizeof(float) * 2 * (size_t)G);
  size_t o_c64 = take(sizeof(double) * (size_t)G);
  size_t o_lg = take(sizeof(double) * (size_t)G * D);
  size_t o_w64 = take(cov == GMM_COV_FULL ? sizeof(double) * (size_t)D * D * G : 0);
  const size_t nfr = cov == GMM_COV_FULL ? full_frag_count(D, G) : 0;
  const size_t ndf = diag_frag_count(D, G);  // also the k-means fragments (any cov)
  size_t o_bx = take(sizeof(double) * ndf);
  size_t o_cq = take(ndf ? sizeof(double) * 2 * (size_t)G : 0);
  size_t o_wf = take(sizeof(double) * nfr);
  size_t o_bw = take(nfr ? sizeof(double) * (size_t)G * 16 * ((D + 15) / 16) : 0);
  size_t o_p = take(sizeof(double) * (size_t)B * G * P);
  size_t o_sc = take(sizeof(double) * 4 * (size_t)B);
  size_t o_a = take(sizeof(double) * (size_t)N);  // assign, or the seeding's dmin
  size_t o_l64 = take(sizeof(double) * (size_t)D);
  size_t o_l32 = take(sizeof(float) * (size_t)D);
  size_t o_ct = take(sizeof(int64_t) * 8);
  // per-slice arrays of the sliced BF16x3 E-step (diagonal, more components
  // than the one-pass kernel holds)
  const int nsl = cov == GMM_COV_DIAG && !em_fast_supported(D, G, GMM_PREC_BF16X3)
                      ? em2s_slices(D, G) : 0;
  size_t o_wm = take(sizeof(float) * (size_t)nsl * N);
  size_t o_wd = take(sizeof(float) * (size_t)nsl * N);
  size_t o_ws = take(sizeof(float) * (size_t)nsl * N);
  size_t o_wr = take(sizeof(float) * (size_t)nsl * ((N + 15) / 16) * 64);
  w->bytes = off;
  if (!base) return true;
  if (avail < off) return false;
  char* b = (char*)base;
  w->s = (float*)(b + o_s);
  w->m = (float*)(b + o_m);
  w->c = (float*)(b + o_c);
  w->W = (float*)(b + o_W);
  w->prm = (float*)(b + o_prm);
  w->Bhi = (uint16_t*)(b + o_bh);
  w->Blo = (uint16_t*)(b + o_bl);
  w->cexp = (float*)(b + o_ce);
  w->c64 = (double*)(b + o_c64);
  w->lamg64 = (double*)(b + o_lg);
  w->W64 = (double*)(b + o_w64);
  w->Bx64 = (double*)(b + o_bx);
  w->cq64 = (double*)(b + o_cq);
  w->Wf64 = (double*)(b + o_wf);
  w->b64 = (double*)(b + o_bw);
  w->partials = (double*)(b + o_p);
  w->scalars = (double*)(b + o_sc);
  w->assign = (int32_t*)(b + o_a);
  w->dmin = (double*)(b + o_a);
  w->lam64 = (double*)(b + o_l64);
  w->lam32 = (float*)(b + o_l32);
  w->counters = (int64_t*)(b + o_ct);
  w->wM = nsl ? (float*)(b + o_wm) : nullptr;
  w->wD = nsl ? (float*)(b + o_wd) : nullptr;
  w->wR = nsl ? (float*)(b + o_wr) : nullptr;
  w->wS = nsl ? (float*)(b + o_ws) : nullptr;
  return true;
}

// ---- many-model (batched) workspace ---------------------------------------

struct BatchItemDev {
  int32_t model;
  int32_t first_of_model;
  int64_t i0, i1;
};

constexpr int kBatchMaxD = 128;
constexpr int kBatchMaxG = 128;

// A descriptor the batched kernels may use: the host sized the launch and the
// workspace from Ns/Gs, so a model outside that envelope is skipped (its
// status gets GMM_DEV_BADDESC from the plan kernel) rather than overrun it.
__device__ inline bool batch_desc_ok(const gmm_model_desc& m, int Gmax) {
  return m.N >= 1 && m.G >= 1 && m.G <= Gmax && m.X != nullptr;
}

struct BatchWorkspace {
  int n_models, D, Gmax, RBmax, KS, cap;  // cap: item capacity
  BatchItemDev* items;
  int2* mitems;
  int* n_items;
  // EM constants (stride per model)
  float* prm;      // 2 * Gmax * (D+1)
  float* cc;       // 2 * Gmax
  float* cexp;     // 2 * Gmax
  void* Whi;       // RBmax * KS * 64 * 16 bytes
  void* Wlo;
  double* c64;     // Gmax
  double* lam64;   // Gmax * D
  // k-means constants (stride per model)
  float* kmprm;    // kpstride: [Gmax][D+1] m of the FP32 k-means form, or the
                   // [16 RBmax][4] table of the matrix-core form
  size_t kpstride;
  float* ksd;      // D
  double* klam64;  // D
  float* kmnorm;   // 1
  int64_t* kscratch;  // 2 * Gmax (resurrection)
  double* partials;   // cap * Gmax * (2D+1)
  double* sparts;     // cap
  size_t bytes;
};

inline bool carve_batched(void* base, size_t avail, int n_models, int D, int Gmax, int cap,
                          BatchWorkspace* w) {
  size_t off = 0;
  auto take = [&](size_t n) {
    size_t o = off;
    off = align_up(off + n);
    return o;
  };
  const size_t M = (size_t)n_models;
  const int RBmax = (Gmax + 15) / 16;
  const int KS = D <= 64 ? 4 : ((2 * D + 31) / 32 <= 8 ? 8 : (2 * D + 31) / 32);
  const size_t o_it = take(sizeof(BatchItemDev) * (size_t)cap);
  const size_t o_mi = take(sizeof(int2) * M);
  const size_t o_ni = take(sizeof(int) * 4);
  const size_t o_prm = take(sizeof(float) * M * 2 * Gmax * (D + 1));
  const size_t o_cc = take(sizeof(float) * M * 2 * Gmax);
  const size_t o_ce = take(sizeof(float) * M * 2 * Gmax);
  const size_t o_wh = take(M * RBmax * KS * 64 * 16);
  const size_t o_wl = take(M * RBmax * KS * 64 * 16);
  const size_t o_c64 = take(sizeof(double) * M * Gmax);
  const size_t o_l64 = take(sizeof(double) * M * Gmax * D);
  const size_t kps = (size_t)Gmax * (D + 1) > (size_t)64 * RBmax ? (size_t)Gmax * (D + 1)
                                                                   : (size_t)64 * RBmax;
  const size_t o_kp = take(sizeof(float) * M * kps);
  const size_t o_ks = take(sizeof(float) * M * D);
  const size_t o_kl = take(sizeof(double) * M * D);
  const size_t o_kn = take(sizeof(float) * M);
  const size_t o_kx = take(sizeof(int64_t) * M * 2 * Gmax);
  const size_t o_p = take(sizeof(double) * (size_t)cap * Gmax * (2 * D + 1));
  const size_t o_sp = take(sizeof(double) * (size_t)cap);
  w->n_models = n_models;
  w->D = D;
  w->Gmax = Gmax;
  w->RBmax = RBmax;
  w->KS = KS;
  w->cap = cap;
  w->kpstride = kps;
  w->bytes = off;
  if (!base) return true;
  if (avail < off) return false;
  char* b = (char*)base;
  w->items = (BatchItemDev*)(b + o_it);
  w->mitems = (int2*)(b + o_mi);
  w->n_items = (int*)(b + o_ni);
  w->prm = (float*)(b + o_prm);
  w->cc = (float*)(b + o_cc);
  w->cexp = (float*)(b + o_ce);
  w->Whi = b + o_wh;
  w->Wlo = b + o_wl;
  w->c64 = (double*)(b + o_c64);
  w->lam64 = (double*)(b + o_l64);
  w->kmprm = (float*)(b + o_kp);
  w->ksd = (float*)(b + o_ks);
  w->klam64 = (double*)(b + o_kl);
  w->kmnorm = (float*)(b + o_kn);
  w->kscratch = (int64_t*)(b + o_kx);
  w->partials = (double*)(b + o_p);
  w->sparts = (double*)(b + o_sp);
  return true;
}

int batch_item_count(int32_t n_models, const int64_t* Ns, int64_t chunk);
hipError_t launch_batch_plan(const gmm_model_desc* models, int n_models, int64_t chunk,
                             const BatchWorkspace& bw, hipStream_t st);
bool em_fast_supported(int D, int G, int prec);
bool km_fast_supported(int D, int G);
hipError_t launch_em_batched(const gmm_model_desc* models, int n_models, int n_items_host, int D,
                             float var_floor, int prec, bool mstep, const BatchWorkspace& bw,
                             hipStream_t st);
hipError_t launch_kmeans_batched(const gmm_model_desc* models, int n_models, int n_items_host,
                                 int D, int dist, float var_floor, const BatchWorkspace& bw,
                                 hipStream_t st);
hipError_t launch_global_stats_batched(const gmm_model_desc* models, int n_models, int D,
                                       double* mean_out, double* var_out, hipStream_t st);

// ---- device helpers -------------------------------------------------------

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Fixed-order FP64 block reduction (tree over LDS).  All threads must call it;
// returns the sum in thread 0 (others get an unspecified value).
template <int NT>
__device__ __forceinline__ double block_sum_d(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// Fixed-order combination of one component's per-block Welford partials
// (Eqs. 12-14 in the pairwise form): block b's partials [L_b, m_b[D], Q_b[D]]
// start at base + b * stride; blocks are taken in order b = 0..nb-1, empty ones
// skipped, the first non-empty one as is, every later one by L' = L + L_b,
// m += (m_b - m) L_b / L', Q += Q_b + (m_b - m)^2 L L_b / L'.  The running
// totals L depend on the counts alone, so they are taken first (one thread, in
// block order) and each block's two weights computed from them in parallel;
// then thread d runs the chain of dimension d with the loads of FLY blocks in
// flight (32 for a few large reductions, 8 where many workgroups share the GPU
// and registers decide occupancy).  The arithmetic is that of the plain block-by-block loop.  Needs
// D <= NT; every thread must call it.  Returns the total L; thread d < D gets
// its (m, Q).
constexpr int kWcChunk = 256;  // blocks per pass
struct WelfordLds {
  double lb[kWcChunk], la[kWcChunk], w1[kWcChunk], w2[kWcChunk];
  int kind[kWcChunk];
  double run;
};
template <int NT, int FLY>
__device__ double welford_combine(const double* __restrict__ base, size_t stride, int nb, int D,
                                  WelfordLds& S, double& m, double& Q) {
  const int tid = threadIdx.x;
  const int d = tid;
  if (tid == 0) S.run = 0.0;
  m = 0.0;
  Q = 0.0;
  __syncthreads();
  for (int c0 = 0; c0 < nb; c0 += kWcChunk) {
    const int nc = min(kWcChunk, nb - c0);
    for (int i = tid; i < nc; i += NT) S.lb[i] = base[(size_t)(c0 + i) * stride];
    __syncthreads();
    if (tid == 0) {
      double L = S.run;
      for (int i = 0; i < nc; ++i) {
        const double Lb = S.lb[i];
        S.la[i] = L;
        if (Lb != 0.0) L = L == 0.0 ? Lb : L + Lb;
      }
      S.run = L;
    }
    __syncthreads();
    for (int i = tid; i < nc; i += NT) {
      const double Lb = S.lb[i], La = S.la[i];
      const double Ln = La + Lb;
      S.kind[i] = Lb == 0.0 ? 0 : (La == 0.0 ? 1 : 2);
      S.w1[i] = Lb / Ln;
      S.w2[i] = La * Lb / Ln;
    }
    __syncthreads();
    if (d < D) {
      constexpr int kFly = FLY;  // blocks whose loads are in flight together
      const double* q = base + (size_t)c0 * stride + 1 + d;
      for (int i0 = 0; i0 < nc; i0 += kFly) {
        double mb[kFly], Qb[kFly];
#pragma unroll
        for (int j = 0; j < kFly; ++j) {
          const int i = min(i0 + j, nc - 1);
          mb[j] = q[(size_t)i * stride];
          Qb[j] = q[(size_t)i * stride + D];
        }
#pragma unroll
        for (int j = 0; j < kFly; ++j) {
          const int i = i0 + j;
          if (i >= nc) break;
          const int k = S.kind[i];
          if (k == 1) {
            m = mb[j];
            Q = Qb[j];
          } else if (k == 2) {
            const double dl = mb[j] - m;
            m += dl * S.w1[i];
            Q += Qb[j] + dl * dl * S.w2[i];
          }
        }
      }
    }
    __syncthreads();  // the chunk's arrays are rewritten by the next pass
  }
  return S.run;
}

namespace {
// First level of the reduce of the Welford partials [nb][G][1 + 2D] when
// there are many blocks: workgroup (g, s) combines blocks s seg ..
// min((s + 1) seg, nb) - 1 of component g in order (welford_combine) and
// leaves the segment's (L, m, Q) in place of the segment's first block, so
// that the chains of the final reduce are nb / seg long instead of nb.
__global__ void __launch_bounds__(256) k_welford_seg(double* __restrict__ part, int nb, int seg,
                                                     int D, int G) {
  __shared__ WelfordLds S;
  const int g = blockIdx.x, b0 = blockIdx.y * seg;
  const int n = min(seg, nb - b0);
  if (n <= 0) return;
  const int P = 2 * D + 1;
  double* const base = part + (size_t)b0 * G * P + (size_t)g * P;
  double m, Q;
  const double L = welford_combine<256, 32>(base, (size_t)G * P, n, D, S, m, Q);
  // welford_combine ends with a barrier: every read of the segment is done
  const int d = threadIdx.x;
  if (d == 0) base[0] = L;
  if (d < D) {
    base[1 + d] = L > 0.0 ? m : 0.0;
    base[1 + D + d] = L > 0.0 ? Q : 0.0;
  }
}

}  // namespace

// Sum of v[0..n) in index order, by thread 0, with the values staged through
// LDS by the whole workgroup so that their loads overlap (the same arithmetic
// as one thread's plain loop).  Every thread must call it; the sum is valid in
// thread 0.  sh: kWcChunk doubles of LDS.
template <int NT>
__device__ double ordered_sum(const double* __restrict__ v, int n, double* sh) {
  double s = 0.0;
  for (int c0 = 0; c0 < n; c0 += kWcChunk) {
    const int nc = min(kWcChunk, n - c0);
    for (int i = threadIdx.x; i < nc; i += NT) sh[i] = v[c0 + i];
    __syncthreads();
    if (threadIdx.x == 0)
      for (int i = 0; i < nc; ++i) s += sh[i];
    __syncthreads();
  }
  return s;
}

// ---- optional event timing of the data-pass kernels (gmm_profile.hip) ------

constexpr int kProfKinds = 8;
enum ProfKind {
  kProfEM = GMM_PROF_EM,
  kProfKmAssign = GMM_PROF_KM_ASSIGN,
  kProfKmAccum = GMM_PROF_KM_ACCUM,
  kProfLoglik = GMM_PROF_LOGLIK,
  kProfStats = GMM_PROF_STATS,
  kProfBatched = GMM_PROF_BATCHED,
};

// While one of these lives on a thread, ProfScope records nothing there (for
// entry points that must not create events).
struct ProfSuppress {
  ProfSuppress();
  ~ProfSuppress();
};

// Records an event pair around its lifetime when profiling is on.
class ProfScope {
 public:
  ProfScope(int kind, hipStream_t st);
  ~ProfScope();

 private:
  int kind_;
  hipStream_t st_;
  hipEvent_t a_, b_;
};

// ---- launchers (defined in the kernel sources) ----------------------------

hipError_t launch_global_stats(const float* X, int64_t N, int D, int64_t ldx, double* mean,
                               double* var, const Workspace& w, hipStream_t st);

hipError_t launch_pre_diag(const float* hefts, const float* means, const float* covs, int D,
                           int G, const Workspace& w, hipStream_t st);

bool em_fast_supported(int D, int G, int prec);
hipError_t launch_em_fast(const float* X, int64_t N, int D, int64_t ldx, int G, const float* hefts,
                          const float* means, const float* covs, int prec, bool mstep,
                          int64_t* n_recomputed, float* per_sample, int32_t* dev_status,
                          const Workspace& w, hipStream_t st, int* nb_out);

// EM / log-likelihood over component slices (BF16x3, D <= 128, any G): see
// em2_range; nb_out: work ranges of the partials
bool em2s_supported(int D, int G);
hipError_t launch_em_sliced(const float* X, int64_t N, int D, int64_t ldx, int G,
                            const float* hefts, const float* means, const float* covs, bool mstep,
                            int64_t* n_recomputed, float* per_sample, int32_t* dev_status,
                            const Workspace& w, hipStream_t st, int* nb_out);

hipError_t launch_fin_welford(int nb, int64_t N, int D, int G, float var_floor, float* hefts,
                              float* means, float* covs, double* mean_loglik, int32_t* dev_status,
                              const Workspace& w, hipStream_t st);

hipError_t launch_em_diag(const float* X, int64_t N, int D, int64_t ldx, int G, float* hefts,
                          float* means, float* covs, float var_floor, int prec,
                          double* mean_loglik, int64_t* n_recomputed, int32_t* dev_status,
                          const Workspace& w, hipStream_t st);

hipError_t launch_loglik_diag(const float* X, int64_t N, int D, int64_t ldx, int G,
                              const float* hefts, const float* means, const float* covs, int prec,
                              double* mean_loglik, float* per_sample, int32_t* dev_status,
                              const Workspace& w, hipStream_t st);

// FP64 data (diagonal): the tile kernels in FP64 throughout
bool em_f64_supported(int D, int G);
hipError_t launch_em_diag_f64(const double* X, int64_t N, int D, int64_t ldx, int G,
                              double* hefts, double* means, double* covs, double var_floor,
                              double* mean_loglik, int32_t* dev_status, const Workspace& w,
                              hipStream_t st);
hipError_t launch_loglik_diag_f64(const double* X, int64_t N, int D, int64_t ldx, int G,
                                  const double* hefts, const double* means, const double* covs,
                                  double* mean_loglik, double* per_sample, int32_t* dev_status,
                                  const Workspace& w, hipStream_t st);

hipError_t launch_global_stats_f64(const double* X, int64_t N, int D, int64_t ldx, double* mean,
                                   double* var, const Workspace& w, hipStream_t st);
bool kmeans_f64_supported(int D);
hipError_t launch_kmeans_f64(const double* X, int64_t N, int D, int64_t ldx, int G, int dist,
                             const double* gvar, double var_floor, double* means, double* dcovs,
                             double* hefts, int64_t* counts, int32_t* assign, double* inertia,
                             int64_t* n_recomputed, int32_t* dev_status, const Workspace& w,
                             hipStream_t st);

hipError_t launch_em_full(const float* X, int64_t N, int D, int64_t ldx, int G, float* hefts,
                          float* means, float* covs, float var_floor, double* mean_loglik,
                          int64_t* n_recomputed, int32_t* dev_status, const Workspace& w,
                          hipStream_t st);

hipError_t launch_loglik_full(const float* X, int64_t N, int D, int64_t ldx, int G,
                              const float* hefts, const float* means, const float* covs,
                              double* mean_loglik, float* per_sample, int32_t* dev_status,
                              const Workspace& w, hipStream_t st);

bool km_fast_supported(int D, int G);
bool km2_supported(int D, int G);
// kernel family (GMM_PATH_*) of gmm_em_iter / gmm_loglik (diagonal) and of
// gmm_kmeans_iter; the launchers dispatch on these
int em_diag_path(int D, int G, int prec);
int kmeans_path(int D, int G, int prec);
hipError_t launch_kmeans_fast(const float* X, int64_t N, int D, int64_t ldx, int G, int dist,
                              const double* gvar, float var_floor, float* means, float* dcovs,
                              float* hefts, int64_t* counts, int32_t* assign, double* inertia,
                              int64_t* n_recomputed, int32_t* dev_status, const Workspace& w,
                              hipStream_t st, int prec);

hipError_t launch_kmeans(const float* X, int64_t N, int D, int64_t ldx, int G, int dist,
                         const double* gvar, float var_floor, float* means, float* dcovs,
                         float* hefts, int64_t* counts, int32_t* assign, double* inertia,
                         int prec, int64_t* n_recomputed, int32_t* dev_status, const Workspace& w,
                         hipStream_t st);

hipError_t launch_log_p_gaussian(const float* X, int64_t N, int D, int64_t ldx, int g,
                                 const float* means, const float* dcovs, double* mean_out,
                                 float* per_sample, int32_t* dev_status, const Workspace& w,
                                 hipStream_t st);

hipError_t launch_seed_means(const float* X, int64_t N, int D, int64_t ldx, int G, int mode,
                             const double* gvar, float var_floor, int64_t first,
                             const int64_t* idx, float* means, int32_t* dev_status,
                             const Workspace& w, hipStream_t st);

hipError_t launch_assign(const float* X, int64_t N, int D, int64_t ldx, int G, int mode,
                         const float* hefts, const float* means, const float* dcovs,
                         int32_t* assign, int64_t* hist, int32_t* dev_status, const Workspace& w,
                         hipStream_t st);

}  // namespace gmm
