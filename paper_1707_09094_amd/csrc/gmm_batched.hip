// gmm_batched.hip -- shared pieces of the many-model entry points: the
// on-device work list (a model's samples cut into consecutive items of
// `chunk` samples, grouped by the model's component-block count, largest
// first) and per-model status reset.
// Building the list on the device keeps an iteration free of host copies,
// so a sequence of batched calls can be captured into a graph.
#include "gmm_internal.hpp"

namespace gmm {

namespace {

// One workgroup.  mitems[m] = (first item, item count).  Items are grouped
// by the model's block count RB = ceil(G / 16), largest first: an item's cost
// grows with RB, so the persistent grid takes the longest items first and
// neighbouring workgroups run the same kernel variant; models keep index
// order within a group and a model's items stay consecutive.  A model whose
// descriptor is unusable gets no items; if the descriptors ask for more items
// than the host sized (`cap`), no model gets any.
// Exclusive prefix sum over the 1024 threads of the workgroup (Hillis-Steele
// in LDS, exact in 64-bit integers); *total receives the sum.  Every thread
// must call it.
__device__ long long block_scan_excl(long long v, long long* sh, long long* total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const long long t = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += t;
    __syncthreads();
  }
  const long long incl = sh[tid];
  *total = sh[1023];
  __syncthreads();  // sh is reused by the next call
  return incl - v;
}

__global__ void __launch_bounds__(1024) k_batch_plan(const gmm_model_desc* models, int n_models,
                                                     int Gmax, int64_t chunk, int cap,
                                                     BatchItemDev* items, int2* mitems,
                                                     int* n_items) {
  __shared__ long long scan_sh[1024];
  const int tid = threadIdx.x;
  // per-thread contiguous block of models
  const int per = (n_models + 1023) / 1024;
  const int m0 = min(n_models, tid * per), m1 = min(n_models, m0 + per);
  auto count = [&](int m) -> int64_t {
    return batch_desc_ok(models[m], Gmax) ? (models[m].N + chunk - 1) / chunk : 0;
  };
  int64_t local = 0;
  for (int m = m0; m < m1; ++m) local += count(m);
  long long all = 0;
  (void)block_scan_excl((long long)local, scan_sh, &all);
  const bool ovf = all > cap;
  if (tid == 0) *n_items = ovf ? 0 : (int)all;
  for (int m = m0; m < m1; ++m) {
    const gmm_model_desc& md = models[m];
    const bool ok = batch_desc_ok(md, Gmax) && !ovf;
    if (!ok) mitems[m] = make_int2(0, 0);
    if (md.dev_status) *md.dev_status = ok ? 0 : GMM_DEV_BADDESC;
  }
  if (ovf) return;
  const int RBmax = (Gmax + 15) / 16;
  int run = 0;  // items of the groups placed so far
  for (int rb = RBmax; rb >= 1; --rb) {
    auto in_group = [&](int m) { return (models[m].G + 15) / 16 == rb; };
    int mine = 0;
    for (int m = m0; m < m1; ++m)
      if (in_group(m)) mine += (int)count(m);
    long long grp = 0;
    int first = run + (int)block_scan_excl(mine, scan_sh, &grp);
    for (int m = m0; m < m1; ++m) {
      if (!in_group(m)) continue;
      const gmm_model_desc& md = models[m];
      const int cnt = (int)count(m);
      mitems[m] = make_int2(first, cnt);
      for (int k = 0; k < cnt; ++k) {
        BatchItemDev it;
        it.model = m;
        it.first_of_model = first;
        it.i0 = (int64_t)k * chunk;
        it.i1 = min(md.N, (int64_t)(k + 1) * chunk);
        items[first + k] = it;
      }
      first += cnt;
    }
    run += (int)grp;
  }
}

}  // namespace

int batch_item_count(int32_t n_models, const int64_t* Ns, int64_t chunk) {
  int64_t tot = 0;
  for (int m = 0; m < n_models; ++m) tot += (Ns[m] + chunk - 1) / chunk;
  return tot > INT32_MAX ? -1 : (int)tot;
}

hipError_t launch_batch_plan(const gmm_model_desc* models, int n_models, int64_t chunk,
                             const BatchWorkspace& bw, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(1024), 0, st, models, n_models, bw.Gmax, chunk,
                     bw.cap, bw.items, bw.mitems, bw.n_items);
  return hipGetLastError();
}

}  // namespace gmm
