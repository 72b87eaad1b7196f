// gmm_noalloc.hip -- gmm_em_iter_noalloc: gmm_em_iter for callers that cannot
// allocate device memory.  Its scratch space is the file-scope device array
// `scratch` (one copy per GPU, allocated when the library's code object is
// loaded on that GPU and held until the process ends).  The array's name is a
// host-side stand-in in host code: the device address of each GPU's copy is
// taken once per device with hipGetSymbolAddress and only that address is
// handed to the kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gmm_internal.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)GMM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (nullptr on error).
void* scratch_ptr() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" int gmm_em_iter_noalloc(const float* X, int64_t N, int32_t D, int64_t ldx, int32_t G,
                                   int32_t cov, float* hefts, float* means, float* covs,
                                   float var_floor, int32_t prec, double* mean_loglik,
                                   int64_t* n_recomputed, int32_t* dev_status,
                                   gmm_stream_t stream) {
  const size_t need = gmm_workspace_bytes(N, D, G, cov, prec);
  if (need == 0 || need > kScratchBytes) return GMM_EINVAL;
  void* ws = scratch_ptr();
  if (!ws) return GMM_EHIP;
  // the same validation, kernels and scratch layout as gmm_em_iter with a
  // workspace of kScratchBytes at the array's device address; no event
  // timing, whatever gmm_profile_enable said
  gmm::ProfSuppress quiet;
  return gmm_em_iter(X, N, D, ldx, G, cov, hefts, means, covs, var_floor, prec, mean_loglik,
                     n_recomputed, dev_status, ws, kScratchBytes, stream);
}
