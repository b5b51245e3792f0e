// The adjoint without a workspace argument and without any allocation, for
// callers that cannot allocate device memory: code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc.
//
// The adjoint's partials (what bsi_adjoint keeps in the caller's workspace) go
// to `scratch`, a static device array of BSI_ADJOINT_NOALLOC_MAX_BYTES, which
// every GPU the library runs on holds until the process ends.  All calls on
// one GPU share that GPU's array: calls that may overlap on one GPU (several
// streams or host threads) race on it, and the caller must order them.
// Nothing needs clearing between calls: pass 1 writes every partial that
// pass 2 reads.
#include <mutex>
#include <string>

#include "bsi_internal.h"

namespace bsi {

constexpr size_t kScratchBytes = BSI_ADJOINT_NOALLOC_MAX_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mutex;
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};

// This device's address of `scratch`, resolved once per device with that
// device current.  In host code the array's name is a host-side stand-in, not
// a device address: kernels take this pointer instead.
int32_t scratch_ptr(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device index out of range for the scratch array");
    return BSI_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "resolving the scratch array's device address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return BSI_OK;
}

}  // namespace
}  // namespace bsi

using namespace bsi;

extern "C" {

int32_t bsi_adjoint_noalloc(const float* dfield, const int32_t dims[3], const int32_t spacing[3],
                            float* grid_grad, hipStream_t stream) {
  clear_error();
  VolGeom g;
  int32_t rc = make_geom(dims, spacing, &g);
  if (rc) return rc;
  if (!dfield) {
    set_error("dfield must be a non-null device pointer");
    return BSI_ERR_INVALID_ARG;
  }
  if (!grid_grad) {
    set_error("grid_grad must be a non-null device pointer");
    return BSI_ERR_INVALID_ARG;
  }
  const AdjGeom a = make_adj_geom(g);
  const size_t need = adj_workspace_bytes(a);
  if (need > kScratchBytes) {
    set_error("bsi_adjoint_noalloc: this geometry needs " + std::to_string(need) +
              " bytes of scratch, more than its fixed " + std::to_string(kScratchBytes) +
              "; use bsi_adjoint with a workspace");
    return BSI_ERR_UNSUPPORTED;
  }
  int dev = 0;
  if ((rc = current_device(&dev))) return rc;
  const float* lut = nullptr;
  if ((rc = lut_device_ptr(dev, &lut))) return rc;
  void* ws = nullptr;
  if ((rc = scratch_ptr(dev, &ws))) return rc;
  const hipError_t e = launch_adjoint(dfield, grid_grad, a, lut, static_cast<float*>(ws), stream);
  return e == hipSuccess ? BSI_OK : hip_fail(e, "launching the adjoint kernels");
}

}  // extern "C"
