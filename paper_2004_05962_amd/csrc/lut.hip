// Basis look-up table: B0..B3 at every in-tile offset of every spacing.
//
// The grid is aligned to the voxels, so the weights of Eq. 1 depend only on
// the offset o = x mod d within a tile (Sec. 3.4 stores them in look-up
// tables).  They are evaluated here once, in FP64 on the host, rounded to FP32,
// and kept in a static device array for the life of the process, so every
// kernel and every launch reads the same weights.
#include <mutex>

#include "bsi_internal.h"

namespace bsi {

static __device__ float g_lut[kLutFloats];

namespace {

std::mutex g_lut_mutex;
constexpr int kMaxDevices = 64;
const float* g_lut_ptr[kMaxDevices] = {};

// Uniform cubic B-spline basis (Rueckert et al. 1999) at u in [0, 1).
void basis(double u, double b[4]) {
  const double v = 1.0 - u, u2 = u * u, u3 = u2 * u;
  b[0] = v * v * v / 6.0;
  b[1] = (3.0 * u3 - 6.0 * u2 + 4.0) / 6.0;
  b[2] = (-3.0 * u3 + 3.0 * u2 + 3.0 * u + 1.0) / 6.0;
  b[3] = u3 / 6.0;
}

}  // namespace

int32_t lut_device_ptr(int dev, const float** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device index out of range for the basis table");
    return BSI_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_lut_mutex);
  if (!g_lut_ptr[dev]) {
    static float host[kLutFloats];
    for (int d = 1; d <= kMaxSpacing; ++d)
      for (int o = 0; o < d; ++o) {
        double b[4];
        basis((double)o / (double)d, b);
        float* row = host + 4 * ((d * (d - 1)) / 2 + o);
        for (int l = 0; l < 4; ++l) row[l] = (float)b[l];
      }
    // Upload with a plain blocking copy, then resolve this device's address.
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(g_lut), host, sizeof(host), 0, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "uploading the basis table");
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_lut));
    if (e != hipSuccess) return hip_fail(e, "resolving the basis table address");
    g_lut_ptr[dev] = static_cast<const float*>(p);
  }
  *out = g_lut_ptr[dev];
  return BSI_OK;
}

}  // namespace bsi
