// Basis look-up tables at every in-tile offset of every spacing: B0..B3, and
// the weights of the lerp form of Sec. 3.3 / App. B,
//   h0 = B1 / (B0 + B1),  h1 = B3 / (B2 + B3),  g1 = B2 + B3
// (both denominators are at least 1/6).
//
// The grid is aligned to the voxels, so the weights of Eq. 1 depend only on
// the offset o = x mod d within a tile (Sec. 3.4 stores them in look-up
// tables).  They are evaluated here once, in FP64 on the host, rounded to FP32,
// and kept in a static device array for the life of the process, so every
// kernel and every launch reads the same weights.
#include <mutex>

#include "bsi_internal.h"

namespace bsi {

// The basis table, followed by the same rows rotated for the adjoint's
// fixed accumulator slots: row (d, o, ph)[k] = B_((k - ph) & 3)(o/d).
static __device__ float g_lut[kLutFloats + kLutRotFloats];
static __device__ float g_lerp_lut[kLutFloats];  // rows (h0, h1, g1, 0)

namespace {

std::mutex g_lut_mutex;
constexpr int kMaxDevices = 64;
const float* g_lut_ptr[kMaxDevices] = {};
const float* g_lerp_ptr[kMaxDevices] = {};

// Uniform cubic B-spline basis (Rueckert et al. 1999) at u in [0, 1).
void basis(double u, double b[4]) {
  const double v = 1.0 - u, u2 = u * u, u3 = u2 * u;
  b[0] = v * v * v / 6.0;
  b[1] = (3.0 * u3 - 6.0 * u2 + 4.0) / 6.0;
  b[2] = (-3.0 * u3 + 3.0 * u2 + 3.0 * u + 1.0) / 6.0;
  b[3] = u3 / 6.0;
}

// Fill the tables on the host (FP64, rounded once to FP32).
void fill_tables(float* basis_tab, float* lerp_tab) {
  for (int d = 1; d <= kMaxSpacing; ++d)
    for (int o = 0; o < d; ++o) {
      double b[4];
      basis((double)o / (double)d, b);
      float* row = basis_tab + 4 * ((d * (d - 1)) / 2 + o);
      for (int l = 0; l < 4; ++l) row[l] = (float)b[l];
      float* rot = basis_tab + kLutFloats + 16 * ((d * (d - 1)) / 2 + o);
      for (int ph = 0; ph < 4; ++ph)
        for (int k = 0; k < 4; ++k) rot[4 * ph + k] = (float)b[(k - ph) & 3];
      float* lr = lerp_tab + 4 * ((d * (d - 1)) / 2 + o);
      lr[0] = (float)(b[1] / (b[0] + b[1]));
      lr[1] = (float)(b[3] / (b[2] + b[3]));
      lr[2] = (float)(b[2] + b[3]);
      lr[3] = 0.f;
    }
}

int32_t upload(int dev) {
  static float host[kLutFloats + kLutRotFloats], lerp_host[kLutFloats];
  fill_tables(host, lerp_host);
  // Upload with plain blocking copies, then resolve this device's addresses.
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(g_lut), host, sizeof(host), 0, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "uploading the basis table");
  e = hipMemcpyToSymbol(HIP_SYMBOL(g_lerp_lut), lerp_host, sizeof(lerp_host), 0, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "uploading the lerp table");
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_lut));
  if (e != hipSuccess) return hip_fail(e, "resolving the basis table address");
  void* q = nullptr;
  e = hipGetSymbolAddress(&q, HIP_SYMBOL(g_lerp_lut));
  if (e != hipSuccess) return hip_fail(e, "resolving the lerp table address");
  g_lut_ptr[dev] = static_cast<const float*>(p);
  g_lerp_ptr[dev] = static_cast<const float*>(q);
  return BSI_OK;
}

int32_t table_ptr(int dev, bool lerp, const float** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device index out of range for the basis table");
    return BSI_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_lut_mutex);
  if (!g_lut_ptr[dev]) {
    const int32_t rc = upload(dev);
    if (rc) return rc;
  }
  *out = lerp ? g_lerp_ptr[dev] : g_lut_ptr[dev];
  return BSI_OK;
}

}  // namespace

int32_t lut_device_ptr(int dev, const float** out) { return table_ptr(dev, false, out); }

int32_t lerp_lut_device_ptr(int dev, const float** out) { return table_ptr(dev, true, out); }

}  // namespace bsi
