// Trilinear sampling of a scalar image at p = x + T(x) with its analytic
// gradient: the image side of the SSD registration step.
//
// p is formed in FP32 (the precision that decides the cell); corners on voxel
// centres, p clamped to [0, n-1]; at an exact integer p the cell [p, p+1] is
// used; a coordinate on or beyond the border (p <= 0 or p >= n-1) gets zero
// gradient.
#pragma once

#include "bsi_device.h"

namespace bsi {

struct Axis {
  int i0, i1;
  float f;
  float in;  // 1 where p is strictly inside (0, n-1), else 0
};

__device__ __forceinline__ Axis sample_axis(float p, int n) {
  Axis a;
  const float top = (float)(n - 1);
  a.in = (p > 0.f && p < top) ? 1.f : 0.f;
  const float pc = fminf(fmaxf(p, 0.f), top);  // NaN -> 0
  int i = (int)floorf(pc);
  i = min(i, n >= 2 ? n - 2 : 0);
  a.i0 = i;
  a.i1 = min(i + 1, n - 1);
  a.f = n >= 2 ? pc - (float)i : 0.f;
  return a;
}

// Two consecutive floats, 4-byte aligned.
struct __attribute__((packed, aligned(4))) F2 {
  float x, y;
};
__device__ __forceinline__ F2 ldf2(const float* p) { return *reinterpret_cast<const F2*>(p); }

struct Sample {
  float w;            // interpolated value
  float gx, gy, gz;   // dW/dp, masked at the border
};

// The sample in two halves, so that a caller can issue the loads of one
// sample before it finishes the previous one: trilinear_load forms the cell
// and loads its 8 corners, trilinear_finish interpolates.
struct SampleIn {
  float c000, c001, c010, c011, c100, c101, c110, c111;  // corners, x fastest
  float fx, fy, fz;                                      // offsets in the cell
  float inx, iny, inz;                                   // 1 strictly inside, else 0
};

// Pairs: 1 when the caller guarantees nx >= 2 (x-neighbours as one 8-byte
// load, no branch), 0 when nx == 1, -1 to test nx here.
template <int Pairs = -1>
__device__ __forceinline__ SampleIn trilinear_load(const float* __restrict__ img, int nx, int ny, int nz, float px,
                                                   float py, float pz) {
  const Axis ax = sample_axis(px, nx), ay = sample_axis(py, ny), az = sample_axis(pz, nz);
  const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
  const float* p00 = img + az.i0 * sz + ay.i0 * sy;
  const float* p01 = img + az.i0 * sz + ay.i1 * sy;
  const float* p10 = img + az.i1 * sz + ay.i0 * sy;
  const float* p11 = img + az.i1 * sz + ay.i1 * sy;
  SampleIn s;
  if (Pairs == 1 || (Pairs == -1 && nx >= 2)) {
    // i1 = i0 + 1: each pair of x-neighbours is one 8-byte load
    const F2 q00 = ldf2(p00 + ax.i0), q01 = ldf2(p01 + ax.i0);
    const F2 q10 = ldf2(p10 + ax.i0), q11 = ldf2(p11 + ax.i0);
    s.c000 = q00.x, s.c001 = q00.y, s.c010 = q01.x, s.c011 = q01.y;
    s.c100 = q10.x, s.c101 = q10.y, s.c110 = q11.x, s.c111 = q11.y;
  } else {
    s.c000 = s.c001 = p00[0];
    s.c010 = s.c011 = p01[0];
    s.c100 = s.c101 = p10[0];
    s.c110 = s.c111 = p11[0];
  }
  s.fx = ax.f, s.fy = ay.f, s.fz = az.f;
  s.inx = ax.in, s.iny = ay.in, s.inz = az.in;
  return s;
}

__device__ __forceinline__ Sample trilinear_finish(const SampleIn& c) {
  const float fx = c.fx, fy = c.fy, fz = c.fz;
  // interpolate along x, then y, then z
  const float x00 = fmaf(fx, c.c001 - c.c000, c.c000), x01 = fmaf(fx, c.c011 - c.c010, c.c010);
  const float x10 = fmaf(fx, c.c101 - c.c100, c.c100), x11 = fmaf(fx, c.c111 - c.c110, c.c110);
  const float y0 = fmaf(fy, x01 - x00, x00), y1 = fmaf(fy, x11 - x10, x10);
  Sample s;
  s.w = fmaf(fz, y1 - y0, y0);
  // analytic derivatives of the trilinear form
  const float dx00 = c.c001 - c.c000, dx01 = c.c011 - c.c010, dx10 = c.c101 - c.c100, dx11 = c.c111 - c.c110;
  const float dx0 = fmaf(fy, dx01 - dx00, dx00), dx1 = fmaf(fy, dx11 - dx10, dx10);
  s.gx = fmaf(fz, dx1 - dx0, dx0) * c.inx;
  s.gy = fmaf(fz, (x11 - x10) - (x01 - x00), x01 - x00) * c.iny;
  s.gz = (y1 - y0) * c.inz;
  return s;
}

__device__ __forceinline__ Sample trilinear(const float* __restrict__ img, int nx, int ny, int nz, float px, float py,
                                            float pz) {
  return trilinear_finish(trilinear_load(img, nx, ny, nz, px, py, pz));
}

}  // namespace bsi
