// Device-side building blocks shared by the single-volume and batched kernels.
//
// Every arithmetic step is written with explicit fmaf() in a fixed order and the
// library is compiled with -ffp-contract=off, so one routine gives the same bits
// wherever it is inlined (single-volume launch, batched persistent launch, graph).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bsi {

constexpr int kWave = 64;
constexpr int kMaxSpacing = 64;
// Basis table for every spacing d in [1, kMaxSpacing]: row (d, o) holds
// B0..B3(o/d), the weights of Eq. 1 at in-tile offset o.
constexpr int kLutFloats = 4 * kMaxSpacing * (kMaxSpacing + 1) / 2;
constexpr int kNumXcd = 8;  // MI355X: 8 accelerator complex dies, 32 CUs each

// 12-byte vector of the three displacement components.  Packed with 4-byte
// alignment so one lane moves it with a single global_{load,store}_dwordx3.
struct __attribute__((packed, aligned(4))) F3 {
  float x, y, z;
};

struct VolGeom {
  int32_t nx, ny, nz;  // voxels
  int32_t dx, dy, dz;  // spacing (voxels per tile)
  int32_t gx, gy, gz;  // control points = ceil(n/d) + 3
};

// Brick decomposition of the adjoint (see adjoint.hip).  A pure function of the
// geometry, so the summation order, and thus the bits, depend on the inputs only.
struct AdjGeom {
  VolGeom g;
  int32_t xb, yb, zb;     // brick extent in voxels
  int32_t nbx, nby, nbz;  // bricks per axis
  int32_t cxm, cym, czm;  // partial-window strides (upper bound of a brick window)
};

__device__ __forceinline__ const float* lut_row(const float* lut, int d, int o) {
  return lut + 4 * ((d * (d - 1)) / 2 + o);
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Workgroups are dispatched round-robin over the 8 XCDs (id % 8).  Remap so that
// each XCD receives one contiguous range of logical work items: neighbouring
// items share control points, which then stay in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int id, int n) {
  const int q = n / kNumXcd, r = n % kNumXcd;
  const int xcd = id % kNumXcd, k = id / kNumXcd;
  return xcd * q + (xcd < r ? xcd : r) + k;
}

__device__ __forceinline__ F3 ldf3(const float* p) { return *reinterpret_cast<const F3*>(p); }
__device__ __forceinline__ void stf3(float* p, F3 v) { *reinterpret_cast<F3*>(p) = v; }

// ----------------------------------------------------------------------------
// Forward BSI for one wave: 64 consecutive voxels x0..x0+63 of row y, planes
// z0..z1-1 (x0, y, z0, z1 wave-uniform).
//
// Sum factorisation of Eq. 1, per lane: for control plane cz,
//   Q(cz) = sum_m By_m(v) * (sum_l Bx_l(u) * phi[cz][ty+m][tx+l])
// and for each voxel plane z of tile tz,
//   T = sum_n Bz_n(w) * Q(tz+n).
// Q is kept for a rolling window of 4 planes in registers, so each control
// plane is contracted once per row and reused by the dz voxel planes of each of
// the 4 tiles that read it.  The raw control points of the next plane are
// prefetched while the current tile is written.  Each voxel is one 12-byte
// store, so a wave writes 768 contiguous bytes per plane.
// ----------------------------------------------------------------------------
__device__ __forceinline__ F3 fwd_contract(const F3 (&r)[16], float bx0, float bx1, float bx2,
                                           float bx3, float by0, float by1, float by2, float by3) {
  F3 row[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const F3 a = r[4 * m], b = r[4 * m + 1], c = r[4 * m + 2], d = r[4 * m + 3];
    row[m].x = fmaf(bx3, d.x, fmaf(bx2, c.x, fmaf(bx1, b.x, bx0 * a.x)));
    row[m].y = fmaf(bx3, d.y, fmaf(bx2, c.y, fmaf(bx1, b.y, bx0 * a.y)));
    row[m].z = fmaf(bx3, d.z, fmaf(bx2, c.z, fmaf(bx1, b.z, bx0 * a.z)));
  }
  F3 q;
  q.x = fmaf(by3, row[3].x, fmaf(by2, row[2].x, fmaf(by1, row[1].x, by0 * row[0].x)));
  q.y = fmaf(by3, row[3].y, fmaf(by2, row[2].y, fmaf(by1, row[1].y, by0 * row[0].y)));
  q.z = fmaf(by3, row[3].z, fmaf(by2, row[2].z, fmaf(by1, row[1].z, by0 * row[0].z)));
  return q;
}

__device__ __forceinline__ void fwd_load_plane(const float* __restrict__ base, size_t row_stride,
                                               F3 (&r)[16]) {
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int l = 0; l < 4; ++l) r[4 * m + l] = ldf3(base + m * row_stride + 3 * l);
}

__device__ __forceinline__ void fwd_wave(const float* __restrict__ grid, float* __restrict__ field,
                                         const VolGeom& g, const float* __restrict__ lut, int x0,
                                         int y, int z0, int z1, int lane) {
  const int x = x0 + lane;
  const bool active = x < g.nx;
  const int xc = active ? x : g.nx - 1;  // idle lanes read a valid column, store nothing
  const int tx = xc / g.dx;
  const int ox = xc - tx * g.dx;
  const float* wx = lut_row(lut, g.dx, ox);
  const float bx0 = wx[0], bx1 = wx[1], bx2 = wx[2], bx3 = wx[3];
  const int ty = y / g.dy;
  const int oy = y - ty * g.dy;
  const float* wy = lut_row(lut, g.dy, oy);
  const float by0 = wy[0], by1 = wy[1], by2 = wy[2], by3 = wy[3];

  const size_t row_stride = (size_t)g.gx * 3;
  const size_t plane_stride = (size_t)g.gy * row_stride;
  const float* gbase = grid + (size_t)ty * row_stride + (size_t)tx * 3;

  int tz = z0 / g.dz;
  int oz = z0 - tz * g.dz;
  F3 raw[16];
  fwd_load_plane(gbase + (size_t)tz * plane_stride, row_stride, raw);
  F3 q0 = fwd_contract(raw, bx0, bx1, bx2, bx3, by0, by1, by2, by3);
  fwd_load_plane(gbase + (size_t)(tz + 1) * plane_stride, row_stride, raw);
  F3 q1 = fwd_contract(raw, bx0, bx1, bx2, bx3, by0, by1, by2, by3);
  fwd_load_plane(gbase + (size_t)(tz + 2) * plane_stride, row_stride, raw);
  F3 q2 = fwd_contract(raw, bx0, bx1, bx2, bx3, by0, by1, by2, by3);
  fwd_load_plane(gbase + (size_t)(tz + 3) * plane_stride, row_stride, raw);

  const size_t zstride = (size_t)g.ny * g.nx * 3;
  float* out = field + (((size_t)z0 * g.ny + y) * g.nx + x) * 3;
  int z = z0;
  for (;;) {
    const F3 q3 = fwd_contract(raw, bx0, bx1, bx2, bx3, by0, by1, by2, by3);
    const int left = z1 - z;
    const int oend = (g.dz - oz < left) ? g.dz : oz + left;
    // Another tile follows inside this range: prefetch its new plane (tz + 4 is
    // then at most ceil(nz/dz) + 2 = gz - 1, in bounds).
    if (g.dz - oz < left) fwd_load_plane(gbase + (size_t)(tz + 4) * plane_stride, row_stride, raw);
    for (; oz < oend; ++oz, ++z) {
      const float* wz = lut_row(lut, g.dz, oz);
      const float w0 = wz[0], w1 = wz[1], w2 = wz[2], w3 = wz[3];
      F3 t;
      t.x = fmaf(w3, q3.x, fmaf(w2, q2.x, fmaf(w1, q1.x, w0 * q0.x)));
      t.y = fmaf(w3, q3.y, fmaf(w2, q2.y, fmaf(w1, q1.y, w0 * q0.y)));
      t.z = fmaf(w3, q3.z, fmaf(w2, q2.z, fmaf(w1, q1.z, w0 * q0.z)));
      if (active) stf3(out, t);
      out += zstride;
    }
    if (z >= z1) break;
    oz = 0;
    ++tz;
    q0 = q1;
    q1 = q2;
    q2 = q3;
  }
}

}  // namespace bsi
