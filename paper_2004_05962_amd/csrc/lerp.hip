// Forward BSI in the lerp form of Sec. 3.3 / App. B: an ablation of the
// paper's own evaluation against the sum-factorised kernel (forward.hip).
//
// Per axis the four-tap B-spline filter is rewritten as three linear
// interpolations,
//   sum_l B_l p_l = lerp(lerp(p0, p1, h0), lerp(p2, p3, h1), g1),
//   h0 = B1 / (B0 + B1),  h1 = B3 / (B2 + B3),  g1 = B2 + B3,
// and, as in the paper, applied per voxel to the whole 4x4x4 window: one
// trilinear interpolation of each of the 8 2x2x2 sub-cubes with the h weights,
// then one trilinear interpolation of the 8 results with the g1 weights, i.e.
// 9 x 7 = 63 lerps (126 vector operations) per component and voxel, with no
// sharing between voxels.  The sum-factorised kernel shares the x- and
// y-contractions of a control plane across the voxel planes of a tile and
// needs about 22 FMA per voxel instead.
//
// Layout as the forward: a workgroup is 4 rows of one 64-voxel x-strip (lane
// = voxel) over a chunk of z; the control points of the 4 planes a tile reads
// sit in LDS (a ring of 5 plane slots: the next plane is staged while the
// current tile is evaluated), so each voxel's 64 points are LDS reads.
#include "bsi_internal.h"

namespace bsi {

namespace {

constexpr int kLerpSlots = 5;

struct LerpSmem {
  float ring[kLerpSlots][fwd_loads<3>() * kFwdThreads];
};

__device__ __forceinline__ float lerp(float a, float b, float t) { return fmaf(t, b - a, a); }

struct Axis3 {
  float h0, h1, g1;
};

__device__ __forceinline__ Axis3 lerp_weights(const float* __restrict__ lerp_lut, int d, int o) {
  const float* w = lut_row(lerp_lut, d, o);
  return Axis3{w[0], w[1], w[2]};
}

// One component of the window's lerp-form value.  pl[n] points at this lane's
// window origin in the slot of control plane tz + n; c selects the component.
__device__ __forceinline__ float ttli(const float* const (&pl)[4], int c, const Axis3& wx, const Axis3& wy,
                                     const Axis3& wz) {
  float sub[2][2][2];
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const float hx = i ? wx.h1 : wx.h0, hy = j ? wy.h1 : wy.h0, hz = k ? wz.h1 : wz.h0;
        float zz[2];
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          const float* p = pl[2 * k + n];
          float yy[2];
#pragma unroll
          for (int m = 0; m < 2; ++m) {
            const float* q = p + (2 * j + m) * fwd_pitch<3>() + (2 * i) * 3 + c;
            yy[m] = lerp(q[0], q[3], hx);
          }
          zz[n] = lerp(yy[0], yy[1], hy);
        }
        sub[k][j][i] = lerp(zz[0], zz[1], hz);
      }
  const float y00 = lerp(sub[0][0][0], sub[0][0][1], wx.g1), y01 = lerp(sub[0][1][0], sub[0][1][1], wx.g1);
  const float y10 = lerp(sub[1][0][0], sub[1][0][1], wx.g1), y11 = lerp(sub[1][1][0], sub[1][1][1], wx.g1);
  return lerp(lerp(y00, y01, wy.g1), lerp(y10, y11, wy.g1), wz.g1);
}

__global__ __launch_bounds__(kFwdThreads) void lerp_kernel(const float* __restrict__ grid,
                                                            float* __restrict__ field, VolGeom g,
                                                            const float* __restrict__ lerp_lut, FwdLaunch L) {
  __shared__ LerpSmem sm;
  int id = xcd_remap(blockIdx.x, gridDim.x);
  const int bxi = id % L.nbx;
  id /= L.nbx;
  const int byi = id % L.nby;
  const int bzi = id / L.nby;
  const int tid = threadIdx.x;
  const int x0 = bxi * kWave, y0 = byi * kFwdRows;
  const int z0 = bzi * L.zchunk, z1 = min(g.nz, z0 + L.zchunk);
  const int lane = tid & (kWave - 1);
  const int wave = uniform(tid / kWave);
  const int cx0 = x0 / g.dx;
  const int ncx = (min(x0 + kWave, g.nx) - 1) / g.dx - cx0 + 4;
  const int cy0 = y0 / g.dy;
  const int ncy = (min(y0 + kFwdRows, g.ny) - 1) / g.dy - cy0 + 4;
  const FwdStage<3> map = fwd_stage_map<3>(g, cx0, ncx, cy0, ncy, tid);

  const int x = x0 + lane, y = y0 + wave;
  const bool active = x < g.nx && y < g.ny;
  const int xc = min(x, g.nx - 1), yc = min(y, g.ny - 1);
  const int tx = xc / g.dx, ty = yc / g.dy;
  const Axis3 wx = lerp_weights(lerp_lut, g.dx, xc - tx * g.dx);
  const Axis3 wy = lerp_weights(lerp_lut, g.dy, yc - ty * g.dy);
  const int base = (ty - cy0) * fwd_pitch<3>() + (tx - cx0) * 3;

  int tz = z0 / g.dz;
  int oz = z0 - tz * g.dz;
  float r[fwd_loads<3>()];
  // planes tz .. tz+3 in slots (tz + n) % 5
#pragma unroll 1
  for (int n = 0; n < 4; ++n) {
    fwd_fetch<3>(grid, g, map, tz + n, r);
    fwd_stage<3>(sm.ring[(tz + n) % kLerpSlots], tid, r);
  }
  __syncthreads();

  const size_t zstride = (size_t)g.ny * g.nx * 3;
  float* out = field + (((size_t)z0 * g.ny + yc) * g.nx + xc) * 3;
  int z = z0;
  for (;;) {
    const int left = z1 - z;
    const bool more = g.dz - oz < left;  // another tile follows inside this range
    // its new plane tz + 4 is then at most ceil(nz/dz) + 2 = gz - 1: in bounds
    if (more) fwd_fetch<3>(grid, g, map, tz + 4, r);
    const float* pl[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) pl[n] = sm.ring[(tz + n) % kLerpSlots] + base;
    const int oend = more ? g.dz : oz + left;
    for (; oz < oend; ++oz, ++z) {
      const Axis3 wz = lerp_weights(lerp_lut, g.dz, oz);
      // one component at a time (its 64 window values in flight, not 192)
      float t[3] = {0.f, 0.f, 0.f};
#pragma unroll 1
      for (int c = 0; c < 3; ++c) {
        const float v = ttli(pl, c, wx, wy, wz);
        t[0] = c == 0 ? v : t[0];
        t[1] = c == 1 ? v : t[1];
        t[2] = c == 2 ? v : t[2];
      }
      if (active) fwd_store<3>(out, t);
      out += zstride;
    }
    if (!more) break;
    // plane tz + 4 replaces plane tz - 1 (slot (tz + 4) % 5), which no wave
    // has read since the previous tile's barrier
    fwd_stage<3>(sm.ring[(tz + 4) % kLerpSlots], tid, r);
    __syncthreads();
    oz = 0;
    ++tz;
  }
}

}  // namespace

hipError_t launch_forward_lerp(const float* grid, float* field, const VolGeom& g, const float* lerp_lut,
                               hipStream_t s) {
  const FwdLaunch L = make_fwd_launch(g);
  const long blocks = (long)L.nbx * L.nby * L.nbz;
  hipLaunchKernelGGL(lerp_kernel, dim3((unsigned)blocks), dim3(kFwdThreads), 0, s, grid, field, g, lerp_lut, L);
  return hipGetLastError();
}

}  // namespace bsi
