// Adjoint BSI kernels for one volume: pass 1 (bricks -> partials) and pass 2
// (fixed-order gather per control point).  See adjoint_device.h.
#include "adjoint_device.h"
#include "bsi_internal.h"

namespace bsi {

__global__ __launch_bounds__(kAdjThreads) void adj_pass1_kernel(const float* __restrict__ dfield,
                                                                 float* __restrict__ part, AdjGeom a,
                                                                 const float* __restrict__ lut) {
  __shared__ AdjSmem sm;
  const int nbricks = a.nbx * a.nby * a.nbz;
  const int brick = xcd_remap(blockIdx.x, gridDim.x);
  if (brick >= nbricks) return;  // uniform over the workgroup
  adj_brick(dfield, part, a, lut, brick, sm, threadIdx.x);
}

constexpr int kGatherThreads = 256;

__global__ __launch_bounds__(kGatherThreads) void adj_pass2_kernel(const float* __restrict__ part,
                                                                    float* __restrict__ grad, AdjGeom a) {
  const int64_t n = (int64_t)a.g.gx * a.g.gy * a.g.gz;
  const int64_t i = (int64_t)blockIdx.x * kGatherThreads + threadIdx.x;
  if (i >= n) return;
  const int cx = (int)(i % a.g.gx);
  const int64_t r = i / a.g.gx;
  const int cy = (int)(r % a.g.gy);
  const int cz = (int)(r / a.g.gy);
  stf3(grad + i * 3, adj_gather_point(part, a, cx, cy, cz));
}

AdjGeom make_adj_geom(const VolGeom& g) {
  AdjGeom a;
  a.g = g;
  // Tile-aligned bricks where the spacing divides into the brick bound.
  a.xb = g.dx * (kAdjMaxX / g.dx);  // dx <= 64, so >= 1 tile and <= 64 voxels
  a.yb = g.dy <= kAdjMaxY ? g.dy * (kAdjMaxY / g.dy) : kAdjMaxY;
  a.zb = g.dz * (kAdjTargetZ / g.dz > 0 ? kAdjTargetZ / g.dz : 1);
  a.nbx = (g.nx + a.xb - 1) / a.xb;
  a.nby = (g.ny + a.yb - 1) / a.yb;
  a.nbz = (g.nz + a.zb - 1) / a.zb;
  a.cxm = (a.xb - 1) / g.dx + 5;
  a.cym = (a.yb - 1) / g.dy + 5;
  a.czm = (a.zb - 1) / g.dz + 5;
  return a;
}

size_t adj_workspace_bytes(const AdjGeom& a) {
  return (size_t)a.nbx * a.nby * a.nbz * a.czm * a.cym * a.cxm * 3 * sizeof(float);
}

hipError_t launch_adjoint(const float* dfield, float* grad, const AdjGeom& a, const float* lut,
                          float* part, hipStream_t s) {
  const long nbricks = (long)a.nbx * a.nby * a.nbz;
  hipLaunchKernelGGL(adj_pass1_kernel, dim3((unsigned)nbricks), dim3(kAdjThreads), 0, s, dfield, part,
                     a, lut);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long npts = (long)a.g.gx * a.g.gy * a.g.gz;
  hipLaunchKernelGGL(adj_pass2_kernel, dim3((unsigned)((npts + kGatherThreads - 1) / kGatherThreads)),
                     dim3(kGatherThreads), 0, s, part, grad, a);
  return hipGetLastError();
}

}  // namespace bsi
