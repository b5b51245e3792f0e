// Adjoint BSI kernels for one volume: pass 1 (bricks -> partials) and pass 2
// (fixed-order gather per control point).  See adjoint_device.h.
#include "adjoint_device.h"
#include "bsi_internal.h"

namespace bsi {

template <int DX>
__global__ __launch_bounds__(kAdjThreads) __attribute__((amdgpu_waves_per_eu(BSI_ADJ_WPE))) void adj_pass1_kernel(
    const float* __restrict__ dfield, float* __restrict__ part, AdjGeom a, const float* __restrict__ lut) {
  __shared__ AdjSmem<DX> sm;
  const int nbricks = a.x.nb * a.y.nb * a.z.nb;
  const int brick = xcd_remap(blockIdx.x, gridDim.x);
  if (brick >= nbricks) return;  // uniform over the workgroup
  if (adj_stage_all(a))  // uniform: a function of the geometry
    adj_brick<DX, true, true>(dfield, part, a, lut, brick, sm, threadIdx.x);
  else
    adj_brick<DX, true, false>(dfield, part, a, lut, brick, sm, threadIdx.x);
}

__global__ __launch_bounds__(kGatherThreads) void adj_pass2_kernel(const float* __restrict__ part,
                                                                    float* __restrict__ grad, AdjGeom a) {
  adj_gather_block(part, grad, a, blockIdx.x, threadIdx.x);
}

namespace {
// k units of u voxels per brick.
AdjAxis make_axis(int n, int d, int u, int k) {
  AdjAxis a;
  a.u = u;
  a.U = (n + u - 1) / u;
  a.k = k < a.U ? k : a.U;
  a.nb = (a.U + a.k - 1) / a.k;
  a.w = a.k * u;
  // a brick of k whole tiles meets k + 3 control points; a brick of rows that
  // may start inside a tile meets at most (w - 1)/d + 2 tiles, plus 3
  a.cm = u == d ? a.k + 3 : (a.w - 1) / d + 5;
  return a;
}
}  // namespace

#ifndef BSI_ADJ_FIT
#define BSI_ADJ_FIT 1
#endif

// Bricks of pass 1: kAdjBX voxels (one per lane) by kAdjBY rows by whole
// z-tiles, about kAdjTargetZ planes deep (at least one tile).  Where fewer
// tiles, but at least half as many, let a brick's whole window of partials fit
// the LDS stage, the brick takes that depth: its partials are then stored
// after its last load instead of one plane at a time between its loads.
AdjGeom make_adj_geom(const VolGeom& g) {
  AdjGeom a;
  a.g = g;
  a.x = make_axis(g.nx, g.dx, 1, kAdjBX);
  a.y = make_axis(g.ny, g.dy, 1, kAdjBY);
  int kz = kAdjTargetZ / g.dz > 0 ? kAdjTargetZ / g.dz : 1;
  const int kfit = kAdjStageFloats / (a.y.cm * a.x.cm * 3) - 3;  // deepest brick whose window fits
  if (BSI_ADJ_FIT == 1 && kfit < kz && 2 * kfit >= kz) kz = kfit;
  if (BSI_ADJ_FIT == 2 && kfit < kz && kfit >= 1) kz = kfit;
  a.z = make_axis(g.nz, g.dz, g.dz, kz);
  return a;
}

size_t adj_workspace_bytes(const AdjGeom& a) {
  return (size_t)a.x.nb * a.y.nb * a.z.nb * a.x.cm * a.y.cm * a.z.cm * 3 * sizeof(float);
}

hipError_t launch_adjoint_partials(const float* dfield, const AdjGeom& a, const float* lut, float* part,
                                  hipStream_t s) {
  const long nbricks = (long)a.x.nb * a.y.nb * a.z.nb;
  const dim3 grid((unsigned)nbricks), block(kAdjThreads);
  static_assert(kAdjMaxDX == 12, "one case per specialised spacing");
  switch (a.g.dx) {
    case 1: hipLaunchKernelGGL(adj_pass1_kernel<1>, grid, block, 0, s, dfield, part, a, lut); break;
    case 2: hipLaunchKernelGGL(adj_pass1_kernel<2>, grid, block, 0, s, dfield, part, a, lut); break;
    case 3: hipLaunchKernelGGL(adj_pass1_kernel<3>, grid, block, 0, s, dfield, part, a, lut); break;
    case 4: hipLaunchKernelGGL(adj_pass1_kernel<4>, grid, block, 0, s, dfield, part, a, lut); break;
    case 5: hipLaunchKernelGGL(adj_pass1_kernel<5>, grid, block, 0, s, dfield, part, a, lut); break;
    case 6: hipLaunchKernelGGL(adj_pass1_kernel<6>, grid, block, 0, s, dfield, part, a, lut); break;
    case 7: hipLaunchKernelGGL(adj_pass1_kernel<7>, grid, block, 0, s, dfield, part, a, lut); break;
    case 8: hipLaunchKernelGGL(adj_pass1_kernel<8>, grid, block, 0, s, dfield, part, a, lut); break;
    case 9: hipLaunchKernelGGL(adj_pass1_kernel<9>, grid, block, 0, s, dfield, part, a, lut); break;
    case 10: hipLaunchKernelGGL(adj_pass1_kernel<10>, grid, block, 0, s, dfield, part, a, lut); break;
    case 11: hipLaunchKernelGGL(adj_pass1_kernel<11>, grid, block, 0, s, dfield, part, a, lut); break;
    case 12: hipLaunchKernelGGL(adj_pass1_kernel<12>, grid, block, 0, s, dfield, part, a, lut); break;
    default: hipLaunchKernelGGL(adj_pass1_kernel<0>, grid, block, 0, s, dfield, part, a, lut); break;
  }
  return hipGetLastError();
}

hipError_t launch_adjoint_reduce(const float* part, float* grad, const AdjGeom& a, hipStream_t s) {
  const int64_t nblk = adj_gather_blocks(a.g);
  if (nblk >= ((int64_t)1 << 31)) return hipErrorInvalidConfiguration;  // a field far beyond device memory
  hipLaunchKernelGGL(adj_pass2_kernel, dim3((unsigned)nblk), dim3(kGatherThreads), 0, s, part, grad, a);
  return hipGetLastError();
}

hipError_t launch_adjoint(const float* dfield, float* grad, const AdjGeom& a, const float* lut,
                          float* part, hipStream_t s) {
  hipError_t e = launch_adjoint_partials(dfield, a, lut, part, s);
  if (e != hipSuccess) return e;
  return launch_adjoint_reduce(part, grad, a, s);
}

}  // namespace bsi
