// SSD registration step around BSI: trilinear warp, SSD loss + gradient with
// respect to the displacement field, and the gradient-descent update.
//
// p(x) = x + T(x) is formed in FP32 (the precision that decides the cell);
// corners on voxel centres, p clamped to [0, n-1]; at an exact integer p the
// cell [p, p+1] is used; a coordinate on or beyond the border (p <= 0 or
// p >= n-1) gets zero gradient.
#include "bsi_internal.h"
#include "warp_device.h"

namespace bsi {

namespace {

constexpr int kRowThreads = 256;

__global__ __launch_bounds__(kRowThreads) void warp_kernel(const float* __restrict__ field,
                                                            const float* __restrict__ image, VolGeom g,
                                                            float* __restrict__ out, int nbx) {
  const int row = blockIdx.x / nbx;  // row = z * ny + y
  const int x = (blockIdx.x - row * nbx) * kRowThreads + threadIdx.x;
  if (x >= g.nx) return;
  const int z = row / g.ny, y = row - z * g.ny;
  const size_t v = (size_t)row * g.nx + x;
  const F3 t = ldf3(field + v * 3);
  const Sample s = trilinear(image, g.nx, g.ny, g.nz, (float)x + t.x, (float)y + t.y, (float)z + t.z);
  out[v] = s.w;
}

__global__ __launch_bounds__(kRowThreads) void ssd_kernel(const float* __restrict__ field,
                                                           const float* __restrict__ moving,
                                                           const float* __restrict__ fixed, VolGeom g,
                                                           float* __restrict__ dfield,
                                                           float* __restrict__ partials, int nbx) {
  __shared__ float red[kRowThreads];
  const int row = blockIdx.x / nbx;
  const int x = (blockIdx.x - row * nbx) * kRowThreads + threadIdx.x;
  float r2 = 0.f;
  if (x < g.nx) {
    const int z = row / g.ny, y = row - z * g.ny;
    const size_t v = (size_t)row * g.nx + x;
    const F3 t = ldf3(field + v * 3);
    const Sample s = trilinear(moving, g.nx, g.ny, g.nz, (float)x + t.x, (float)y + t.y, (float)z + t.z);
    const float r = s.w - fixed[v];
    r2 = r * r;
    const float two_r = 2.f * r;
    stf3(dfield + v * 3, F3{two_r * s.gx, two_r * s.gy, two_r * s.gz});
  }
  // fixed-order tree reduction of r^2 over the workgroup
  red[threadIdx.x] = r2;
  __syncthreads();
  for (int h = kRowThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

constexpr int kReduceThreads = 1024;

__global__ __launch_bounds__(kReduceThreads) void sum_kernel(const float* __restrict__ partials, long n,
                                                              float* __restrict__ out) {
  __shared__ float red[kReduceThreads];
  float s = 0.f;
  for (long i = threadIdx.x; i < n; i += kReduceThreads) s += partials[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = kReduceThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

constexpr int kAxpyThreads = 256;

__global__ __launch_bounds__(kAxpyThreads) void descent_kernel(float* __restrict__ grid,
                                                                const float* __restrict__ grad, float eta,
                                                                int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kAxpyThreads;
  for (int64_t i = (int64_t)blockIdx.x * kAxpyThreads + threadIdx.x; i < n; i += stride)
    grid[i] = fmaf(-eta, grad[i], grid[i]);
}

int row_blocks(const VolGeom& g) { return (g.nx + kRowThreads - 1) / kRowThreads; }

}  // namespace

size_t ssd_partial_count(const VolGeom& g) { return (size_t)row_blocks(g) * g.ny * g.nz; }

hipError_t launch_warp(const float* field, const float* image, const VolGeom& g, float* out,
                       hipStream_t s) {
  const int nbx = row_blocks(g);
  const long blocks = (long)nbx * g.ny * g.nz;
  hipLaunchKernelGGL(warp_kernel, dim3((unsigned)blocks), dim3(kRowThreads), 0, s, field, image, g, out, nbx);
  return hipGetLastError();
}

hipError_t launch_ssd_grad(const float* field, const float* moving, const float* fixed,
                           const VolGeom& g, float* dfield, float* loss, float* partials,
                           hipStream_t s) {
  const int nbx = row_blocks(g);
  const long blocks = (long)nbx * g.ny * g.nz;
  hipLaunchKernelGGL(ssd_kernel, dim3((unsigned)blocks), dim3(kRowThreads), 0, s, field, moving, fixed, g,
                     dfield, partials, nbx);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sum(partials, blocks, loss, s);
}

hipError_t launch_sum(const float* partials, long n, float* out, hipStream_t s) {
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(kReduceThreads), 0, s, partials, n, out);
  return hipGetLastError();
}

hipError_t launch_descent(float* grid, const float* grad, float eta, int64_t count, hipStream_t s) {
  int64_t blocks = (count + kAxpyThreads - 1) / kAxpyThreads;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(descent_kernel, dim3((unsigned)blocks), dim3(kAxpyThreads), 0, s, grid, grad, eta, count);
  return hipGetLastError();
}

}  // namespace bsi
