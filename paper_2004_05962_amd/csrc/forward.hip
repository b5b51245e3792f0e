// Forward BSI kernel (Eq. 1) for one volume: C = 3 for a displacement grid,
// C = 1 for a scalar image (B-spline upsampling).
//
// Workgroup = kFwdRows waves = kFwdRows consecutive rows of one 64-voxel x-strip
// (256 voxels, 4 per lane, for scalar images), over one chunk of z; it runs
// fwd_block (bsi_device.h): per-lane sum factorisation with a rolling window of
// 4 contracted control planes in registers, control points staged per plane in
// LDS, and one coalesced 12-byte store per voxel (16 bytes per 4 scalar voxels).  The field write is the dominant HBM traffic (12 bytes per
// voxel against 12 bytes per control point).
#include "bsi_internal.h"

namespace bsi {

template <int C, class T, bool Edge>
__global__ __launch_bounds__(T::threads) void fwd_kernel(const float* __restrict__ grid, float* __restrict__ field,
                                                          VolGeom g, const float* __restrict__ lut, FwdLaunch L) {
  __shared__ FwdSmem<C, T> sm;
  int id = xcd_remap(blockIdx.x, gridDim.x);
  const int bx = id % L.nbx;
  id /= L.nbx;
  const int by = id % L.nby;
  const int bz = id / L.nby;
  const int z0 = bz * L.zchunk;
  const int z1 = min(g.nz, z0 + L.zchunk);
  fwd_block<C, T, Edge>(grid, field, g, lut, bx * T::width, by * T::rows, z0, z1, sm, threadIdx.x);
}

template <int C, class T, bool Edge>
hipError_t launch_fwd(const float* grid, float* field, const VolGeom& g, const float* lut, hipStream_t s) {
  const FwdLaunch L = make_fwd_launch(g, kFwdTargetBlocks, T::width, T::rows);
  const long blocks = (long)L.nbx * L.nby * L.nbz;
  hipLaunchKernelGGL((fwd_kernel<C, T, Edge>), dim3((unsigned)blocks), dim3(T::threads), 0, s, grid, field, g, lut, L);
  return hipGetLastError();
}

// One span (rows [yb * R, yb * R + R) of plane z) per workgroup, workgroup id =
// z * nyb + yb: ids follow the field's addresses.
template <int C>
__global__ __launch_bounds__(kSpanThreads) void fwd_span_kernel(const float* __restrict__ grid,
                                                                 float* __restrict__ field, VolGeom g,
                                                                 const float* __restrict__ lut, int R, int nyb) {
  extern __shared__ float span_smem[];
  const int z = blockIdx.x / nyb;
  const int yb = blockIdx.x - z * nyb;
  const int y0 = yb * R;
  fwd_span<C>(grid, field, g, lut, z, y0, min(g.ny, y0 + R), span_smem, threadIdx.x);
}

#ifndef BSI_FWD_SPAN_VOXELS
#define BSI_FWD_SPAN_VOXELS 2048
#endif
#ifndef BSI_FWD_SPAN_LDS
#define BSI_FWD_SPAN_LDS 32768
#endif

// Rows per span: the most (up to about BSI_FWD_SPAN_VOXELS voxels) whose LDS
// fits BSI_FWD_SPAN_LDS bytes; 0 when not even one row fits (very wide rows).
int span_rows(const VolGeom& g, int C) {
  int R = BSI_FWD_SPAN_VOXELS / g.nx;
  if (R < 1) R = 1;
  if (R > g.ny) R = g.ny;
  while (R >= 1 && fwd_span_lds(R, g.dy, g.gx, C) > BSI_FWD_SPAN_LDS) --R;
  if (R >= 1 && (double)R * g.nx * C * 4 >= 2147483648.0) return 0;
  return R;
}

template <int C>
hipError_t launch_span(const float* grid, float* field, const VolGeom& g, const float* lut, int R, hipStream_t s) {
  const int nyb = (g.ny + R - 1) / R;
  const long blocks = (long)nyb * g.nz;
  hipLaunchKernelGGL(fwd_span_kernel<C>, dim3((unsigned)blocks), dim3(kSpanThreads),
                     fwd_span_lds(R, g.dy, g.gx, C), s, grid, field, g, lut, R, nyb);
  return hipGetLastError();
}

FwdLaunch make_fwd_launch(const VolGeom& g, long target, int width, int rows) {
  FwdLaunch L;
  L.nbx = (g.nx + width - 1) / width;
  L.nby = (g.ny + rows - 1) / rows;
  // Split z (at tile boundaries) until there are >= target workgroups: enough
  // waves to keep the stores flowing, and no more (each chunk restages the 3
  // control planes before its first tile).  The split does not change the
  // arithmetic of any voxel.
  const int tiles_z = (g.nz + g.dz - 1) / g.dz;
  const long base = (long)L.nbx * L.nby;
  int chunks = (int)((target + base - 1) / base);
  if (chunks > tiles_z) chunks = tiles_z;
  if (chunks < 1) chunks = 1;
  const int tiles_per_chunk = (tiles_z + chunks - 1) / chunks;
  L.zchunk = tiles_per_chunk * g.dz;
  L.nbz = (g.nz + L.zchunk - 1) / L.zchunk;
  return L;
}

// Rows that start on 64-byte boundaries (every one, when nx * 12 bytes and the
// field pointer are multiples of 64) are written whole segment by segment.
// Wider than 256 voxels and with z-tiles of at least 5 planes, a workgroup of
// 2 rows x 8 strips covers 512 voxels of each of its rows (at 512 x 512 x 256,
// spacing 5: 167 against 172 us inside the forward + adjoint step).  Its 16
// waves meet at one barrier per z-tile, which cost more than it gained at
// spacing 3 (0.224 against 0.189 ms).  Other rows take edge stores (fwd_block).
hipError_t launch_forward(const float* grid, float* field, const VolGeom& g, const float* lut,
                          hipStream_t s) {
#if BSI_FWD_SPAN
  {
    const int R = span_rows(g, 3);
    if (R > 0 && (long)((g.ny + R - 1) / R) * g.nz < 0x7fffffffL) return launch_span<3>(grid, field, g, lut, R, s);
  }
#endif
  const bool aligned = (g.nx * 12) % 64 == 0 && reinterpret_cast<uintptr_t>(field) % 64 == 0;
  if (aligned && g.nx > 256 && g.dz >= 5)
    return launch_fwd<3, FwdTile<2, 8, 1>, false>(grid, field, g, lut, s);
  if (aligned) return launch_fwd<3, FwdTileDefault, false>(grid, field, g, lut, s);
  return launch_fwd<3, FwdTileDefault, true>(grid, field, g, lut, s);
}

hipError_t launch_forward_scalar(const float* grid, float* image, const VolGeom& g, const float* lut,
                                 hipStream_t s) {
  // Rows starting on 16-byte boundaries: 4 voxels per lane, one 16-byte store
  // each.  Otherwise one voxel per lane (4 stores per lane would each cover
  // only every fourth dword of the wave's span), with edge stores.
  if (g.nx % 4 == 0 && reinterpret_cast<uintptr_t>(image) % 16 == 0)
    return launch_fwd<1, FwdTile<kFwdRows, 1, 4>, false>(grid, image, g, lut, s);
  return launch_fwd<1, FwdTileDefault, true>(grid, image, g, lut, s);
}

}  // namespace bsi
