// Fused SSD gradient: BSI (Eq. 1) -> trilinear warp -> SSD -> adjoint of Eq. 1
// in one pass over the voxels, so neither the displacement field nor its
// gradient is ever written to memory.  Merging the other FFD steps into BSI is
// the direction the paper's conclusion (Sec. 8) names for further speed-up.
//
//   T(x)      = sum_{l,m,n} Bx_l By_m Bz_n phi                 (Eq. 1)
//   W(x)      = moving(x + T(x))        trilinear, see warp_device.h
//   L         = sum_x (W(x) - fixed(x))^2
//   dL/dphi   = B^T [ 2 (W - fixed) dW/dp ]                    (the adjoint)
//
// Pass 1 keeps the adjoint's decomposition (adjoint_device.h): one workgroup
// per brick, each thread one x-tile row marching z, the 16 lanes of a row
// holding the brick's 16 x-tiles.  Per thread, T is evaluated sum-factorised:
//   R_n(c)  = sum_m By_m(v) phi[tz+n][ty+m][c]   for the thread's own control
//             column c (and column c + 16 for lanes < 3), control planes
//             tz..tz+3 kept in a rolling window, one new plane per z-tile;
//   P(c)    = sum_n Bz_n(w) R_n(c)               once per voxel plane;
//   T(o)    = sum_l Bx_l(o) P(tx + l)            per voxel.
// For spacings up to kFusedMaxDX the per-voxel work runs in voxel layout: each
// wave publishes its rows' P in LDS, every lane takes voxels k * 64 + lane of
// the wave's 4 rows (consecutive lanes on consecutive voxels, so the image
// loads coalesce), evaluates T, samples the moving image and writes the
// voxel's gradient 2 (W - fixed) dW/dp into the wave's transpose buffer, from
// which the tile lanes read their rows: from there on it is the adjoint's
// pass 1 with this gradient in place of dfield.  Larger spacings do the same
// per tile lane, the three neighbouring columns of P taken from the row's
// other lanes (DPP).
// Each workgroup also sums its voxels' squared residuals in a fixed order into
// one loss partial; pass 2 is the adjoint's fixed-order gather, and the loss is
// the fixed-order sum of the partials.  No atomics: the bits depend on the
// inputs only.
#include "adjoint_device.h"
#include "bsi_internal.h"
#include "warp_device.h"

namespace bsi {

namespace {

// Spacings that take the warp in voxel layout (below); larger ones evaluate it
// in tile layout.
constexpr int kFusedMaxDX = 8;
constexpr int kFusedCols = kAdjTilesX + 3;  // window columns of one brick row

__host__ __device__ constexpr bool fused_voxel_layout(int dx) { return dx >= 1 && dx <= kFusedMaxDX; }

template <int DX>
struct FusedSmem {
  AdjEmitSmem e;
  float red[kAdjThreads];
  // per wave: column values P of its 4 rows, and the transpose buffer that
  // carries each voxel's gradient from voxel lanes to tile lanes
  float P[fused_voxel_layout(DX) ? kAdjWaves * kAdjRowsPerWave * kFusedCols * 3 : 1];
  float T[fused_voxel_layout(DX) ? kAdjWaves * adj_wave_buf(DX) : 1];
  float wx[fused_voxel_layout(DX) ? 4 * DX : 1];  // x weights of the offsets 0..DX-1
};

// Value of lane (i + L) mod 16 of this lane's row of 16 lanes.
template <int L>
__device__ __forceinline__ F3 row_from_right(const F3& v) {
  return F3{row_ror<kAdjTilesX - L>(v.x), row_ror<kAdjTilesX - L>(v.y), row_ror<kAdjTilesX - L>(v.z)};
}

template <int L>
__device__ __forceinline__ F3 column_right(int txl, const F3& pm, const F3& pw) {
  const F3 m = row_from_right<L>(pm), w = row_from_right<L>(pw);
  return txl + L < kAdjTilesX ? m : w;
}

__device__ __forceinline__ F3 zcombine(const float* __restrict__ wz, const F3 (&R)[4]) {
  F3 p;
  p.x = fmaf(wz[3], R[3].x, fmaf(wz[2], R[2].x, fmaf(wz[1], R[1].x, wz[0] * R[0].x)));
  p.y = fmaf(wz[3], R[3].y, fmaf(wz[2], R[2].y, fmaf(wz[1], R[1].y, wz[0] * R[0].y)));
  p.z = fmaf(wz[3], R[3].z, fmaf(wz[2], R[2].z, fmaf(wz[1], R[1].z, wz[0] * R[0].z)));
  return p;
}

template <int DX>
__device__ __forceinline__ void fused_brick(const float* __restrict__ grid, const float* __restrict__ moving,
                                            const float* __restrict__ fixed, float* __restrict__ part,
                                            float* __restrict__ lpart, const AdjGeom& a,
                                            const float* __restrict__ lut, int brick, FusedSmem<DX>& sm,
                                            int tid) {
  const VolGeom& g = a.g;
  const int dx = DX > 0 ? DX : g.dx;
  const AdjBrick b = adj_brick_geom(a, brick);
  float* pbase = part + (size_t)brick * a.z.cm * a.y.cm * a.x.cm * 3;
  if constexpr (fused_voxel_layout(DX)) {
    if (tid < 4 * DX) sm.wx[tid] = lut_row(lut, DX, 0)[tid];  // ordered by adj_tables' barrier
  }
  adj_tables(a, b, lut, sm.e, tid);

  const int txl = tid % kAdjTilesX;
  const int yl = tid / kAdjTilesX;
  const int y = b.y0 + yl;
  const int tx = b.cx0 + txl;
  const bool row_in = y < b.ye;
  const bool act = txl < b.ntx && row_in;
  const int x0 = tx * dx;
  const int nval = act ? min(dx, g.nx - x0) : 0;
  const float* lutx = lut_row(lut, dx, 0);

  // Control columns this thread contracts over y: its own (cx0 + txl) and, for
  // txl < 3, cx0 + 16 + txl; both only when inside the brick's window (< Cx),
  // which keeps every index below gx.  Rows outside the brick contract nothing.
  const bool need_m = row_in && txl < b.Cx;
  const bool need_w = row_in && txl < 3 && kAdjTilesX + txl < b.Cx;
  const int yc = row_in ? y : b.y0;
  const int ty = yc / g.dy;  // ty + 3 <= gy - 1
  const float* wy = lut_row(lut, g.dy, yc - ty * g.dy);
  const float by0 = wy[0], by1 = wy[1], by2 = wy[2], by3 = wy[3];
  const size_t gplane = (size_t)g.gy * g.gx * 3, grow = (size_t)g.gx * 3;
  const float* colm = grid + ((size_t)ty * g.gx + (need_m ? tx : 0)) * 3;
  const float* colw = grid + ((size_t)ty * g.gx + (need_w ? tx + kAdjTilesX : 0)) * 3;
  auto ycontract = [&](const float* col, int cz, bool need) {
    F3 r{0.f, 0.f, 0.f};
    if (need) {
      const float* p = col + (size_t)cz * gplane;
      const F3 q0 = ldf3(p), q1 = ldf3(p + grow), q2 = ldf3(p + 2 * grow), q3 = ldf3(p + 3 * grow);
      r.x = fmaf(by3, q3.x, fmaf(by2, q2.x, fmaf(by1, q1.x, by0 * q0.x)));
      r.y = fmaf(by3, q3.y, fmaf(by2, q2.y, fmaf(by1, q1.y, by0 * q0.y)));
      r.z = fmaf(by3, q3.z, fmaf(by2, q2.z, fmaf(by1, q1.z, by0 * q0.z)));
    }
    return r;
  };

  int tz = b.cz0;
  int oz = b.z0 - tz * g.dz;
  F3 R[4], Rw[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    R[n] = ycontract(colm, tz + n, need_m);
    Rw[n] = ycontract(colw, tz + n, need_w);
  }
  F3 acc[4], accw[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) acc[n] = accw[n] = F3{0.f, 0.f, 0.f};
  float l2 = 0.f;
  const size_t izs = (size_t)g.ny * g.nx;
  const float* fix = fixed + (size_t)b.z0 * izs + (size_t)(act ? y : 0) * g.nx + (act ? x0 : 0);

  for (int z = b.z0; z < b.ze; ++z) {
    const float* wz = lut_row(lut, g.dz, oz);
    F3 M[4];
    const F3 pm = zcombine(wz, R);  // P of column tx (every lane takes part)
    const F3 pw = zcombine(wz, Rw); // P of column tx + 16 (lanes txl < 3)
    if constexpr (fused_voxel_layout(DX)) {
      const int lane = tid & (kWave - 1), wave = tid / kWave;
      float* pl = sm.P + wave * (kAdjRowsPerWave * kFusedCols * 3);
      float* tb = sm.T + wave * adj_wave_buf(DX);
      const int ywave = b.y0 + wave * kAdjRowsPerWave;
      wave_lds_sync();  // the previous plane's readers of pl and tb are done
      {
        const int r = lane / kAdjTilesX;
        stf3(pl + (r * kFusedCols + txl) * 3, pm);
        if (txl < 3) stf3(pl + (r * kFusedCols + kAdjTilesX + txl) * 3, pw);
      }
      wave_lds_sync();
#if BSI_FUSED_FULL_UNROLL
#pragma unroll
#else
#pragma unroll 2
#endif
      for (int k = 0; k < DX; ++k) {
        const int v = k * kWave + lane;
        const int r = v / (kAdjTilesX * DX);
        const int xl = v - r * (kAdjTilesX * DX);
        const int tl = xl / DX, o = xl - tl * DX;
        const int xv = b.x0 + xl, yv = ywave + r;
        F3 d{0.f, 0.f, 0.f};
        if (xv < b.xe && yv < b.ye) {
          const float* bx = sm.wx + 4 * o;
          const float* pp = pl + (r * kFusedCols + tl) * 3;  // columns tl .. tl + 3 (<= 18)
          F3 t;
          t.x = fmaf(bx[3], pp[9], fmaf(bx[2], pp[6], fmaf(bx[1], pp[3], bx[0] * pp[0])));
          t.y = fmaf(bx[3], pp[10], fmaf(bx[2], pp[7], fmaf(bx[1], pp[4], bx[0] * pp[1])));
          t.z = fmaf(bx[3], pp[11], fmaf(bx[2], pp[8], fmaf(bx[1], pp[5], bx[0] * pp[2])));
          const Sample smp = trilinear(moving, g.nx, g.ny, g.nz, (float)xv + t.x, (float)yv + t.y, (float)z + t.z);
          const float res = smp.w - fixed[((size_t)z * g.ny + yv) * g.nx + xv];
          l2 = fmaf(res, res, l2);
          const float two_r = 2.f * res;
          d = F3{two_r * smp.gx, two_r * smp.gy, two_r * smp.gz};
        }
        stf3(tb + v * 3, d);
      }
      wave_lds_sync();
      adj_plane_moments<DX>(tb, lane, nval, lutx, M);
    } else {
      // P of the four columns tx..tx+3 of this plane (every lane takes part)
      F3 P[4];
      P[0] = pm;
      P[1] = column_right<1>(txl, pm, pw);
      P[2] = column_right<2>(txl, pm, pw);
      P[3] = column_right<3>(txl, pm, pw);
#pragma unroll
      for (int l = 0; l < 4; ++l) M[l] = F3{0.f, 0.f, 0.f};
      auto voxel = [&](int o) {
        const float* bx = lutx + 4 * o;
        F3 t;
        t.x = fmaf(bx[3], P[3].x, fmaf(bx[2], P[2].x, fmaf(bx[1], P[1].x, bx[0] * P[0].x)));
        t.y = fmaf(bx[3], P[3].y, fmaf(bx[2], P[2].y, fmaf(bx[1], P[1].y, bx[0] * P[0].y)));
        t.z = fmaf(bx[3], P[3].z, fmaf(bx[2], P[2].z, fmaf(bx[1], P[1].z, bx[0] * P[0].z)));
        const Sample smp = trilinear(moving, g.nx, g.ny, g.nz, (float)(x0 + o) + t.x, (float)y + t.y,
                                     (float)z + t.z);
        const float res = smp.w - fix[o];
        l2 = fmaf(res, res, l2);
        const float two_r = 2.f * res;
        const F3 d{two_r * smp.gx, two_r * smp.gy, two_r * smp.gz};
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          M[l].x = fmaf(bx[l], d.x, M[l].x);
          M[l].y = fmaf(bx[l], d.y, M[l].y);
          M[l].z = fmaf(bx[l], d.z, M[l].z);
        }
      };
#pragma unroll 1
      for (int o = 0; o < nval; ++o) voxel(o);
    }
    fix += izs;

    F3 cm, cw;
    adj_xcombine(txl, M, cm, cw);
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const float w = wz[n];
      acc[n].x = fmaf(w, cm.x, acc[n].x);
      acc[n].y = fmaf(w, cm.y, acc[n].y);
      acc[n].z = fmaf(w, cm.z, acc[n].z);
      accw[n].x = fmaf(w, cw.x, accw[n].x);
      accw[n].y = fmaf(w, cw.y, accw[n].y);
      accw[n].z = fmaf(w, cw.z, accw[n].z);
    }
    if (++oz == g.dz && z + 1 < b.ze) {
      adj_emit(a, b, pbase, sm.e, tid, tz - b.cz0, tz - b.cz0, false, acc[0], accw[0]);
#pragma unroll
      for (int n = 0; n < 3; ++n) {
        acc[n] = acc[n + 1];
        accw[n] = accw[n + 1];
        R[n] = R[n + 1];
        Rw[n] = Rw[n + 1];
      }
      acc[3] = accw[3] = F3{0.f, 0.f, 0.f};
      // the next tile tz + 1 lies inside the brick, so its last plane
      // tz + 4 <= ceil(nz/dz) + 2 = gz - 1
      R[3] = ycontract(colm, tz + 4, need_m);
      Rw[3] = ycontract(colw, tz + 4, need_w);
      oz = 0;
      ++tz;
    }
  }
#pragma unroll 1
  for (int n = 0; n < 4; ++n) {
    adj_emit(a, b, pbase, sm.e, tid, tz - b.cz0 + n, tz - b.cz0 + n, n == 3, acc[0], accw[0]);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      acc[j] = acc[j + 1];
      accw[j] = accw[j + 1];
    }
  }

  // loss partial of the brick: fixed-order tree over the workgroup
  sm.red[tid] = l2;
  __syncthreads();
  for (int h = kAdjThreads / 2; h > 0; h >>= 1) {
    if (tid < h) sm.red[tid] += sm.red[tid + h];
    __syncthreads();
  }
  if (tid == 0) lpart[brick] = sm.red[0];
}

template <int DX>
__global__ __launch_bounds__(kAdjThreads) __attribute__((amdgpu_waves_per_eu(4))) void fused_pass1_kernel(const float* __restrict__ grid,
                                                                   const float* __restrict__ moving,
                                                                   const float* __restrict__ fixed,
                                                                   float* __restrict__ part,
                                                                   float* __restrict__ lpart, AdjGeom a,
                                                                   const float* __restrict__ lut) {
  __shared__ FusedSmem<DX> sm;
  const int nbricks = a.x.nb * a.y.nb * a.z.nb;
  const int brick = xcd_remap(blockIdx.x, gridDim.x);
  if (brick >= nbricks) return;  // uniform over the workgroup
  fused_brick<DX>(grid, moving, fixed, part, lpart, a, lut, brick, sm, threadIdx.x);
}

}  // namespace

size_t fused_workspace_bytes(const AdjGeom& a) {
  const size_t p = (adj_workspace_bytes(a) + 255) / 256 * 256;
  return p + (size_t)a.x.nb * a.y.nb * a.z.nb * sizeof(float);
}

hipError_t launch_ssd_fused(const float* grid, const float* moving, const float* fixed, float* grad, float* loss,
                            const AdjGeom& a, const float* lut, void* workspace, hipStream_t s) {
  float* part = static_cast<float*>(workspace);
  float* lpart = reinterpret_cast<float*>(static_cast<char*>(workspace) +
                                          (adj_workspace_bytes(a) + 255) / 256 * 256);
  const long nbricks = (long)a.x.nb * a.y.nb * a.z.nb;
  const dim3 gridd((unsigned)nbricks), block(kAdjThreads);
#define BSI_FUSED_CASE(D)                                                                           \
  case D:                                                                                          \
    hipLaunchKernelGGL(fused_pass1_kernel<D>, gridd, block, 0, s, grid, moving, fixed, part, lpart, a, \
                       lut);                                                                       \
    break;
  switch (a.g.dx) {
    BSI_FUSED_CASE(1)
    BSI_FUSED_CASE(2)
    BSI_FUSED_CASE(3)
    BSI_FUSED_CASE(4)
    BSI_FUSED_CASE(5)
    BSI_FUSED_CASE(6)
    BSI_FUSED_CASE(7)
    BSI_FUSED_CASE(8)
    default: BSI_FUSED_CASE(0)
  }
#undef BSI_FUSED_CASE
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_adjoint_reduce(part, grad, a, s)) != hipSuccess) return e;
  return launch_sum(lpart, nbricks, loss, s);
}

}  // namespace bsi
