// Adjoint of Eq. 1 (its transpose), as a deterministic two-pass gather.
//
// Pass 1 (one workgroup per brick), z-first.  A brick is kAdjBX = 64
// consecutive x-voxels (one per lane) by kAdjBY rows by a run of whole
// z-tiles.  Wave w of the workgroup owns rows y0 + w R .. y0 + w R + R - 1
// (R = kAdjRows), so each lane owns one voxel column per row and marches z.
// Per voxel plane it loads its R voxels (a wave reads 768 contiguous bytes per
// row) and accumulates the z-contraction in registers,
//   A_r[n] += Bz_n(w) * dfield[z][y_r][x]        (n = cz - tz, 4 planes),
// the only per-voxel work.  When a z-tile ends, plane A[0] is finished for the
// brick's voxel rows and is contracted in LDS:
//   over x, per wave (its own rows), on tile lanes: lane (row, t) forms the
//     x-moments of tile t, M_l = sum_o Bx_l(o) A0[row][t dx + o], and the 16
//     lanes of a row combine them with row shifts (DPP):
//     H[row][cx] = sum_l M_l(tile cx - l);
//   then, after one workgroup barrier, over y, the same way on y-tile lanes:
//     G[cy][cx] = sum_m N_m(tile cy - m),  N_m = sum_oy By_m(oy) H[t dy + oy][cx].
// G is the brick's partial gradient of that control plane.  H is double-
// buffered, so the barrier of plane k also orders the y-contraction of plane
// k - 1 before the x-contraction of plane k + 1.  A brick's partials are staged
// in LDS and stored after its last load (see kAdjStageFloats).
//
// Pass 2 (one thread per control point) sums, in fixed brick order, the
// partials of the bricks whose voxels meet the point's support.  No atomics
// anywhere: the bits depend on the inputs only.
#pragma once

#include <type_traits>

#include "bsi_device.h"

namespace bsi {

#ifndef BSI_ADJ_ROWS
#define BSI_ADJ_ROWS 2
#endif
#ifndef BSI_ADJ_WAVES
#define BSI_ADJ_WAVES 8
#endif
#ifndef BSI_ADJ_TARGET_Z
#define BSI_ADJ_TARGET_Z 48
#endif
// Waves per SIMD the pass-1 kernels are compiled for (a register bound of
// 512 / this): 6 keeps three 512-thread workgroups per CU.
#ifndef BSI_ADJ_WPE
#define BSI_ADJ_WPE 6
#endif
constexpr int kAdjRows = BSI_ADJ_ROWS;             // rows per lane (R)
constexpr int kAdjWaves = BSI_ADJ_WAVES;           // waves per workgroup
constexpr int kAdjThreads = kAdjWaves * kWave;
constexpr int kAdjBX = kWave;                      // brick width (voxels): one lane per voxel
constexpr int kAdjBY = kAdjWaves * kAdjRows;       // brick height (rows)
constexpr int kAdjTargetZ = BSI_ADJ_TARGET_Z;      // brick depth bound (voxels, at least one tile)
constexpr int kAdjMaxDX = 12;                      // largest x spacing with its own kernel
constexpr int kAdjTiles = 16;                      // tile lanes per row of lanes (DPP rows)
// A brick of at most 16 rows meets at most 16 y-tiles (16 at spacing 1, at
// most (kAdjBY - 1)/dy + 2 otherwise): one row of 16 y-tile lanes per column.
static_assert(kAdjBY <= kAdjTiles, "a brick's y-tiles fit one row of tile lanes");

// The kernels are specialised per x spacing DX = 1..kAdjMaxDX; DX = 0 is the
// generic kernel for spacings above kAdjMaxDX, and DX = kAdjAnyTile a kernel
// for any spacing 4..kAdjMaxDX taken at run time (the same operations, in the
// same order, as the specialisation of that spacing).
constexpr int kAdjAnyTile = -1;

// Window columns of a brick of kAdjBX voxels at x spacing dx (0: any spacing
// above kAdjMaxDX; kAdjAnyTile: any of 4..kAdjMaxDX): a run of w voxels meets
// at most (w - 1)/dx + 2 tiles, and exactly w / dx when the run is whole tiles
// (spacing 1).
__host__ __device__ constexpr int adj_cx_max(int dx) {
  return dx == 1 ? kAdjBX + 3
                 : (kAdjBX - 1) / (dx == kAdjAnyTile ? 4 : dx > 0 ? dx : kAdjMaxDX + 1) + 5;
}
// The x-contraction runs on tile lanes (16 x-tiles per row of 16 lanes) when a
// brick row holds at most 16 tiles: x spacing 4 (bricks start on multiples of
// 64, so exactly 16 tiles), 5..12, and the generic kernel (spacing 13 or more,
// at most 6 tiles).  Spacings 1..3 sum each column directly (adj_xsum).
__host__ __device__ constexpr bool adj_tile_lanes(int dx) { return dx == 0 || dx == kAdjAnyTile || dx >= 4; }

// Finished partial planes are staged in LDS and stored once per brick.  On
// this chip loads and stores share one counter of outstanding memory
// operations, and a store issued while loads are in flight makes the next wait
// for a load wait for everything: a store per finished plane would drain the
// planes of loads in flight at every z-tile.  With the partials of a whole
// brick staged (spacings of 5 and more at the default brick size), they are
// stored after the brick's last load.
#ifndef BSI_ADJ_STAGE_FLOATS
#define BSI_ADJ_STAGE_FLOATS 6144
#endif
constexpr int kAdjStageFloats = BSI_ADJ_STAGE_FLOATS;  // 24 KB

// Rows of H the y-contraction loads at once (one LDS round trip per group).
#ifndef BSI_ADJ_YGROUP
#define BSI_ADJ_YGROUP 1
#endif
constexpr int kAdjYGroup = BSI_ADJ_YGROUP;

// Rows of the finished-plane buffer F carry dx - 1 voxels of zeros on each
// side at x spacings 4..12, so a tile that reaches past the brick is
// contracted without a test per voxel: its voxels outside the brick read zero
// (the voxels of a ragged brick's row past its end are written as zeros too).
__host__ __device__ constexpr int adj_fpad(int dx) {
  return dx == kAdjAnyTile ? kAdjMaxDX - 1 : dx >= 4 && dx <= kAdjMaxDX ? dx - 1 : 0;
}
__host__ __device__ constexpr int adj_frow(int dx) { return kWave + 2 * adj_fpad(dx); }  // row stride (voxels)

template <int DX>
struct AdjSmem {
  float F[kAdjBY * adj_frow(DX) * 3];        // finished plane, row by row (each wave writes its own rows)
  float H[2][kAdjBY * adj_cx_max(DX) * 3];   // x-contracted rows, double-buffered
  float P[kAdjStageFloats];                  // the brick's partial planes awaiting their store
};

struct AdjBrick {
  int x0, y0, z0, xe, ye, ze;  // voxel range [x0, xe) etc.
  int cx0, cy0, cz0;           // first control index of the window
  int Cx, Cy;                  // window extent in x, y
  int ntx;                     // x-tiles of the brick inside the volume
};

__host__ __device__ inline AdjBrick adj_brick_geom(const AdjGeom& a, int brick) {
  const VolGeom& g = a.g;
  AdjBrick b;
  const int bx = brick % a.x.nb;
  const int t = brick / a.x.nb;
  const int by = t % a.y.nb;
  const int bz = t / a.y.nb;
  b.x0 = adj_brick_begin(a.x, g.nx, bx);
  b.y0 = adj_brick_begin(a.y, g.ny, by);
  b.z0 = adj_brick_begin(a.z, g.nz, bz);
  b.xe = adj_brick_begin(a.x, g.nx, bx + 1);
  b.ye = adj_brick_begin(a.y, g.ny, by + 1);
  b.ze = adj_brick_begin(a.z, g.nz, bz + 1);
  b.cx0 = b.x0 / g.dx;
  b.cy0 = b.y0 / g.dy;
  b.cz0 = b.z0 / g.dz;
  b.Cx = (b.xe - 1) / g.dx - b.cx0 + 4;
  b.Cy = (b.ye - 1) / g.dy - b.cy0 + 4;
  b.ntx = (b.xe - 1) / g.dx - b.cx0 + 1;
  return b;
}

// Control planes of a brick's window: the z-tiles of its voxels plus 3.
__host__ __device__ inline int adj_brick_cz(const AdjGeom& a, const AdjBrick& b) {
  return (b.ze - 1) / a.g.dz - b.cz0 + 4;
}

// Floats per brick in the workspace, and the offset of window point
// (czl, cyl, cxl) within its brick's partials.
__host__ __device__ inline size_t adj_brick_stride(const AdjGeom& a) {
  return (size_t)a.z.cm * a.y.cm * a.x.cm * 3;
}
__host__ __device__ inline size_t adj_part_offset(const AdjGeom& a, int czl, int cyl, int cxl) {
  return ((size_t)(czl * a.y.cm + cyl) * a.x.cm + cxl) * 3;
}

// Whether a brick's whole window of partials (cm_z planes of cm_y * cm_x
// points) fits the LDS stage; otherwise each plane is stored as it is finished.
__host__ __device__ inline bool adj_stage_all(const AdjGeom& a) {
  return (long)a.z.cm * a.y.cm * a.x.cm * 3 <= kAdjStageFloats;
}

// Voxel 0 of brick row `row` in F (voxels -fpad .. 63 + fpad are addressable).
template <int DX>
__device__ __forceinline__ float* adj_frow_ptr(AdjSmem<DX>& sm, int row) {
  return sm.F + (row * adj_frow(DX) + adj_fpad(DX)) * 3;
}

// This wave's R rows of F get voxel `lane` of the finished plane (zero past
// the brick's end).
template <int DX, int R>
__device__ __forceinline__ void adj_put_f(AdjSmem<DX>& sm, const AdjBrick& b, int wave, int lane, int r, F3 v) {
  if (lane >= b.xe - b.x0) v = F3{0.f, 0.f, 0.f};
  stf3(adj_frow_ptr<DX>(sm, wave * R + r) + lane * 3, v);
}

// Zero the pads of this wave's R rows of F (wave-local: the wave's next
// wave_lds_sync orders it before the x-contraction reads them).
template <int DX, int R>
__device__ __forceinline__ void adj_zero_fpad(AdjSmem<DX>& sm, int wave, int lane) {
  constexpr int P = adj_fpad(DX);
  if constexpr (P > 0) {
    for (int i = lane; i < R * 2 * P * 3; i += kWave) {
      const int r = i / (2 * P * 3), j = i - r * (2 * P * 3);  // j: float within the row's two pads
      const int v = j / 3, c = j - v * 3;                       // pad voxel, component
      const int xl = v < P ? v - P : kWave + (v - P);
      adj_frow_ptr<DX>(sm, wave * R + r)[xl * 3 + c] = 0.f;
    }
  }
}

// Value of lane i - N of this lane's row of 16 lanes, 0 for i < N (DPP
// row_shr); row_shl: lane i + N, 0 for i + N >= 16.  Lanes past the row's
// edge read the zero `old` operand.
template <int N>
__device__ __forceinline__ float row_shr(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x110 + N, 0xF, 0xF, true));
}
template <int N>
__device__ __forceinline__ float row_shl(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x100 + N, 0xF, 0xF, true));
}

// Window column of tile lanes: lane t of a row of 16 holds the moments M_l of
// tile t; this forms
//   cm = S[t]      = sum_{l <= t} M_l(tile t - l)
//   cw = S[16 + t] = sum_{l > t}  M_l(tile 16 + t - l)   (t < 3)
// l ascending.  The shifts bring in zero for the terms a lane does not take
// (row_shr by l for l > t, row_shl by 16 - l for l <= t), and adding zero is
// exact, so no per-lane selects are needed.  Idle lanes hold M = 0, so columns
// past the last tile come out right.  Every lane of the wave takes part (no
// lane may be inactive).
__device__ __forceinline__ void adj_combine(const F3 (&M)[4], F3& cm, F3& cw) {
  cm = M[0];
  cm.x += row_shr<1>(M[1].x);
  cm.y += row_shr<1>(M[1].y);
  cm.z += row_shr<1>(M[1].z);
  cm.x += row_shr<2>(M[2].x);
  cm.y += row_shr<2>(M[2].y);
  cm.z += row_shr<2>(M[2].z);
  cm.x += row_shr<3>(M[3].x);
  cm.y += row_shr<3>(M[3].y);
  cm.z += row_shr<3>(M[3].z);
  cw.x = row_shl<15>(M[1].x);
  cw.y = row_shl<15>(M[1].y);
  cw.z = row_shl<15>(M[1].z);
  cw.x += row_shl<14>(M[2].x);
  cw.y += row_shl<14>(M[2].y);
  cw.z += row_shl<14>(M[2].z);
  cw.x += row_shl<13>(M[3].x);
  cw.y += row_shl<13>(M[3].y);
  cw.z += row_shl<13>(M[3].z);
  // cm is formed here, not sunk into the callers' conditional stores (which
  // keeps all nine shifted values live at once and spills)
  asm volatile("" : "+v"(cm.x), "+v"(cm.y), "+v"(cm.z));
}

// Moments += w_l * v for l = 0..3.
__device__ __forceinline__ void adj_moment_step(const float* __restrict__ w, const F3& v, F3 (&M)[4]) {
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    M[l].x = fmaf(w[l], v.x, M[l].x);
    M[l].y = fmaf(w[l], v.y, M[l].y);
    M[l].z = fmaf(w[l], v.z, M[l].z);
  }
}

// Streaming load of one voxel of dfield: non-temporal, since every voxel is
// read once; the read stream then does not leave the caches full of dfield
// lines that the next kernel's writes have to displace.
template <bool Stream>
__device__ __forceinline__ F3 ldf3_dfield(const float* p) {
  if constexpr (Stream)
    return F3{__builtin_nontemporal_load(p), __builtin_nontemporal_load(p + 1), __builtin_nontemporal_load(p + 2)};
  else
    return ldf3(p);
}

// Offsets (floats, within a voxel plane) of this lane's R voxels: row
// y0 + wave R + r, column x0 + lane, both clamped into the brick so that every
// lane loads from a valid address without a branch.  A clamped lane's values
// are never read: the x-contraction reads only columns inside the brick and
// the y-contraction only rows inside it.  A plane holds < 2^32 floats.
template <int R>
__host__ __device__ inline void adj_offsets(const AdjBrick& b, int nx, int wave, int lane, uint32_t (&off)[R]) {
  const int x = imin(b.x0 + lane, b.xe - 1);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int y = imin(b.y0 + wave * R + r, b.ye - 1);
    off[r] = ((uint32_t)y * (uint32_t)nx + (uint32_t)x) * 3u;
  }
}

// x-contraction of one window column cx for one brick row (spacings 1..3):
//   sum over voxels x of the brick in cx's support [(cx-3)dx, (cx+1)dx),
//   ascending, of Bx_{cx - floor(x/dx)}(x - floor(x/dx) dx) * F[x - x0].
template <int DX>
__device__ __forceinline__ F3 adj_xsum(const float* __restrict__ Fr, const AdjBrick& b, int cx,
                                       const float* __restrict__ lut) {
  F3 s{0.f, 0.f, 0.f};
#pragma unroll 1
  for (int j = 0; j < 4; ++j) {  // tile cx - 3 + j, weight index l = 3 - j
    const int xt = (cx - 3 + j) * DX - b.x0;  // the tile's first voxel, brick-relative
#pragma unroll
    for (int o = 0; o < DX; ++o) {
      const int xl = xt + o;
      if (xl >= 0 && xl < b.xe - b.x0) {
        const float w = lut_row(lut, DX, o)[3 - j];  // uniform: a scalar load
        const float* q = Fr + xl * 3;
        s.x = fmaf(w, q[0], s.x);
        s.y = fmaf(w, q[1], s.y);
        s.z = fmaf(w, q[2], s.z);
      }
    }
  }
  return s;
}

// First half of a finished plane's emission (collective over the workgroup,
// wave-local work) for workgroups of W waves of R rows each (W R = kAdjBY):
// this wave's rows of the plane (lane = voxel; get(r) gives row r) go through
// its rows of the LDS buffer F and are contracted over x into H[czl & 1].  The caller then places one
// workgroup barrier and calls adj_emit_y.
template <int DX, int R>
__device__ __forceinline__ void adj_emit_xf(const AdjBrick& b, AdjSmem<DX>& sm, const float* __restrict__ lut,
                                            int dx, int tid, int czl);

template <int DX, int R, class Get>
__device__ __forceinline__ void adj_emit_x(const AdjBrick& b, AdjSmem<DX>& sm, const float* __restrict__ lut,
                                           int dx, int tid, int czl, Get get) {
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  wave_lds_sync();  // this wave's x-contraction of the previous plane is done with its rows of F
#pragma unroll
  for (int r = 0; r < R; ++r) adj_put_f<DX, R>(sm, b, wave, lane, r, get(r));
  wave_lds_sync();
  adj_emit_xf<DX, R>(b, sm, lut, dx, tid, czl);
}

// The x-contraction of this wave's rows, already in F.
template <int DX, int R>
__device__ __forceinline__ void adj_emit_xf(const AdjBrick& b, AdjSmem<DX>& sm, const float* __restrict__ lut,
                                            int dx, int tid, int czl) {
  static_assert(kWave / kAdjTiles >= R, "a wave's rows fit its rows of 16 tile lanes");
  constexpr int CXM = adj_cx_max(DX);
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  float* H = sm.H[czl & 1];  // czl counts the brick's finished planes
  const int nrow = b.ye - b.y0 - wave * R;  // this wave's rows inside the brick
  if constexpr (adj_tile_lanes(DX)) {
    // lane (rr, t) = (lane / 16, lane % 16): tile cx0 + t of row rr,
    //   M_l = sum_o Bx_l(o) F[rr][t dx + o - x0]   (o ascending, voxels in the brick)
    const int rr = lane / kAdjTiles, t = lane % kAdjTiles;
    const bool act = rr < R && rr < nrow && t < b.ntx;
    F3 M[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) M[l] = F3{0.f, 0.f, 0.f};
    if (act) {
      const int xt = (b.cx0 + t) * dx - b.x0;  // the tile's first voxel, brick-relative (may be < 0)
      const float* Fr = adj_frow_ptr<DX>(sm, wave * R + rr);
      if constexpr (adj_fpad(DX) > 0) {
        // voxels xt .. xt + dx - 1 lie in -(dx - 1) .. 63 + dx - 1: no tests
        if constexpr (DX > 0) {
#pragma unroll
          for (int o = 0; o < DX; ++o) adj_moment_step(lut_row(lut, DX, o), ldf3(Fr + (xt + o) * 3), M);
        } else {  // kAdjAnyTile: dx from the geometry, the same operations in the same order
#pragma unroll 1
          for (int o = 0; o < dx; ++o) adj_moment_step(lut_row(lut, dx, o), ldf3(Fr + (xt + o) * 3), M);
        }
      } else {
        const int nxb = b.xe - b.x0;
        auto voxel = [&](int o) {
          const int xl = xt + o;
          if (xl >= 0 && xl < nxb) adj_moment_step(lut_row(lut, dx, o), ldf3(Fr + xl * 3), M);
        };
        // pairs of voxels in flight: few registers while the z-accumulators
        // and the next planes' loads are live
#pragma unroll 1
        for (int o = 0; o < dx; o += 2) {
          voxel(o);
          if (o + 1 < dx) voxel(o + 1);
        }
      }
    }
    F3 cm, cw;
    adj_combine(M, cm, cw);  // every lane of the wave takes part
    if (rr < R && rr < nrow) {
      float* hrow = H + (wave * R + rr) * CXM * 3;
      if (t < b.Cx) stf3(hrow + t * 3, cm);
      if (t < 3 && kAdjTiles + t < b.Cx) stf3(hrow + (kAdjTiles + t) * 3, cw);
    }
  } else {
    const int items = imin(nrow, R) * b.Cx;
    for (int it = lane; it < items; it += kWave) {
      const int r = it / b.Cx, cxl = it - r * b.Cx;
      stf3(H + ((wave * R + r) * CXM + cxl) * 3, adj_xsum<DX>(adj_frow_ptr<DX>(sm, wave * R + r), b, b.cx0 + cxl, lut));
    }
  }
}

// Second half (after the workgroup barrier), for workgroups of W waves: the
// y-contraction of H[czl & 1] into window plane czl of the brick's partials,
// on y-tile lanes: lane (c4, ty) = (lane / 16, lane % 16) of wave w takes
// column cxl = 4 w + c4 (then + 4 W ...) and y-tile cy0 + ty; it forms
//   N_m = sum over the tile's rows y in the brick (ascending) of By_m(v(y)) H[y][cxl]
// and the 16 lanes of a row finish window rows ty and, for ty < 3, 16 + ty.
// StageAll: the partials go to the LDS stage, and after the brick's last
// plane (last) the whole staged window is stored as one contiguous run of
// padded planes; otherwise straight to the workspace.
template <int DX, int W, bool StageAll>
__device__ __forceinline__ void adj_emit_y(const AdjGeom& a, const AdjBrick& b, float* __restrict__ pbase,
                                           AdjSmem<DX>& sm, const float* __restrict__ lut, int tid, int czl,
                                           bool last) {
  constexpr int CXM = adj_cx_max(DX);
  const VolGeom& g = a.g;
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  const float* H = sm.H[czl & 1];
  const int nty = b.Cy - 3;  // y-tiles meeting the brick (<= 16)
  const int c4 = lane / kAdjTiles, ty = lane % kAdjTiles;
  for (int c0 = wave * 4; c0 < b.Cx; c0 += W * 4) {  // uniform over the wave
    const int cxl = c0 + c4;
    const bool act = cxl < b.Cx && ty < nty;
    F3 N[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) N[m] = F3{0.f, 0.f, 0.f};
    const int y1 = (b.cy0 + ty) * g.dy;  // the tile's first row
    const float* hc = H + (act ? cxl : 0) * 3;
    // rows in groups of kAdjYGroup, loaded together (a row outside the brick, or of
    // an idle lane, reads a valid row and counts as zero); the trip counts are
    // uniform, so the weights are scalar loads
#pragma unroll 1
    for (int oy0 = 0; oy0 < g.dy; oy0 += kAdjYGroup) {
      F3 v[kAdjYGroup];
#pragma unroll
      for (int j = 0; j < kAdjYGroup; ++j) {
        const int y = y1 + oy0 + j;
        const bool ok = act && oy0 + j < g.dy && y >= b.y0 && y < b.ye;
        v[j] = ldf3(hc + (ok ? y - b.y0 : 0) * CXM * 3);
        if (!ok) v[j] = F3{0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int j = 0; j < kAdjYGroup; ++j)
        if (oy0 + j < g.dy) adj_moment_step(lut_row(lut, g.dy, oy0 + j), v[j], N);
    }
    F3 gm, gw;
    adj_combine(N, gm, gw);  // every lane of the wave takes part
    if (cxl < b.Cx) {
      float* dst = StageAll ? sm.P : pbase;
      if (ty < b.Cy) stf3(dst + adj_part_offset(a, czl, ty, cxl), gm);
      if (ty < 3 && kAdjTiles + ty < b.Cy) stf3(dst + adj_part_offset(a, czl, kAdjTiles + ty, cxl), gw);
    }
  }
  if constexpr (StageAll) {
    if (last) {
      // a following brick of this workgroup writes the stage only after the
      // barrier at its start
      __syncthreads();
      const int n = (czl + 1) * a.y.cm * a.x.cm;
      for (int i = tid; i < n; i += W * kWave) stf3(pbase + i * 3, ldf3(sm.P + i * 3));
    }
  }
}

template <bool Stream>
__device__ __forceinline__ void adj_load(const float* __restrict__ plane, const uint32_t (&off)[kAdjRows],
                                         F3 (&d)[kAdjRows]) {
#pragma unroll
  for (int r = 0; r < kAdjRows; ++r) d[r] = ldf3_dfield<Stream>(plane + off[r]);
}

// Pass 1 for one brick.  Collective over the workgroup (kAdjThreads threads).
// Stream: dfield is read with non-temporal loads.  StageAll: adj_stage_all(a).
template <int DX, bool Stream, bool StageAll>
__device__ __forceinline__ void adj_brick(const float* __restrict__ dfield, float* __restrict__ part,
                                          const AdjGeom& a, const float* __restrict__ lut, int brick,
                                          AdjSmem<DX>& sm, int tid) {
  constexpr int R = kAdjRows;
  const VolGeom& g = a.g;
  const int dx = DX > 0 ? DX : g.dx;
  const AdjBrick b = adj_brick_geom(a, brick);
  float* pbase = part + (size_t)brick * adj_brick_stride(a);
  __syncthreads();  // a previous brick of this workgroup may still read the LDS buffers

  const int lane = tid & (kWave - 1), wave = uniform(tid / kWave);
  uint32_t off[R];
  adj_offsets<R>(b, g.nx, wave, lane, off);
  const size_t zs = (size_t)g.ny * g.nx * 3;
  const float* plane0 = dfield + (size_t)b.z0 * zs;

  // acc[k][r]: the z-accumulation of control plane c for row r, in slot
  // k = (c - cz0) & 3, so the accumulators never move: in tile t (phase
  // ph = t & 3) slot k takes weight Bz_((k - ph) & 3), and slot ph holds the
  // plane that finishes with the tile.  (The slot code below is written out
  // in this function, not in lambdas: every access to acc must be visible
  // with a constant index when it is promoted to registers.)
  F3 acc[4][R];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int r = 0; r < R; ++r) acc[k][r] = F3{0.f, 0.f, 0.f};
  adj_zero_fpad<DX, R>(sm, wave, lane);
  int t = 0;   // tile index within the brick (z-bricks are whole tiles: b.z0 = cz0 dz)
  int oz = 0;  // offset within the tile
  const float* ahead = plane0 + 2 * zs;  // the plane two ahead of the next one

// Control plane CZL, in slot PH (uniform), goes to this wave's rows of F and
// the slot is cleared, then the shared emission.
// A scalar branch to the slot's own code: constant register indices, no selects.
#define BSI_ADJ_PUT_SLOT(K)                                                                \
  _Pragma("unroll") for (int r = 0; r < R; ++r) {                                        \
    adj_put_f<DX, R>(sm, b, wave, lane, r, acc[K][r]);                                   \
    acc[K][r] = F3{0.f, 0.f, 0.f};                                                       \
  }
#define BSI_ADJ_PUT(PH)                                                                    \
  switch (PH) {                                                                          \
    case 0: BSI_ADJ_PUT_SLOT(0) break;                                                   \
    case 1: BSI_ADJ_PUT_SLOT(1) break;                                                   \
    case 2: BSI_ADJ_PUT_SLOT(2) break;                                                   \
    default: BSI_ADJ_PUT_SLOT(3) break;                                                  \
  }
// The emission runs at raised wave priority: the work before and after the
// tile's barrier then takes issue slots ahead of waves that are only streaming
// planes (they wait on memory anyway), so the workgroup's waves reach the
// barrier sooner.
#define BSI_ADJ_EMIT(CZL, PH, LAST)                                                        \
  {                                                                                      \
    __builtin_amdgcn_s_setprio(2);                                                       \
    wave_lds_sync(); /* this wave's x-contraction of the previous plane is done with F */ \
    BSI_ADJ_PUT(PH)                                                                      \
    wave_lds_sync();                                                                     \
    adj_emit_xf<DX, R>(b, sm, lut, dx, tid, (CZL));                                      \
    __syncthreads();                                                                     \
    adj_emit_y<DX, kAdjWaves, StageAll>(a, b, pbase, sm, lut, tid, (CZL), (LAST));       \
    __builtin_amdgcn_s_setprio(0);                                                       \
  }

// One voxel plane Z from register set D: z-accumulation, the loads of the
// plane two ahead into the same registers (when LOAD), then the emission when
// a z-tile ends.
#define BSI_ADJ_PLANE(D, Z, LOAD)                                                          \
  {                                                                                      \
    const int ph = t & 3;                                                                \
    const float* ws_ = lut_rot_row(lut, g.dz, oz, ph); /* Bz_((k - ph) & 3): one scalar load */ \
    _Pragma("unroll") for (int k = 0; k < 4; ++k) {                                      \
      const float w = ws_[k];                                                            \
      _Pragma("unroll") for (int r = 0; r < R; ++r) {                                    \
        acc[k][r].x = fmaf(w, D[r].x, acc[k][r].x);                                      \
        acc[k][r].y = fmaf(w, D[r].y, acc[k][r].y);                                      \
        acc[k][r].z = fmaf(w, D[r].z, acc[k][r].z);                                      \
      }                                                                                  \
    }                                                                                    \
    if (LOAD) adj_load<Stream>(ahead, off, D);                                           \
    ahead += zs;                                                                         \
    if (++oz == g.dz && (Z) + 1 < b.ze) {                                                \
      BSI_ADJ_EMIT(t, ph, false)                                                         \
      oz = 0;                                                                            \
      ++t;                                                                               \
    }                                                                                    \
  }

  // Two register sets, each holding one plane's loads.  The loop is unrolled
  // over them, and its main part runs only while every plane of the pair and
  // every plane two ahead exists, so its loads are unconditional: each set
  // keeps fixed registers, and waiting for one set's loads leaves the other
  // set's in flight.  (Both sets are first loaded unconditionally, from the
  // brick's last plane when it is one plane deep, so the loop is entered with
  // the same loads in flight on every path.)
  F3 d0[R], d1[R];
  adj_load<Stream>(plane0, off, d0);
  adj_load<Stream>(plane0 + (b.ze - b.z0 > 1 ? zs : 0), off, d1);
  int z = b.z0;
  for (; z + 4 <= b.ze; z += 2) {
    BSI_ADJ_PLANE(d0, z, true)
    BSI_ADJ_PLANE(d1, z + 1, true)
  }
  for (; z < b.ze; z += 2) {
    BSI_ADJ_PLANE(d0, z, z + 2 < b.ze)
    if (z + 1 < b.ze) BSI_ADJ_PLANE(d1, z + 1, z + 3 < b.ze)
  }
  // The brick's last four control planes, t .. t + 3 (the last three are
  // shared with the next brick), in slots (t + n) & 3, in ascending order.
#pragma unroll 1
  for (int n = 0; n < 4; ++n) BSI_ADJ_EMIT(t + n, (t + n) & 3, n == 3)
#undef BSI_ADJ_PLANE
#undef BSI_ADJ_EMIT
#undef BSI_ADJ_PUT
#undef BSI_ADJ_PUT_SLOT
}

// Pass 2 for one control point (cx, cy, cz): fixed-order sum of brick partials.
// Bricks whose voxels meet the point's support [(c-3)d, (c+1)d) on each axis,
// summed bz, then by, then bx ascending.  When no axis has more than two such
// bricks all 8 loads are issued at once from clamped addresses and the valid
// ones added in that order; otherwise a loop.
struct AdjSpan {
  int lo, hi;  // brick range
};

// First control index of brick b's window (b < nb): its first voxel's tile,
// b * k when the units are whole tiles.
__host__ __device__ inline int adj_brick_c0(const AdjAxis& ax, int b, int d) {
  return ax.u == d ? b * ax.k : (b * ax.w) / d;
}

__host__ __device__ inline AdjSpan adj_span(const AdjAxis& ax, int c, int d, int n) {
  return AdjSpan{adj_brick_of_voxel(ax, imax(0, (c - 3) * d)), adj_brick_of_voxel(ax, imin(n, (c + 1) * d) - 1)};
}

// Workspace offset (floats) of control point (cx, cy, cz) in brick (bx, by, bz)'s partials.
__host__ __device__ inline size_t adj_part_addr(const AdjGeom& a, int bx, int by, int bz, int cx, int cy, int cz) {
  const int cxl = cx - adj_brick_c0(a.x, bx, a.g.dx);
  const int cyl = cy - adj_brick_c0(a.y, by, a.g.dy);
  const int czl = cz - adj_brick_c0(a.z, bz, a.g.dz);
  return (size_t)((bz * a.y.nb + by) * a.x.nb + bx) * adj_brick_stride(a) + adj_part_offset(a, czl, cyl, cxl);
}

__device__ __forceinline__ F3 adj_gather_point(const float* __restrict__ part, const AdjGeom& a, int cx,
                                               int cy, int cz) {
  const VolGeom& g = a.g;
  const AdjSpan sx = adj_span(a.x, cx, g.dx, g.nx), sy = adj_span(a.y, cy, g.dy, g.ny),
                sz = adj_span(a.z, cz, g.dz, g.nz);
  auto addr = [&](int bx, int by, int bz) { return part + adj_part_addr(a, bx, by, bz, cx, cy, cz); };
  F3 s{0.f, 0.f, 0.f};
  if (sx.hi - sx.lo <= 1 && sy.hi - sy.lo <= 1 && sz.hi - sz.lo <= 1) {
    F3 v[2][2][2];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i)
          v[k][j][i] = ldf3(addr(min(sx.lo + i, sx.hi), min(sy.lo + j, sy.hi), min(sz.lo + k, sz.hi)));
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i)
          if (sz.lo + k <= sz.hi && sy.lo + j <= sy.hi && sx.lo + i <= sx.hi) {
            s.x += v[k][j][i].x;
            s.y += v[k][j][i].y;
            s.z += v[k][j][i].z;
          }
    return s;
  }
  for (int bz = sz.lo; bz <= sz.hi; ++bz)
    for (int by = sy.lo; by <= sy.hi; ++by)
      for (int bx = sx.lo; bx <= sx.hi; ++bx) {
        const F3 v = ldf3(addr(bx, by, bz));
        s.x += v.x;
        s.y += v.y;
        s.z += v.z;
      }
  return s;
}

// Pass 2's workgroups: a wave takes up to 64 control points along x of one
// control row (cy, cz), so the y- and z-brick spans, and their address terms,
// are uniform over the wave (scalar).  A workgroup holds kGatherWaves rows.
constexpr int kGatherWaves = 4;
constexpr int kGatherThreads = kGatherWaves * kWave;

__host__ __device__ inline int adj_gather_xblocks(const VolGeom& g) { return (g.gx + kWave - 1) / kWave; }
__host__ __device__ inline int adj_gather_yblocks(const VolGeom& g) {
  return (g.gy + kGatherWaves - 1) / kGatherWaves;
}
__host__ __device__ inline int64_t adj_gather_blocks(const VolGeom& g) {
  return (int64_t)adj_gather_xblocks(g) * adj_gather_yblocks(g) * g.gz;
}

// Control point of lane `lane` of wave `wave` of pass-2 workgroup blk
// (blk < adj_gather_blocks < 2^31); false for a lane past the grid.
__host__ __device__ inline bool adj_gather_index(const VolGeom& g, int blk, int wave, int lane, int& cx, int& cy,
                                                 int& cz) {
  const int nxb = adj_gather_xblocks(g), nyb = adj_gather_yblocks(g);
  const int xb = blk % nxb;
  blk /= nxb;
  cy = (blk % nyb) * kGatherWaves + wave;
  cz = blk / nyb;
  cx = xb * kWave + lane;
  return cy < g.gy && cx < g.gx;
}

// Workgroup blk of pass 2, thread tid.
__device__ __forceinline__ void adj_gather_block(const float* __restrict__ part, float* __restrict__ grad,
                                                 const AdjGeom& a, int blk, int tid) {
  int cx, cy, cz;
  if (!adj_gather_index(a.g, blk, uniform(tid / kWave), tid & (kWave - 1), cx, cy, cz)) return;
  const size_t i = ((size_t)cz * a.g.gy + cy) * a.g.gx + cx;
  stf3(grad + i * 3, adj_gather_point(part, a, cx, cy, cz));
}

}  // namespace bsi
