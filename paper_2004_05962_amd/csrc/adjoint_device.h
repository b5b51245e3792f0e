// Adjoint of Eq. 1 (its transpose), as a deterministic two-pass gather.
//
// Pass 1 (one workgroup per brick).  Each axis is cut into bricks of a fixed
// number of whole tiles (rows instead when a y-tile is taller than a brick),
// the last brick holding the rest: kAdjTilesX x-tiles, at most kAdjMaxY rows
// and about kAdjTargetZ planes per brick.  A workgroup reads its brick's dfield
// exactly once.  Each thread owns one x-tile of one row (lane = x-tile, 16 tiles x 4
// rows per wave) and marches along z.  At every voxel plane it loads the tile
// row's dx voxels (contiguous) and forms the four x-moments
//   M_l = sum_o Bx_l(o) * dfield[z][y][tx*dx + o]          (l = 0..3)
// with weights that are the same for every lane.  The 16 lanes of a row hold
// the brick's 16 x-tiles, so the x-contraction of the plane row is finished
// right there, with row rotations across lanes (DPP):
//   S[cx] = sum_l M_l of tile (cx - l)                         (l ascending)
// lane t forms column t and, for t < 3, column 16 + t (the columns past the
// last tile).  These two columns are accumulated into the four control planes
// the current z-tile touches,
//   A[n] += Bz_n(w) * S                                        (n = cz - tz).
// When a z-tile ends, plane A[0] is finished and goes to an LDS slot; after
// every second finished plane the workgroup contracts the buffered pair over y
// (one barrier per pair),
//   G[cy][cx] = sum_m sum_{y in tile cy-m} By_m(v(y)) * A[0][y][cx],
// and writes G, the brick's partial gradient of those control planes.  Every
// brick writes its whole window of (cz, cy, cx) partials to the workspace.
//
// Pass 2 (one thread per control point) sums the partials of the bricks whose
// voxels touch the point (at most 2 per axis when a brick spans >= 3 tiles), in
// fixed brick order.  No atomics anywhere: the bits depend on the inputs only.
//
// The x-tile loop is specialised for spacings 1..kAdjMaxDX (fully unrolled, so
// every load of a tile row is in flight at once); larger spacings use a generic
// loop over chunks of kAdjChunk.  Both perform the same operations in the same
// order.
#pragma once

#include "bsi_device.h"

namespace bsi {

#ifndef BSI_ADJ_TILES_X
#define BSI_ADJ_TILES_X 16
#endif
constexpr int kAdjTilesX = BSI_ADJ_TILES_X;        // x-tiles per brick (= lanes per row)
constexpr int kAdjThreads = 512;
constexpr int kAdjMaxY = kAdjThreads / kAdjTilesX;  // rows per brick
constexpr int kAdjMaxCx = kAdjTilesX + 4;           // window bound in x
// The decomposition is a function of the geometry and these constants only,
// never of the device, so the bits never depend on the GPU it runs on.
#ifndef BSI_ADJ_TARGET_Z
#define BSI_ADJ_TARGET_Z 24
#endif
constexpr int kAdjTargetZ = BSI_ADJ_TARGET_Z;       // brick depth bound (voxels)
constexpr int kAdjMaxDX = 12;                       // largest specialised x spacing
constexpr int kAdjChunk = 4;                        // generic path: voxels per step
// Voxel planes of loads in flight per wave.  Two cost 3 DX more VGPRs per
// lane: up to DX = 7 that stays within 128 (two 512-thread workgroups per CU,
// as many as the LDS allows); from DX = 8 the LDS admits one workgroup per CU,
// which leaves 256 VGPRs per lane.
#ifndef BSI_ADJ_PREFETCH_MAX_DX
#define BSI_ADJ_PREFETCH_MAX_DX 12
#endif
__host__ __device__ constexpr int adj_prefetch(int dx) { return dx <= BSI_ADJ_PREFETCH_MAX_DX ? 2 : 1; }
static_assert(kWave % kAdjTilesX == 0, "a wave holds whole rows of tiles");

constexpr int kAdjWaves = kAdjThreads / kWave;
constexpr int kAdjRowsPerWave = kWave / kAdjTilesX;  // a wave holds whole rows of tiles
constexpr int kAdjSlotsX = 4;  // x-combined planes buffered in LDS (two pairs)

// Per-wave LDS region: the wave's tile rows of one voxel plane (64 * DX voxels)
// on their way from coalesced loads to tile-owning lanes.  Each wave only ever
// touches its own region.  The generic path (DX == 0) reads global memory
// directly and needs none.
__host__ __device__ constexpr int adj_wave_buf(int dx) { return dx > 0 ? kWave * dx * 3 : 1; }

constexpr int kAdjMaxCy = kAdjMaxY + 4;  // y-window bound (32 one-row units)

// LDS of the emission (finished control planes and the brick's y tables).
struct AdjEmitSmem {
  float Sx[kAdjSlotsX * kAdjMaxY * kAdjMaxCx * 3];     // finished planes, x-contracted
  float WYC[kAdjMaxCy * kAdjMaxY];                    // By weight of brick row y for window row cy
  int YR[kAdjMaxCy * 2];                              // rows [ya, yb) of the brick in cy's support
};

template <int DX>
struct AdjSmem {
  float T[kAdjWaves * adj_wave_buf(DX)];              // per-wave transpose buffers
  AdjEmitSmem e;
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

// Finished control plane number k of the brick (czl = cz - cz0).  Collective:
// every thread of the workgroup calls it with its (row, column) values of
// A[0]: cm for column txl, cw for column 16 + txl (lanes txl < 3); zero for
// idle threads.
//  1. Every thread writes its columns of the plane into LDS slot k % 4.
//  2. After every second plane (and after the brick's last one) one barrier,
//     then the y-contraction of the buffered planes, over the brick rows in
//     cy's support in ascending order:
//       G[cy][cx] = sum_y By_{cy - floor(y/dy)}(v(y)) * Sx[y][cx]
//     written to the brick's partials.
// Slot reuse: plane k + 4 overwrites slot k % 4 only after the barrier of the
// pair k + 2, k + 3, which every thread passes after its y-contraction of k.
__device__ __forceinline__ void adj_emit(const AdjGeom& a, const AdjBrick& b, float* __restrict__ pbase,
                                         AdjEmitSmem& sm, int tid, int k, int czl, bool last, const F3& cm,
                                         const F3& cw) {
  {
    const int txl = tid % kAdjTilesX;
    const int yl = tid / kAdjTilesX;
    float* row = sm.Sx + (k % kAdjSlotsX) * (kAdjMaxY * kAdjMaxCx * 3) + yl * (kAdjMaxCx * 3);
    if (yl < b.ye - b.y0) {
      if (txl < b.Cx) stf3(row + txl * 3, cm);
      if (txl < 3 && kAdjTilesX + txl < b.Cx) stf3(row + (kAdjTilesX + txl) * 3, cw);
    }
  }
  if (!(k & 1) && !last) return;  // the y-contraction waits for the pair

  __syncthreads();
  const int npend = (k & 1) ? 2 : 1;  // planes k-1, k  or  k alone
  // item -> (plane p, window row cyl, window column cxl < Cx): every thread
  // of a round has an item (Cx <= 19 columns, not a 32-wide slot)
  const int per_plane = b.Cy * b.Cx;
  for (int it = tid; it < npend * per_plane; it += kAdjThreads) {
    const int p = it >= per_plane ? 1 : 0;
    const int r = it - p * per_plane;
    const int cyl = r / b.Cx;
    const int cxl = r - cyl * b.Cx;
    const int kk = k - (npend - 1) + p;
    const float* sp = sm.Sx + (kk % kAdjSlotsX) * (kAdjMaxY * kAdjMaxCx * 3) + cxl * 3;
    const float* wrow = sm.WYC + cyl * kAdjMaxY;
    const int ya = sm.YR[2 * cyl], yb = sm.YR[2 * cyl + 1];
    float ax = 0.f, ay = 0.f, az = 0.f;
#pragma unroll 4
    for (int yl = ya; yl < yb; ++yl) {
      const float wv = wrow[yl];
      const float* q = sp + yl * (kAdjMaxCx * 3);
      ax = fmaf(wv, q[0], ax);
      ay = fmaf(wv, q[1], ay);
      az = fmaf(wv, q[2], az);
    }
    const int cz_l = czl - (k - kk);
    stf3(pbase + adj_part_offset(a, cz_l, cyl, cxl), F3{ax, ay, az});
  }
}

// Value of lane (i - N) mod 16 of this lane's row of 16 lanes (DPP row_ror).
template <int N>
__device__ __forceinline__ float row_ror(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x120 + N, 0xF, 0xF, false));
}

template <int L>
__device__ __forceinline__ void adj_xcombine_term(int txl, const F3& m, F3& cm, F3& cw) {
  const F3 r{row_ror<L>(m.x), row_ror<L>(m.y), row_ror<L>(m.z)};  // M_L of tile txl - L (mod 16)
  if (txl >= L) {
    cm.x += r.x;
    cm.y += r.y;
    cm.z += r.z;
  } else {
    cw.x += r.x;
    cw.y += r.y;
    cw.z += r.z;
  }
}

// x-contraction of one plane row across the 16 tile lanes of a row:
//   cm = S[txl]      = sum_{l <= txl} M_l(tile txl - l)
//   cw = S[16 + txl] = sum_{l > txl}  M_l(tile 16 + txl - l)   (txl < 3)
// l ascending.  Idle lanes hold M = 0, so columns past the brick's last tile
// come out right.  Every lane of the wave takes part (no lane may be inactive).
__device__ __forceinline__ void adj_xcombine(int txl, const F3 (&M)[4], F3& cm, F3& cw) {
  cm = M[0];
  cw = F3{0.f, 0.f, 0.f};
  adj_xcombine_term<1>(txl, M[1], cm, cw);
  adj_xcombine_term<2>(txl, M[2], cm, cw);
  adj_xcombine_term<3>(txl, M[3], cm, cw);
}

// One step of the x-moments: voxel o of the tile row with value d.
__device__ __forceinline__ void adj_xmoment_step(int o, const float* __restrict__ w, const F3& d, F3 (&M)[4]) {
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    if (o == 0) {
      M[l].x = w[l] * d.x;
      M[l].y = w[l] * d.y;
      M[l].z = w[l] * d.z;
    } else {
      M[l].x = fmaf(w[l], d.x, M[l].x);
      M[l].y = fmaf(w[l], d.y, M[l].y);
      M[l].z = fmaf(w[l], d.z, M[l].z);
    }
  }
}

// x-moments of one tile row: M_l = sum_o Bx_l(o) d(o), o ascending, over the
// voxels o < nval of the tile (nval < dx only for the volume's last tile; 0
// for idle threads, which then keep M = 0).  DX > 0: compile-time spacing, all
// loads issued together (adj_row_load / adj_row_moments, so the next plane's
// row can be in flight while this one is reduced).  DX == 0: runtime spacing,
// chunks of kAdjChunk loads.
// Coalesced loads of the wave's part of one voxel plane, for DX <= kAdjMaxDX:
// the wave's kAdjRowsPerWave rows x (kAdjTilesX * DX) voxels, enumerated
// v = row * kAdjTilesX * DX + x; lane j loads v = k * 64 + j (k < DX), i.e.
// consecutive lanes read consecutive 12-byte voxels.
template <int DX>
__host__ __device__ inline void adj_plane_offsets(const AdjBrick& b, int nx, int ywave, int lane,
                                                  uint32_t (&off)[DX]) {
  // Every lane loads from a valid address, clamped into the brick, with no
  // branch or select around the load (the data is only consumed one plane
  // later).  A clamped slot holds a copy of another voxel, but no lane reads
  // it: tile rows stop at the volume (nval) and rows outside the brick belong
  // to idle lanes.  The offsets (in floats, within a voxel plane) are the same
  // for every plane of the brick, so they are formed once.
#pragma unroll
  for (int k = 0; k < DX; ++k) {
    const int v = k * kWave + lane;
    const int r = v / (kAdjTilesX * DX);
    const int xl = v - r * (kAdjTilesX * DX);
    const int x = imin(b.x0 + xl, b.xe - 1), y = imin(ywave + r, b.ye - 1);
    off[k] = ((uint32_t)y * (uint32_t)nx + (uint32_t)x) * 3u;  // a plane holds < 2^32 floats (make_geom)
  }
}

// Streaming load of one voxel of dfield: non-temporal, since every voxel is
// read once.  The read stream then does not leave the caches full of dfield
// lines that the following kernel's writes have to displace (measured: the
// next forward 0.180 -> 0.171 ms, pass 1 itself a few percent faster).
template <bool Stream>
__device__ __forceinline__ F3 ldf3_dfield(const float* p) {
  if constexpr (Stream)
    return F3{__builtin_nontemporal_load(p), __builtin_nontemporal_load(p + 1), __builtin_nontemporal_load(p + 2)};
  else
    return ldf3(p);
}

template <int DX, bool Stream>
__device__ __forceinline__ void adj_plane_load(const float* __restrict__ plane, const uint32_t (&off)[DX],
                                               F3 (&d)[DX]) {
#pragma unroll
  for (int k = 0; k < DX; ++k) d[k] = ldf3_dfield<Stream>(plane + off[k]);
}

// Stage a loaded plane in the wave's LDS region (lanes exchange data: tile rows
// come out of coalesced loads).
template <int DX>
__device__ __forceinline__ void adj_plane_stage(float* __restrict__ buf, int lane, const F3 (&d)[DX]) {
  wave_lds_sync();  // previous readers of the region are done
#pragma unroll
  for (int k = 0; k < DX; ++k) stf3(buf + (k * kWave + lane) * 3, d[k]);
  wave_lds_sync();
}

// x-moments of this lane's tile row (row r = lane / kAdjTilesX, tile
// txl = lane % kAdjTilesX), read from the staged plane: rows of up to 5 voxels
// at once, longer rows in chunks of kAdjChunk (the chunk loop stays rolled, so
// the register footprint does not grow with the spacing).  Same
// operations, same order as adj_xmoments_generic.
template <int DX>
__device__ __forceinline__ void adj_plane_moments(const float* __restrict__ buf, int lane, int nval,
                                                  const float* __restrict__ lutx, F3 (&M)[4]) {
  constexpr int C = DX <= 5 ? DX : kAdjChunk;  // short rows in one chunk
  const int r = lane / kAdjTilesX, txl = lane % kAdjTilesX;
  const float* p = buf + (r * kAdjTilesX * DX + txl * DX) * 3;
#pragma unroll
  for (int l = 0; l < 4; ++l) M[l] = F3{0.f, 0.f, 0.f};
#pragma unroll 1
  for (int o0 = 0; o0 < DX; o0 += C) {
    F3 v[C];
#pragma unroll
    for (int j = 0; j < C; ++j) v[j] = o0 + j < DX ? ldf3(p + 3 * (o0 + j)) : F3{0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < C; ++j)
      if (o0 + j < nval) adj_xmoment_step(o0 + j, lutx + 4 * (o0 + j), v[j], M);
  }
}


template <bool Stream>
__device__ __forceinline__ void adj_xmoments_generic(const float* __restrict__ row, int nval,
                                                     const float* __restrict__ lutx, F3 (&M)[4]) {
#pragma unroll
  for (int l = 0; l < 4; ++l) M[l] = F3{0.f, 0.f, 0.f};
  for (int o0 = 0; o0 < nval; o0 += kAdjChunk) {
    F3 d[kAdjChunk];
#pragma unroll
    for (int j = 0; j < kAdjChunk; ++j) d[j] = o0 + j < nval ? ldf3_dfield<Stream>(row + 3 * (o0 + j)) : F3{0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < kAdjChunk; ++j)
      if (o0 + j < nval) adj_xmoment_step(o0 + j, lutx + 4 * (o0 + j), d[j], M);
  }
}

// Per-brick y tables of the emission: WYC[cyl][yl] = By weight of brick row yl
// for window row cyl (0 outside cy's support), YR[cyl] = the support's rows.
// Collective; the first y-contraction's barrier orders these writes before any read.
__device__ __forceinline__ void adj_tables(const AdjGeom& a, const AdjBrick& b, const float* __restrict__ lut,
                                           AdjEmitSmem& sm, int tid) {
  const VolGeom& g = a.g;
  __syncthreads();  // a previous brick of this workgroup may still read the tables
  // Window row cyl (cy = cy0 + cyl) collects brick rows y with
  // cy - 3 <= floor(y/dy) <= cy, a contiguous range; weight By_{cy - floor(y/dy)}.
  for (int i = tid; i < b.Cy * kAdjMaxY; i += kAdjThreads) {
    const int cyl = i / kAdjMaxY, yl = i - cyl * kAdjMaxY;
    const int y = b.y0 + yl;
    float wv = 0.f;
    if (y < b.ye) {
      const int t = y / g.dy;
      const int m = b.cy0 + cyl - t;
      if (m >= 0 && m < 4) wv = lut_row(lut, g.dy, y - t * g.dy)[m];
    }
    sm.WYC[i] = wv;
  }
  for (int cyl = tid; cyl < b.Cy; cyl += kAdjThreads) {
    const int cy = b.cy0 + cyl;
    sm.YR[2 * cyl] = max(max(0, (cy - 3) * g.dy), b.y0) - b.y0;
    sm.YR[2 * cyl + 1] = max(min((cy + 1) * g.dy, b.ye) - b.y0, sm.YR[2 * cyl]);
  }
}

// Pass 1 for one brick.  Collective over the workgroup (kAdjThreads threads).
// Stream: dfield is read with non-temporal loads.
template <int DX, bool Stream = true>
__device__ __forceinline__ void adj_brick(const float* __restrict__ dfield, float* __restrict__ part,
                                          const AdjGeom& a, const float* __restrict__ lut, int brick,
                                          AdjSmem<DX>& sm, int tid) {
  const VolGeom& g = a.g;
  const int dx = DX > 0 ? DX : g.dx;
  const AdjBrick b = adj_brick_geom(a, brick);
  float* pbase = part + (size_t)brick * adj_brick_stride(a);

  adj_tables(a, b, lut, sm.e, tid);
  // (the first y-contraction's barrier orders these writes before any read)

  const int txl = tid % kAdjTilesX;
  const int yl = tid / kAdjTilesX;
  const int y = b.y0 + yl;
  const int tx = b.cx0 + txl;
  const bool act = txl < b.ntx && y < b.ye;
  const int x = tx * dx;
  const int nval = act ? min(dx, g.nx - x) : 0;  // voxels of this tile row
  const size_t zs = (size_t)g.ny * g.nx * 3;
  const float* src = dfield + (((size_t)b.z0 * g.ny + (act ? y : 0)) * g.nx + (act ? x : 0)) * 3;
  const float* lutx = lut_row(lut, dx, 0);

  F3 acc[4], accw[4];  // columns txl and 16 + txl of control planes tz + n
#pragma unroll
  for (int n = 0; n < 4; ++n) acc[n] = accw[n] = F3{0.f, 0.f, 0.f};

  int tz = b.cz0;
  int oz = b.z0 - tz * g.dz;
  const int lane = tid & (kWave - 1);
  const int ywave = b.y0 + (tid / kWave) * kAdjRowsPerWave;
  float* wbuf = sm.T + (tid / kWave) * adj_wave_buf(DX);
  const float* plane0 = dfield + (size_t)b.z0 * zs;

  // One voxel plane: x-moments of this lane's tile row, z-accumulation, and the
  // emission of the finished control plane when a z-tile ends.
  auto step = [&](const F3 (&M)[4], int z) {
    F3 cm, cw;
    adj_xcombine(txl, M, cm, cw);
    const float* wz = lut_row(lut, g.dz, oz);
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
      }
      acc[3] = accw[3] = F3{0.f, 0.f, 0.f};
      oz = 0;
      ++tz;
    }
  };

  if constexpr (DX > 0) {
    // Per plane: wait for its loads (issued kAhead planes earlier), stage them
    // in LDS, which frees their registers, issue the loads of the plane kAhead
    // ahead into them, then read back this lane's tile row and reduce it.
    // kAhead planes of loads are in flight while a plane is reduced (and
    // emitted).  With two, the loop is unrolled by two so that
    // each register set keeps fixed names.
    uint32_t off[DX];
    adj_plane_offsets<DX>(b, g.nx, ywave, lane, off);
    auto plane = [&](int z) { return plane0 + (size_t)(z - b.z0) * zs; };
    constexpr int kAhead = adj_prefetch(DX);
    auto consume = [&](F3 (&d)[DX], int z) {
      adj_plane_stage<DX>(wbuf, lane, d);
      if (z + kAhead < b.ze) adj_plane_load<DX, Stream>(plane(z + kAhead), off, d);
      F3 M[4];
      adj_plane_moments<DX>(wbuf, lane, nval, lutx, M);
      step(M, z);
    };
    F3 d0[DX];
    adj_plane_load<DX, Stream>(plane0, off, d0);
    if constexpr (kAhead == 1) {
      for (int z = b.z0; z < b.ze; ++z) consume(d0, z);
    } else {
      F3 d1[DX];
      if (b.z0 + 1 < b.ze) adj_plane_load<DX, Stream>(plane(b.z0 + 1), off, d1);
      for (int z = b.z0; z < b.ze; z += 2) {
        consume(d0, z);
        if (z + 1 >= b.ze) break;
        consume(d1, z + 1);
      }
    }
  } else {
    for (int z = b.z0; z < b.ze; ++z) {
      F3 M[4];
      adj_xmoments_generic<Stream>(src, nval, lutx, M);
      src += zs;
      step(M, z);
    }
  }
  // The last tile's four planes (the last three are shared with the next brick),
  // shifted through acc[0] so the emission is instantiated once more, not four times.
#pragma unroll 1
  for (int n = 0; n < 4; ++n) {
    adj_emit(a, b, pbase, sm.e, tid, tz - b.cz0 + n, tz - b.cz0 + n, n == 3, acc[0], accw[0]);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      acc[j] = acc[j + 1];
      accw[j] = accw[j + 1];
    }
  }
}

// ----------------------------------------------------------------------------
// Pass 1, z-first ("column march").  A brick is kAdjZBX = 64 consecutive
// x-voxels (one per lane) by kAdjZBY rows by a run of whole z-tiles.  Wave w of
// the workgroup owns rows y0 + w R .. y0 + w R + R - 1 (R = kAdjZRows), so each
// lane owns one voxel column per row and marches z.  Per voxel plane it loads
// its R voxels (a wave reads 768 contiguous bytes per row, coalesced) and
// accumulates the z-contraction of Eq. 1's transpose in registers,
//   A_r[n] += Bz_n(w) * dfield[z][y_r][x]        (n = cz - tz, 4 planes),
// the only per-voxel work.  When a z-tile ends, plane A[0] is finished for the
// brick's voxel rows: it is contracted over x and y in LDS,
//   H[y][cx]  = sum_x Bx_{cx - floor(x/dx)}(u(x)) A0[y][x]   (x ascending)
//   G[cy][cx] = sum_y By_{cy - floor(y/dy)}(v(y)) H[y][cx]   (y ascending)
// and G is written as the brick's partial gradient of that control plane.  The
// x-contraction is per wave (its own rows, wave-private LDS); H is
// double-buffered, so one workgroup barrier per finished plane orders the
// x-contraction of plane k before the y-contraction of plane k, and the
// y-contraction of plane k - 1 before the x-contraction of plane k + 1.
// Pass 2 (unchanged) sums the partials of the bricks meeting each point.
// ----------------------------------------------------------------------------
#ifndef BSI_ADJZ_ROWS
#define BSI_ADJZ_ROWS 2
#endif
#ifndef BSI_ADJZ_WAVES
#define BSI_ADJZ_WAVES 8
#endif
#ifndef BSI_ADJZ_TARGET_Z
#define BSI_ADJZ_TARGET_Z 48
#endif
constexpr int kAdjZRows = BSI_ADJZ_ROWS;              // rows per lane (R)
constexpr int kAdjZWaves = BSI_ADJZ_WAVES;            // waves per workgroup
constexpr int kAdjZThreads = kAdjZWaves * kWave;
constexpr int kAdjZBX = kWave;                         // brick width (voxels)
constexpr int kAdjZBY = kAdjZWaves * kAdjZRows;        // brick height (rows)
constexpr int kAdjZTargetZ = BSI_ADJZ_TARGET_Z;        // brick depth bound (voxels, at least one tile)
#ifndef BSI_ADJZ_WPE
#define BSI_ADJZ_WPE 6
#endif
#ifndef BSI_ADJZ_AHEAD
#define BSI_ADJZ_AHEAD 2
#endif
constexpr int kAdjZAhead = BSI_ADJZ_AHEAD;             // voxel planes of loads in flight per wave

// Window columns of a brick of kAdjZBX voxels at x spacing dx (0: any spacing
// above kAdjMaxDX): a run of w voxels meets at most (w - 1)/dx + 2 tiles, and
// exactly w / dx when the run is whole tiles (spacing 1).
__host__ __device__ constexpr int adjz_cx_max(int dx) {
  return dx == 1 ? kAdjZBX + 3 : (kAdjZBX - 1) / (dx > 0 ? dx : kAdjMaxDX + 1) + 5;
}
constexpr int kAdjZCyMax = kAdjZBY + 3;  // window rows at spacing 1 (the most)
// Finished partial planes are staged in LDS and stored in batches.  On this
// chip loads and stores share one counter of outstanding memory operations,
// and a store issued while loads are in flight makes the next wait for a load
// wait for everything: a store per finished plane would drain the planes of
// loads in flight at every z-tile.  With the partials of a whole brick staged
// (spacings of 5 and more), they are stored once, after the brick's last load.
#ifndef BSI_ADJZ_STAGE_FLOATS
#define BSI_ADJZ_STAGE_FLOATS 6144
#endif
constexpr int kAdjZStageFloats = BSI_ADJZ_STAGE_FLOATS;  // 24 KB
// The x-contraction of a finished plane runs on tile lanes (16 x-tiles per row
// of 16 lanes) when a brick row holds at most 16 tiles: x spacing 4 (bricks
// start on multiples of 64, so exactly 16 tiles), 5..12, and the generic path
// (spacing 13 or more, at most 6 tiles).  Spacings 1..3 sum each column
// directly (adjz_xsum).
__host__ __device__ constexpr bool adjz_tile_lanes(int dx) { return dx == 0 || dx >= 4; }
static_assert(kAdjTilesX == 16 && kWave / kAdjTilesX >= kAdjZRows, "a wave's rows fit its rows of 16 tile lanes");

template <int DX>
struct AdjZSmem {
  float F[kAdjZWaves][kAdjZRows * kWave * 3];       // finished plane, this wave's rows (wave-private)
  float H[2][kAdjZBY * adjz_cx_max(DX) * 3];         // x-contracted rows, double-buffered
  float WYC[kAdjZCyMax * kAdjZBY];                  // By weight of brick row y for window row cy
  int YR[kAdjZCyMax * 2];                           // rows [ya, yb) of the brick in cy's support
  float P[kAdjZStageFloats];                        // finished partial planes awaiting their store
};

// Whether a brick's whole window of partials (cm_z planes of cm_y * cm_x
// points) fits the LDS stage; otherwise each plane is stored as it is finished.
__host__ __device__ inline bool adjz_stage_all(const AdjGeom& a) {
  return (long)a.z.cm * a.y.cm * a.x.cm * 3 <= kAdjZStageFloats;
}

// Per-brick y tables: WYC[cyl][yl] = By weight of brick row yl for window row
// cyl (0 outside cy's support), YR[cyl] = the support's rows within the brick.
// Collective; a leading barrier keeps a previous brick's readers safe, and the
// first finished plane's barrier orders these writes before any read.
__device__ __forceinline__ void adjz_tables(const AdjGeom& a, const AdjBrick& b, const float* __restrict__ lut,
                                            float* __restrict__ WYC, int* __restrict__ YR, int tid) {
  const VolGeom& g = a.g;
  __syncthreads();
  for (int i = tid; i < b.Cy * kAdjZBY; i += kAdjZThreads) {
    const int cyl = i / kAdjZBY, yl = i - cyl * kAdjZBY;
    const int y = b.y0 + yl;
    float wv = 0.f;
    if (y < b.ye) {
      const int t = y / g.dy;
      const int m = b.cy0 + cyl - t;
      if (m >= 0 && m < 4) wv = lut_row(lut, g.dy, y - t * g.dy)[m];
    }
    WYC[i] = wv;
  }
  for (int cyl = tid; cyl < b.Cy; cyl += kAdjZThreads) {
    const int cy = b.cy0 + cyl;
    YR[2 * cyl] = max(max(0, (cy - 3) * g.dy), b.y0) - b.y0;
    YR[2 * cyl + 1] = max(min((cy + 1) * g.dy, b.ye) - b.y0, YR[2 * cyl]);
  }
}

// Offsets (floats, within a voxel plane) of this lane's R voxels: row
// y0 + wave R + r, column x0 + lane, both clamped into the brick so that every
// lane loads from a valid address without a branch.  A clamped lane's values
// are never read: the x-contraction reads only columns inside the brick and
// the y-contraction only rows inside it.  A plane holds < 2^32 floats.
template <int R>
__host__ __device__ inline void adjz_offsets(const AdjBrick& b, int nx, int wave, int lane, uint32_t (&off)[R]) {
  const int x = imin(b.x0 + lane, b.xe - 1);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int y = imin(b.y0 + wave * R + r, b.ye - 1);
    off[r] = ((uint32_t)y * (uint32_t)nx + (uint32_t)x) * 3u;
  }
}

// x-contraction of one window column cxl for brick row r of this wave:
//   sum over voxels x of the brick in cx's support [(cx-3)dx, (cx+1)dx),
//   ascending, of Bx_{cx - floor(x/dx)}(x - floor(x/dx) dx) * F[r][x - x0].
template <int DX>
__device__ __forceinline__ F3 adjz_xsum(const float* __restrict__ Fr, const AdjBrick& b, int dx, int cx,
                                        const float* __restrict__ lut) {
  F3 s{0.f, 0.f, 0.f};
  if constexpr (DX > 0) {
    // one tile at a time: its DX voxel loads in flight together, few registers
    // (the emission runs while the z-accumulators and the next planes' loads
    // are live)
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
  } else {
    const int lo = imax((cx - 3) * dx, b.x0), hi = imin((cx + 1) * dx, b.xe);
    for (int x = lo; x < hi; ++x) {
      const int t = x / dx;
      const float w = lut_row(lut, dx, x - t * dx)[cx - t];
      const float* q = Fr + (x - b.x0) * 3;
      s.x = fmaf(w, q[0], s.x);
      s.y = fmaf(w, q[1], s.y);
      s.z = fmaf(w, q[2], s.z);
    }
  }
  return s;
}

// Values of the neighbouring lanes within a quad (DPP quad_perm): lane ^ 1 and
// lane ^ 2.  After s += swap1(s) and then s += swap2(s), every lane of the quad
// holds (l0 + l1) + (l2 + l3) with the same bits (addition is commutative).
__device__ __forceinline__ float quad_swap1(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ float quad_swap2(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, false));
}

// Finished control plane number k of the brick (czl = its window index).
// Collective over the workgroup; f[r] is this lane's value of A0 for row r.
template <int DX, bool StageAll>
__device__ __forceinline__ void adjz_emit(const AdjGeom& a, const AdjBrick& b, float* __restrict__ pbase,
                                          AdjZSmem<DX>& sm, const float* __restrict__ lut, int tid, int czl,
                                          bool last, const F3 (&f)[kAdjZRows]) {
  constexpr int CXM = adjz_cx_max(DX);
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  const int dx = DX > 0 ? DX : a.g.dx;
  float* Fw = sm.F[wave];
  wave_lds_sync();  // this wave's x-contraction of the previous plane is done with Fw
#pragma unroll
  for (int r = 0; r < kAdjZRows; ++r) stf3(Fw + (r * kWave + lane) * 3, f[r]);
  wave_lds_sync();
  float* H = sm.H[czl & 1];  // czl counts the brick's finished planes
  const int nrow = b.ye - b.y0 - wave * kAdjZRows;  // this wave's rows inside the brick
  if constexpr (adjz_tile_lanes(DX)) {
    // Tile lanes: lane (rr, t) = (lane / 16, lane % 16) forms the x-moments of
    // tile cx0 + t in row rr of this wave,
    //   M_l = sum_o Bx_l(o) F[rr][t dx + o - x0]    (o ascending, voxels in the brick)
    // each voxel read once; the 16 lanes of a row then finish the columns with
    // row rotations (adj_xcombine): column t and, for t < 3, column 16 + t.
    const int rr = lane / kAdjTilesX, t = lane % kAdjTilesX;
    const bool act = rr < kAdjZRows && rr < nrow && t < b.ntx;
    F3 M[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) M[l] = F3{0.f, 0.f, 0.f};
    if (act) {
      const int xt = (b.cx0 + t) * dx - b.x0;  // the tile's first voxel, brick-relative (may be < 0)
      const float* Fr = Fw + rr * kWave * 3;
      const int nxb = b.xe - b.x0;
      auto voxel = [&](int o) {
        const int xl = xt + o;
        if (xl >= 0 && xl < nxb) {
          const float* w = lut_row(lut, dx, o);
          const F3 v = ldf3(Fr + xl * 3);
#pragma unroll
          for (int l = 0; l < 4; ++l) {
            M[l].x = fmaf(w[l], v.x, M[l].x);
            M[l].y = fmaf(w[l], v.y, M[l].y);
            M[l].z = fmaf(w[l], v.z, M[l].z);
          }
        }
      };
      // pairs of voxels in flight: few registers while the z-accumulators and
      // the next planes' loads are live
#pragma unroll 1
      for (int o = 0; o < dx; o += 2) {
        voxel(o);
        if (o + 1 < dx) voxel(o + 1);
      }
    }
    F3 cm, cw;
    adj_xcombine(t, M, cm, cw);  // every lane of the wave takes part
    if (rr < kAdjZRows && rr < nrow) {
      float* hrow = H + (wave * kAdjZRows + rr) * CXM * 3;
      if (t < b.Cx) stf3(hrow + t * 3, cm);
      if (t < 3 && kAdjTilesX + t < b.Cx) stf3(hrow + (kAdjTilesX + t) * 3, cw);
    }
  } else {
    const int items = imin(nrow, kAdjZRows) * b.Cx;
    for (int it = lane; it < items; it += kWave) {
      const int r = it / b.Cx, cxl = it - r * b.Cx;
      stf3(H + ((wave * kAdjZRows + r) * CXM + cxl) * 3, adjz_xsum<DX>(Fw + r * kWave * 3, b, dx, b.cx0 + cxl, lut));
    }
  }
  __syncthreads();
  // y-contraction: wave w takes window rows cyl = w, w + kAdjZWaves, ...;
  // lane j takes columns cxl = j, j + 64, ...  Every row y of cy's support
  // inside the brick is summed in ascending order with its By weight, which
  // is the same for the whole wave (a scalar load of the basis table).
  {
    const VolGeom& g = a.g;
    for (int cyl = wave; cyl < b.Cy; cyl += kAdjZWaves) {
      const int cy = b.cy0 + cyl;
      const int ya = imax(imax(0, (cy - 3) * g.dy), b.y0), yb = imin((cy + 1) * g.dy, b.ye);
      for (int cxl = lane; cxl < b.Cx; cxl += kWave) {
        const float* hp = H + cxl * 3;
        float ax = 0.f, ay = 0.f, az = 0.f;
        // tiles t of the support, ascending; rows y of each with offset y - t dy
        int t = ya / g.dy, oy = ya - t * g.dy;
#pragma unroll 1
        for (int y = ya; y < yb; ++y) {
          const float wv = lut_row(lut, g.dy, oy)[cy - t];
          const float* hq = hp + (y - b.y0) * CXM * 3;
          ax = fmaf(wv, hq[0], ax);
          ay = fmaf(wv, hq[1], ay);
          az = fmaf(wv, hq[2], az);
          if (++oy == g.dy) {
            oy = 0;
            ++t;
          }
        }
        if constexpr (StageAll)
          stf3(sm.P + adj_part_offset(a, czl, cyl, cxl), F3{ax, ay, az});
        else
          stf3(pbase + adj_part_offset(a, czl, cyl, cxl), F3{ax, ay, az});
      }
    }
  }
  // After the brick's last plane (its loads all done), the staged window goes
  // out as one contiguous run of whole (padded) planes.  A following brick of
  // this workgroup writes the stage only after adjz_tables' barrier.
  if constexpr (StageAll) {
    if (last) {
      __syncthreads();
      const int n = (czl + 1) * a.y.cm * a.x.cm;
      for (int i = tid; i < n; i += kAdjZThreads) stf3(pbase + i * 3, ldf3(sm.P + i * 3));
    }
  }
}

template <bool Stream>
__device__ __forceinline__ void adjz_load(const float* __restrict__ plane, const uint32_t (&off)[kAdjZRows],
                                          F3 (&d)[kAdjZRows]) {
#pragma unroll
  for (int r = 0; r < kAdjZRows; ++r) d[r] = ldf3_dfield<Stream>(plane + off[r]);
}

// Pass 1 for one brick, z-first.  Collective over the workgroup (kAdjZThreads
// threads).  Stream: dfield is read with non-temporal loads.
template <int DX, bool Stream = true, bool StageAll = false>
__device__ __forceinline__ void adjz_brick(const float* __restrict__ dfield, float* __restrict__ part,
                                           const AdjGeom& a, const float* __restrict__ lut, int brick,
                                           AdjZSmem<DX>& sm, int tid) {
  constexpr int R = kAdjZRows;
  const VolGeom& g = a.g;
  const AdjBrick b = adj_brick_geom(a, brick);
  float* pbase = part + (size_t)brick * adj_brick_stride(a);
  adjz_tables(a, b, lut, sm.WYC, sm.YR, tid);

  const int lane = tid & (kWave - 1), wave = uniform(tid / kWave);
  uint32_t off[R];
  adjz_offsets<R>(b, g.nx, wave, lane, off);
  const size_t zs = (size_t)g.ny * g.nx * 3;
  const float* plane0 = dfield + (size_t)b.z0 * zs;
  auto plane = [&](int z) { return plane0 + (size_t)(z - b.z0) * zs; };

  F3 acc[R][4];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int n = 0; n < 4; ++n) acc[r][n] = F3{0.f, 0.f, 0.f};
  int tz = b.cz0;        // z-bricks are whole tiles: b.z0 = tz * dz
  int oz = 0;
  auto emit0 = [&](int czl, bool last) {
    F3 f[R];
#pragma unroll
    for (int r = 0; r < R; ++r) f[r] = acc[r][0];
    adjz_emit<DX, StageAll>(a, b, pbase, sm, lut, tid, czl, last, f);
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int n = 0; n < 3; ++n) acc[r][n] = acc[r][n + 1];
      acc[r][3] = F3{0.f, 0.f, 0.f};
    }
  };
  // One voxel plane: z-accumulation, then the loads of the plane kAdjZAhead
  // planes ahead into the same registers (when that plane exists: Load), then
  // the emission when a z-tile ends.
  const float* ahead = nullptr;  // the plane kAdjZAhead ahead of the one consumed next
  auto consume = [&](F3 (&d)[R], int z, bool load) {
    const float* wz = lut_row(lut, g.dz, oz);
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const float w = wz[n];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        acc[r][n].x = fmaf(w, d[r].x, acc[r][n].x);
        acc[r][n].y = fmaf(w, d[r].y, acc[r][n].y);
        acc[r][n].z = fmaf(w, d[r].z, acc[r][n].z);
      }
    }
    if (load) adjz_load<Stream>(ahead, off, d);
    ahead += zs;  // plane z + 1 + kAdjZAhead
    if (++oz == g.dz && z + 1 < b.ze) {
      emit0(tz - b.cz0, false);
      oz = 0;
      ++tz;
    }
  };
  // kAdjZAhead register sets, each holding one plane's loads.  The loop is
  // unrolled over them, and its main part runs only while every plane of the
  // group and every plane kAdjZAhead ahead exists, so its loads are
  // unconditional: each set keeps fixed registers, and waiting for one set's
  // loads leaves the other sets' loads in flight.
  // (The first sets are loaded unconditionally, from the brick's last plane
  // when it is shallower, so the loop is entered with the same loads in flight
  // on every path and its waits count them exactly.)
  F3 d[kAdjZAhead][R];
#pragma unroll
  for (int j = 0; j < kAdjZAhead; ++j) adjz_load<Stream>(plane(imin(b.z0 + j, b.ze - 1)), off, d[j]);
  ahead = plane0 + (size_t)kAdjZAhead * zs;
  int z = b.z0;
  for (; z + 2 * kAdjZAhead <= b.ze; z += kAdjZAhead) {
#pragma unroll
    for (int j = 0; j < kAdjZAhead; ++j) consume(d[j], z + j, true);
  }
  for (; z < b.ze; z += kAdjZAhead) {
#pragma unroll
    for (int j = 0; j < kAdjZAhead; ++j)
      if (z + j < b.ze) consume(d[j], z + j, z + j + kAdjZAhead < b.ze);
  }
  // the last tile's four planes (the last three are shared with the next brick)
#pragma unroll 1
  for (int n = 0; n < 4; ++n) emit0(tz - b.cz0 + n, n == 3);
}

// Pass 2 for one control point (cx, cy, cz): fixed-order sum of brick partials.
// Bricks whose voxels meet the point's support [(c-3)d, (c+1)d) on each axis,
// summed bz, then by, then bx ascending.  When no axis has more than two such
// bricks (bricks of at least 3 tiles) all 8 loads are issued at once from
// clamped addresses and the valid ones added in that order; otherwise a loop.
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

}  // namespace bsi
