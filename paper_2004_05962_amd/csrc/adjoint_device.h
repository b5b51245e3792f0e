// Adjoint of Eq. 1 (its transpose), as a deterministic two-pass gather.
//
// Pass 1 (one workgroup per brick).  The volume is cut into bricks of
// xb x yb x zb voxels, aligned to tiles where the spacing allows.  A workgroup
// reads its brick's dfield exactly once, in coalesced 12-byte-per-lane loads
// (lane = x, 8 waves x 4 rows = 32 rows), marching along z.  Each column keeps
// the z-contraction for the 4 control planes its current tile touches,
//   A[n] += Bz_n(w) * dfield[z][y][x]       (n = cz - tz),
// and when a tile ends the finished plane is contracted over x and y in LDS:
//   Sx[y][cx] = sum_l sum_{x in tile cx-l} Bx_l(u(x)) * A(x, y)
//   G[cy][cx] = sum_m sum_{y in tile cy-m} By_m(v(y)) * Sx[y][cx]
// G is the brick's partial gradient for that control plane; every brick writes
// its whole window of (cz, cy, cx) partials to the workspace.
//
// Pass 2 (one thread per control point) sums the partials of the bricks whose
// voxels touch the point (at most 2 per axis when a brick spans >= 3 tiles), in
// fixed brick order.  No atomics anywhere, so the bits depend on the inputs only.
#pragma once

#include "bsi_device.h"

namespace bsi {

// Workgroup shape of pass 1 (compile-time; the brick is always at most 64 x 32
// voxels in x, y, so these knobs change scheduling, never the summation order).
#ifndef BSI_ADJ_WAVES
#define BSI_ADJ_WAVES 8
#endif
#ifndef BSI_ADJ_PREFETCH
#define BSI_ADJ_PREFETCH 2
#endif
constexpr int kAdjWaves = BSI_ADJ_WAVES;
constexpr int kAdjThreads = kWave * kAdjWaves;
constexpr int kAdjMaxX = kWave;                  // 64
constexpr int kAdjMaxY = 32;
constexpr int kAdjRows = kAdjMaxY / kAdjWaves;   // rows per thread
constexpr int kAdjPrefetch = BSI_ADJ_PREFETCH;   // z-planes loaded ahead
constexpr int kAdjMaxCx = (kAdjMaxX - 1) + 5;    // window bound at spacing 1
constexpr int kAdjTargetZ = 24;
static_assert(kAdjRows * kAdjWaves == kAdjMaxY, "rows must tile the 32-row brick");
static_assert(kAdjPrefetch >= 1 && kAdjPrefetch <= 4, "prefetch depth 1..4");

struct AdjSmem {
  float V[kAdjMaxY * kAdjMaxX * 3];    // finished plane A(x, y), per component
  float Sx[kAdjMaxY * kAdjMaxCx * 3];  // x-contracted plane
  float WX[kAdjMaxX * 4];              // Bx_l at each x of the brick
  float WY[kAdjMaxY * 4];              // By_m at each y of the brick
};

struct AdjBrick {
  int x0, y0, z0, xe, ye, ze;  // voxel range [x0, xe) etc.
  int cx0, cy0, cz0;           // first control index of the window
  int Cx, Cy;                  // window extent in x, y
};

__device__ __forceinline__ AdjBrick adj_brick_geom(const AdjGeom& a, int brick) {
  const VolGeom& g = a.g;
  AdjBrick b;
  const int bx = brick % a.nbx;
  const int t = brick / a.nbx;
  const int by = t % a.nby;
  const int bz = t / a.nby;
  b.x0 = bx * a.xb;
  b.y0 = by * a.yb;
  b.z0 = bz * a.zb;
  b.xe = min(b.x0 + a.xb, g.nx);
  b.ye = min(b.y0 + a.yb, g.ny);
  b.ze = min(b.z0 + a.zb, g.nz);
  b.cx0 = b.x0 / g.dx;
  b.cy0 = b.y0 / g.dy;
  b.cz0 = b.z0 / g.dz;
  b.Cx = (b.xe - 1) / g.dx - b.cx0 + 4;
  b.Cy = (b.ye - 1) / g.dy - b.cy0 + 4;
  return b;
}

// Contract one finished control plane (czl = cz - cz0) of the brick over x and
// y and write the partials.  Collective: every thread of the workgroup calls it.
__device__ __forceinline__ void adj_emit(const AdjGeom& a, const AdjBrick& b, float* __restrict__ pbase,
                                         AdjSmem& sm, int tid, int czl, const F3 (&v)[kAdjRows],
                                         const bool (&act)[kAdjRows]) {
  const VolGeom& g = a.g;
  const int lane = tid & (kWave - 1), w = tid / kWave;
#pragma unroll
  for (int k = 0; k < kAdjRows; ++k) {
    const int yl = k * kAdjWaves + w;
    float* d = sm.V + (yl * kAdjMaxX + lane) * 3;
    d[0] = act[k] ? v[k].x : 0.f;
    d[1] = act[k] ? v[k].y : 0.f;
    d[2] = act[k] ? v[k].z : 0.f;
  }
  __syncthreads();

  // x-contraction: one item per (row, cx), all three components
  const int txlo = b.x0 / g.dx, txhi = (b.xe - 1) / g.dx;
  const int n1 = (b.ye - b.y0) * b.Cx;
  for (int it = tid; it < n1; it += kAdjThreads) {
    const int yl = it / b.Cx;
    const int cxl = it - yl * b.Cx;
    const int cx = b.cx0 + cxl;
    const float* vrow = sm.V + yl * kAdjMaxX * 3;
    float sx = 0.f, sy = 0.f, sz = 0.f;
    for (int l = 0; l < 4; ++l) {
      const int tile = cx - l;
      if (tile < txlo || tile > txhi) continue;
      const int xa = max(tile * g.dx, b.x0) - b.x0;
      const int xb = min(tile * g.dx + g.dx, b.xe) - b.x0;
#pragma unroll 4
      for (int xl = xa; xl < xb; ++xl) {
        const float wv = sm.WX[xl * 4 + l];
        const float* v = vrow + xl * 3;
        sx = fmaf(wv, v[0], sx);
        sy = fmaf(wv, v[1], sy);
        sz = fmaf(wv, v[2], sz);
      }
    }
    float* o = sm.Sx + (yl * kAdjMaxCx + cxl) * 3;
    o[0] = sx;
    o[1] = sy;
    o[2] = sz;
  }
  __syncthreads();

  // y-contraction: one item per (cy, cx), all three components
  const int tylo = b.y0 / g.dy, tyhi = (b.ye - 1) / g.dy;
  const int n2 = b.Cy * b.Cx;
  for (int it = tid; it < n2; it += kAdjThreads) {
    const int cyl = it / b.Cx;
    const int cxl = it - cyl * b.Cx;
    const int cy = b.cy0 + cyl;
    float sx = 0.f, sy = 0.f, sz = 0.f;
    for (int m = 0; m < 4; ++m) {
      const int tile = cy - m;
      if (tile < tylo || tile > tyhi) continue;
      const int ya = max(tile * g.dy, b.y0) - b.y0;
      const int yb = min(tile * g.dy + g.dy, b.ye) - b.y0;
#pragma unroll 4
      for (int yl = ya; yl < yb; ++yl) {
        const float wv = sm.WY[yl * 4 + m];
        const float* v = sm.Sx + (yl * kAdjMaxCx + cxl) * 3;
        sx = fmaf(wv, v[0], sx);
        sy = fmaf(wv, v[1], sy);
        sz = fmaf(wv, v[2], sz);
      }
    }
    stf3(pbase + ((size_t)(czl * a.cym + cyl) * a.cxm + cxl) * 3, F3{sx, sy, sz});
  }
  // No trailing barrier: the next emit's first barrier orders these LDS reads
  // before its Sx writes, and its V writes come after this emit's second barrier.
}

// Pass 1 for one brick.  Collective over the workgroup (kAdjThreads threads).
__device__ __forceinline__ void adj_brick(const float* __restrict__ dfield, float* __restrict__ part,
                                          const AdjGeom& a, const float* __restrict__ lut, int brick,
                                          AdjSmem& sm, int tid) {
  const VolGeom& g = a.g;
  const AdjBrick b = adj_brick_geom(a, brick);
  float* pbase = part + (size_t)brick * a.czm * a.cym * a.cxm * 3;

  __syncthreads();  // a previous brick of this workgroup may still read WX / WY
  for (int i = tid; i < kAdjMaxX * 4; i += kAdjThreads) {
    const int x = b.x0 + (i >> 2);
    float wv = 0.f;
    if (x < b.xe) {
      const int t = x / g.dx;
      wv = lut_row(lut, g.dx, x - t * g.dx)[i & 3];
    }
    sm.WX[i] = wv;
  }
  for (int i = tid; i < kAdjMaxY * 4; i += kAdjThreads) {
    const int y = b.y0 + (i >> 2);
    float wv = 0.f;
    if (y < b.ye) {
      const int t = y / g.dy;
      wv = lut_row(lut, g.dy, y - t * g.dy)[i & 3];
    }
    sm.WY[i] = wv;
  }
  // (the first adj_emit barrier orders these writes before any read)

  const int lane = tid & (kWave - 1), w = tid / kWave;
  const int x = b.x0 + lane;
  const size_t zs = (size_t)g.ny * g.nx * 3;
  bool act[kAdjRows];
  const float* src[kAdjRows];
#pragma unroll
  for (int k = 0; k < kAdjRows; ++k) {
    const int y = b.y0 + k * kAdjWaves + w;
    act[k] = (x < b.xe) && (y < b.ye);
    src[k] = dfield + (((size_t)b.z0 * g.ny + (act[k] ? y : 0)) * g.nx + (act[k] ? x : 0)) * 3;
  }

  F3 acc[kAdjRows][4];
#pragma unroll
  for (int k = 0; k < kAdjRows; ++k)
#pragma unroll
    for (int n = 0; n < 4; ++n) acc[k][n] = F3{0.f, 0.f, 0.f};

  const F3 zero{0.f, 0.f, 0.f};
  // ring of the next kAdjPrefetch z-planes of every row (registers)
  F3 pf[kAdjPrefetch][kAdjRows];
#pragma unroll
  for (int j = 0; j < kAdjPrefetch; ++j)
#pragma unroll
    for (int k = 0; k < kAdjRows; ++k)
      pf[j][k] = (act[k] && b.z0 + j < b.ze) ? ldf3(src[k] + (size_t)j * zs) : zero;

  int tz = b.cz0;
  int oz = b.z0 - tz * g.dz;
  for (int z = b.z0; z < b.ze; ++z) {
    F3 cur[kAdjRows];
#pragma unroll
    for (int k = 0; k < kAdjRows; ++k) {
      cur[k] = pf[0][k];
#pragma unroll
      for (int j = 0; j + 1 < kAdjPrefetch; ++j) pf[j][k] = pf[j + 1][k];
      const int zn = z + kAdjPrefetch;
      pf[kAdjPrefetch - 1][k] = (act[k] && zn < b.ze) ? ldf3(src[k] + (size_t)(zn - b.z0) * zs) : zero;
    }
    const float* wz = lut_row(lut, g.dz, oz);
    const float w0 = wz[0], w1 = wz[1], w2 = wz[2], w3 = wz[3];
#pragma unroll
    for (int k = 0; k < kAdjRows; ++k) {
      acc[k][0].x = fmaf(w0, cur[k].x, acc[k][0].x);
      acc[k][0].y = fmaf(w0, cur[k].y, acc[k][0].y);
      acc[k][0].z = fmaf(w0, cur[k].z, acc[k][0].z);
      acc[k][1].x = fmaf(w1, cur[k].x, acc[k][1].x);
      acc[k][1].y = fmaf(w1, cur[k].y, acc[k][1].y);
      acc[k][1].z = fmaf(w1, cur[k].z, acc[k][1].z);
      acc[k][2].x = fmaf(w2, cur[k].x, acc[k][2].x);
      acc[k][2].y = fmaf(w2, cur[k].y, acc[k][2].y);
      acc[k][2].z = fmaf(w2, cur[k].z, acc[k][2].z);
      acc[k][3].x = fmaf(w3, cur[k].x, acc[k][3].x);
      acc[k][3].y = fmaf(w3, cur[k].y, acc[k][3].y);
      acc[k][3].z = fmaf(w3, cur[k].z, acc[k][3].z);
    }
    if (++oz == g.dz && z + 1 < b.ze) {
      F3 fin[kAdjRows];
#pragma unroll
      for (int k = 0; k < kAdjRows; ++k) fin[k] = acc[k][0];
      adj_emit(a, b, pbase, sm, tid, tz - b.cz0, fin, act);
#pragma unroll
      for (int k = 0; k < kAdjRows; ++k) {
        acc[k][0] = acc[k][1];
        acc[k][1] = acc[k][2];
        acc[k][2] = acc[k][3];
        acc[k][3] = zero;
      }
      oz = 0;
      ++tz;
    }
  }
  // The last tile's four planes (the last three are shared with the next brick).
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    F3 fin[kAdjRows];
#pragma unroll
    for (int k = 0; k < kAdjRows; ++k) fin[k] = acc[k][n];
    adj_emit(a, b, pbase, sm, tid, tz - b.cz0 + n, fin, act);
  }
}

// Pass 2 for one control point (cx, cy, cz): fixed-order sum of brick partials.
__device__ __forceinline__ F3 adj_gather_point(const float* __restrict__ part, const AdjGeom& a, int cx,
                                               int cy, int cz) {
  const VolGeom& g = a.g;
  // bricks whose voxels touch the point's support [(c-3)d, (c+1)d) on each axis
  const int bxlo = max(0, (cx - 3) * g.dx) / a.xb, bxhi = (min(g.nx, (cx + 1) * g.dx) - 1) / a.xb;
  const int bylo = max(0, (cy - 3) * g.dy) / a.yb, byhi = (min(g.ny, (cy + 1) * g.dy) - 1) / a.yb;
  const int bzlo = max(0, (cz - 3) * g.dz) / a.zb, bzhi = (min(g.nz, (cz + 1) * g.dz) - 1) / a.zb;
  const size_t bstride = (size_t)a.czm * a.cym * a.cxm * 3;
  F3 s{0.f, 0.f, 0.f};
  for (int bz = bzlo; bz <= bzhi; ++bz) {
    const int czl = cz - (bz * a.zb) / g.dz;
    for (int by = bylo; by <= byhi; ++by) {
      const int cyl = cy - (by * a.yb) / g.dy;
      for (int bx = bxlo; bx <= bxhi; ++bx) {
        const int cxl = cx - (bx * a.xb) / g.dx;
        const float* p = part + (size_t)((bz * a.nby + by) * a.nbx + bx) * bstride +
                         ((size_t)(czl * a.cym + cyl) * a.cxm + cxl) * 3;
        const F3 v = ldf3(p);
        s.x += v.x;
        s.y += v.y;
        s.z += v.z;
      }
    }
  }
  return s;
}

}  // namespace bsi
