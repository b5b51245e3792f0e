// Real-spacing grid: the exact window-start decision shared by host and
// device, and the geometry of the z-first adjoint's bricks (used by the
// kernels in general.hip and by the host index checker).
#pragma once

#include "bsi_device.h"
#include "bsi_internal.h"

namespace bsi {

// a + b = s + e exactly (Knuth's two-sum; round to nearest, no overflow).
__host__ __device__ inline void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Exact sign of D(i) = (x - o) - i s for integers 0 <= x, |i| < 2^24, and the
// FP32 value of D rounded from its exact expansion.  x - o = A + a and i s =
// P + p are error-free; growing the nonoverlapping expansion (a, A) by -p and
// then by -P (Shewchuk's grow-expansion) gives four nonoverlapping components
// whose largest nonzero one carries the sign of the exact sum.
__host__ __device__ inline int gen_residual(float X, float o, float s, int i, float& D) {
  float A, a;
  two_sum(X, -o, A, a);
  const float I = (float)i;
  const float P = I * s;
  const float p = fmaf(I, s, -P);
  float Q, h0, h1, k0, k1, k2;
  two_sum(-p, a, Q, h0);
  two_sum(Q, A, Q, h1);
  const float h2 = Q;
  two_sum(-P, h0, Q, k0);
  two_sum(Q, h1, Q, k1);
  two_sum(Q, h2, Q, k2);
  const float k3 = Q;
  D = k3 + k2;
  const float top = k3 != 0.f ? k3 : k2 != 0.f ? k2 : k1 != 0.f ? k1 : k0;
  return top > 0.f ? 1 : top < 0.f ? -1 : 0;
}

// Window start i = floor((v - o)/s) of voxel v (exact) and u = (v - o)/s - i
// in FP32.  The FP32 quotient is within 1/8 of the exact one for v < 2^21, so
// the floor is its floor, one below or one above; the exact residual decides.
__host__ __device__ inline int gen_locate(const GenAxis& a, int v, float& u) {
  const float X = (float)v;
  int i = (int)floorf((X - a.o) / a.s);
  float D;
  if (gen_residual(X, a.o, a.s, i, D) < 0) {
    --i;
    (void)gen_residual(X, a.o, a.s, i, D);
  } else {
    float D1;
    if (gen_residual(X, a.o, a.s, i + 1, D1) >= 0) {
      ++i;
      D = D1;
    }
  }
  u = D / a.s;
  return i;
}

__host__ __device__ inline int gen_tile(const GenAxis& a, int v) {
  float u;
  return gen_locate(a, v, u);
}


// ---------------------------------------------------------------------------
// Bricks of the z-first adjoint (general.hip): 64 x-voxels by 16 rows by the
// voxels of kz whole z-tiles.
constexpr int kGzBX = kWave;             // brick width (voxels)
constexpr int kGzRows = 2;               // rows per lane
constexpr int kGzWaves = 8;
constexpr int kGzBY = kGzRows * kGzWaves;  // brick height (rows)
constexpr int kGzThreads = kGzWaves * kWave;
constexpr int kGzTargetZ = 48;           // about this many voxel planes per brick
constexpr int kGzStage = 6144;           // floats of staged partials (24 KB)

struct GenAdj {
  int nbx, nby, nbz;  // bricks per axis
  int kz;             // z-tiles per brick
  int cmx, cmy, cmz;  // window extents (the largest over the bricks)
  int stage_all;      // the whole window of partials fits the LDS stage
};

// LDS of one workgroup (floats): F, H[2], the brick's x and y weight rows and
// first-voxel tables, the stage.
struct GzLayout {
  int F, H, wx, fx, wy, fy, P, total;
};
__host__ __device__ inline GzLayout gz_layout(const GenAdj& a) {
  GzLayout L;
  int o = 0;
  L.F = o;
  o += kGzBY * kGzBX * 3;
  L.H = o;
  o += 2 * kGzBY * a.cmx * 3;
  L.wx = o;
  o += kGzBX * 4;
  L.fx = o;
  o += a.cmx + 4;
  L.wy = o;
  o += kGzBY * 4;
  L.fy = o;
  o += a.cmy + 4;
  L.P = o;
  o += a.stage_all ? a.cmz * a.cmy * a.cmx * 3 : 0;
  L.total = o;
  return L;
}

struct GzTables {
  const int* tile[3];
  const float* w[3];
  const int* first[3];
};

// Brick (bx, by, bz): its voxel range and the first control index of its window per axis.
struct GzBrick {
  int x0, xe, y0, ye, z0, ze;
  int cx0, cy0, cz0;
  int Cx, Cy;
};

__host__ __device__ inline GzBrick gz_brick(const GenGeom& q, const GenAdj& a, const GzTables& T, int id) {
  GzBrick b;
  const int bx = id % a.nbx;
  const int r = id / a.nbx;
  const int by = r % a.nby;
  const int bz = r / a.nby;
  b.x0 = bx * kGzBX;
  b.xe = min(q.x.n, b.x0 + kGzBX);
  b.y0 = by * kGzBY;
  b.ye = min(q.y.n, b.y0 + kGzBY);
  b.cz0 = bz * a.kz;
  b.z0 = T.first[2][b.cz0];
  b.ze = T.first[2][min(b.cz0 + a.kz, q.z.g - 3)];
  b.cx0 = T.tile[0][b.x0];
  b.Cx = T.tile[0][b.xe - 1] - b.cx0 + 4;
  b.cy0 = T.tile[1][b.y0];
  b.Cy = T.tile[1][b.ye - 1] - b.cy0 + 4;
  return b;
}


// Bricks of the z-first adjoint: about kGzTargetZ planes of whole z-tiles,
// fewer (at least half as many) when that lets a brick's window of partials
// fit the LDS stage.  A pure function of the geometry.
inline GenAdj make_gen_adj(const GenGeom& q) {
  GenAdj a;
  a.nbx = (q.x.n + kGzBX - 1) / kGzBX;
  a.nby = (q.y.n + kGzBY - 1) / kGzBY;
  a.cmx = a.cmy = 0;
  for (int bx = 0; bx < a.nbx; ++bx) {
    const int x0 = bx * kGzBX, xe = imin(q.x.n, x0 + kGzBX);
    a.cmx = imax(a.cmx, gen_tile(q.x, xe - 1) - gen_tile(q.x, x0) + 4);
  }
  for (int by = 0; by < a.nby; ++by) {
    const int y0 = by * kGzBY, ye = imin(q.y.n, y0 + kGzBY);
    a.cmy = imax(a.cmy, gen_tile(q.y, ye - 1) - gen_tile(q.y, y0) + 4);
  }
  const int tiles = q.z.g - 3;  // z-tiles holding voxels
  int kz = imax(1, (int)(kGzTargetZ / q.z.s));
  kz = imin(kz, tiles);
  const int kfit = kGzStage / (a.cmy * a.cmx * 3) - 3;
  if (kfit < kz && 2 * kfit >= kz) kz = kfit;
  a.kz = kz;
  a.nbz = (tiles + kz - 1) / kz;
  a.cmz = kz + 3;
  a.stage_all = (long)a.cmz * a.cmy * a.cmx * 3 <= kGzStage;
  return a;
}

// Bricks whose voxels meet the support [first(c - 3), first(c + 1)) of
// control index c along one axis, for bricks of `width` voxels (x, y).
struct GzSpan {
  int lo, hi;
};
__host__ __device__ inline GzSpan gz_span(const int* first, int c, int width) {
  return GzSpan{first[c >= 3 ? c - 3 : 0] / width, (first[c + 1] - 1) / width};
}
// Along z: bricks of kz tiles; tiles c - 3 .. c that hold voxels (g - 3 of them).
__host__ __device__ inline GzSpan gz_span_z(const GenAdj& a, int c, int gz) {
  return GzSpan{(c >= 3 ? c - 3 : 0) / a.kz, (c < gz - 4 ? c : gz - 4) / a.kz};
}

}  // namespace bsi
