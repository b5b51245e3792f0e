// BSI for a control grid with real spacing and an origin offset: the paper's
// method needs the grid aligned to the voxels with integer spacing (Sec. 3.4),
// the limitation its conclusion names (Sec. 8).  Per axis:
//   control point a sits at voxel o + (a - 1) s      (s >= 1, -s < o <= 0),
//   voxel x: t = (x - o) / s, window i = floor(t) .. i + 3, weights B(t - i),
//   g = floor((n - 1 - o) / s) + 4 points.
// The window start i = floor((x - o)/s) is decided exactly, from the FP32
// values of s and o, with FP32 error-free transformations (gen_locate); the
// same code runs on the host (grid size) and the device, so every decision
// agrees.  The offset u = t - i and the weights are FP32.  Nothing on the
// device is FP64.
//
// Forward: the aligned kernel's pipeline (forward.hip) with weights computed
// per coordinate instead of looked up per offset: x weights once per lane, y
// weights once per wave, and the window start and z weights of every plane of
// the workgroup's z range once, into an LDS table.  Tiles have varying voxel
// counts; the window of 4 contracted planes advances whenever floor(t_z) does
// (by one, since s >= 1), with the next plane loaded while the current tile is
// written and one barrier per tile.
//
// Adjoint: the per-axis tables i(x), B(u(x)) and the first voxel of every
// tile are computed once per call into the workspace; then the aligned
// adjoint's two passes, z-first, with the tables in place of equal tiles
// (gen_zf_pass1_kernel: bricks of 64 x 16 voxels by whole z-tiles, the
// z-contraction in registers, each finished control plane contracted over x
// and y in LDS; gen_zf_pass2_kernel: the fixed-order sum of brick partials per
// control point).  Deterministic, no atomics.
#include <cmath>

#include "adjoint_device.h"
#include "general_device.h"

namespace bsi {

namespace {

// Window start and the four FP32 basis weights at u (B0..B3 of Eq. 1).
__device__ __forceinline__ int gen_weights(const GenAxis& a, int v, float (&w)[4]) {
  float u;
  const int i = gen_locate(a, v, u);
  const float r = 1.f - u, u2 = u * u;
  const float sixth = 1.f / 6.f;
  w[0] = r * r * r * sixth;
  w[1] = fmaf(3.f * u2, u - 2.f, 4.f) * sixth;
  w[2] = fmaf(3.f * u, fmaf(-u, u, u) + 1.f, 1.f) * sixth;
  w[3] = u2 * u * sixth;
  return i;
}

constexpr int kGenMaxZ = 256;  // voxel planes per workgroup (z table in LDS)

struct GenFwdSmem {
  FwdSmem<3> f;
  float zw[kGenMaxZ][4];  // z weights of the workgroup's planes
  int zt[kGenMaxZ];       // their window start floor(t_z)
};

// Edge: rows off 64-byte boundaries, written with edge stores (FwdEdgeStore).
template <bool Edge>
__global__ __launch_bounds__(kFwdThreads) void gen_fwd_kernel(const float* __restrict__ grid,
                                                               float* __restrict__ field, VolGeom g, GenGeom q,
                                                               int nbx, int nby, int zchunk) {
  __shared__ GenFwdSmem sm;
  int id = xcd_remap(blockIdx.x, gridDim.x);
  const int bxi = id % nbx;
  id /= nbx;
  const int byi = id % nby;
  const int bzi = id / nby;
  const int tid = threadIdx.x;
  const int x0 = bxi * kWave, y0 = byi * kFwdRows;
  const int z0 = bzi * zchunk, z1 = min(g.nz, z0 + zchunk);  // z1 - z0 <= kGenMaxZ
  const int lane = tid & (kWave - 1);
  const int wave = uniform(tid / kWave);
  // s >= 1: 64 voxels span at most 63 tile steps, so the window fits the
  // staging layout (at most kFwdMaxCx x kFwdMaxCy points)
  const int cx0 = gen_tile(q.x, x0);
  const int ncx = gen_tile(q.x, min(x0 + kWave, g.nx) - 1) - cx0 + 4;
  const int cy0 = gen_tile(q.y, y0);
  const int ncy = gen_tile(q.y, min(y0 + kFwdRows, g.ny) - 1) - cy0 + 4;
  const FwdStage<3> map = fwd_stage_map<3>(g, cx0, ncx, cy0, ncy, tid);
  for (int i = tid; i < z1 - z0; i += kFwdThreads) {
    float w[4];
    sm.zt[i] = gen_weights(q.z, z0 + i, w);
#pragma unroll
    for (int n = 0; n < 4; ++n) sm.zw[i][n] = w[n];
  }
  // (the warm-up's first barrier orders the table before any read)

  const int x = x0 + lane, y = y0 + wave;
  const bool active = x < g.nx && y < g.ny;
  const int xc = min(x, g.nx - 1), yc = min(y, g.ny - 1);
  float bx[4], wy[4];
  const int tx = gen_weights(q.x, xc, bx);
  const int ty = gen_weights(q.y, yc, wy);
  const int base = (ty - cy0) * fwd_pitch<3>() + (tx - cx0) * 3;

  int tz = gen_tile(q.z, z0);
  float r[fwd_loads<3>()];
  // Warm-up as in the aligned forward: planes tz, tz+1, tz+2 through slots
  // 0, 1, 0 into q0..q2, then plane tz+3 staged into slot 1.
  FwdVal<3> q0, q1, q2;
#pragma unroll
  for (int c = 0; c < 3; ++c) q0.v[c] = q1.v[c] = q2.v[c] = 0.f;
#pragma unroll 1
  for (int j = 0; j < 3; ++j) {
    __syncthreads();
    fwd_fetch<3>(grid, g, map, tz + j, r);
    fwd_stage<3>(sm.f.ring[j & 1], tid, r);
    __syncthreads();
    const FwdVal<3> qn = fwd_contract<3>(sm.f.ring[j & 1], base, bx[0], bx[1], bx[2], bx[3], wy);
    q0 = q1;
    q1 = q2;
    q2 = qn;
  }
  __syncthreads();
  fwd_fetch<3>(grid, g, map, tz + 3, r);
  fwd_stage<3>(sm.f.ring[1], tid, r);
  __syncthreads();
  int slot3 = 1;

  const size_t zstride = (size_t)g.ny * g.nx * 3;
  float* out = field + (((size_t)z0 * g.ny + yc) * g.nx + xc) * 3;
  FwdEdgeStore<3> edge(field, g, z0, yc, x0, xc);
  int z = z0;
  for (;;) {
    const FwdVal<3> q3 = fwd_contract<3>(sm.f.ring[slot3], base, bx[0], bx[1], bx[2], bx[3], wy);
    int zend = z;  // the planes of tile tz in this chunk (s >= 1: the next one is tz + 1)
    while (zend < z1 && sm.zt[zend - z0] == tz) ++zend;
    const bool more = zend < z1;
    // its new plane tz + 4 = t_z(zend) + 3 <= gz - 1: in bounds
    if (more) fwd_fetch<3>(grid, g, map, tz + 4, r);
    for (; z < zend; ++z, out += zstride) {
      const float* wz = sm.zw[z - z0];
      float t[3];
#pragma unroll
      for (int c = 0; c < 3; ++c)
        t[c] = fmaf(wz[3], q3.v[c], fmaf(wz[2], q2.v[c], fmaf(wz[1], q1.v[c], wz[0] * q0.v[c])));
      if constexpr (Edge) edge.store(active, t);
      else if (active) fwd_store<3>(out, t);
    }
    if (!more) break;
    fwd_stage<3>(sm.f.ring[slot3 ^ 1], tid, r);
    __syncthreads();
    slot3 ^= 1;
    ++tz;
    q0 = q1;
    q1 = q2;
    q2 = q3;
  }
}

// The three axes' tables in one launch: workgroups [0, nb[0]) take x, then y, then z.
struct GenTables3 {
  GenAxis ax[3];
  int* tile[3];
  float* w[3];
  int* first[3];
  int nb[3];  // workgroups per axis
};

// Thread k of an axis's workgroups writes entry k of its tables: tile[k] =
// i(k) and w[k] = B(u(k)) for k < n, and first[k] = min{v : i(v) >= k} for
// k <= g (first[g] = n), found by bisection on the exact i(v), so the three
// tables need no order between them.  The z weights are stored in pass 1's
// accumulator order: entry s of voxel k is the weight of control plane c with
// c mod 4 = s, i.e. B_{(s - i(k)) mod 4}.
__global__ __launch_bounds__(256) void gen_tables3_kernel(GenTables3 p) {
  int blk = blockIdx.x, i = 0;
  while (i < 2 && blk >= p.nb[i]) blk -= p.nb[i++];
  const GenAxis a = p.ax[i];
  const int k = blk * 256 + threadIdx.x;
  if (k < a.n) {
    float b[4];
    const int tk = gen_weights(a, k, b);
    p.tile[i][k] = tk;
    const int rot = i == 2 ? tk & 3 : 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) p.w[i][4 * k + s] = b[(s - rot) & 3];
  }
  if (k <= a.g) {
    int lo = 0, hi = a.n;  // i(v) is nondecreasing in v
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (gen_tile(a, mid) < k) lo = mid + 1;
      else hi = mid;
    }
    p.first[i][k] = lo;
  }
}

// ---------------------------------------------------------------------------
// The adjoint, z-first (as the aligned pass 1 in adjoint_device.h), with the
// per-axis tables instead of tiles of equal length.  A brick is 64 x-voxels
// (one per lane) by 16 rows (8 waves of 2 rows) by the voxels of kz whole
// z-tiles, [first_z[b kz], first_z[(b+1) kz]).  Per voxel plane a lane adds
// its 2 voxels into the 4 control planes they meet, with the plane's z
// weights (scalar loads of the z table); slot k of the accumulators holds
// control plane c with c mod 4 = k.  When the plane's z-tile ends,
// control plane t is finished and is contracted in LDS: over x, output
// column c of a row sums the brick's voxels v in [first_x[c-3], first_x[c+1])
// (ascending) with weight B_{c - i(v)}(u(v)); then, after a workgroup barrier,
// over y the same way, giving the brick's partial of that plane.  Pass 2
// sums, per control point, the partials of the bricks meeting its support in
// fixed order.  No atomics.
// XTiles: every brick meets at most 16 x-tiles (window width cmx <= 19), so
// the x-contraction runs on tile lanes.
// Waves per SIMD pass 1 is compiled for (a register bound of 512 / this).
#ifndef BSI_GZ_WPE
#define BSI_GZ_WPE 6
#endif
template <bool XTiles>
__global__ __launch_bounds__(kGzThreads) __attribute__((amdgpu_waves_per_eu(BSI_GZ_WPE))) void gen_zf_pass1_kernel(const float* __restrict__ dfield,
                                                                   float* __restrict__ part, GenGeom q, GenAdj a,
                                                                   GzTables T) {
  extern __shared__ float gz_smem[];
  const int nbricks = a.nbx * a.nby * a.nbz;
  const int brick = xcd_remap(blockIdx.x, gridDim.x);
  if (brick >= nbricks) return;  // uniform over the workgroup
  const GzLayout L = gz_layout(a);
  float* F = gz_smem + L.F;
  float* wxT = gz_smem + L.wx;
  int* fxT = reinterpret_cast<int*>(gz_smem + L.fx);
  float* wyT = gz_smem + L.wy;
  int* fyT = reinterpret_cast<int*>(gz_smem + L.fy);
  const GzBrick b = gz_brick(q, a, T, brick);
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = uniform(tid / kWave);
  const int nxb = b.xe - b.x0, nyb = b.ye - b.y0;
  // the brick's x and y tables; fxT[j] = first_x[cx0 + j - 3] (clamped at 0),
  // so output column cx0 + j takes the voxels [fxT[j], fxT[j + 4])
  if (tid < nxb) {
#pragma unroll
    for (int l = 0; l < 4; ++l) wxT[4 * tid + l] = T.w[0][4 * (b.x0 + tid) + l];
  }
  if (tid < nyb) {
#pragma unroll
    for (int l = 0; l < 4; ++l) wyT[4 * tid + l] = T.w[1][4 * (b.y0 + tid) + l];
  }
  if (tid < b.Cx + 4) fxT[tid] = T.first[0][max(b.cx0 + tid - 3, 0)];
  if (tid < b.Cy + 4) fyT[tid] = T.first[1][max(b.cy0 + tid - 3, 0)];
  __syncthreads();

  const size_t plane = (size_t)q.x.n * q.y.n * 3;
  uint32_t off[kGzRows];
#pragma unroll
  for (int r = 0; r < kGzRows; ++r)
    off[r] = ((uint32_t)min(b.y0 + wave * kGzRows + r, b.ye - 1) * (uint32_t)q.x.n +
              (uint32_t)min(b.x0 + lane, b.xe - 1)) * 3u;
  float* pbase = part + (size_t)brick * a.cmz * a.cmy * a.cmx * 3;
  float* P = a.stage_all ? gz_smem + L.P : pbase;

  F3 acc[4][kGzRows];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int r = 0; r < kGzRows; ++r) acc[k][r] = F3{0.f, 0.f, 0.f};

  // the x- and y-contractions of brick-relative control plane czl, whose
  // rows the waves have put in F, into the partials
  auto contract = [&](int czl, bool last) {
    float* H = gz_smem + L.H + (czl & 1) * kGzBY * a.cmx * 3;
    // x.  Tile lanes when the brick meets at most 16 x-tiles (as in the aligned
    // pass 1): lane (rr, t) of this wave forms the 4 moments of tile cx0 + t
    // of its row rr, M_l = sum over the tile's voxels (ascending) of
    // B_l(u(v)) F[v], and DPP row shifts combine them into the window
    // columns, H[j] = sum_l M_l(tile j - l).  Otherwise one lane per (row,
    // column), summing the column's voxels tile by tile.
    if constexpr (XTiles) {
      const int rr = lane / kAdjTiles, tt = lane % kAdjTiles;
      const int row = wave * kGzRows + rr;
      const bool rowok = rr < kGzRows && row < nyb;
      F3 M[4];
#pragma unroll
      for (int l = 0; l < 4; ++l) M[l] = F3{0.f, 0.f, 0.f};
      if (rowok && tt < b.Cx - 3) {
        const int va = max(fxT[tt + 3], b.x0) - b.x0, vb = min(fxT[tt + 4], b.xe) - b.x0;
        const float* Fr = F + row * kGzBX * 3;
#pragma unroll 2
        for (int v = va; v < vb; ++v) adj_moment_step(wxT + 4 * v, ldf3(Fr + 3 * v), M);
      }
      F3 cm, cw;
      adj_combine(M, cm, cw);  // every lane of the wave takes part
      if (rowok) {
        float* hrow = H + row * a.cmx * 3;
        if (tt < b.Cx) stf3(hrow + tt * 3, cm);
        if (tt < 3 && kAdjTiles + tt < b.Cx) stf3(hrow + (kAdjTiles + tt) * 3, cw);
      }
    } else {
      for (int it = lane; it < kGzRows * b.Cx; it += kWave) {
        const int r = it / b.Cx, j = it - r * b.Cx;
        const int row = wave * kGzRows + r;
        if (row < nyb) {
          float sx = 0.f, sy = 0.f, sz = 0.f;
          const float* Fr = F + row * kGzBX * 3;
          // tiles c-3 .. c (weight index l = 3 .. 0): the voxels in ascending order
#pragma unroll
          for (int l = 3; l >= 0; --l) {
            const int va = max(fxT[j + 3 - l], b.x0) - b.x0, vb = min(fxT[j + 4 - l], b.xe) - b.x0;
#pragma unroll 2
            for (int v = va; v < vb; ++v) {
              const float wgt = wxT[4 * v + l];
              sx = fmaf(wgt, Fr[3 * v], sx);
              sy = fmaf(wgt, Fr[3 * v + 1], sy);
              sz = fmaf(wgt, Fr[3 * v + 2], sz);
            }
          }
          stf3(H + (row * a.cmx + j) * 3, F3{sx, sy, sz});
        }
      }
    }
    __syncthreads();
    // y, on y-tile lanes (a brick of 16 rows meets at most 16 y-tiles): lane
    // (c4, ty) of wave w takes window column 4 w + c4 (then + 32 ...) and
    // y-tile cy0 + ty, forms N_m = sum over the tile's rows (ascending) of
    // B_m(v(y)) H[y][column], and the shifts give window rows ty and
    // (ty < 3) 16 + ty.
    {
      const int c4 = lane / kAdjTiles, ty = lane % kAdjTiles;
      const int nty = b.Cy - 3;
      for (int c0 = wave * 4; c0 < b.Cx; c0 += kGzWaves * 4) {  // uniform over the wave
        const int j = c0 + c4;
        F3 N[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) N[m] = F3{0.f, 0.f, 0.f};
        if (j < b.Cx && ty < nty) {
          const int ya = max(fyT[ty + 3], b.y0) - b.y0, yb = min(fyT[ty + 4], b.ye) - b.y0;
#pragma unroll 2
          for (int y = ya; y < yb; ++y) adj_moment_step(wyT + 4 * y, ldf3(H + (y * a.cmx + j) * 3), N);
        }
        F3 gm, gw;
        adj_combine(N, gm, gw);  // every lane of the wave takes part
        if (j < b.Cx) {
          if (ty < b.Cy) stf3(P + ((size_t)(czl * a.cmy + ty) * a.cmx + j) * 3, gm);
          if (ty < 3 && kAdjTiles + ty < b.Cy) stf3(P + ((size_t)(czl * a.cmy + kAdjTiles + ty) * a.cmx + j) * 3, gw);
        }
      }
    }
    if (a.stage_all && last) {
      __syncthreads();
      const int n = (czl + 1) * a.cmy * a.cmx * 3;
      for (int i = tid; i < n; i += kGzThreads) pbase[i] = P[i];
    }
  };

// Slot K (a constant) goes to this wave's rows of F and is cleared.
#define BSI_GZ_PUT_SLOT(K)                                                                    \
  _Pragma("unroll") for (int r = 0; r < kGzRows; ++r) {                                       \
    stf3(F + ((wave * kGzRows + r) * kGzBX + lane) * 3, acc[K][r]);                           \
    acc[K][r] = F3{0.f, 0.f, 0.f};                                                            \
  }
// Control plane CZL (brick-relative), held in slot PH (uniform): its rows go
// to F by a scalar branch to that slot's own code, then the x- and
// y-contractions into the partials.
#define BSI_GZ_EMIT(CZL, PH, LAST)                                                              \
  {                                                                                           \
    wave_lds_sync(); /* this wave's x-contraction of the previous plane is done with F */      \
    switch (PH) {                                                                             \
      case 0: BSI_GZ_PUT_SLOT(0) break;                                                       \
      case 1: BSI_GZ_PUT_SLOT(1) break;                                                       \
      case 2: BSI_GZ_PUT_SLOT(2) break;                                                       \
      default: BSI_GZ_PUT_SLOT(3) break;                                                      \
    }                                                                                         \
    wave_lds_sync();                                                                          \
    contract((CZL), (LAST));                                                                  \
  }

// One voxel plane Z from register set D: the z-accumulation (slot k holds
// control plane c with c mod 4 = k, and the table holds the plane's weights
// in that order: one scalar load), the loads of the plane two ahead into the
// same registers (when LOAD), then, when Z is the last plane of tile t
// (tend = first_z[t+1]), the contraction of control plane t, in slot t mod 4;
// s >= 1, so the next tile is t + 1.
#define BSI_GZ_PLANE(D, Z, LOAD)                                                              \
  {                                                                                           \
    const float* ws = T.w[2] + 4 * (Z);                                                       \
    _Pragma("unroll") for (int k = 0; k < 4; ++k)                                             \
      _Pragma("unroll") for (int r = 0; r < kGzRows; ++r) {                                   \
        acc[k][r].x = fmaf(ws[k], D[r].x, acc[k][r].x);                                       \
        acc[k][r].y = fmaf(ws[k], D[r].y, acc[k][r].y);                                       \
        acc[k][r].z = fmaf(ws[k], D[r].z, acc[k][r].z);                                       \
      }                                                                                       \
    if (LOAD) {                                                                               \
      _Pragma("unroll") for (int r = 0; r < kGzRows; ++r) D[r] = ldf3_dfield<true>(ahead + off[r]); \
    }                                                                                         \
    ahead += plane;                                                                           \
    if ((Z) + 1 == tend && (Z) + 1 < b.ze) {                                                  \
      BSI_GZ_EMIT(t - b.cz0, t & 3, false)                                                    \
      ++t;                                                                                    \
      tend = T.first[2][t + 1];                                                               \
    }                                                                                         \
  }

  // two register sets, each holding one plane's loads (as the aligned pass 1):
  // in the main loop every load is unconditional, so waiting for one set
  // leaves the other set's loads in flight
  const float* base0 = dfield + (size_t)b.z0 * plane;
  F3 d0[kGzRows], d1[kGzRows];
#pragma unroll
  for (int r = 0; r < kGzRows; ++r) d0[r] = ldf3_dfield<true>(base0 + off[r]);
#pragma unroll
  for (int r = 0; r < kGzRows; ++r) d1[r] = ldf3_dfield<true>(base0 + (b.ze - b.z0 > 1 ? plane : 0) + off[r]);
  const float* ahead = base0 + 2 * plane;
  int t = b.cz0;                    // the z-tile of the plane at hand (the brick starts on a tile)
  int tend = T.first[2][t + 1];     // its end
  int z = b.z0;
  for (; z + 4 <= b.ze; z += 2) {
    BSI_GZ_PLANE(d0, z, true)
    BSI_GZ_PLANE(d1, z + 1, true)
  }
  for (; z < b.ze; z += 2) {
    BSI_GZ_PLANE(d0, z, z + 2 < b.ze)
    if (z + 1 < b.ze) BSI_GZ_PLANE(d1, z + 1, z + 3 < b.ze)
  }
#undef BSI_GZ_PLANE
  // the brick's last four control planes, t .. t + 3, in ascending order
#pragma unroll 1
  for (int n = 0; n < 4; ++n) BSI_GZ_EMIT(t - b.cz0 + n, (t + n) & 3, n == 3)
#undef BSI_GZ_EMIT
#undef BSI_GZ_PUT_SLOT
}

// Pass 2: one thread per control point; a wave takes 64 points of one (cy, cz) row.
__global__ __launch_bounds__(256) void gen_zf_pass2_kernel(const float* __restrict__ part, float* __restrict__ grad,
                                                           GenGeom q, GenAdj a, GzTables T) {
  const int nxb = (q.x.g + kWave - 1) / kWave, nyb = (q.y.g + 3) / 4;
  int blk = blockIdx.x;
  const int xb = blk % nxb;
  blk /= nxb;
  const int cy = (blk % nyb) * 4 + uniform(threadIdx.x / kWave);
  const int cz = blk / nyb;
  const int cx = xb * kWave + (threadIdx.x & (kWave - 1));
  if (cy >= q.y.g || cx >= q.x.g) return;
  // bricks meeting the support [first(c-3), first(c+1)) of each axis
  const GzSpan spx = gz_span(T.first[0], cx, kGzBX), spy = gz_span(T.first[1], cy, kGzBY),
               spz = gz_span_z(a, cz, q.z.g);
  const int xa = spx.lo, xb2 = spx.hi, ya = spy.lo, yb2 = spy.hi, za = spz.lo, zb2 = spz.hi;
  const size_t stride = (size_t)a.cmz * a.cmy * a.cmx * 3;
  float sx = 0.f, sy = 0.f, sz = 0.f;
  for (int bz = za; bz <= zb2; ++bz)
    for (int by = ya; by <= yb2; ++by) {
      const int cyl = cy - T.tile[1][by * kGzBY];
      for (int bx = xa; bx <= xb2; ++bx) {
        const int cxl = cx - T.tile[0][bx * kGzBX];
        const size_t id = ((size_t)bz * a.nby + by) * a.nbx + bx;
        const float* p = part + id * stride + ((size_t)((cz - bz * a.kz) * a.cmy + cyl) * a.cmx + cxl) * 3;
        sx += p[0];
        sy += p[1];
        sz += p[2];
      }
    }
  float* g = grad + (((size_t)cz * q.y.g + cy) * q.x.g + cx) * 3;
  g[0] = sx;
  g[1] = sy;
  g[2] = sz;
}

constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }

struct GenWork {
  int* tile[3];
  float* w[3];
  int* first[3];  // first voxel of every tile, per axis (g + 1 entries)
  float* part;    // brick partials of the z-first adjoint
};

size_t gen_layout(const GenGeom& q, void* base, GenWork* wk) {
  char* p = static_cast<char*>(base);
  size_t off = 0;
  const GenAxis* ax[3] = {&q.x, &q.y, &q.z};
  for (int i = 0; i < 3; ++i) {
    if (wk) wk->tile[i] = reinterpret_cast<int*>(p + off);
    off += align256((size_t)ax[i]->n * sizeof(int));
    if (wk) wk->w[i] = reinterpret_cast<float*>(p + off);
    off += align256((size_t)ax[i]->n * 4 * sizeof(float));
  }
  for (int i = 0; i < 3; ++i) {
    if (wk) wk->first[i] = reinterpret_cast<int*>(p + off);
    off += align256((size_t)(ax[i]->g + 1) * sizeof(int));
  }
  const GenAdj a = make_gen_adj(q);
  if (wk) wk->part = reinterpret_cast<float*>(p + off);
  off += align256((size_t)a.nbx * a.nby * a.nbz * a.cmz * a.cmy * a.cmx * 3 * sizeof(float));
  return off;
}

unsigned blocks_for(long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

int32_t make_gen_geom(const int32_t dims[3], const float spacing[3], const float origin[3], GenGeom* q, VolGeom* g) {
  if (!dims || !spacing || !origin) {
    set_error("dims, spacing and origin must be non-null");
    return BSI_ERR_INVALID_ARG;
  }
  GenAxis* ax[3] = {&q->x, &q->y, &q->z};
  for (int i = 0; i < 3; ++i) {
    const double s = spacing[i], o = origin[i];
    if (dims[i] < 1 || !std::isfinite(s) || !std::isfinite(o) || s < 1.0 || !(o <= 0.0 && o > -s)) {
      set_error("need dims >= 1, spacing >= 1 and -spacing < origin <= 0 on every axis");
      return BSI_ERR_INVALID_ARG;
    }
    if (s > BSI_MAX_SPACING || dims[i] > BSI_MAX_DIM) {
      set_error("spacing above BSI_MAX_SPACING or an axis above BSI_MAX_DIM");
      return BSI_ERR_UNSUPPORTED;
    }
    ax[i]->s = s;
    ax[i]->o = o;
    ax[i]->n = dims[i];
    ax[i]->g = gen_tile(*ax[i], dims[i] - 1) + 4;
  }
  const double rows = (double)dims[1] * dims[2];
  if (rows > 2.0e9 || rows * dims[0] * 3 > 9.0e18 / 16) {
    set_error("volume too large");
    return BSI_ERR_UNSUPPORTED;
  }
  g->nx = dims[0];
  g->ny = dims[1];
  g->nz = dims[2];
  g->dx = g->dy = g->dz = 1;  // unused: the general kernels take tiles from q
  g->gx = q->x.g;
  g->gy = q->y.g;
  g->gz = q->z.g;
  // the forward's staging map is the aligned forward's (signed 32-bit offsets)
  if ((double)g->nx * g->ny * 3 >= 4294967296.0) {
    set_error("a voxel plane (nx * ny) above 1.43e9 voxels");
    return BSI_ERR_UNSUPPORTED;
  }
  return check_control_plane(g->gx, g->gy);
}

hipError_t launch_forward_general(const float* grid, float* field, const VolGeom& g, const GenGeom& q,
                                  hipStream_t s) {
  const int nbx = (g.nx + kWave - 1) / kWave, nby = (g.ny + kFwdRows - 1) / kFwdRows;
  const long base = (long)nbx * nby;
  int chunks = (int)((kFwdTargetBlocks + base - 1) / base);
  chunks = std::max(chunks, (g.nz + kGenMaxZ - 1) / kGenMaxZ);  // the z table holds kGenMaxZ planes
  chunks = std::max(1, std::min(chunks, g.nz));
  const int zchunk = (g.nz + chunks - 1) / chunks;
  const int nbz = (g.nz + zchunk - 1) / zchunk;
  // rows on 64-byte boundaries: non-temporal stores; otherwise edge stores
  if ((g.nx * 12) % 64 == 0 && reinterpret_cast<uintptr_t>(field) % 64 == 0)
    hipLaunchKernelGGL(gen_fwd_kernel<false>, dim3((unsigned)(base * nbz)), dim3(kFwdThreads), 0, s, grid, field,
                       g, q, nbx, nby, zchunk);
  else
    hipLaunchKernelGGL(gen_fwd_kernel<true>, dim3((unsigned)(base * nbz)), dim3(kFwdThreads), 0, s, grid, field,
                       g, q, nbx, nby, zchunk);
  return hipGetLastError();
}

size_t general_workspace_bytes(const GenGeom& q) { return gen_layout(q, nullptr, nullptr); }

hipError_t launch_adjoint_general(const float* dfield, float* grad, const GenGeom& q, void* workspace,
                                  hipStream_t s) {
  GenWork wk;
  gen_layout(q, workspace, &wk);
  GenTables3 tp;
  const GenAxis* ax[3] = {&q.x, &q.y, &q.z};
  for (int i = 0; i < 3; ++i) {
    tp.ax[i] = *ax[i];
    tp.tile[i] = wk.tile[i];
    tp.w[i] = wk.w[i];
    tp.first[i] = wk.first[i];
    tp.nb[i] = (int)blocks_for(std::max(ax[i]->n, ax[i]->g + 1));
  }
  hipLaunchKernelGGL(gen_tables3_kernel, dim3((unsigned)(tp.nb[0] + tp.nb[1] + tp.nb[2])), dim3(256), 0, s, tp);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  const GenAdj a = make_gen_adj(q);
  GzTables T;
  for (int i = 0; i < 3; ++i) {
    T.tile[i] = wk.tile[i];
    T.w[i] = wk.w[i];
    T.first[i] = wk.first[i];
  }
  const long nbricks = (long)a.nbx * a.nby * a.nbz;
  const int nxb = (q.x.g + kWave - 1) / kWave, nyb = (q.y.g + 3) / 4;
  const long nblk = (long)nxb * nyb * q.z.g;
  if (nbricks > 0x7fffffffL || nblk > 0x7fffffffL) return hipErrorInvalidValue;
  const size_t lds = (size_t)gz_layout(a).total * sizeof(float);
  if (a.cmx - 3 <= kAdjTiles)
    hipLaunchKernelGGL(gen_zf_pass1_kernel<true>, dim3((unsigned)nbricks), dim3(kGzThreads), lds, s, dfield, wk.part, q,
                       a, T);
  else
    hipLaunchKernelGGL(gen_zf_pass1_kernel<false>, dim3((unsigned)nbricks), dim3(kGzThreads), lds, s, dfield, wk.part,
                       q, a, T);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gen_zf_pass2_kernel, dim3((unsigned)nblk), dim3(256), 0, s, wk.part, grad, q, a, T);
  return hipGetLastError();
}

}  // namespace bsi
