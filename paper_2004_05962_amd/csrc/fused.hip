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
// Pass 1 is the adjoint's z-first pass 1 (adjoint_device.h: the same bricks,
// lanes, z-accumulation and emission) with dfield replaced by the voxel's
// SSD gradient, computed on the spot.  T is evaluated as the forward kernel
// does (fwd_block): per control plane, Q = sum_m By_m sum_l Bx_l phi from the
// plane's window staged in LDS, kept for the 4 planes of the current z-tile,
// and T = sum_n Bz_n Q per voxel plane, with the same operations in the same
// order; the sampling and gradient are the SSD kernel's.  So the field, the
// per-voxel gradient and the adjoint's accumulation are bit-identical to the
// separate forward, SSD and adjoint kernels, and so is the control-grid
// gradient; only the loss is summed in another order.
//
// Each workgroup sums its voxels' squared residuals in a fixed order into one
// loss partial per brick; pass 2 is the adjoint's fixed-order gather, and the
// loss is the fixed-order sum of the partials.  No atomics.
#include "adjoint_device.h"
#include "bsi_internal.h"
#include "warp_device.h"

namespace bsi {

namespace {

// The fused pass uses the adjoint's bricks with one row per lane: kAdjBY
// waves of 64 lanes, so each lane keeps the forward's 4 contracted planes and
// the adjoint's 4 accumulators for a single voxel column.
constexpr int kFusedWaves = kAdjBY;
constexpr int kFusedThreads = kFusedWaves * kWave;

// A staged control plane: the brick's window of at most kAdjBY + 3 rows by
// adj_cx_max(DX) columns (pitch adj_cx_max(DX) points).
template <int DX>
__host__ __device__ constexpr int fused_slot_floats() {
  return (kAdjBY + 3) * adj_cx_max(DX) * 3;
}
template <int DX>
__host__ __device__ constexpr int fused_loads() {  // staged floats per thread
  return (fused_slot_floats<DX>() + kFusedThreads - 1) / kFusedThreads;
}

template <int DX>
struct FusedSmem {
  AdjSmem<DX> adj;
  float ring[2][fused_slot_floats<DX>()];
  float red[kFusedThreads];
};

// Loads of control plane cz's window into registers (thread tid takes floats
// e = tid + k kFusedThreads of the Cy x Cx x 3 window), and their store into a
// slot with row pitch adj_cx_max(DX) points.
template <int DX>
struct FusedStage {
  int src[fused_loads<DX>()];  // float offset within a control plane, -1 outside the window
  int dst[fused_loads<DX>()];
};

template <int DX>
__device__ __forceinline__ FusedStage<DX> fused_stage_map(const VolGeom& g, const AdjBrick& b, int tid) {
  constexpr int CXM = adj_cx_max(DX);
  FusedStage<DX> m;
  const int wrow = b.Cx * 3;
#pragma unroll
  for (int k = 0; k < fused_loads<DX>(); ++k) {
    const int e = tid + k * kFusedThreads;
    const int cyl = e / wrow, i = e - cyl * wrow;
    const bool in = cyl < b.Cy;
    m.src[k] = in ? ((b.cy0 + cyl) * g.gx + b.cx0) * 3 + i : -1;
    m.dst[k] = cyl * CXM * 3 + i;
  }
  return m;
}

template <int DX>
__device__ __forceinline__ void fused_fetch(const float* __restrict__ grid, const VolGeom& g, const FusedStage<DX>& m,
                                            int cz, float (&r)[fused_loads<DX>()]) {
  const float* plane = grid + (size_t)cz * g.gy * g.gx * 3;
#pragma unroll
  for (int k = 0; k < fused_loads<DX>(); ++k) r[k] = m.src[k] >= 0 ? plane[m.src[k]] : 0.f;
}

template <int DX>
__device__ __forceinline__ void fused_stage(float* __restrict__ slot, const FusedStage<DX>& m,
                                            const float (&r)[fused_loads<DX>()]) {
#pragma unroll
  for (int k = 0; k < fused_loads<DX>(); ++k)
    if (m.src[k] >= 0) slot[m.dst[k]] = r[k];
}

// Q = sum_m By_m (sum_l Bx_l phi[row + m][col + l]) from a staged plane: the
// operations of the forward kernel's contraction (fwd_contract), in its order.
template <int DX>
__device__ __forceinline__ F3 fused_contract(const float* __restrict__ slot, int base, const float (&bx)[4],
                                             const float (&by)[4]) {
  constexpr int P = adj_cx_max(DX) * 3;  // floats per staged row
  float q[3];
  {
    const float* p = slot + base;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      q[c] = by[0] * fmaf(bx[3], p[9 + c], fmaf(bx[2], p[6 + c], fmaf(bx[1], p[3 + c], bx[0] * p[c])));
  }
#pragma unroll 1
  for (int m = 1; m < 4; ++m) {
    const float* p = slot + base + m * P;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float r = fmaf(bx[3], p[9 + c], fmaf(bx[2], p[6 + c], fmaf(bx[1], p[3 + c], bx[0] * p[c])));
      q[c] = fmaf(by[m], r, q[c]);
    }
  }
  return F3{q[0], q[1], q[2]};
}

// Pairs: the sampler's x-neighbour loads (trilinear_load): 1 for nx >= 2, 0 for nx == 1.
template <int DX, bool StageAll, int Pairs>
__device__ __forceinline__ void fused_brick(const float* __restrict__ grid, const float* __restrict__ moving,
                                            const float* __restrict__ fixed, float* __restrict__ part,
                                            float* __restrict__ lpart, const AdjGeom& a,
                                            const float* __restrict__ lut, int brick, FusedSmem<DX>& sm, int tid) {
  constexpr int R = 1;
  constexpr int CXM = adj_cx_max(DX);
  const VolGeom& g = a.g;
  const int dx = DX > 0 ? DX : g.dx;
  const AdjBrick b = adj_brick_geom(a, brick);
  float* pbase = part + (size_t)brick * adj_brick_stride(a);
  const int lane = tid & (kWave - 1), wave = uniform(tid / kWave);

  // this lane's voxels: column x, rows y[r]; forward weights and window bases
  const int x = b.x0 + lane;
  const int xc = imin(x, b.xe - 1);
  const int tx = xc / dx;
  float bx[4];
  {
    const float* w = lut_row(lut, dx, xc - tx * dx);
#pragma unroll
    for (int l = 0; l < 4; ++l) bx[l] = w[l];
  }
  int yv[R], base[R];
  bool act[R];
  float by[R][4];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    yv[r] = b.y0 + wave * R + r;
    act[r] = x < b.xe && yv[r] < b.ye;
    const int yc = imin(yv[r], b.ye - 1);
    const int ty = yc / g.dy;
    const float* w = lut_row(lut, g.dy, yc - ty * g.dy);
#pragma unroll
    for (int m = 0; m < 4; ++m) by[r][m] = w[m];
    base[r] = ((ty - b.cy0) * CXM + (tx - b.cx0)) * 3;
  }
  const FusedStage<DX> map = fused_stage_map<DX>(g, b, tid);
  adj_zero_fpad<DX, R>(sm.adj, wave, lane);

  // Q of the 4 control planes of the first z-tile, one plane staged at a time
  int tz = b.cz0;  // z-bricks are whole tiles: b.z0 = tz * dz
  F3 Q[R][4];
  float st[fused_loads<DX>()];
#pragma unroll 1
  for (int j = 0; j < 4; ++j) {
    __syncthreads();  // the slot's previous plane has been contracted (or a previous brick is done)
    fused_fetch<DX>(grid, g, map, tz + j, st);
    fused_stage<DX>(sm.ring[(tz + j) & 1], map, st);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const F3 q = fused_contract<DX>(sm.ring[(tz + j) & 1], base[r], bx, by[r]);
#pragma unroll
      for (int n = 0; n < 3; ++n) Q[r][n] = Q[r][n + 1];
      Q[r][3] = q;
    }
  }
  // the next tile's new plane tz + 4 (when another tile follows inside the
  // brick, it is at most ceil(nz/dz) + 2 = gz - 1)
  bool more = (tz + 1) * g.dz < b.ze;
  if (more) fused_fetch<DX>(grid, g, map, tz + 4, st);

  F3 acc[R][4];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int n = 0; n < 4; ++n) acc[r][n] = F3{0.f, 0.f, 0.f};
  float l2 = 0.f;
  auto finish = [&](int czl, bool last) {
    F3 f[R];
#pragma unroll
    for (int r = 0; r < R; ++r) f[r] = acc[r][0];
    adj_emit_x<DX, R>(b, sm.adj, lut, dx, tid, czl, [&](int r) { return f[r]; });
    __syncthreads();
    adj_emit_y<DX, kFusedWaves, StageAll>(a, b, pbase, sm.adj, lut, tid, czl, last);
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int n = 0; n < 3; ++n) acc[r][n] = acc[r][n + 1];
      acc[r][3] = F3{0.f, 0.f, 0.f};
    }
  };

  // Per voxel plane, in two stages: (a) T from the 4 contracted planes, the
  // sample's cell and the loads of its corners and of `fixed`; (b) the
  // residual, the gradient and the z-accumulation.  Within a z-tile, (a) of
  // the next plane is issued before (b) of the current one, so a wave keeps
  // one plane's loads in flight while it finishes the previous plane.  Every
  // lane loads (a lane outside the brick from its clamped column and row, and
  // a clamped sample position), so that no load is conditional and waiting
  // for one plane's loads leaves the next plane's in flight; (b) ignores the
  // values of such lanes.
  static_assert(R == 1, "one voxel row per lane");
  struct Pending {
    SampleIn s;
    float fx;
    float w[4];  // Bz_0..3 of the plane's offset in its tile
  };
  const size_t izs = (size_t)g.ny * g.nx;
  const int y = yv[0];
  const size_t fxy = (size_t)imin(y, b.ye - 1) * g.nx + xc;  // the lane's (clamped) voxel column
  auto stage_a = [&](int z, int oz) {
    Pending p;
    const float* wz = lut_row(lut, g.dz, oz);
#pragma unroll
    for (int n = 0; n < 4; ++n) p.w[n] = wz[n];
    p.fx = fixed[(size_t)z * izs + fxy];
    // T as the forward kernel forms it
    const F3 t{fmaf(p.w[3], Q[0][3].x, fmaf(p.w[2], Q[0][2].x, fmaf(p.w[1], Q[0][1].x, p.w[0] * Q[0][0].x))),
               fmaf(p.w[3], Q[0][3].y, fmaf(p.w[2], Q[0][2].y, fmaf(p.w[1], Q[0][1].y, p.w[0] * Q[0][0].y))),
               fmaf(p.w[3], Q[0][3].z, fmaf(p.w[2], Q[0][2].z, fmaf(p.w[1], Q[0][1].z, p.w[0] * Q[0][0].z)))};
    p.s = trilinear_load<Pairs>(moving, g.nx, g.ny, g.nz, (float)x + t.x, (float)y + t.y, (float)z + t.z);
    return p;
  };
  auto stage_b = [&](const Pending& p) {
    F3 d{0.f, 0.f, 0.f};
    if (act[0]) {
      // the SSD kernel's residual and gradient
      const Sample s = trilinear_finish(p.s);
      const float res = s.w - p.fx;
      l2 = fmaf(res, res, l2);
      const float two_r = 2.f * res;
      d = F3{two_r * s.gx, two_r * s.gy, two_r * s.gz};
    }
    // the adjoint's z-accumulation
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      acc[0][n].x = fmaf(p.w[n], d.x, acc[0][n].x);
      acc[0][n].y = fmaf(p.w[n], d.y, acc[0][n].y);
      acc[0][n].z = fmaf(p.w[n], d.z, acc[0][n].z);
    }
  };

  for (int z = b.z0; z < b.ze;) {  // one z-tile (the brick's last may be partial)
    const int np = imin(g.dz, b.ze - z);
    // two register sets, used in turn (a copy from one to the other would
    // wait for the loads it copies)
    Pending p0 = stage_a(z, 0);
    int k = 0;
    for (; k + 2 < np; k += 2) {
      const Pending p1 = stage_a(z + k + 1, k + 1);
      stage_b(p0);
      p0 = stage_a(z + k + 2, k + 2);
      stage_b(p1);
    }
    if (k + 1 < np) {
      const Pending p1 = stage_a(z + k + 1, k + 1);
      stage_b(p0);
      stage_b(p1);
    } else {
      stage_b(p0);
    }
    z += np;
    if (np == g.dz && z < b.ze) {
      // plane tz + 4 goes to the slot of plane tz + 2, contracted before the
      // previous tile's barrier; the emission's barrier orders the store
      // before the contraction below
      fused_stage<DX>(sm.ring[(tz + 4) & 1], map, st);
      F3 f[R];
#pragma unroll
      for (int r = 0; r < R; ++r) f[r] = acc[r][0];
      adj_emit_x<DX, R>(b, sm.adj, lut, dx, tid, tz - b.cz0, [&](int r) { return f[r]; });
      __syncthreads();
      adj_emit_y<DX, kFusedWaves, StageAll>(a, b, pbase, sm.adj, lut, tid, tz - b.cz0, false);
#pragma unroll
      for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int n = 0; n < 3; ++n) {
          acc[r][n] = acc[r][n + 1];
          Q[r][n] = Q[r][n + 1];
        }
        acc[r][3] = F3{0.f, 0.f, 0.f};
        Q[r][3] = fused_contract<DX>(sm.ring[(tz + 4) & 1], base[r], bx, by[r]);
      }
      ++tz;
      more = (tz + 1) * g.dz < b.ze;
      if (more) fused_fetch<DX>(grid, g, map, tz + 4, st);
    }
  }
#pragma unroll 1
  for (int n = 0; n < 4; ++n) finish(tz - b.cz0 + n, n == 3);

  // loss partial of the brick: fixed-order tree over the workgroup
  sm.red[tid] = l2;
  __syncthreads();
  for (int h = kFusedThreads / 2; h > 0; h >>= 1) {
    if (tid < h) sm.red[tid] += sm.red[tid + h];
    __syncthreads();
  }
  if (tid == 0) lpart[brick] = sm.red[0];
}

template <int DX, int Pairs = 1>
__global__ __launch_bounds__(kFusedThreads) void fused_pass1_kernel(const float* __restrict__ grid,
                                                                  const float* __restrict__ moving,
                                                                  const float* __restrict__ fixed,
                                                                  float* __restrict__ part,
                                                                  float* __restrict__ lpart, AdjGeom a,
                                                                  const float* __restrict__ lut) {
  __shared__ FusedSmem<DX> sm;
  const int nbricks = a.x.nb * a.y.nb * a.z.nb;
  const int brick = xcd_remap(blockIdx.x, gridDim.x);
  if (brick >= nbricks) return;  // uniform over the workgroup
  if (adj_stage_all(a))
    fused_brick<DX, true, Pairs>(grid, moving, fixed, part, lpart, a, lut, brick, sm, threadIdx.x);
  else
    fused_brick<DX, false, Pairs>(grid, moving, fixed, part, lpart, a, lut, brick, sm, threadIdx.x);
}

}  // namespace

size_t fused_workspace_bytes(const AdjGeom& a) {
  const size_t p = (adj_workspace_bytes(a) + 255) / 256 * 256;
  return p + (size_t)a.x.nb * a.y.nb * a.z.nb * sizeof(float);
}

// The fused step's tail in one launch: workgroups [0, nblk) are pass 2 (the
// fixed-order gather of each control point's partials), and with `descend`
// also the descent update grid -= eta grad of the points they gather (pass 1
// has finished reading the grid: it ran before, on the same stream); workgroup
// nblk sums the bricks' loss partials in a fixed order.
constexpr int kTailThreads = kGatherThreads;

__global__ __launch_bounds__(kTailThreads) void fused_tail_kernel(const float* __restrict__ part,
                                                                   float* __restrict__ grad, float* __restrict__ grid,
                                                                   float eta, int descend,
                                                                   const float* __restrict__ lpart, int nlp,
                                                                   float* __restrict__ loss, AdjGeom a, int nblk) {
  if ((int)blockIdx.x == nblk) {
    __shared__ float red[kTailThreads];
    float acc = 0.f;
    for (int i = threadIdx.x; i < nlp; i += kTailThreads) acc += lpart[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kTailThreads / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0];
    return;
  }
  int cx, cy, cz;
  if (!adj_gather_index(a.g, blockIdx.x, uniform(threadIdx.x / kWave), threadIdx.x & (kWave - 1), cx, cy, cz))
    return;
  const size_t i = ((size_t)cz * a.g.gy + cy) * a.g.gx + cx;
  const F3 gv = adj_gather_point(part, a, cx, cy, cz);
  stf3(grad + i * 3, gv);
  if (descend) {  // the descent kernel's update, on the same values
    float* p = grid + i * 3;
    stf3(p, F3{fmaf(-eta, gv.x, p[0]), fmaf(-eta, gv.y, p[1]), fmaf(-eta, gv.z, p[2])});
  }
}

hipError_t launch_ssd_fused(const float* grid, const float* moving, const float* fixed, float* grad, float* loss,
                            const AdjGeom& a, const float* lut, void* workspace, hipStream_t s, float* descend_grid,
                            float eta) {
  float* part = static_cast<float*>(workspace);
  float* lpart = reinterpret_cast<float*>(static_cast<char*>(workspace) +
                                          (adj_workspace_bytes(a) + 255) / 256 * 256);
  const long nbricks = (long)a.x.nb * a.y.nb * a.z.nb;
  const dim3 gridd((unsigned)nbricks), block(kFusedThreads);
#define BSI_FUSED_CASE(D)                                                                               \
  case D:                                                                                               \
    hipLaunchKernelGGL(fused_pass1_kernel<D>, gridd, block, 0, s, grid, moving, fixed, part, lpart, a, lut); \
    break;
  static_assert(kAdjMaxDX == 12, "one case per specialised spacing");
  // a volume one voxel wide samples its x-neighbours one by one (generic kernel)
  switch (a.g.nx >= 2 ? a.g.dx : -1) {
    case -1:
      hipLaunchKernelGGL((fused_pass1_kernel<0, 0>), gridd, block, 0, s, grid, moving, fixed, part, lpart, a, lut);
      break;
    BSI_FUSED_CASE(1)
    BSI_FUSED_CASE(2)
    BSI_FUSED_CASE(3)
    BSI_FUSED_CASE(4)
    BSI_FUSED_CASE(5)
    BSI_FUSED_CASE(6)
    BSI_FUSED_CASE(7)
    BSI_FUSED_CASE(8)
    BSI_FUSED_CASE(9)
    BSI_FUSED_CASE(10)
    BSI_FUSED_CASE(11)
    BSI_FUSED_CASE(12)
    default: BSI_FUSED_CASE(0)
  }
#undef BSI_FUSED_CASE
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t nblk = adj_gather_blocks(a.g);
  if (nblk + 1 >= ((int64_t)1 << 31) || nbricks >= ((int64_t)1 << 31))
    return hipErrorInvalidConfiguration;  // a field far beyond device memory
  hipLaunchKernelGGL(fused_tail_kernel, dim3((unsigned)(nblk + 1)), dim3(kTailThreads), 0, s, part, grad, descend_grid,
                     eta, descend_grid != nullptr ? 1 : 0, lpart, (int)nbricks, loss, a, (int)nblk);
  return hipGetLastError();
}

}  // namespace bsi
