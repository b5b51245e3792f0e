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
// Adjoint: three separable gathers in a fixed order, one output per thread:
//   A[z][y][cx]  = sum_x  Bx(x; cx)  dfield[z][y][x]       x ascending
//   Bm[z][cy][cx] = sum_y By(y; cy)  A[z][y][cx]           y ascending
//   grad[cz][cy][cx] = sum_z Bz(z; cz) Bm[z][cy][cx]        z ascending
// where B(x; c) = B_{c - i(x)}(u(x)) for the voxels whose window holds c.  The
// per-axis tables i(x), B(u(x)) are computed once per call into the workspace.
#include <cmath>

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

// Per-axis tables: tile[v] = i(v), w[v][0..3] = B(u(v)), for v < n.
__global__ __launch_bounds__(256) void gen_table_kernel(GenAxis a, int* __restrict__ tile,
                                                         float* __restrict__ w) {
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (v >= a.n) return;
  float b[4];
  tile[v] = gen_weights(a, v, b);
#pragma unroll
  for (int l = 0; l < 4; ++l) w[4 * v + l] = b[l];
}

constexpr int kGatherChunk = 8;  // voxels loaded together per output

// One separable gather along an axis.  The input is viewed as [outer][n][inner]
// F3 values (n along the axis), the output as [outer][g][inner]; output
// (o, c, k) sums the inputs (o, v, k) whose window holds c, v ascending.
__global__ __launch_bounds__(256) void gen_gather_kernel(const float* __restrict__ in, float* __restrict__ out,
                                                          GenAxis a, const int* __restrict__ tile,
                                                          const int* __restrict__ first, const float* __restrict__ w,
                                                          long outer, int inner) {
  const long id = (long)blockIdx.x * 256 + threadIdx.x;
  const long total = outer * a.g * (long)inner;
  if (id >= total) return;
  const int k = (int)(id % inner);
  const long rest = id / inner;
  const int c = (int)(rest % a.g);
  const long o = rest / a.g;
  // the voxels whose window holds c: c - 3 <= i(v) <= c, i.e. [first[c-3], first[c+1])
  const int va = first[max(c - 3, 0)], vb = first[c + 1];
  float sx = 0.f, sy = 0.f, sz = 0.f;
  const float* src = in + ((size_t)o * a.n * inner + k) * 3;
  // a chunk's loads are all issued before its sums (clamped indices, valid
  // voxels summed in ascending order)
  for (int v0 = va; v0 < vb; v0 += kGatherChunk) {
    int vi[kGatherChunk];
#pragma unroll
    for (int j = 0; j < kGatherChunk; ++j) vi[j] = min(v0 + j, vb - 1);
    float b[kGatherChunk];
    F3 d[kGatherChunk];
#pragma unroll
    for (int j = 0; j < kGatherChunk; ++j) {
      b[j] = w[4 * vi[j] + (c - tile[vi[j]])];
      d[j] = ldf3(src + (size_t)vi[j] * inner * 3);
    }
#pragma unroll
    for (int j = 0; j < kGatherChunk; ++j) {
      if (v0 + j < vb) {
        sx = fmaf(b[j], d[j].x, sx);
        sy = fmaf(b[j], d[j].y, sy);
        sz = fmaf(b[j], d[j].z, sz);
      }
    }
  }
  float* dst = out + (((size_t)o * a.g + c) * inner + k) * 3;
  dst[0] = sx;
  dst[1] = sy;
  dst[2] = sz;
}

// First voxel of every tile of an axis: first[t] = min{v : i(v) >= t} for t = 0..g
// (first[g] = n), from the nondecreasing table of window starts.
__global__ __launch_bounds__(256) void gen_first_kernel(GenAxis a, const int* __restrict__ tile,
                                                         int* __restrict__ first) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t > a.g) return;
  int lo = 0, hi = a.n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (tile[mid] < t) lo = mid + 1;
    else hi = mid;
  }
  first[t] = lo;
}

// The x pass of the adjoint by tile moments.  Along x, tile t is the run of
// voxels [first[t], first[t+1]), and output c = sum_l M_l(c - l) (l ascending)
// with M_l(t) = sum_{v in tile t} B_l(u(v)) d(v) (v ascending).  A wave takes
// one row and kGxTiles consecutive tiles t0 .. t0+63 (t0 = c0 - 3): lane j
// forms the moments of tile t0 + j from global memory (its tile's voxels are
// contiguous, so the wave's loads cover a contiguous run), publishes them in
// the wave's LDS region, and lanes j < kGxTiles - 3 then form output c0 + j.
constexpr int kGxRows = 4;                 // rows per workgroup, one per wave
constexpr int kGxThreads = kGxRows * kWave;
constexpr int kGxTiles = kWave;            // tiles per wave
constexpr int kGxOut = kGxTiles - 3;       // outputs per wave
constexpr int kGxChunk = 6;                // voxels loaded together per lane

__global__ __launch_bounds__(kGxThreads) void gen_gather_x_kernel(const float* __restrict__ in,
                                                                   float* __restrict__ out, GenAxis a,
                                                                   const int* __restrict__ first,
                                                                   const float* __restrict__ w, long rows) {
  __shared__ float sm[kGxRows][kGxTiles * 12];
  const int nseg = (a.g + kGxOut - 1) / kGxOut;
  const long rblk = blockIdx.x / nseg;
  const int seg = blockIdx.x - (int)(rblk * nseg);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const long row = rblk * kGxRows + wave;
  if (row >= rows) return;  // wave-uniform; no workgroup barrier below
  const int c0 = seg * kGxOut;
  const int t = c0 - 3 + lane;  // this lane's tile
  float mm[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) mm[k] = 0.f;
  if (t >= 0 && t < a.g - 3) {  // tiles 0 .. g-4 hold voxels
    const float* src = in + (size_t)row * a.n * 3;
    const int v1 = first[t + 1];
    // a chunk's loads are all issued before its sums (clamped addresses, valid
    // voxels summed in ascending order): several loads in flight per lane
    for (int v0 = first[t]; v0 < v1; v0 += kGxChunk) {
      F3 d[kGxChunk];
      float b[kGxChunk][4];
#pragma unroll
      for (int j = 0; j < kGxChunk; ++j) {
        const int v = min(v0 + j, v1 - 1);
        d[j] = ldf3(src + (size_t)v * 3);
#pragma unroll
        for (int l = 0; l < 4; ++l) b[j][l] = w[4 * v + l];
      }
#pragma unroll
      for (int j = 0; j < kGxChunk; ++j) {
        if (v0 + j < v1) {
#pragma unroll
          for (int l = 0; l < 4; ++l) {
            mm[3 * l] = fmaf(b[j][l], d[j].x, mm[3 * l]);
            mm[3 * l + 1] = fmaf(b[j][l], d[j].y, mm[3 * l + 1]);
            mm[3 * l + 2] = fmaf(b[j][l], d[j].z, mm[3 * l + 2]);
          }
        }
      }
    }
  }
  float* mv = sm[wave];
#pragma unroll
  for (int k = 0; k < 12; ++k) mv[lane * 12 + k] = mm[k];
  wave_lds_sync();
  const int c = c0 + lane;
  if (lane < kGxOut && c < a.g) {
    float sx = 0.f, sy = 0.f, sz = 0.f;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const float* m = mv + (lane + 3 - l) * 12 + 3 * l;  // tile c - l (zero when it has no voxels)
      sx += m[0];
      sy += m[1];
      sz += m[2];
    }
    float* dst = out + ((size_t)row * a.g + c) * 3;
    dst[0] = sx;
    dst[1] = sy;
    dst[2] = sz;
  }
}

constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }

struct GenWork {
  int* tile[3];
  float* w[3];
  int* first[3];  // first voxel of every tile, per axis (g + 1 entries)
  float* A;   // [nz][ny][gx][3]
  float* Bm;  // [nz][gy][gx][3]
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
  if (wk) wk->A = reinterpret_cast<float*>(p + off);
  off += align256((size_t)q.z.n * q.y.n * q.x.g * 3 * sizeof(float));
  if (wk) wk->Bm = reinterpret_cast<float*>(p + off);
  off += align256((size_t)q.z.n * q.y.g * q.x.g * 3 * sizeof(float));
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
  const GenAxis* ax[3] = {&q.x, &q.y, &q.z};
  for (int i = 0; i < 3; ++i) {
    hipLaunchKernelGGL(gen_table_kernel, dim3(blocks_for(ax[i]->n)), dim3(256), 0, s, *ax[i], wk.tile[i], wk.w[i]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gen_first_kernel, dim3(blocks_for(ax[i]->g + 1)), dim3(256), 0, s, *ax[i], wk.tile[i],
                       wk.first[i]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // x: [nz*ny][nx] -> A [nz*ny][gx] by tile moments: kGxRows rows and kGxOut
  // outputs per workgroup
  hipError_t e;
  const long rows = (long)q.z.n * q.y.n;
  const long nseg = (q.x.g + kGxOut - 1) / kGxOut;
  const long blocks = (rows + kGxRows - 1) / kGxRows * nseg;
  if (blocks > 0x7fffffffL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gen_gather_x_kernel, dim3((unsigned)blocks), dim3(kGxThreads), 0, s, dfield, wk.A, q.x,
                     wk.first[0], wk.w[0], rows);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // y: [nz][ny][gx] -> Bm [nz][gy][gx]
  hipLaunchKernelGGL(gen_gather_kernel, dim3(blocks_for((long)q.z.n * q.y.g * q.x.g)), dim3(256), 0, s, wk.A,
                     wk.Bm, q.y, wk.tile[1], wk.first[1], wk.w[1], (long)q.z.n, q.x.g);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // z: [1][nz][gy*gx] -> grad [gz][gy*gx]
  hipLaunchKernelGGL(gen_gather_kernel, dim3(blocks_for((long)q.z.g * q.y.g * q.x.g)), dim3(256), 0, s, wk.Bm,
                     grad, q.z, wk.tile[2], wk.first[2], wk.w[2], 1L, q.y.g * q.x.g);
  return hipGetLastError();
}

}  // namespace bsi
