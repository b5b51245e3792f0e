// Device-side building blocks shared by the single-volume and batched kernels.
//
// Every arithmetic step is written with explicit fmaf() in a fixed order and the
// library is compiled with -ffp-contract=off, so one routine gives the same bits
// wherever it is inlined (single-volume launch, batched persistent launch, graph).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bsi {

constexpr int kWave = 64;
constexpr int kMaxSpacing = 64;
// Basis table for every spacing d in [1, kMaxSpacing]: row (d, o) holds
// B0..B3(o/d), the weights of Eq. 1 at in-tile offset o.
constexpr int kLutFloats = 4 * kMaxSpacing * (kMaxSpacing + 1) / 2;
// Rotated rows (lut_rot_row), stored after the basis table in the same array.
constexpr int kLutRotFloats = 4 * kLutFloats;
constexpr int kNumXcd = 8;  // MI355X: 8 accelerator complex dies, 32 CUs each

// 12-byte vector of the three displacement components.  Packed with 4-byte
// alignment so one lane moves it with a single global_{load,store}_dwordx3.
struct __attribute__((packed, aligned(4))) F3 {
  float x, y, z;
};

struct VolGeom {
  int32_t nx, ny, nz;  // voxels
  int32_t dx, dy, dz;  // spacing (voxels per tile)
  int32_t gx, gy, gz;  // control points = ceil(n/d) + 3
};

// Brick decomposition of the adjoint along one axis: the axis is cut into U
// units of u voxels (a tile, or a single voxel when a tile is taller than a
// brick may be), and brick b of nb holds the k units [b*k, (b+1)*k), the last
// brick the rest.  A brick is w = k*u voxels wide, so brick boundaries sit at
// multiples of w: with k = 16 x-tiles of d voxels a brick row is 192 d bytes,
// a multiple of 64, and rows that start on a 64-byte boundary are cut only at
// 64-byte boundaries.  cm bounds the number of control points whose support
// meets one brick (the partial-window stride).
struct AdjAxis {
  int32_t u, U, k, nb, w, cm;
};

// The adjoint's bricks (see adjoint_device.h).  A pure function of the
// geometry, so the summation order, and thus the bits, depend on the inputs only.
struct AdjGeom {
  VolGeom g;
  AdjAxis x, y, z;
};

// First voxel of brick b (b <= nb; brick nb begins at the axis end n).  For
// b < nb this is b * w < n, since b * k < U.  Axes hold at most 2^20 voxels,
// so b * w fits 32 bits.
__host__ __device__ __forceinline__ int adj_brick_begin(const AdjAxis& a, int n, int b) {
  const int v = b * a.w;
  return v < n ? v : n;
}
__host__ __device__ __forceinline__ int adj_brick_of_voxel(const AdjAxis& a, int v) { return v / a.w; }

// Integer min / max callable from host code too (the host index checker runs
// the kernels' address arithmetic on the CPU).
__host__ __device__ constexpr int imin(int a, int b) { return a < b ? a : b; }
__host__ __device__ constexpr int imax(int a, int b) { return a > b ? a : b; }

__device__ __forceinline__ const float* lut_row(const float* lut, int d, int o) {
  return lut + 4 * ((d * (d - 1)) / 2 + o);
}
// Row (d, o) rotated by ph: element k is B_((k - ph) & 3)(o/d).  `lut` is the
// basis table's device pointer; the rotated rows follow it.
__device__ __forceinline__ const float* lut_rot_row(const float* lut, int d, int o, int ph) {
  return lut + kLutFloats + 16 * ((d * (d - 1)) / 2 + o) + 4 * ph;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// A pointer read from memory (not a kernel argument) is taken as a generic
// pointer, and accesses through it become flat instructions, which also count
// against the LDS wait counter.  Rebuilt from its bits in the global address
// space, the accesses derived from it are global ones.
template <class T>
__device__ __forceinline__ T* as_global(T* p) {
  using G = __attribute__((address_space(1))) T;
  return (T*)(G*)(uintptr_t)p;
}

// Workgroups are dispatched round-robin over the 8 XCDs (id % 8).  Remap so that
// each XCD receives one contiguous range of logical work items: neighbouring
// items share control points, which then stay in that XCD's L2.
__host__ __device__ __forceinline__ int xcd_remap(int id, int n) {
  const int q = n / kNumXcd, r = n % kNumXcd;
  const int xcd = id % kNumXcd, k = id / kNumXcd;
  return xcd * q + (xcd < r ? xcd : r) + k;
}

// Work items of workgroup `block` of `grid` over [0, total) in a batched
// launch: first, first + step, ... while below total.  A persistent grid
// steps by its size; a grid of one workgroup per item (grid = total) takes
// its one item and steps past the end.
struct ItemRange {
  int64_t first, step;
};
__host__ __device__ inline ItemRange batch_items(int block, int grid, int64_t total, bool persistent) {
  return ItemRange{xcd_remap(block, grid), persistent ? (int64_t)grid : total};
}

// Order this wave's LDS writes before its following LDS reads (and vice versa):
// lanes exchange data through the wave's own region, no workgroup barrier.
// The fences name the LDS ("local") address space only: a fence without an
// address space would also order global memory, i.e. wait for the wave's
// outstanding prefetch loads.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

__device__ __forceinline__ F3 ldf3(const float* p) { return *reinterpret_cast<const F3*>(p); }
__device__ __forceinline__ void stf3(float* p, F3 v) { *reinterpret_cast<F3*>(p) = v; }

// ----------------------------------------------------------------------------
// Forward BSI for one workgroup: kFwdRows consecutive rows y0.. of the 64-voxel
// x-strip x0..x0+63 (lane = x), voxel planes z0..z1-1.  All bounds are
// workgroup-uniform.
//
// Sum factorisation of Eq. 1, per lane: for control plane cz,
//   Q(cz) = sum_m By_m(v) * (sum_l Bx_l(u) * phi[cz][ty+m][tx+l])
// and for each voxel plane z of tile tz,
//   T = sum_n Bz_n(w) * Q(tz+n).
// Q is kept for a rolling window of 4 planes in registers, so each control
// plane is contracted once per row and reused by the dz voxel planes of each of
// the 4 tiles that read it.  The control points the workgroup needs from a plane
// (a window of at most kFwdMaxCy x kFwdMaxCx points) are staged once in a
// two-slot LDS ring: the next plane is loaded into registers (a few floats per
// thread, coalesced rows) while the current tile is written, then stored to the
// free slot; one barrier per tile.  Each voxel is one 12-byte store, so a wave
// writes 768 contiguous bytes per plane.  For scalar images a lane owns 4
// consecutive voxels instead (one 16-byte store; a wave writes 1 KB per plane).
// ----------------------------------------------------------------------------
#ifndef BSI_FWD_ROWS
#define BSI_FWD_ROWS 4
#endif
constexpr int kFwdRows = BSI_FWD_ROWS;                 // waves (rows) per workgroup
constexpr int kFwdThreads = kWave * kFwdRows;
constexpr int kFwdMaxCx = (kWave - 1) + 4;             // window width at spacing 1
constexpr int kFwdMaxCy = (kFwdRows - 1) + 4;          // window height at spacing 1
// Workgroup shape: R rows of S consecutive strips, one wave per (row, strip);
// a lane owns V consecutive x-voxels, so a strip is 64 V voxels and a
// workgroup row 64 S V.  The staged window is sized for spacing 1.
template <int R, int S, int V>
struct FwdTile {
  static constexpr int rows = R, strips = S, lane_voxels = V;
  static constexpr int threads = kWave * R * S;
  static constexpr int width = kWave * S * V;  // voxels per workgroup row
  static constexpr int max_cx = width - 1 + 4, max_cy = R - 1 + 4;
};
using FwdTileDefault = FwdTile<kFwdRows, 1, 1>;
// Staged window of one control plane for C components per point.
template <int C, class T = FwdTileDefault>
__host__ __device__ constexpr int fwd_pitch() { return T::max_cx * C; }  // floats per staged control row
template <int C, class T = FwdTileDefault>
__host__ __device__ constexpr int fwd_loads() {  // staged floats per thread
  return (T::max_cy * fwd_pitch<C, T>() + T::threads - 1) / T::threads;
}

template <int C, class T = FwdTileDefault>
struct FwdSmem {
  float ring[2][fwd_loads<C, T>() * T::threads];
};

// Control points a forward workgroup of `width` voxels x `rows` rows at
// (x0, y0) reads from each plane: columns cx0 .. cx0 + ncx - 1, rows
// cy0 .. cy0 + ncy - 1 (the tiles of its voxels plus 3).
struct FwdWindow {
  int cx0, ncx, cy0, ncy;
};
__host__ __device__ inline FwdWindow fwd_window(const VolGeom& g, int x0, int y0, int width, int rows) {
  FwdWindow w;
  w.cx0 = x0 / g.dx;
  w.ncx = (imin(x0 + width, g.nx) - 1) / g.dx - w.cx0 + 4;
  w.cy0 = y0 / g.dy;
  w.ncy = (imin(y0 + rows, g.ny) - 1) / g.dy - w.cy0 + 4;
  return w;
}

// Staging map: thread tid moves floats e = tid + k * threads of the window,
// e = row * pitch + col; goff[k] is its grid offset within a plane, or -1 when
// e lies outside this workgroup's window.
template <int C, class T = FwdTileDefault>
struct FwdStage {
  int goff[fwd_loads<C, T>()];
};

template <int C, class T = FwdTileDefault>
__host__ __device__ inline FwdStage<C, T> fwd_stage_map(const VolGeom& g, int cx0, int ncx, int cy0, int ncy,
                                                        int tid) {
  FwdStage<C, T> m;
#pragma unroll
  for (int k = 0; k < fwd_loads<C, T>(); ++k) {
    const int e = tid + k * T::threads;
    const int row = e / fwd_pitch<C, T>();
    const int col = e - row * fwd_pitch<C, T>();
    m.goff[k] = (row < ncy && col < ncx * C) ? ((cy0 + row) * g.gx + cx0) * C + col : -1;
  }
  return m;
}

template <int C, class T = FwdTileDefault>
__device__ __forceinline__ void fwd_fetch(const float* __restrict__ grid, const VolGeom& g,
                                          const FwdStage<C, T>& m, int cz, float (&r)[fwd_loads<C, T>()]) {
  const float* plane = grid + (size_t)cz * g.gy * g.gx * C;
#pragma unroll
  for (int k = 0; k < fwd_loads<C, T>(); ++k) r[k] = m.goff[k] >= 0 ? plane[m.goff[k]] : 0.f;
}

template <int C, class T = FwdTileDefault>
__device__ __forceinline__ void fwd_stage(float* __restrict__ slot, int tid, const float (&r)[fwd_loads<C, T>()]) {
#pragma unroll
  for (int k = 0; k < fwd_loads<C, T>(); ++k) slot[tid + k * T::threads] = r[k];
}

template <int C>
struct FwdVal {
  float v[C];
};

// Q for this lane's (x, y) from a staged plane: the x-contraction of each of the
// 4 control rows, then the y-contraction with weights wy[0..3].  The row loop is
// kept rolled so only one row is in flight: a small register footprint, i.e.
// more waves per SIMD to hide LDS and memory latency.
template <int C, class T = FwdTileDefault>
__device__ __forceinline__ FwdVal<C> fwd_contract(const float* __restrict__ slot, int base, float bx0,
                                                  float bx1, float bx2, float bx3,
                                                  const float* __restrict__ wy) {
  // row 0 outside the rolled loop: q = By_0 * row0, then q = fma(By_m, row_m, q)
  FwdVal<C> q;
  {
    const float* p = slot + base;
    const float b = wy[0];
#pragma unroll
    for (int c = 0; c < C; ++c)
      q.v[c] = b * fmaf(bx3, p[3 * C + c], fmaf(bx2, p[2 * C + c], fmaf(bx1, p[C + c], bx0 * p[c])));
  }
#pragma unroll 1
  for (int m = 1; m < 4; ++m) {
    const float* p = slot + base + m * fwd_pitch<C, T>();
    const float b = wy[m];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const float r = fmaf(bx3, p[3 * C + c], fmaf(bx2, p[2 * C + c], fmaf(bx1, p[C + c], bx0 * p[c])));
      q.v[c] = fmaf(b, r, q.v[c]);
    }
  }
  return q;
}

// Streaming store of one voxel's C values: non-temporal, so the write stream
// does not evict the control points that neighbouring waves still read from L2.
// (12-byte stores straight from the lanes measured faster than staging the
// wave's row through LDS into 16-byte stores.)
template <int C>
__device__ __forceinline__ void fwd_store(float* p, const float (&t)[C]) {
#pragma unroll
  for (int c = 0; c < C; ++c) __builtin_nontemporal_store(t[c], p + c);
}

typedef float fwd_f4 __attribute__((ext_vector_type(4)));
typedef float fwd_f3 __attribute__((ext_vector_type(3)));

// Buffer stores (edge stores below): resource word 3 for raw 32-bit access on
// CDNA3/4, and the non-temporal cache-policy bit.
constexpr int kBufferFlags = 0x00020000;
constexpr int kCpolNT = 2;
template <int C>
__device__ __forceinline__ void fwd_buffer_store(__amdgpu_buffer_rsrc_t rs, int off, const float (&t)[C], int cpol);
template <>
__device__ __forceinline__ void fwd_buffer_store<3>(__amdgpu_buffer_rsrc_t rs, int off, const float (&t)[3],
                                                    int cpol) {
  if (cpol) __builtin_amdgcn_raw_buffer_store_b96(fwd_f3{t[0], t[1], t[2]}, rs, off, 0, kCpolNT);
  else __builtin_amdgcn_raw_buffer_store_b96(fwd_f3{t[0], t[1], t[2]}, rs, off, 0, 0);
}
template <>
__device__ __forceinline__ void fwd_buffer_store<1>(__amdgpu_buffer_rsrc_t rs, int off, const float (&t)[1],
                                                    int cpol) {
  if (cpol) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, t[0]), rs, off, 0, kCpolNT);
  else __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, t[0]), rs, off, 0, 0);
}

// Edge stores for a wave that writes one voxel per lane of a contiguous row
// span, voxels [xw, xw + nw) of its row, once per plane.  A 64-byte segment
// only partly inside that span is shared with the neighbouring span (another
// wave, possibly another workgroup); written with non-temporal stores, its two
// halves reach HBM separately, which measured 50% slower overall.  The lanes
// that write into such a segment use ordinary stores instead, so the halves
// meet in L2; the other lanes stream with non-temporal stores.  m is the span's
// offset in its first segment; it moves by the plane size each plane.  Both
// kinds are buffer stores over the wave's row (a global store of each kind on
// the two sides of a branch would be merged by the compiler into one ordinary
// store); a row holds at most 2^20 voxels (the ABI's axis limit), so its byte
// offsets fit 32 bits.
template <int C>
struct FwdEdgeStore {
  static constexpr int kVB = 4 * C;  // bytes per voxel
  float* row;                        // the wave's row in the current plane
  size_t zstride;                    // floats per plane
  uint32_t m, mstep;
  int row_bytes, nw, vl, lane_off;

  // field: the volume; (z0, yc): the wave's first plane and its row; xw: the
  // span's first voxel; x: this lane's voxel (clamped into the row by the caller
  // when idle).
  __device__ __forceinline__ FwdEdgeStore(float* field, const VolGeom& g, int z0, int yc, int xw, int x) {
    zstride = (size_t)g.ny * g.nx * C;
    row = field + ((size_t)z0 * g.ny + yc) * g.nx * C;
    row_bytes = g.nx * kVB;
    nw = max(0, min(kWave, g.nx - xw));
    vl = x - xw;
    lane_off = x * kVB;
    m = (uint32_t)uniform((int)(reinterpret_cast<uintptr_t>(row + (size_t)min(xw, g.nx - 1) * C) & 63));
    mstep = (uint32_t)((zstride * 4) & 63);
  }
  // Store this lane's voxel of the current plane (if active), then step to the next plane.
  __device__ __forceinline__ void store(bool active, const float (&t)[C]) {
    const int head = m ? (int)(64 - m + kVB - 1) / kVB : 0;               // lanes in the first partial segment
    const int end = (int)m + kVB * nw;
    const int tail = (end & 63) ? ((end & ~63) - (int)m) / kVB : nw;     // lanes from here on: the last one
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(row, 0, row_bytes, kBufferFlags);
    if (active) {
      if (vl < head || vl >= tail)
        fwd_buffer_store<C>(rs, lane_off, t, 0);
      else
        fwd_buffer_store<C>(rs, lane_off, t, kCpolNT);
    }
    m = (m + mstep) & 63;
    row += zstride;
  }
};

// Collective over the workgroup (T::threads threads, all bounds uniform).
// C = 3 for displacement grids, C = 1 for scalar images.  x0, y0: the
// workgroup's first voxel and row.  The lane of strip k owns the V consecutive
// voxels x0 + 64 V k + V lane + (0 .. V-1) of its row; each voxel goes through
// exactly the same operations whatever the shape.  V = 4 (C = 1 only) requires
// every row to start on a 16-byte boundary: a lane whose 4 voxels all lie in
// the volume writes them with one 16-byte store.  Edge (V = 1): lanes whose
// voxel lies in a 64-byte segment shared with the neighbouring span use
// ordinary stores (FwdEdgeStore); for rows that do not start on 64-byte boundaries.
// Plain (V = 1, no Edge): ordinary stores for every voxel.
template <int C, class T = FwdTileDefault, bool Edge = false, bool Plain = false>
__device__ __forceinline__ void fwd_block(const float* __restrict__ grid, float* __restrict__ field,
                                          const VolGeom& g, const float* __restrict__ lut, int x0, int y0,
                                          int z0, int z1, FwdSmem<C, T>& sm, int tid) {
  constexpr int V = T::lane_voxels;
  static_assert(V == 1 || (V == 4 && C == 1), "wide lanes are for scalar images");
  static_assert(!Edge || V == 1, "edge stores assume one voxel per lane");
  const int lane = tid & (kWave - 1);
  const int wave = uniform(tid / kWave);
  const FwdWindow win = fwd_window(g, x0, y0, T::width, T::rows);
  const int cx0 = win.cx0, cy0 = win.cy0;
  const FwdStage<C, T> map = fwd_stage_map<C, T>(g, cx0, win.ncx, cy0, win.ncy, tid);

  const int xl = x0 + (wave % T::strips) * kWave * V + V * lane;  // the lane's first voxel
  const int y = y0 + wave / T::strips;
  const int yc = min(y, g.ny - 1);
  const int ty = yc / g.dy;
  const int oy = yc - ty * g.dy;
  const float* wy = lut_row(lut, g.dy, oy);  // wave-uniform
  bool active[V];
  float bx[V][4];
  int base[V];
#pragma unroll
  for (int k = 0; k < V; ++k) {
    const int x = xl + k;
    active[k] = x < g.nx && y < g.ny;
    const int xc = min(x, g.nx - 1);  // idle lanes read a valid column, store nothing
    const int tx = xc / g.dx;
    const float* wx = lut_row(lut, g.dx, xc - tx * g.dx);
#pragma unroll
    for (int l = 0; l < 4; ++l) bx[k][l] = wx[l];
    base[k] = (ty - cy0) * fwd_pitch<C, T>() + (tx - cx0) * C;
  }
  auto contract = [&](const float* slot, int k) {
    return fwd_contract<C, T>(slot, base[k], bx[k][0], bx[k][1], bx[k][2], bx[k][3], wy);
  };

  int tz = z0 / g.dz;
  int oz = z0 - tz * g.dz;
  float r[fwd_loads<C, T>()];
  // Warm-up: stage planes tz, tz+1, tz+2 one at a time (slots 0, 1, 0) and shift
  // their contractions into q0..q2; then stage plane tz+3 into slot 1 (its
  // contraction is the loop head).  One plane in flight keeps registers low.
  FwdVal<C> q0[V], q1[V], q2[V];
#pragma unroll
  for (int k = 0; k < V; ++k)
#pragma unroll
    for (int c = 0; c < C; ++c) q0[k].v[c] = q1[k].v[c] = q2[k].v[c] = 0.f;
#pragma unroll 1
  for (int j = 0; j < 3; ++j) {
    __syncthreads();  // the slot may still be read (previous item or iteration)
    fwd_fetch<C, T>(grid, g, map, tz + j, r);
    fwd_stage<C, T>(sm.ring[j & 1], tid, r);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const FwdVal<C> qn = contract(sm.ring[j & 1], k);
      q0[k] = q1[k];
      q1[k] = q2[k];
      q2[k] = qn;
    }
  }
  __syncthreads();
  fwd_fetch<C, T>(grid, g, map, tz + 3, r);
  fwd_stage<C, T>(sm.ring[1], tid, r);
  __syncthreads();
  int slot3 = 1;  // slot holding plane tz + 3

  const size_t zstride = (size_t)g.ny * g.nx * C;
  float* out = field + (((size_t)z0 * g.ny + yc) * g.nx + min(xl, g.nx - 1)) * C;
  bool all = true;
#pragma unroll
  for (int k = 0; k < V; ++k) all = all && active[k];
  const bool wide = V == 4 && all;
  // Used by the Edge path only (elsewhere the compiler drops it).  One voxel per
  // lane, so the wave's span is its strip.
  FwdEdgeStore<C> edge(field, g, z0, yc, x0 + (wave % T::strips) * kWave * V, min(xl, g.nx - 1));
  int z = z0;
  for (;;) {
    FwdVal<C> q3[V];
#pragma unroll
    for (int k = 0; k < V; ++k) q3[k] = contract(sm.ring[slot3], k);
    const int left = z1 - z;
    const bool more = g.dz - oz < left;  // another tile follows inside this range
    // its new plane tz + 4 is then at most ceil(nz/dz) + 2 = gz - 1: in bounds
    if (more) fwd_fetch<C, T>(grid, g, map, tz + 4, r);
    const int oend = more ? g.dz : oz + left;
    for (; oz < oend; ++oz, ++z) {
      const float* wz = lut_row(lut, g.dz, oz);
      const float w0 = wz[0], w1 = wz[1], w2 = wz[2], w3 = wz[3];
      float t[V][C];
#pragma unroll
      for (int k = 0; k < V; ++k)
#pragma unroll
        for (int c = 0; c < C; ++c)
          t[k][c] = fmaf(w3, q3[k].v[c], fmaf(w2, q2[k].v[c], fmaf(w1, q1[k].v[c], w0 * q0[k].v[c])));
      if constexpr (V == 4) {
        if (wide) {
          __builtin_nontemporal_store(fwd_f4{t[0][0], t[1][0], t[2][0], t[3][0]}, reinterpret_cast<fwd_f4*>(out));
        } else {
#pragma unroll
          for (int k = 0; k < V; ++k)
            if (active[k]) fwd_store<C>(out + k * C, t[k]);
        }
      } else if constexpr (Edge) {
        edge.store(active[0], t[0]);
      } else if constexpr (Plain) {
        if (active[0]) {
#pragma unroll
          for (int c = 0; c < C; ++c) out[c] = t[0][c];
        }
      } else {
        if (active[0]) fwd_store<C>(out, t[0]);
      }
      out += zstride;
    }
    if (!more) break;
    // plane tz + 4 goes to the slot of plane tz + 2, consumed one tile ago
    fwd_stage<C, T>(sm.ring[slot3 ^ 1], tid, r);
    __syncthreads();
    slot3 ^= 1;
    oz = 0;
    ++tz;
#pragma unroll
    for (int k = 0; k < V; ++k) {
      q0[k] = q1[k];
      q1[k] = q2[k];
      q2[k] = q3[k];
    }
  }
}

// ----------------------------------------------------------------------------
// Forward BSI, one span per workgroup: rows [y0, y1) of voxel plane z, i.e.
// (y1 - y0) * nx consecutive voxels, a contiguous range of the field.  The
// workgroup writes its span and exits; consecutive workgroups take consecutive
// spans, so the writes in flight at any moment cover one compact range of
// addresses, as in a plain fill.
//
// Sum factorisation of Eq. 1 in the order z, y, x, through LDS:
//   P[r][c]  = sum_n Bz_n(w) * phi[tz+n][ty0+r][c]          (control rows r < nry)
//   Q[ry][c] = sum_m By_m(v(y0+ry)) * P[ty(y0+ry)-ty0+m][c] (span rows ry)
//   T        = sum_l Bx_l(u(x)) * Q[ry][tx+l]               (per voxel)
// (c runs over the gx * C floats of a control row).  The four control planes
// of the span stay in L2 for the neighbouring spans of the same planes.
// Lane = voxel: each of the 256 threads takes voxels x = tid + 256 k of every
// row, so a wave writes 64 consecutive voxels per store instruction.  Stores
// are non-temporal, except for voxels in a 64-byte segment the span shares with
// the neighbouring span (its first and last segment, when the span does not
// start or end on a 64-byte boundary), which use ordinary stores so that the
// two halves meet in L2.  LDS: (nry + rows) * gx * C floats (fwd_span_lds).
// ----------------------------------------------------------------------------
constexpr int kSpanThreads = 256;

__host__ __device__ constexpr int fwd_span_ctl_rows(int rows, int dy) { return (rows - 1) / dy + 5; }
__host__ __device__ constexpr size_t fwd_span_lds(int rows, int dy, int gx, int C) {
  return (size_t)(fwd_span_ctl_rows(rows, dy) + rows) * gx * C * sizeof(float);
}

// The control window of span (z, rows [y0, y1)): planes tz .. tz+3, control
// rows ty0 .. ty0 + nry - 1, all gx columns.
struct FwdSpanWindow {
  int tz, ty0, nry;
};
__host__ __device__ inline FwdSpanWindow fwd_span_window(const VolGeom& g, int z, int y0, int y1) {
  FwdSpanWindow w;
  w.tz = z / g.dz;
  w.ty0 = y0 / g.dy;
  w.nry = (y1 - 1) / g.dy - w.ty0 + 4;
  return w;
}

template <int C>
__device__ __forceinline__ void fwd_span(const float* __restrict__ grid, float* __restrict__ field, const VolGeom& g,
                                         const float* __restrict__ lut, int z, int y0, int y1,
                                         float* __restrict__ smem, int tid) {
  const int W = g.gx * C;  // floats per control row
  const FwdSpanWindow win = fwd_span_window(g, z, y0, y1);
  const int tz = win.tz, ty0 = win.ty0, nry = win.nry;
  const float* wz = lut_row(lut, g.dz, z - tz * g.dz);
  const float z0 = wz[0], z1 = wz[1], z2 = wz[2], z3 = wz[3];
  const int rows = y1 - y0;
  float* P = smem;             // [nry][W]
  float* Q = smem + nry * W;   // [rows][W]
  const size_t pstride = (size_t)g.gy * W;
  const float* g0 = grid + ((size_t)tz * g.gy + ty0) * W;
  for (int e = tid; e < nry * W; e += kSpanThreads) {
    const float* q = g0 + e;  // control row ty0 + e / W, float e % W of plane tz
    P[e] = fmaf(z3, q[3 * pstride], fmaf(z2, q[2 * pstride], fmaf(z1, q[pstride], z0 * q[0])));
  }
  __syncthreads();
  for (int e = tid; e < rows * W; e += kSpanThreads) {
    const int ry = e / W;
    const int i = e - ry * W;
    const int y = y0 + ry;
    const int ty = y / g.dy;
    const float* wy = lut_row(lut, g.dy, y - ty * g.dy);
    const float* p = P + (ty - ty0) * W + i;
    Q[e] = fmaf(wy[3], p[3 * W], fmaf(wy[2], p[2 * W], fmaf(wy[1], p[W], wy[0] * p[0])));
  }
  __syncthreads();
  // the span's bytes [sb, se) relative to a 64-byte boundary below them
  const uintptr_t sb = reinterpret_cast<uintptr_t>(field + ((size_t)z * g.ny + y0) * g.nx * C);
  const int m = (int)(sb & 63);
  const long nvox = (long)rows * g.nx;
  const long head = m ? (64 - m + 4 * C - 1) / (4 * C) : 0;         // voxels in the shared first segment
  const long end = m + nvox * 4 * C;
  const long tail = (end & 63) ? ((end & ~63L) - m) / (4 * C) : nvox;  // first voxel in the shared last segment
  // both kinds of store are buffer stores over the span (a span holds fewer
  // than 2^32 bytes: rows * nx * C * 4 with rows * nx below 2^28)
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      field + ((size_t)z * g.ny + y0) * g.nx * C, 0, (int)(nvox * 4 * C), kBufferFlags);
  for (int ry = 0; ry < rows; ++ry) {
    const float* q = Q + ry * W;
    for (int x = tid; x < g.nx; x += kSpanThreads) {
      const int tx = x / g.dx;
      const float* wx = lut_row(lut, g.dx, x - tx * g.dx);
      const float* p = q + tx * C;
      float t[C];
#pragma unroll
      for (int c = 0; c < C; ++c)
        t[c] = fmaf(wx[3], p[3 * C + c], fmaf(wx[2], p[2 * C + c], fmaf(wx[1], p[C + c], wx[0] * p[c])));
      const long v = (long)ry * g.nx + x;
      if (v >= head && v < tail) fwd_buffer_store<C>(rs, (int)(v * 4 * C), t, kCpolNT);
      else fwd_buffer_store<C>(rs, (int)(v * 4 * C), t, 0);
    }
  }
}

}  // namespace bsi
