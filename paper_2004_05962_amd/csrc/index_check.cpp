// Host-side check of the kernels' index arithmetic (test infrastructure).
//
// Runs, on the CPU, the same geometry functions and __host__ __device__
// address helpers the kernels use, for every workgroup / lane / control point
// of a launch, and checks that every global load and store lies inside its
// buffer (dfield, field, grid, workspace), that every LDS index lies inside
// its array, and that pass 2 reads only partials pass 1 wrote.  Nothing here
// touches a device.  Built next to libbsi.so and called by the CPU tests.
#include <cstdio>
#include <string>
#include <vector>

#include "adjoint_device.h"
#include "bsi_internal.h"
#include "general_device.h"

namespace bsi {
namespace {

struct Check {
  std::string msg;
  bool ok = true;
  bool fail(const std::string& m) {
    if (ok) msg = m;
    ok = false;
    return false;
  }
};

#define REQUIRE(c, what)                                                         \
  do {                                                                           \
    if (!(c)) return ck.fail(std::string(what) + " [" #c "]");                   \
  } while (0)

// Loads and LDS indices of pass 1 (adj_brick) for one brick.
bool check_adj_brick(const AdjGeom& a, const AdjBrick& b, Check& ck) {
  const size_t plane = (size_t)a.g.nx * a.g.ny * 3;
  REQUIRE(b.z0 == b.cz0 * a.g.dz, "z-bricks start on tile boundaries (the march starts at offset 0)");
  REQUIRE(b.xe - b.x0 <= kAdjBX && b.ye - b.y0 <= kAdjBY, "brick within one lane per voxel and row");
  const int dxc = a.g.dx <= kAdjMaxDX ? a.g.dx : 0;
  REQUIRE(b.Cx <= adj_cx_max(dxc), "x window within the H buffer's row");
  REQUIRE(b.Cy - 3 <= kAdjTiles, "y-tiles within one row of tile lanes");
  if (adj_tile_lanes(dxc)) REQUIRE(b.ntx <= kAdjTiles, "x-tiles within one row of tile lanes");
  if (a.g.dx >= 4 && a.g.dx <= kAdjMaxDX) {  // the run-time-spacing kernel (batched pass 1) reads the same bricks
    REQUIRE(b.Cx <= adj_cx_max(kAdjAnyTile), "x window within the run-time-spacing kernel's H row");
    for (int t = 0; t < b.ntx; ++t) {
      const int xt = (b.cx0 + t) * a.g.dx - b.x0;
      REQUIRE(xt >= -adj_fpad(kAdjAnyTile) && xt + a.g.dx <= kWave + adj_fpad(kAdjAnyTile),
              "x-tile within the run-time-spacing kernel's padded F row");
    }
  }
  if (adj_fpad(dxc) > 0)  // a tile's voxels, read without tests, lie within the row and its zero pads
    for (int t = 0; t < b.ntx; ++t) {
      const int xt = (b.cx0 + t) * a.g.dx - b.x0;
      REQUIRE(xt >= -adj_fpad(dxc) && xt + a.g.dx <= kWave + adj_fpad(dxc), "x-tile within the padded F row");
    }
  if (adj_stage_all(a)) REQUIRE((size_t)adj_brick_cz(a, b) * a.y.cm * a.x.cm * 3 <= (size_t)kAdjStageFloats,
                                "staged partials within the LDS stage");
  for (int w = 0; w < kAdjWaves; ++w)
    for (int lane = 0; lane < kWave; ++lane) {
      uint32_t off[kAdjRows];
      adj_offsets<kAdjRows>(b, a.g.nx, w, lane, off);
      for (int r = 0; r < kAdjRows; ++r) {
        REQUIRE((size_t)off[r] + 3 <= plane, "pass-1 load outside its voxel plane");
        const int x = (int)(off[r] / 3 % a.g.nx), y = (int)(off[r] / 3 / a.g.nx);
        REQUIRE(x >= b.x0 && x < b.xe && y >= b.y0 && y < b.ye, "pass-1 load outside its brick");
      }
    }
  // the fused step stages each control plane's window (Cy rows x Cx points)
  REQUIRE(b.Cy <= kAdjBY + 3, "fused staging rows");
  return true;
}

// Pass 1 (its bricks, via `brick_check`) and pass 2 of a two-pass adjoint with
// brick geometry `a`.
template <class BrickCheck>
bool check_adjoint(const AdjGeom& a, BrickCheck brick_check, Check& ck) {
  const VolGeom& g = a.g;
  const size_t ws = adj_workspace_bytes(a) / sizeof(float);
  const int nb = a.x.nb * a.y.nb * a.z.nb;
  REQUIRE(a.x.nb >= 1 && a.y.nb >= 1 && a.z.nb >= 1, "brick counts");
  REQUIRE((size_t)nb * adj_brick_stride(a) == ws, "workspace holds the bricks");
  // the window of every brick, as pass 1 writes it
  std::vector<int> Cx(nb), Cy(nb), Cz(nb);
  long voxels = 0;
  for (int id = 0; id < nb; ++id) {
    const AdjBrick b = adj_brick_geom(a, id);
    REQUIRE(0 <= b.x0 && b.x0 < b.xe && b.xe <= g.nx, "brick x range");
    REQUIRE(0 <= b.y0 && b.y0 < b.ye && b.ye <= g.ny, "brick y range");
    REQUIRE(0 <= b.z0 && b.z0 < b.ze && b.ze <= g.nz, "brick z range");
    REQUIRE(b.Cx <= a.x.cm, "x window (partials stride)");
    REQUIRE(b.Cy <= a.y.cm, "y window (partials stride)");
    const int cz = adj_brick_cz(a, b);
    REQUIRE(cz <= a.z.cm, "z window (partials stride)");
    REQUIRE(b.cx0 + b.Cx <= g.gx && b.cy0 + b.Cy <= g.gy && b.cz0 + cz <= g.gz, "window inside the grid");
    REQUIRE(b.cx0 == adj_brick_c0(a.x, id % a.x.nb, g.dx), "x window start");
    REQUIRE(b.cy0 == adj_brick_c0(a.y, id / a.x.nb % a.y.nb, g.dy), "y window start");
    REQUIRE(b.cz0 == adj_brick_c0(a.z, id / (a.x.nb * a.y.nb), g.dz), "z window start");
    const size_t last = (size_t)id * adj_brick_stride(a) + adj_part_offset(a, cz - 1, b.Cy - 1, b.Cx - 1);
    REQUIRE(last + 3 <= ws, "partial store outside the workspace");
    if (!brick_check(a, b, ck)) return false;
    Cx[id] = b.Cx;
    Cy[id] = b.Cy;
    Cz[id] = cz;
    voxels += (long)(b.xe - b.x0) * (b.ye - b.y0) * (b.ze - b.z0);
  }
  REQUIRE(voxels == (long)g.nx * g.ny * g.nz, "bricks tile the volume");
  // per axis: brick b meets the support [(c-3)d, (c+1)d) of control index c
  // exactly when b lies in c's span (pass 2 misses no brick and adds no other)
  const AdjAxis* axes[3] = {&a.x, &a.y, &a.z};
  const int nn[3] = {g.nx, g.ny, g.nz}, dd[3] = {g.dx, g.dy, g.dz}, gg[3] = {g.gx, g.gy, g.gz};
  for (int ax = 0; ax < 3; ++ax)
    for (int c = 0; c < gg[ax]; ++c) {
      const AdjSpan sp = adj_span(*axes[ax], c, dd[ax], nn[ax]);
      const int lo = imax(0, (c - 3) * dd[ax]), hi = imin(nn[ax], (c + 1) * dd[ax]);
      for (int b = 0; b < axes[ax]->nb; ++b) {
        const int b0 = adj_brick_begin(*axes[ax], nn[ax], b), b1 = adj_brick_begin(*axes[ax], nn[ax], b + 1);
        const bool meets = b0 < hi && lo < b1;
        REQUIRE(meets == (b >= sp.lo && b <= sp.hi), "pass-2 span differs from the bricks meeting the support");
      }
    }
  // pass 2's workgroups take every control point exactly once
  {
    std::vector<unsigned char> hit((size_t)g.gx * g.gy * g.gz, 0);
    const int64_t nblk = adj_gather_blocks(g);
    REQUIRE(nblk < ((int64_t)1 << 31), "pass-2 grid above 2^31 workgroups");
    for (int64_t blk = 0; blk < nblk; ++blk)
      for (int w = 0; w < kGatherWaves; ++w)
        for (int l = 0; l < kWave; ++l) {
          int cx, cy, cz;
          if (!adj_gather_index(g, (int)blk, w, l, cx, cy, cz)) continue;
          REQUIRE(0 <= cx && cx < g.gx && 0 <= cy && cy < g.gy && 0 <= cz && cz < g.gz, "pass-2 point off the grid");
          unsigned char& h = hit[((size_t)cz * g.gy + cy) * g.gx + cx];
          REQUIRE(h == 0, "pass-2 point taken twice");
          h = 1;
        }
    for (unsigned char h : hit) REQUIRE(h == 1, "pass-2 point never taken");
  }
  // pass 2: every brick a control point reads holds that point in its window
  for (int cz = 0; cz < g.gz; ++cz)
    for (int cy = 0; cy < g.gy; ++cy)
      for (int cx = 0; cx < g.gx; ++cx) {
        const AdjSpan sx = adj_span(a.x, cx, g.dx, g.nx), sy = adj_span(a.y, cy, g.dy, g.ny),
                      sz = adj_span(a.z, cz, g.dz, g.nz);
        REQUIRE(0 <= sx.lo && sx.lo <= sx.hi && sx.hi < a.x.nb, "x span");
        REQUIRE(0 <= sy.lo && sy.lo <= sy.hi && sy.hi < a.y.nb, "y span");
        REQUIRE(0 <= sz.lo && sz.lo <= sz.hi && sz.hi < a.z.nb, "z span");
        for (int bz = sz.lo; bz <= sz.hi; ++bz)
          for (int by = sy.lo; by <= sy.hi; ++by)
            for (int bx = sx.lo; bx <= sx.hi; ++bx) {
              const int id = (bz * a.y.nb + by) * a.x.nb + bx;
              const int cxl = cx - adj_brick_c0(a.x, bx, g.dx), cyl = cy - adj_brick_c0(a.y, by, g.dy),
                        czl = cz - adj_brick_c0(a.z, bz, g.dz);
              REQUIRE(0 <= cxl && cxl < Cx[id] && 0 <= cyl && cyl < Cy[id] && 0 <= czl && czl < Cz[id],
                      "pass 2 reads a partial pass 1 did not write");
              REQUIRE(adj_part_addr(a, bx, by, bz, cx, cy, cz) + 3 <= ws, "pass-2 load outside the workspace");
            }
      }
  return true;
}

bool check_adjoints(const VolGeom& g, Check& ck) { return check_adjoint(make_adj_geom(g), check_adj_brick, ck); }

// The marching forward (fwd_block) with workgroup shape T and C components.
template <int C, class T>
bool check_forward_march(const VolGeom& g, Check& ck, long target = kFwdTargetBlocks) {
  const FwdLaunch L = make_fwd_launch(g, target, T::width, T::rows);
  REQUIRE(L.zchunk % g.dz == 0 && L.zchunk > 0, "z chunks of whole tiles");
  REQUIRE((long)L.nbz * L.zchunk >= g.nz && (long)(L.nbz - 1) * L.zchunk < g.nz, "z chunks cover the volume");
  const size_t cplane = (size_t)g.gx * g.gy * C;
  for (int bz = 0; bz < L.nbz; ++bz)
    for (int by = 0; by < L.nby; ++by)
      for (int bx = 0; bx < L.nbx; ++bx) {
        const int x0 = bx * T::width, y0 = by * T::rows, z0 = bz * L.zchunk, z1 = imin(g.nz, z0 + L.zchunk);
        REQUIRE(x0 < g.nx && y0 < g.ny && z0 < z1, "forward workgroup inside the volume");
        const FwdWindow w = fwd_window(g, x0, y0, T::width, T::rows);
        REQUIRE(w.ncx <= T::max_cx && w.ncy <= T::max_cy, "forward window within the staging capacity");
        REQUIRE(w.cx0 + w.ncx <= g.gx && w.cy0 + w.ncy <= g.gy, "forward window inside the grid");
        // planes read: tiles z0/dz .. (z1-1)/dz, each with its 3 successors
        REQUIRE((z1 - 1) / g.dz + 3 < g.gz, "forward planes inside the grid");
        if (bz == 0 && by == 0)  // the staging map depends on the column window only through cx0, ncx
          for (int tid = 0; tid < T::threads; ++tid) {
            const FwdStage<C, T> m = fwd_stage_map<C, T>(g, w.cx0, w.ncx, w.cy0, w.ncy, tid);
            for (int k = 0; k < fwd_loads<C, T>(); ++k)
              REQUIRE(m.goff[k] < 0 || (size_t)m.goff[k] < cplane, "staged load outside its control plane");
          }
      }
  return true;
}

// The span forward: every span's control window and LDS request.
template <int C>
bool check_forward_span(const VolGeom& g, Check& ck) {
  const int R = span_rows(g, C);
  if (R == 0) return true;  // the span kernel is not used for this geometry
  REQUIRE((double)R * g.nx * C * 4 < 2147483648.0, "span bytes fit the buffer record");
  REQUIRE((g.nx - 1) / g.dx + 3 < g.gx, "span columns inside the grid");
  const int nyb = (g.ny + R - 1) / R;
  for (int yb = 0; yb < nyb; ++yb) {
    const int y0 = yb * R, y1 = imin(g.ny, y0 + R);
    REQUIRE(y0 < y1, "span rows inside the volume");
    for (int z = 0; z < g.nz; ++z) {
      const FwdSpanWindow w = fwd_span_window(g, z, y0, y1);
      REQUIRE(w.tz + 3 < g.gz, "span planes inside the grid");
      REQUIRE(w.ty0 + w.nry <= g.gy, "span control rows inside the grid");
      REQUIRE(w.nry <= fwd_span_ctl_rows(R, g.dy), "span window within its LDS request");
      REQUIRE((size_t)(w.nry + (y1 - y0)) * g.gx * C * sizeof(float) <= fwd_span_lds(R, g.dy, g.gx, C),
              "span LDS use within the request");
    }
  }
  return true;
}

// The batched forward's shapes and z-split targets (the schedule knobs).
bool check_forward_batched(const VolGeom& g, Check& ck) {
  for (long target : {512L, 2048L, 8192L})
    if (!(check_forward_march<3, FwdTile<4, 1, 1>>(g, ck, target) &&
          check_forward_march<3, FwdTile<2, 2, 1>>(g, ck, target) &&
          check_forward_march<3, FwdTile<8, 1, 1>>(g, ck, target)))
      return false;
  return true;
}

bool check_forward(const VolGeom& g, Check& ck) {
  return check_forward_march<3, FwdTileDefault>(g, ck) && check_forward_march<3, FwdTile<2, 8, 1>>(g, ck) &&
         check_forward_march<1, FwdTile<kFwdRows, 1, 4>>(g, ck) && check_forward_march<1, FwdTileDefault>(g, ck) &&
         check_forward_span<3>(g, ck) && check_forward_span<1>(g, ck) && check_forward_batched(g, ck);
}

// The z-first adjoint of the real-spacing grid (general.hip): its bricks,
// LDS request, table reads, partial offsets and pass-2 spans, with host
// tables built by the same exact window-start function the device uses.
bool check_general_adjoint(const GenGeom& q, Check& ck) {
  const GenAxis* ax[3] = {&q.x, &q.y, &q.z};
  std::vector<int> tile[3], first[3];
  for (int i = 0; i < 3; ++i) {
    const GenAxis& A = *ax[i];
    tile[i].resize((size_t)A.n);
    for (int v = 0; v < A.n; ++v) tile[i][(size_t)v] = gen_tile(A, v);
    REQUIRE(tile[i][0] == 0 && tile[i][(size_t)A.n - 1] == A.g - 4, "window starts span the grid");
    for (int v = 1; v < A.n; ++v) {
      const int d = tile[i][(size_t)v] - tile[i][(size_t)v - 1];
      REQUIRE(d == 0 || d == 1, "window starts step by 0 or 1 (spacing >= 1)");
    }
    first[i].resize((size_t)A.g + 1);
    for (int t = 0; t <= A.g; ++t) {
      int lo = 0, hi = A.n;
      while (lo < hi) {
        const int mid = (lo + hi) / 2;
        if (tile[i][(size_t)mid] < t) lo = mid + 1;
        else hi = mid;
      }
      first[i][(size_t)t] = lo;
    }
  }
  GzTables T;
  for (int i = 0; i < 3; ++i) {
    T.tile[i] = tile[i].data();
    T.w[i] = nullptr;
    T.first[i] = first[i].data();
  }
  const GenAdj a = make_gen_adj(q);
  const GzLayout L = gz_layout(a);
  REQUIRE((size_t)L.total * sizeof(float) <= 65536, "pass-1 LDS request within 64 KB");
  REQUIRE(a.kz >= 1 && a.nbz * a.kz >= q.z.g - 3 && (a.nbz - 1) * a.kz < q.z.g - 3, "z-bricks cover the z-tiles");
  const bool xtiles = a.cmx - 3 <= kAdjTiles;
  const long nbricks = (long)a.nbx * a.nby * a.nbz;
  REQUIRE(nbricks < (1L << 31), "pass-1 grid");
  std::vector<int> last((size_t)a.nbz);
  for (long id = 0; id < nbricks; ++id) {
    const GzBrick b = gz_brick(q, a, T, (int)id);
    REQUIRE(b.x0 < b.xe && b.xe - b.x0 <= kGzBX && b.y0 < b.ye && b.ye - b.y0 <= kGzBY, "brick inside the volume");
    REQUIRE(b.z0 < b.ze && b.ze <= q.z.n, "brick planes inside the volume");
    REQUIRE(b.Cx <= a.cmx && b.Cy <= a.cmy, "window within the partials' extents");
    REQUIRE(b.Cx + 4 <= kGzThreads && b.Cy + 4 <= kGzThreads, "table fill within the workgroup");
    REQUIRE(b.cx0 + b.Cx <= q.x.g && b.cy0 + b.Cy <= q.y.g, "first-voxel reads within the tables");
    REQUIRE(!xtiles || b.Cx - 3 <= kAdjTiles, "x-tiles within one row of tile lanes");
    REQUIRE(b.Cy - 3 <= kAdjTiles, "y-tiles within one row of tile lanes");
    const int tl = tile[2][(size_t)b.ze - 1];
    REQUIRE(tl - b.cz0 >= 0 && tl - b.cz0 + 3 < a.cmz, "the brick's last control plane within its window");
    if (a.stage_all) REQUIRE((tl - b.cz0 + 4) * a.cmy * a.cmx * 3 <= kGzStage, "staged partials within the stage");
    last[(size_t)(id / ((long)a.nbx * a.nby))] = tl;
  }
  // pass 2: every brick a control point reads holds it in its window
  for (int c = 0; c < q.x.g; ++c) {
    const GzSpan sp = gz_span(T.first[0], c, kGzBX);
    REQUIRE(0 <= sp.lo && sp.lo <= sp.hi && sp.hi < a.nbx, "x span");
    for (int bx = sp.lo; bx <= sp.hi; ++bx) {
      const GzBrick b = gz_brick(q, a, T, bx);
      REQUIRE(c - b.cx0 >= 0 && c - b.cx0 < b.Cx, "pass 2 reads an x column outside the brick's window");
    }
  }
  for (int c = 0; c < q.y.g; ++c) {
    const GzSpan sp = gz_span(T.first[1], c, kGzBY);
    REQUIRE(0 <= sp.lo && sp.lo <= sp.hi && sp.hi < a.nby, "y span");
    for (int by = sp.lo; by <= sp.hi; ++by) {
      const GzBrick b = gz_brick(q, a, T, by * a.nbx);
      REQUIRE(c - b.cy0 >= 0 && c - b.cy0 < b.Cy, "pass 2 reads a y row outside the brick's window");
    }
  }
  for (int c = 0; c < q.z.g; ++c) {
    const GzSpan sp = gz_span_z(a, c, q.z.g);
    REQUIRE(0 <= sp.lo && sp.lo <= sp.hi && sp.hi < a.nbz, "z span");
    for (int bz = sp.lo; bz <= sp.hi; ++bz) {
      const int czl = c - bz * a.kz;
      REQUIRE(czl >= 0 && czl <= last[(size_t)bz] - bz * a.kz + 3, "pass 2 reads a control plane the brick did not emit");
    }
  }
  const long nblk = (long)((q.x.g + kWave - 1) / kWave) * ((q.y.g + 3) / 4) * q.z.g;
  REQUIRE(nblk < (1L << 31), "pass-2 grid");
  return true;
}

}  // namespace
}  // namespace bsi

using namespace bsi;

extern "C" {

// 0: every check passed; 1: a check failed (message in msg); -1: invalid geometry.
int bsi_check_indices(const int32_t dims[3], const int32_t spacing[3], char* msg, int msglen) {
  VolGeom g;
  if (make_geom(dims, spacing, &g)) {
    std::snprintf(msg, msglen, "invalid geometry");
    return -1;
  }
  Check ck;
  check_adjoints(g, ck) && check_forward(g, ck);
  std::snprintf(msg, msglen, "%s", ck.msg.c_str());
  return ck.ok ? 0 : 1;
}

// 0: every check of the real-spacing adjoint passed; 1: one failed; -1: invalid geometry.
int bsi_check_general_indices(const int32_t dims[3], const float spacing[3], const float origin[3], char* msg,
                              int msglen) {
  GenGeom q;
  VolGeom g;
  if (make_gen_geom(dims, spacing, origin, &q, &g)) {
    std::snprintf(msg, msglen, "invalid geometry");
    return -1;
  }
  Check ck;
  check_general_adjoint(q, ck);
  std::snprintf(msg, msglen, "%s", ck.msg.c_str());
  return ck.ok ? 0 : 1;
}

// The batched kernels' item loops (batch_items): over several totals and
// grids, one workgroup per item and persistent, every item is taken exactly
// once and every workgroup's loop ends within ceil(total / grid) passes.
int bsi_check_batch_items(char* msg, int msglen) {
  Check ck;
  auto run = [&](int64_t total, int grid, bool persistent) -> bool {
    std::vector<int> hit((size_t)total, 0);
    const int64_t max_pass = (total + grid - 1) / grid;
    for (int b = 0; b < grid; ++b) {
      int64_t passes = 0;
      for (ItemRange r = batch_items(b, grid, total, persistent); r.first < total; r.first += r.step) {
        REQUIRE(r.first >= 0, "item below zero");
        REQUIRE(++passes <= max_pass, "a workgroup's item loop does not end");
        ++hit[(size_t)r.first];
      }
    }
    for (int h : hit) REQUIRE(h == 1, "an item taken other than once");
    return true;
  };
  for (int64_t total : {1L, 2L, 7L, 8L, 9L, 100L, 1000L, 4097L, 20000L}) {
    if (!run(total, (int)total, false)) break;
    for (int grid : {1, 3, 8, 256, 512, 1024})
      if (grid <= total && !run(total, grid, true)) break;
    if (!ck.ok) break;
  }
  std::snprintf(msg, msglen, "%s", ck.msg.c_str());
  return ck.ok ? 0 : 1;
}

}  // extern "C"
