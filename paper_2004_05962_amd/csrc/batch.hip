// Batched forward + adjoint BSI over many volumes of different sizes and
// spacings, in persistent launches that can be captured into one HIP graph.
//
// The plan holds a device descriptor table (geometry, buffers and the first
// global work-item index of every volume for each pass).  Each persistent
// workgroup walks a static slice of the concatenated work list and runs the
// same per-wave / per-brick / per-point routines as the single-volume kernels,
// so every volume's output is bit-identical to bsi_forward / bsi_adjoint.
// The schedule (forward workgroup shape and z split, persistent grid sizes of
// each pass, how many streams the pass-1 classes spread over, whether the
// forward runs beside the adjoint) is chosen by timing and never changes the
// arithmetic.
//
// Graph shape: the forward (grid -> field) and the adjoint (dfield -> grad) are
// independent, so they run as parallel branches (fork/join with events); the
// adjoint's pass-1 launches, one per x-spacing class, are spread over several
// streams as well, so that their tails overlap, and join before pass 2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <unistd.h>
#include <sstream>
#include <string>
#include <vector>

#include "adjoint_device.h"
#include "bsi_internal.h"

namespace bsi {

struct VolDesc {
  AdjGeom a;  // a.g is the volume geometry
  FwdLaunch f;
  const float* grid;
  float* field;
  const float* dfield;
  float* grad;
  float* part;
  int64_t first[4];  // first global work item of this volume: forward, pass 1 (its class), pass 2,
                     // pass 1 (spacings 4..12 in one launch)
};

enum Pass { kFwd = 0, kAdj1 = 1, kAdj2 = 2, kAdj1Tiles = 3 };
constexpr int kNumClasses = kAdjMaxDX + 1;  // class dx for dx <= kAdjMaxDX, class 0 otherwise
constexpr int kTilesLo = 4;                  // classes kTilesLo..kAdjMaxDX: the tile-lane spacings
inline int dx_class(int dx) { return dx <= kAdjMaxDX ? dx : 0; }
constexpr int kPtThreads = kGatherThreads;  // pass 2's workgroup
constexpr int kClassStreams = 3;  // pass-1 class launches run on the caller's stream and these

// ---- schedule knobs: each a small table of values, none changes a result bit
enum Knob {
  kKFwdShape, kKFwdItems, kKFwdPerCu, kKAdjPerCu, kKPtsPerCu, kKBranches, kKBeside, kKFwdNT, kKAdjOne, kNumKnobs
};
// forward workgroup shapes R x S (R rows of S 64-voxel strips: FwdTile<R, S, 1>)
constexpr int kNumFwdShapes = 3;
static const char* const kFwdShapeName[kNumFwdShapes] = {"4x1", "2x2", "8x1"};
static const int kFwdShapeWidth[kNumFwdShapes] = {64, 128, 64};
static const int kFwdShapeRows[kNumFwdShapes] = {4, 2, 8};
static const int kFwdItems[] = {512, 2048, 8192};  // forward items per volume (the z split aims at this)
static const int kFwdPerCu[] = {0, 2, 4, 8};       // forward workgroups per CU (0: one per item)
static const int kAdjPerCu[] = {0, 1, 2, 3};       // pass-1 workgroups per CU (0: one per brick)
static const int kPtsPerCu[] = {0, 8};             // pass-2 workgroups per CU (0: one per block)
static const int kBranches[] = {1, 2, 4};          // streams the pass-1 classes are spread over
static const int kBeside[] = {1, 0};               // 1: forward beside the adjoint; 0: forward first
static const int kFwdNT[] = {0, 1};                // forward stores: 0 ordinary, 1 non-temporal
static const int kAdjOne[] = {0, 1};               // 1: spacings 4..12 in one pass-1 launch (run-time spacing)
static const int kKnobSize[kNumKnobs] = {kNumFwdShapes, 3, 4, 4, 2, 3, 2, 2, 2};
static const char* const kKnobName[kNumKnobs] = {"fwd_tile",      "fwd_items",     "fwd_wg_per_cu",
                                                 "adj_wg_per_cu", "pts_wg_per_cu", "pass1_streams",
                                                 "fwd_beside",    "fwd_nt_stores", "pass1_one_launch"};
static_assert(kClassStreams + 1 >= 4, "the largest pass1_streams value");

struct BatchConfig {
  int k[kNumKnobs];  // value index of each knob
};
// The starting point of the search: 8x1 forward, 512 items per volume, one
// workgroup per item in every pass, pass 1 in one launch for the spacings
// 4..12 and per class for the rest over 4 streams, forward first with
// ordinary stores (among the fastest graphs measured on the 32-volume
// workload).
static const BatchConfig kDefaultConfig = {{2, 0, 0, 0, 0, 2, 1, 0, 1}};

int config_count() {
  int n = 1;
  for (int i = 0; i < kNumKnobs; ++i) n *= kKnobSize[i];
  return n;
}
int encode_config(const BatchConfig& c) {
  int v = 0;
  for (int i = kNumKnobs - 1; i >= 0; --i) v = v * kKnobSize[i] + c.k[i];
  return v;
}
BatchConfig decode_config(int v) {
  BatchConfig c;
  for (int i = 0; i < kNumKnobs; ++i) {
    c.k[i] = v % kKnobSize[i];
    v /= kKnobSize[i];
  }
  return c;
}
std::string describe_config(const BatchConfig& c) {
  std::string out;
  for (int i = 0; i < kNumKnobs; ++i) {
    if (i) out += ' ';
    out += kKnobName[i];
    out += '=';
    switch (i) {
      case kKFwdShape: out += kFwdShapeName[c.k[i]]; break;
      case kKFwdItems: out += std::to_string(kFwdItems[c.k[i]]); break;
      case kKFwdPerCu: out += std::to_string(kFwdPerCu[c.k[i]]); break;
      case kKAdjPerCu: out += std::to_string(kAdjPerCu[c.k[i]]); break;
      case kKPtsPerCu: out += std::to_string(kPtsPerCu[c.k[i]]); break;
      case kKBranches: out += std::to_string(kBranches[c.k[i]]); break;
      case kKBeside: out += std::to_string(kBeside[c.k[i]]); break;
      case kKFwdNT: out += std::to_string(kFwdNT[c.k[i]]); break;
      default: out += std::to_string(kAdjOne[c.k[i]]); break;
    }
  }
  return out;
}

__device__ __forceinline__ int find_volume(const VolDesc* __restrict__ v, int count, int64_t item, int pass) {
  int lo = 0, hi = count - 1;  // last volume whose first item <= item
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (v[mid].first[pass] <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// body(item) for each item of this workgroup (batch_items): a loop over a
// persistent grid; otherwise one test and one call, so that no loop state stays
// live across the body (pass 1's body needs every scalar register it can get:
// with a loop around it, its scalar registers spill to vector registers and
// those to scratch).
template <bool Persistent, class Body>
__device__ __forceinline__ void batch_for_items(int64_t total, Body&& body) {
  const ItemRange r = batch_items(blockIdx.x, gridDim.x, total, Persistent);
  if constexpr (Persistent) {
    for (int64_t item = r.first; item < total; item += r.step) body(item);
  } else {
    if (r.first < total) body(r.first);
  }
}

template <class T, bool NT, bool Persistent>
__global__ __launch_bounds__(T::threads) void batch_fwd_kernel(const VolDesc* __restrict__ vols, int count,
                                                               int64_t total, const float* __restrict__ lut) {
  __shared__ FwdSmem<3, T> sm;
  batch_for_items<Persistent>(total, [&](const int64_t item) {
    const int vi = uniform(find_volume(vols, count, item, kFwd));
    const VolDesc& d = vols[vi];
    const VolGeom g = d.a.g;
    const FwdLaunch L = d.f;
    int id = (int)(item - d.first[kFwd]);
    const int bx = id % L.nbx;
    id /= L.nbx;
    const int by = id % L.nby;
    const int bz = id / L.nby;
    const int z0 = bz * L.zchunk;
    const int z1 = min(g.nz, z0 + L.zchunk);
    fwd_block<3, T, NT, !NT>(as_global(d.grid), as_global(d.field), g, lut, bx * T::width, by * T::rows, z0, z1, sm,
                             threadIdx.x);
  });
}

// Pass 1 over the volumes of one x-spacing class (DX = 1..kAdjMaxDX, or 0 for
// the generic path), each class with its own descriptor sub-table, so every
// launch keeps the register footprint of its own specialisation.
// (DX = kAdjAnyTile: the volumes of every spacing 4..12, item numbering
// first[kAdj1Tiles]; the same bits as each spacing's own kernel.)
template <int DX, bool Persistent>
__global__ __launch_bounds__(kAdjThreads) __attribute__((amdgpu_waves_per_eu(BSI_ADJ_WPE))) void batch_adj1_kernel(
    const VolDesc* __restrict__ vols, int count, int64_t total, const float* __restrict__ lut) {
  __shared__ AdjSmem<DX> sm;
  constexpr int kPass = DX == kAdjAnyTile ? kAdj1Tiles : kAdj1;
  batch_for_items<Persistent>(total, [&](const int64_t item) {
    const int vi = uniform(find_volume(vols, count, item, kPass));
    const VolDesc& d = vols[vi];
    const AdjGeom a = d.a;
    // ordinary loads: with the forward running beside pass 1 in the graph,
    // streaming loads measured 2-5% slower here
    const int brick = (int)(item - d.first[kPass]);
    if (adj_stage_all(a))
      adj_brick<DX, false, true>(as_global(d.dfield), as_global(d.part), a, lut, brick, sm, threadIdx.x);
    else
      adj_brick<DX, false, false>(as_global(d.dfield), as_global(d.part), a, lut, brick, sm, threadIdx.x);
  });
}

template <bool Persistent>
__global__ __launch_bounds__(kPtThreads) void batch_adj2_kernel(const VolDesc* __restrict__ vols, int count,
                                                                 int64_t total) {
  batch_for_items<Persistent>(total, [&](const int64_t item) {
    const int vi = uniform(find_volume(vols, count, item, kAdj2));
    const VolDesc& d = vols[vi];
    const AdjGeom a = d.a;
    adj_gather_block(as_global(d.part), as_global(d.grad), a, (int)(item - d.first[kAdj2]), threadIdx.x);
  });
}

}  // namespace bsi

using namespace bsi;

struct bsi_batch {
  int device = 0;
  int cus = 0;
  int count = 0;
  std::vector<VolDesc> host;  // descriptors (pointers filled by bind)
  std::vector<size_t> part_off;
  int64_t total[3] = {0, 0, 0};
  VolDesc* d_desc = nullptr;
  // Pass 1 runs one launch per x-spacing class (see batch_adj1_kernel): the
  // descriptors again, ordered by class, with pass-1 item indices per class.
  std::vector<VolDesc> cls_host;
  int cls_first[kNumClasses + 1] = {};  // class c holds cls_host[cls_first[c] .. cls_first[c+1])
  int64_t cls_total[kNumClasses] = {};
  int64_t tiles_total = 0;  // pass-1 items of classes kTilesLo.. (first[kAdj1Tiles] numbering)
  VolDesc* d_cls = nullptr;
  float* d_part = nullptr;
  const float* lut = nullptr;
  bool has_fwd = false, has_adj = false;
  BatchConfig cfg = kDefaultConfig;
  int layout_shape = -1, layout_items = -1;  // forward shape and z split the descriptors hold
  std::string key;
  hipStream_t side = nullptr;  // second branch (forward) of run / capture
  hipEvent_t fork = nullptr, join = nullptr;
  hipStream_t cls_side[kClassStreams] = {};  // further branches of adjoint pass 1
  hipEvent_t cls_join[kClassStreams] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

int32_t check_device(const bsi_batch* p) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "querying the current device");
  if (dev != p->device) {
    set_error("the plan belongs to another device than the current one");
    return BSI_ERR_INVALID_ARG;
  }
  return BSI_OK;
}

// Wait until nothing the plan has enqueued is still running: its graph may be
// replaying and its kernels read the descriptor tables, on the caller's streams
// as well as on the plan's own.  A launch on a caller's stream cannot be named
// from here, so the whole device is synchronised.  Called before the graph is
// destroyed or the tables are rewritten (bind, tune, capture, destroy).
int32_t quiesce(bsi_batch* p) {
  const hipError_t e = hipDeviceSynchronize();
  return e == hipSuccess ? BSI_OK : hip_fail(e, "synchronising the plan's device");
}

// Callers quiesce first: an executable graph must not be destroyed while a
// launch of it may still run.
void drop_graph(bsi_batch* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
}

// Workgroups of a pass: one per item, or a persistent grid of per_cu per CU.
// A pass of 2^31 items or more always runs persistent (on the largest grid).
int64_t pass_grid(const bsi_batch* p, int64_t total, int per_cu) {
  int64_t grid = per_cu == 0 ? total : std::min<int64_t>(total, (int64_t)per_cu * p->cus);
  return std::min<int64_t>(grid, 0x7fffffff);
}
bool pass_persistent(int64_t total, int per_cu) { return per_cu > 0 || total > 0x7fffffff; }

template <class T>
void launch_fwd_shape(const bsi_batch* p, int64_t total, int per_cu, bool nt, hipStream_t s) {
  const dim3 gd((unsigned)pass_grid(p, total, per_cu)), bd(T::threads);
  const bool pers = pass_persistent(total, per_cu);
  if (!pers && !nt)
    hipLaunchKernelGGL((batch_fwd_kernel<T, false, false>), gd, bd, 0, s, p->d_desc, p->count, total, p->lut);
  else if (!pers)
    hipLaunchKernelGGL((batch_fwd_kernel<T, true, false>), gd, bd, 0, s, p->d_desc, p->count, total, p->lut);
  else if (!nt)
    hipLaunchKernelGGL((batch_fwd_kernel<T, false, true>), gd, bd, 0, s, p->d_desc, p->count, total, p->lut);
  else
    hipLaunchKernelGGL((batch_fwd_kernel<T, true, true>), gd, bd, 0, s, p->d_desc, p->count, total, p->lut);
}

hipError_t launch_pass(bsi_batch* p, int pass, hipStream_t s) {
  const int64_t total = p->total[pass];
  if (total == 0) return hipSuccess;
  if (pass == kFwd) {
    const int per_cu = kFwdPerCu[p->cfg.k[kKFwdPerCu]];
    const bool nt = kFwdNT[p->cfg.k[kKFwdNT]] != 0;
    static_assert(kNumFwdShapes == 3, "one case per forward shape");
    switch (p->cfg.k[kKFwdShape]) {
      case 0: launch_fwd_shape<FwdTile<4, 1, 1>>(p, total, per_cu, nt, s); break;
      case 1: launch_fwd_shape<FwdTile<2, 2, 1>>(p, total, per_cu, nt, s); break;
      default: launch_fwd_shape<FwdTile<8, 1, 1>>(p, total, per_cu, nt, s); break;
    }
  } else if (pass == kAdj1) {
    return hipErrorInvalidValue;  // pass 1 is launched per class (launch_adj1_class)
  } else {
    const int per_cu = kPtsPerCu[p->cfg.k[kKPtsPerCu]];
    const dim3 gd((unsigned)pass_grid(p, total, per_cu)), bd(kPtThreads);
    if (!pass_persistent(total, per_cu))
      hipLaunchKernelGGL(batch_adj2_kernel<false>, gd, bd, 0, s, p->d_desc, p->count, total);
    else
      hipLaunchKernelGGL(batch_adj2_kernel<true>, gd, bd, 0, s, p->d_desc, p->count, total);
  }
  return hipGetLastError();
}

template <int DX>
void launch_adj1_dx(const bsi_batch* p, const VolDesc* v, int n, int64_t ct, int per_cu, hipStream_t s) {
  const dim3 gd((unsigned)pass_grid(p, ct, per_cu)), bd(kAdjThreads);
  if (!pass_persistent(ct, per_cu))
    hipLaunchKernelGGL((batch_adj1_kernel<DX, false>), gd, bd, 0, s, v, n, ct, p->lut);
  else
    hipLaunchKernelGGL((batch_adj1_kernel<DX, true>), gd, bd, 0, s, v, n, ct, p->lut);
}

// Adjoint pass 1 over the volumes of x-spacing class c, on stream s.
hipError_t launch_adj1_class(bsi_batch* p, int c, hipStream_t s) {
  const int n = p->cls_first[c + 1] - p->cls_first[c];
  const int64_t ct = p->cls_total[c];
  if (n == 0 || ct == 0) return hipSuccess;
  const int per_cu = kAdjPerCu[p->cfg.k[kKAdjPerCu]];
  const VolDesc* v = p->d_cls + p->cls_first[c];
  static_assert(kAdjMaxDX == 12, "one case per specialised spacing");
  switch (c) {
    case 1: launch_adj1_dx<1>(p, v, n, ct, per_cu, s); break;
    case 2: launch_adj1_dx<2>(p, v, n, ct, per_cu, s); break;
    case 3: launch_adj1_dx<3>(p, v, n, ct, per_cu, s); break;
    case 4: launch_adj1_dx<4>(p, v, n, ct, per_cu, s); break;
    case 5: launch_adj1_dx<5>(p, v, n, ct, per_cu, s); break;
    case 6: launch_adj1_dx<6>(p, v, n, ct, per_cu, s); break;
    case 7: launch_adj1_dx<7>(p, v, n, ct, per_cu, s); break;
    case 8: launch_adj1_dx<8>(p, v, n, ct, per_cu, s); break;
    case 9: launch_adj1_dx<9>(p, v, n, ct, per_cu, s); break;
    case 10: launch_adj1_dx<10>(p, v, n, ct, per_cu, s); break;
    case 11: launch_adj1_dx<11>(p, v, n, ct, per_cu, s); break;
    case 12: launch_adj1_dx<12>(p, v, n, ct, per_cu, s); break;
    default: launch_adj1_dx<0>(p, v, n, ct, per_cu, s); break;
  }
  return hipGetLastError();
}

// Adjoint pass 1 (every class) then pass 2, on `s`.  Classes go round-robin
// over `s` and the plan's class streams, largest first; each class stream
// waits for p->fork, which the caller has recorded on `s`, and is joined back
// into `s` before pass 2.
int32_t enqueue_adjoint(bsi_batch* p, hipStream_t s) {
  hipError_t e;
  // launches: one per class, or (pass1_one_launch) classes kTilesLo.. as one
  // launch (index kNumClasses) and the others on their own
  const bool one = kAdjOne[p->cfg.k[kKAdjOne]] != 0;
  int64_t size[kNumClasses + 1] = {};
  int order[kNumClasses + 1];
  int used = 0;
  for (int c = 0; c < kNumClasses; ++c)
    if (p->cls_total[c] > 0 && !(one && c >= kTilesLo)) {
      size[c] = p->cls_total[c];
      order[used++] = c;
    }
  if (one && p->tiles_total > 0) {
    size[kNumClasses] = p->tiles_total;
    order[used++] = kNumClasses;
  }
  std::stable_sort(order, order + used, [&size](int a, int b) { return size[a] > size[b]; });
  const int branches = std::min(used, kBranches[p->cfg.k[kKBranches]]);
  for (int j = 0; j + 1 < branches; ++j)
    if ((e = hipStreamWaitEvent(p->cls_side[j], p->fork, 0)) != hipSuccess) return hip_fail(e, "forking pass 1");
  for (int k = 0; k < used; ++k) {
    const int b = k % branches;
    hipStream_t st = b == 0 ? s : p->cls_side[b - 1];
    if (order[k] == kNumClasses) {
      const int n = p->cls_first[kNumClasses] - p->cls_first[kTilesLo];
      launch_adj1_dx<kAdjAnyTile>(p, p->d_cls + p->cls_first[kTilesLo], n, p->tiles_total,
                                  kAdjPerCu[p->cfg.k[kKAdjPerCu]], st);
      e = hipGetLastError();
    } else {
      e = launch_adj1_class(p, order[k], st);
    }
    if (e != hipSuccess) return hip_fail(e, "launching batched adjoint pass 1");
  }
  for (int j = 0; j + 1 < branches; ++j) {
    if ((e = hipEventRecord(p->cls_join[j], p->cls_side[j])) != hipSuccess) return hip_fail(e, "recording a pass-1 join");
    if ((e = hipStreamWaitEvent(s, p->cls_join[j], 0)) != hipSuccess) return hip_fail(e, "joining pass 1");
  }
  if ((e = launch_pass(p, kAdj2, s)) != hipSuccess) return hip_fail(e, "launching batched adjoint pass 2");
  return BSI_OK;
}

// Forward and adjoint on `s`: with fwd_beside the forward runs on the side
// stream beside the adjoint and is joined back into `s`, otherwise first.
int32_t enqueue(bsi_batch* p, hipStream_t s) {
  hipError_t e;
  const bool beside = p->has_fwd && p->has_adj && kBeside[p->cfg.k[kKBeside]];
  if (p->has_fwd && !beside && (e = launch_pass(p, kFwd, s)) != hipSuccess)
    return hip_fail(e, "launching the batched forward");
  if (p->has_adj && (e = hipEventRecord(p->fork, s)) != hipSuccess) return hip_fail(e, "recording the fork event");
  if (beside) {
    if ((e = hipStreamWaitEvent(p->side, p->fork, 0)) != hipSuccess) return hip_fail(e, "forking");
    if ((e = launch_pass(p, kFwd, p->side)) != hipSuccess) return hip_fail(e, "launching the batched forward");
  }
  if (p->has_adj) {
    const int32_t rc = enqueue_adjoint(p, s);
    if (rc) return rc;
  }
  if (beside) {
    if ((e = hipEventRecord(p->join, p->side)) != hipSuccess) return hip_fail(e, "recording the join event");
    if ((e = hipStreamWaitEvent(s, p->join, 0)) != hipSuccess) return hip_fail(e, "joining");
  }
  return BSI_OK;
}

// The forward's work items for the plan's forward shape and z split (host
// descriptors only); true when they changed.
bool layout_forward(bsi_batch* p) {
  const int sh = p->cfg.k[kKFwdShape], it = p->cfg.k[kKFwdItems];
  if (sh == p->layout_shape && it == p->layout_items) return false;
  int64_t tot = 0;
  for (VolDesc& d : p->host) {
    d.f = make_fwd_launch(d.a.g, kFwdItems[it], kFwdShapeWidth[sh], kFwdShapeRows[sh]);
    d.first[kFwd] = tot;
    tot += (int64_t)d.f.nbx * d.f.nby * d.f.nbz;
  }
  p->total[kFwd] = tot;
  p->layout_shape = sh;
  p->layout_items = it;
  return true;
}

int32_t upload_tables(bsi_batch* p) {
  hipError_t e = hipMemcpy(p->d_desc, p->host.data(), sizeof(VolDesc) * p->host.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "uploading the descriptor table");
  e = hipMemcpy(p->d_cls, p->cls_host.data(), sizeof(VolDesc) * p->cls_host.size(), hipMemcpyHostToDevice);
  return e == hipSuccess ? BSI_OK : hip_fail(e, "uploading the class descriptor table");
}

// Switch the plan to configuration c.  Callers quiesce first: the forward's
// descriptors may be rewritten.  Drops a captured graph.
int32_t set_config(bsi_batch* p, const BatchConfig& c) {
  p->cfg = c;
  drop_graph(p);
  if (layout_forward(p) && (p->has_fwd || p->has_adj)) return upload_tables(p);
  return BSI_OK;
}

// Capture enqueue() on `stream` into the plan's graph and instantiate it.
int32_t build_graph(bsi_batch* p, hipStream_t stream) {
  drop_graph(p);
  hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "beginning stream capture");
  int32_t rc = enqueue(p, stream);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "ending stream capture");
  p->graph = g;
  e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(p);
    return hip_fail(e, "instantiating the graph");
  }
  return BSI_OK;
}

// ---- persisted tuning choice: a flat JSON object {"<key>": <index>, ...}
std::string read_file(const char* path) {
  std::ifstream f(path);
  if (!f) return std::string();
  std::stringstream ss;
  ss << f.rdbuf();
  return ss.str();
}

int cache_lookup(const char* path, const std::string& key) {
  const std::string text = read_file(path);
  const std::string pat = "\"" + key + "\":";
  const size_t at = text.find(pat);
  if (at == std::string::npos) return -1;
  return std::atoi(text.c_str() + at + pat.size());
}

void cache_store(const char* path, const std::string& key, int value) {
  std::string text = read_file(path);
  std::vector<std::pair<std::string, int>> entries;
  size_t pos = 0;
  while ((pos = text.find('"', pos)) != std::string::npos) {
    const size_t end = text.find('"', pos + 1);
    if (end == std::string::npos) break;
    const std::string k = text.substr(pos + 1, end - pos - 1);
    const size_t colon = text.find(':', end);
    if (colon == std::string::npos) break;
    entries.emplace_back(k, std::atoi(text.c_str() + colon + 1));
    pos = colon + 1;
  }
  bool found = false;
  for (auto& kv : entries)
    if (kv.first == key) {
      kv.second = value;
      found = true;
    }
  if (!found) entries.emplace_back(key, value);
  // a temporary file of this process and call, renamed over the cache: two
  // processes tuning at once each replace the file whole (the last one wins)
  static int serial = 0;
  const std::string tmp = std::string(path) + ".tmp." + std::to_string((long)getpid()) + "." +
                          std::to_string(++serial);
  {
    std::ofstream f(tmp);
    f << "{\n";
    for (size_t i = 0; i < entries.size(); ++i)
      f << "  \"" << entries[i].first << "\": " << entries[i].second << (i + 1 < entries.size() ? ",\n" : "\n");
    f << "}\n";
  }
  std::rename(tmp.c_str(), path);
}

// A configuration index in [0, config_count()), written as a plain decimal number.
bool parse_config(const char* text, int* out) {
  char* end = nullptr;
  const long v = std::strtol(text, &end, 10);
  if (end == text || *end != '\0' || v < 0 || v >= config_count()) return false;
  *out = (int)v;
  return true;
}

std::string plan_key(const bsi_batch* p) {
  // FNV-1a over the geometry list, prefixed by the architecture and CU count
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](int32_t v) {
    for (int b = 0; b < 4; ++b) {
      h ^= (uint8_t)(v >> (8 * b));
      h *= 1099511628211ull;
    }
  };
  mix(p->count);
  for (const VolDesc& d : p->host) {
    mix(d.a.g.nx); mix(d.a.g.ny); mix(d.a.g.nz);
    mix(d.a.g.dx); mix(d.a.g.dy); mix(d.a.g.dz);
  }
  char buf[64];
  // "k3": the knob tables of this version (an index means another schedule under other tables)
  std::snprintf(buf, sizeof(buf), "k3-gfx950-cu%d-%016llx", p->cus, (unsigned long long)h);
  return buf;
}

}  // namespace

extern "C" {

int32_t bsi_batch_create(int32_t count, const int32_t* dims3xN, const int32_t* spacing3xN, bsi_batch** out) {
  clear_error();
  if (!out || !dims3xN || !spacing3xN || count < 1) {
    set_error("bsi_batch_create needs count >= 1 and non-null arrays");
    return BSI_ERR_INVALID_ARG;
  }
  *out = nullptr;
  std::vector<VolDesc> host((size_t)count);
  std::vector<size_t> off((size_t)count);
  size_t part_floats = 0;
  int64_t tot[3] = {0, 0, 0};
  std::vector<VolGeom> geoms((size_t)count);
  for (int i = 0; i < count; ++i) {
    int32_t rc = make_geom(dims3xN + 3 * i, spacing3xN + 3 * i, &geoms[i]);
    if (rc) {
      set_error("volume " + std::to_string(i) + ": " + bsi_last_error());
      return rc;
    }
    if (adj_gather_blocks(geoms[i]) >= ((int64_t)1 << 31)) {  // a field far beyond device memory
      set_error("volume " + std::to_string(i) + ": too many control points");
      return BSI_ERR_UNSUPPORTED;
    }
  }
  for (int i = 0; i < count; ++i) {
    const VolGeom& g = geoms[i];
    VolDesc& d = host[i];
    std::memset(&d, 0, sizeof(d));
    d.a = make_adj_geom(g);  // the forward's items are laid out by layout_forward
    off[i] = part_floats;
    part_floats += adj_workspace_bytes(d.a) / sizeof(float);
    d.first[kAdj1] = tot[kAdj1];
    d.first[kAdj2] = tot[kAdj2];
    tot[kAdj1] += (int64_t)d.a.x.nb * d.a.y.nb * d.a.z.nb;
    tot[kAdj2] += adj_gather_blocks(g);
  }
  int dev = 0;
  int32_t rc = current_device(&dev);
  if (rc) return rc;
  const float* lut = nullptr;
  if ((rc = lut_device_ptr(dev, &lut))) return rc;

  bsi_batch* p = new bsi_batch();
  p->device = dev;
  p->count = count;
  p->host = std::move(host);
  p->part_off = std::move(off);
  for (int k = 0; k < 3; ++k) p->total[k] = tot[k];
  p->lut = lut;
  hipError_t e = hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "querying the CU count");
  }
  if (hipMalloc(&p->d_desc, sizeof(VolDesc) * (size_t)count) != hipSuccess ||
      hipMalloc(&p->d_part, sizeof(float) * std::max<size_t>(part_floats, 1)) != hipSuccess) {
    (void)hipGetLastError();
    bsi_batch_destroy(p);
    set_error("out of device memory for the batched plan");
    return BSI_ERR_NOMEM;
  }
  for (int i = 0; i < count; ++i) p->host[i].part = p->d_part + p->part_off[i];
  // class-ordered copy for pass 1, with item indices restarting per class
  for (int c = 0; c < kNumClasses; ++c) {
    p->cls_first[c] = (int)p->cls_host.size();
    for (int i = 0; i < count; ++i) {
      if (dx_class(p->host[i].a.g.dx) != c) continue;
      VolDesc d = p->host[i];
      d.first[kAdj1] = p->cls_total[c];
      p->cls_total[c] += (int64_t)d.a.x.nb * d.a.y.nb * d.a.z.nb;
      p->cls_host.push_back(d);
    }
  }
  p->cls_first[kNumClasses] = (int)p->cls_host.size();
  for (int i = p->cls_first[kTilesLo]; i < p->cls_first[kNumClasses]; ++i) {  // class order
    VolDesc& d = p->cls_host[(size_t)i];
    d.first[kAdj1Tiles] = p->tiles_total;
    p->tiles_total += (int64_t)d.a.x.nb * d.a.y.nb * d.a.z.nb;
  }

  if (hipMalloc(&p->d_cls, sizeof(VolDesc) * (size_t)count) != hipSuccess) {
    (void)hipGetLastError();
    bsi_batch_destroy(p);
    set_error("out of device memory for the batched plan");
    return BSI_ERR_NOMEM;
  }
  if ((e = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&p->join, hipEventDisableTiming)) != hipSuccess) {
    bsi_batch_destroy(p);
    return hip_fail(e, "creating the plan's stream and events");
  }
  for (int j = 0; j < kClassStreams; ++j)
    if ((e = hipStreamCreateWithFlags(&p->cls_side[j], hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&p->cls_join[j], hipEventDisableTiming)) != hipSuccess) {
      bsi_batch_destroy(p);
      return hip_fail(e, "creating the plan's pass-1 streams and events");
    }
  p->key = plan_key(p);
  if (const char* force = std::getenv("BSI_FORCE_CONFIG")) {
    int v = -1;
    if (!parse_config(force, &v)) {
      bsi_batch_destroy(p);
      set_error(std::string("BSI_FORCE_CONFIG=") + force + " is not a configuration index in [0, " +
                std::to_string(config_count()) + ")");
      return BSI_ERR_INVALID_ARG;
    }
    p->cfg = decode_config(v);
  } else if (const char* path = std::getenv("BSI_TUNE_CACHE")) {
    const int v = cache_lookup(path, p->key);
    if (v >= 0 && v < config_count()) p->cfg = decode_config(v);
  }
  layout_forward(p);  // nothing is bound yet: the tables are uploaded by bind
  *out = p;
  return BSI_OK;
}

int32_t bsi_batch_bind(bsi_batch* p, const float* const* grids, float* const* fields,
                       const float* const* dfields, float* const* grid_grads) {
  clear_error();
  if (!p) {
    set_error("plan must be non-null");
    return BSI_ERR_INVALID_ARG;
  }
  if ((grids == nullptr) != (fields == nullptr) || (dfields == nullptr) != (grid_grads == nullptr)) {
    set_error("grids/fields and dfields/grid_grads must be given in pairs");
    return BSI_ERR_INVALID_ARG;
  }
  for (int i = 0; i < p->count; ++i) {
    if ((grids && (!grids[i] || !fields[i])) || (dfields && (!dfields[i] || !grid_grads[i]))) {
      set_error("volume " + std::to_string(i) + ": null buffer pointer");
      return BSI_ERR_INVALID_ARG;
    }
  }
  int32_t rc = check_device(p);
  if (rc) return rc;
  if ((rc = quiesce(p))) return rc;
  for (int i = 0; i < p->count; ++i) {
    VolDesc& d = p->host[i];
    d.grid = grids ? grids[i] : nullptr;
    d.field = grids ? fields[i] : nullptr;
    d.dfield = dfields ? dfields[i] : nullptr;
    d.grad = dfields ? grid_grads[i] : nullptr;
  }
  p->has_fwd = grids != nullptr;
  p->has_adj = dfields != nullptr;
  for (VolDesc& c : p->cls_host) {  // same buffers in the class-ordered copy
    for (int i = 0; i < p->count; ++i)
      if (p->host[i].part == c.part) {
        c.grid = p->host[i].grid;
        c.field = p->host[i].field;
        c.dfield = p->host[i].dfield;
        c.grad = p->host[i].grad;
      }
  }
  drop_graph(p);
  return upload_tables(p);
}

int32_t bsi_batch_config(const bsi_batch* p, int32_t* index, int32_t* count) {
  clear_error();
  if (!p || !index || !count) {
    set_error("null argument");
    return BSI_ERR_INVALID_ARG;
  }
  *index = encode_config(p->cfg);
  *count = config_count();
  return BSI_OK;
}

int32_t bsi_batch_describe(const bsi_batch* p, char* buf, int32_t len) {
  clear_error();
  if (!p || !buf || len < 1) {
    set_error("null argument or empty buffer");
    return BSI_ERR_INVALID_ARG;
  }
  std::snprintf(buf, (size_t)len, "%s", describe_config(p->cfg).c_str());
  return BSI_OK;
}

int32_t bsi_batch_run(bsi_batch* p, hipStream_t stream) {
  clear_error();
  if (!p || (!p->has_fwd && !p->has_adj)) {
    set_error("plan is null or has no bound buffers");
    return BSI_ERR_INVALID_ARG;
  }
  int32_t rc = check_device(p);
  if (rc) return rc;
  return enqueue(p, stream);
}

int32_t bsi_batch_run_separate(bsi_batch* p, hipStream_t stream) {
  clear_error();
  if (!p || (!p->has_fwd && !p->has_adj)) {
    set_error("plan is null or has no bound buffers");
    return BSI_ERR_INVALID_ARG;
  }
  int32_t rc = check_device(p);
  if (rc) return rc;
  for (int i = 0; i < p->count; ++i) {
    const VolDesc& d = p->host[i];
    hipError_t e;
    if (p->has_fwd && (e = launch_forward(d.grid, d.field, d.a.g, p->lut, stream)) != hipSuccess)
      return hip_fail(e, "launching a per-volume forward");
    if (p->has_adj && (e = launch_adjoint(d.dfield, d.grad, d.a, p->lut, d.part, stream)) != hipSuccess)
      return hip_fail(e, "launching a per-volume adjoint");
  }
  return BSI_OK;
}

int32_t bsi_batch_tune(bsi_batch* p, hipStream_t stream) {
  clear_error();
  if (!p || (!p->has_fwd && !p->has_adj)) {
    set_error("plan is null or has no bound buffers");
    return BSI_ERR_INVALID_ARG;
  }
  int32_t rc = check_device(p);
  if (rc) return rc;
  if ((rc = quiesce(p))) return rc;
  if (const char* force = std::getenv("BSI_FORCE_CONFIG")) {
    int v = -1;
    if (!parse_config(force, &v)) {
      set_error(std::string("BSI_FORCE_CONFIG=") + force + " is not a configuration index in [0, " +
                std::to_string(config_count()) + ")");
      return BSI_ERR_INVALID_ARG;
    }
    return set_config(p, decode_config(v));
  }
  hipEvent_t t0, t1;
  hipError_t e;
  if ((e = hipEventCreate(&t0)) != hipSuccess) return hip_fail(e, "creating a timing event");
  if ((e = hipEventCreate(&t1)) != hipSuccess) {
    (void)hipEventDestroy(t0);
    return hip_fail(e, "creating a timing event");
  }
  const bool verbose = std::getenv("BSI_TUNE_VERBOSE") != nullptr;
  // Median of 5 timed runs after one warm-up run.  Every run ends with the
  // wait for t1 on `stream`, into which all of the plan's branches join, so
  // the device is idle whenever set_config rewrites the forward's table.
  auto time_config = [&](const BatchConfig& c, float* ms) -> int32_t {
    int32_t r = set_config(p, c);
    if (r) return r;
    if ((r = enqueue(p, stream))) return r;
    float times[5];
    for (int k = 0; k < 5; ++k) {
      if ((e = hipEventRecord(t0, stream)) != hipSuccess) return hip_fail(e, "recording a timing event");
      if ((r = enqueue(p, stream))) return r;
      if ((e = hipEventRecord(t1, stream)) != hipSuccess || (e = hipEventSynchronize(t1)) != hipSuccess ||
          (e = hipEventElapsedTime(&times[k], t0, t1)) != hipSuccess)
        return hip_fail(e, "timing a configuration");
    }
    std::sort(times, times + 5);
    *ms = times[2];
    if (verbose) std::fprintf(stderr, "bsi_batch_tune: %-110s %.4f ms\n", describe_config(c).c_str(), *ms);
    return BSI_OK;
  };
  // Coordinate descent from the plan's configuration (the default, or the
  // cached choice): each knob in turn takes every value with the others held,
  // and keeps the fastest; sweeps repeat until one changes nothing (at most 3).
  // The winner is then timed once more beside the starting point, which it
  // must still beat.
  const BatchConfig start = p->cfg;
  std::vector<std::pair<int, float>> seen;  // configuration index, time
  auto measure = [&](const BatchConfig& c, float* ms) -> int32_t {
    const int id = encode_config(c);
    for (const auto& kv : seen)
      if (kv.first == id) {
        *ms = kv.second;
        return BSI_OK;
      }
    const int32_t r = time_config(c, ms);
    if (r == BSI_OK) seen.emplace_back(id, *ms);
    return r;
  };
  BatchConfig best = start;
  float best_ms = 0.f;
  rc = measure(best, &best_ms);
  for (int sweep = 0; sweep < 3 && rc == BSI_OK; ++sweep) {
    bool changed = false;
    for (int k = 0; k < kNumKnobs && rc == BSI_OK; ++k)
      for (int v = 0; v < kKnobSize[k] && rc == BSI_OK; ++v) {
        if (v == best.k[k]) continue;
        BatchConfig c = best;
        c.k[k] = v;
        float ms = 0.f;
        if ((rc = measure(c, &ms)) == BSI_OK && ms < best_ms) {
          best = c;
          best_ms = ms;
          changed = true;
        }
      }
    if (!changed) break;
  }
  if (rc == BSI_OK && encode_config(best) != encode_config(start)) {
    float again = 0.f, base = 0.f;
    if ((rc = time_config(best, &again)) == BSI_OK && (rc = time_config(start, &base)) == BSI_OK && base <= again)
      best = start;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  const int32_t rc2 = set_config(p, rc == BSI_OK ? best : start);
  if (rc == BSI_OK) rc = rc2;
  if (rc == BSI_OK)
    if (const char* path = std::getenv("BSI_TUNE_CACHE")) cache_store(path, p->key, encode_config(p->cfg));
  return rc;
}

int32_t bsi_batch_capture(bsi_batch* p, hipStream_t stream) {
  clear_error();
  if (!p || (!p->has_fwd && !p->has_adj)) {
    set_error("plan is null or has no bound buffers");
    return BSI_ERR_INVALID_ARG;
  }
  int32_t rc = check_device(p);
  if (rc) return rc;
  if ((rc = quiesce(p))) return rc;
  return build_graph(p, stream);
}

int32_t bsi_batch_launch(bsi_batch* p, hipStream_t stream) {
  clear_error();
  if (!p || !p->exec) {
    set_error("no captured graph: call bsi_batch_capture first");
    return BSI_ERR_INVALID_ARG;
  }
  int32_t rc = check_device(p);
  if (rc) return rc;
  hipError_t e = hipGraphLaunch(p->exec, stream);
  return e == hipSuccess ? BSI_OK : hip_fail(e, "launching the graph");
}

void bsi_batch_destroy(bsi_batch* p) {
  if (!p) return;
  // Teardown is best effort: errors here have nowhere useful to go.
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(p->device);
  (void)hipDeviceSynchronize();
  drop_graph(p);
  if (p->fork) (void)hipEventDestroy(p->fork);
  if (p->join) (void)hipEventDestroy(p->join);
  if (p->side) (void)hipStreamDestroy(p->side);
  for (int j = 0; j < kClassStreams; ++j) {
    if (p->cls_join[j]) (void)hipEventDestroy(p->cls_join[j]);
    if (p->cls_side[j]) (void)hipStreamDestroy(p->cls_side[j]);
  }
  if (p->d_desc) (void)hipFree(p->d_desc);
  if (p->d_cls) (void)hipFree(p->d_cls);
  if (p->d_part) (void)hipFree(p->d_part);
  if (prev >= 0) (void)hipSetDevice(prev);
  delete p;
}

}  // extern "C"
