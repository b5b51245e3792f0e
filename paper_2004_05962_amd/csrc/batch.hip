// Batched forward + adjoint BSI over many volumes of different sizes and
// spacings, in persistent launches that can be captured into one HIP graph.
//
// The plan holds a device descriptor table (geometry, buffers and the first
// global work-item index of every volume for each pass).  Each persistent
// workgroup walks a static slice of the concatenated work list and runs the
// same per-wave / per-brick / per-point routines as the single-volume kernels,
// so every volume's output is bit-identical to bsi_forward / bsi_adjoint.
// Schedules (persistent grid size, slice order) are chosen by timing and never
// change the arithmetic.
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
  int64_t first[3];  // first global work item of this volume: forward, pass 1, pass 2
};

enum Pass { kFwd = 0, kAdj1 = 1, kAdj2 = 2 };
constexpr int kNumClasses = kAdjMaxDX + 1;  // class dx for dx <= kAdjMaxDX, class 0 otherwise
inline int dx_class(int dx) { return dx <= kAdjMaxDX ? dx : 0; }
constexpr int kPtThreads = kGatherThreads;  // pass 2's workgroup
#ifndef BSI_BATCH_FWD_TARGET
#define BSI_BATCH_FWD_TARGET 2048
#endif
constexpr long kBatchFwdTarget = BSI_BATCH_FWD_TARGET;  // forward items per volume (z split)
constexpr int kClassStreams = 3;  // pass-1 class launches run on the caller's stream and these

struct Schedule {
  int fwd_per_cu;  // persistent workgroups per CU (0 = one workgroup per item)
  int adj_per_cu;
  int pts_per_cu;
  int chunked;     // 0: item = wg + k * G;  1: contiguous slices per workgroup
};

// Candidate schedules; index 0 is the non-persistent reference.  (Persistent
// grids of 1-2 workgroups per CU for pass 1, and contiguous slices, measured
// 8-50% slower once the pass-1 classes run concurrently, and are not offered.)
static const Schedule kSchedules[] = {
    {0, 0, 0, 0},
    {4, 2, 8, 0},
};
constexpr int kNumSchedules = sizeof(kSchedules) / sizeof(kSchedules[0]);
constexpr int kDefaultSchedule = 0;

__device__ __forceinline__ int find_volume(const VolDesc* __restrict__ v, int count, int64_t item, int pass) {
  int lo = 0, hi = count - 1;  // last volume whose first item <= item
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (v[mid].first[pass] <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Static slice of [0, total) for this workgroup.
struct Slice {
  int64_t begin, end, step;
};

__device__ __forceinline__ Slice make_slice(int64_t total, int chunked) {
  const int64_t G = gridDim.x;
  const int64_t w = xcd_remap(blockIdx.x, gridDim.x);
  Slice s;
  if (chunked) {
    const int64_t per = (total + G - 1) / G;
    s.begin = w * per;
    s.end = s.begin + per < total ? s.begin + per : total;
    s.step = 1;
  } else {
    s.begin = w;
    s.end = total;
    s.step = G;
  }
  return s;
}

__global__ __launch_bounds__(kFwdThreads) void batch_fwd_kernel(const VolDesc* __restrict__ vols, int count,
                                                                 int64_t total, int chunked,
                                                                 const float* __restrict__ lut) {
  __shared__ FwdSmem<3> sm;
  const Slice s = make_slice(total, chunked);
  for (int64_t item = s.begin; item < s.end; item += s.step) {
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
    // ordinary stores throughout: beside the adjoint classes in the graph they
    // measured faster than non-temporal (1.31-1.36 against 1.35-1.38 ms for
    // the 32-volume graph) and than edge stores
    fwd_block<3, FwdTileDefault, false, true>(d.grid, d.field, g, lut, bx * kWave, by * kFwdRows, z0, z1, sm,
                                              threadIdx.x);
  }
}

// Pass 1 over the volumes of one x-spacing class (DX = 1..kAdjMaxDX, or 0 for
// the generic path), each class with its own descriptor sub-table, so every
// launch keeps the register footprint of its own specialisation.
template <int DX>
__global__ __launch_bounds__(kAdjThreads) __attribute__((amdgpu_waves_per_eu(BSI_ADJ_WPE))) void batch_adj1_kernel(const VolDesc* __restrict__ vols, int count,
                                                                   int64_t total, int chunked,
                                                                   const float* __restrict__ lut) {
  __shared__ AdjSmem<DX> sm;
  const Slice s = make_slice(total, chunked);
  for (int64_t item = s.begin; item < s.end; item += s.step) {
    const int vi = uniform(find_volume(vols, count, item, kAdj1));
    const VolDesc& d = vols[vi];
    const AdjGeom a = d.a;
    // ordinary loads: with the forward running beside pass 1 in the graph,
    // streaming loads measured 2-5% slower here
    const int brick = (int)(item - d.first[kAdj1]);
    if (adj_stage_all(a))
      adj_brick<DX, false, true>(d.dfield, d.part, a, lut, brick, sm, threadIdx.x);
    else
      adj_brick<DX, false, false>(d.dfield, d.part, a, lut, brick, sm, threadIdx.x);
  }
}

__global__ __launch_bounds__(kPtThreads) void batch_adj2_kernel(const VolDesc* __restrict__ vols, int count,
                                                                 int64_t total, int chunked) {
  const Slice s = make_slice(total, chunked);
  for (int64_t item = s.begin; item < s.end; item += s.step) {
    const int vi = uniform(find_volume(vols, count, item, kAdj2));
    const VolDesc& d = vols[vi];
    const AdjGeom a = d.a;
    adj_gather_block(d.part, d.grad, a, (int)(item - d.first[kAdj2]), threadIdx.x);
  }
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
  VolDesc* d_cls = nullptr;
  float* d_part = nullptr;
  const float* lut = nullptr;
  bool has_fwd = false, has_adj = false;
  int schedule = kDefaultSchedule;
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

hipError_t launch_pass(bsi_batch* p, int pass, hipStream_t s) {
  const Schedule& sc = kSchedules[p->schedule];
  const int64_t total = p->total[pass];
  if (total == 0) return hipSuccess;
  const int per_cu = pass == kFwd ? sc.fwd_per_cu : pass == kAdj1 ? sc.adj_per_cu : sc.pts_per_cu;
  int64_t grid = per_cu == 0 ? total : std::min<int64_t>(total, (int64_t)per_cu * p->cus);
  if (grid > 0x7fffffff) grid = 0x7fffffff;
  const int chunked = per_cu == 0 ? 0 : sc.chunked;
  if (pass == kFwd) {
    hipLaunchKernelGGL(batch_fwd_kernel, dim3((unsigned)grid), dim3(kFwdThreads), 0, s, p->d_desc,
                       p->count, total, chunked, p->lut);
  } else if (pass == kAdj1) {
    return hipErrorInvalidValue;  // pass 1 is launched per class (launch_adj1_class)
  } else {
    hipLaunchKernelGGL(batch_adj2_kernel, dim3((unsigned)grid), dim3(kPtThreads), 0, s, p->d_desc, p->count,
                       total, chunked);
  }
  return hipGetLastError();
}

// Adjoint pass 1 over the volumes of x-spacing class c, on stream s.
hipError_t launch_adj1_class(bsi_batch* p, int c, hipStream_t s) {
  const Schedule& sc = kSchedules[p->schedule];
  const int n = p->cls_first[c + 1] - p->cls_first[c];
  const int64_t ct = p->cls_total[c];
  if (n == 0 || ct == 0) return hipSuccess;
  const int per_cu = sc.adj_per_cu;
  const int chunked = per_cu == 0 ? 0 : sc.chunked;
  const int64_t cg = per_cu == 0 ? ct : std::min<int64_t>(ct, (int64_t)per_cu * p->cus);
  const dim3 gd((unsigned)cg), bd(kAdjThreads);
  const VolDesc* v = p->d_cls + p->cls_first[c];
  static_assert(kAdjMaxDX == 12, "one case per specialised spacing");
  switch (c) {
    case 1: hipLaunchKernelGGL(batch_adj1_kernel<1>, gd, bd, 0, s, v, n, ct, chunked, p->lut); break;
    case 2: hipLaunchKernelGGL(batch_adj1_kernel<2>, gd, bd, 0, s, v, n, ct, chunked, p->lut); break;
    case 3: hipLaunchKernelGGL(batch_adj1_kernel<3>, gd, bd, 0, s, v, n, ct, chunked, p->lut); break;
    case 4: hipLaunchKernelGGL(batch_adj1_kernel<4>, gd, bd, 0, s, v, n, ct, chunked, p->lut); break;
    case 5: hipLaunchKernelGGL(batch_adj1_kernel<5>, gd, bd, 0, s, v, n, ct, chunked, p->lut); break;
    case 6: hipLaunchKernelGGL(batch_adj1_kernel<6>, gd, bd, 0, s, v, n, ct, chunked, p->lut); break;
    case 7: hipLaunchKernelGGL(batch_adj1_kernel<7>, gd, bd, 0, s, v, n, ct, chunked, p->lut); break;
    case 8: hipLaunchKernelGGL(batch_adj1_kernel<8>, gd, bd, 0, s, v, n, ct, chunked, p->lut); break;
    case 9: hipLaunchKernelGGL(batch_adj1_kernel<9>, gd, bd, 0, s, v, n, ct, chunked, p->lut); break;
    case 10: hipLaunchKernelGGL(batch_adj1_kernel<10>, gd, bd, 0, s, v, n, ct, chunked, p->lut); break;
    case 11: hipLaunchKernelGGL(batch_adj1_kernel<11>, gd, bd, 0, s, v, n, ct, chunked, p->lut); break;
    case 12: hipLaunchKernelGGL(batch_adj1_kernel<12>, gd, bd, 0, s, v, n, ct, chunked, p->lut); break;
    default: hipLaunchKernelGGL(batch_adj1_kernel<0>, gd, bd, 0, s, v, n, ct, chunked, p->lut); break;
  }
  return hipGetLastError();
}

// Adjoint pass 1 (every class) then pass 2, on `s`.  Classes go round-robin
// over `s` and the plan's class streams, largest first; each class stream
// waits for p->fork, which the caller has recorded on `s`, and is joined back
// into `s` before pass 2.
int32_t enqueue_adjoint(bsi_batch* p, hipStream_t s) {
  hipError_t e;
  int order[kNumClasses];
  int used = 0;
  for (int c = 0; c < kNumClasses; ++c)
    if (p->cls_total[c] > 0) order[used++] = c;
  std::stable_sort(order, order + used, [p](int a, int b) { return p->cls_total[a] > p->cls_total[b]; });
  const int branches = std::min(used, kClassStreams + 1);
  for (int j = 0; j + 1 < branches; ++j)
    if ((e = hipStreamWaitEvent(p->cls_side[j], p->fork, 0)) != hipSuccess) return hip_fail(e, "forking pass 1");
  for (int k = 0; k < used; ++k) {
    const int b = k % branches;
    hipStream_t st = b == 0 ? s : p->cls_side[b - 1];
    if ((e = launch_adj1_class(p, order[k], st)) != hipSuccess) return hip_fail(e, "launching batched adjoint pass 1");
  }
  for (int j = 0; j + 1 < branches; ++j) {
    if ((e = hipEventRecord(p->cls_join[j], p->cls_side[j])) != hipSuccess) return hip_fail(e, "recording a pass-1 join");
    if ((e = hipStreamWaitEvent(s, p->cls_join[j], 0)) != hipSuccess) return hip_fail(e, "joining pass 1");
  }
  if ((e = launch_pass(p, kAdj2, s)) != hipSuccess) return hip_fail(e, "launching batched adjoint pass 2");
  return BSI_OK;
}

// Forward on the side stream, adjoint on `s`, joined back into `s`.
int32_t enqueue(bsi_batch* p, hipStream_t s) {
  hipError_t e;
  if (p->has_adj && (e = hipEventRecord(p->fork, s)) != hipSuccess) return hip_fail(e, "recording the fork event");
  if (p->has_fwd && p->has_adj) {
    if ((e = hipStreamWaitEvent(p->side, p->fork, 0)) != hipSuccess) return hip_fail(e, "forking");
    if ((e = launch_pass(p, kFwd, p->side)) != hipSuccess) return hip_fail(e, "launching the batched forward");
    const int32_t rc = enqueue_adjoint(p, s);
    if (rc) return rc;
    if ((e = hipEventRecord(p->join, p->side)) != hipSuccess) return hip_fail(e, "recording the join event");
    if ((e = hipStreamWaitEvent(s, p->join, 0)) != hipSuccess) return hip_fail(e, "joining");
    return BSI_OK;
  }
  if (p->has_fwd && (e = launch_pass(p, kFwd, s)) != hipSuccess) return hip_fail(e, "launching the batched forward");
  if (p->has_adj) return enqueue_adjoint(p, s);
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

// A schedule index in [0, kNumSchedules), written as a plain decimal number.
bool parse_schedule(const char* text, int* out) {
  char* end = nullptr;
  const long v = std::strtol(text, &end, 10);
  if (end == text || *end != '\0' || v < 0 || v >= kNumSchedules) return false;
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
  std::snprintf(buf, sizeof(buf), "gfx950-cu%d-%016llx", p->cus, (unsigned long long)h);
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
    d.a = make_adj_geom(g);
    // Each volume's forward is split in z to about kBatchFwdTarget items:
    // fewer than a standalone launch needs (the batch fills the GPU), more than
    // one item per column (short items balance better across the batch).
    d.f = make_fwd_launch(g, kBatchFwdTarget);
    off[i] = part_floats;
    part_floats += adj_workspace_bytes(d.a) / sizeof(float);
    d.first[kFwd] = tot[kFwd];
    d.first[kAdj1] = tot[kAdj1];
    d.first[kAdj2] = tot[kAdj2];
    tot[kFwd] += (int64_t)d.f.nbx * d.f.nby * d.f.nbz;
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
    if (!parse_schedule(force, &v)) {
      bsi_batch_destroy(p);
      set_error(std::string("BSI_FORCE_CONFIG=") + force + " is not a schedule index in [0, " +
                std::to_string(kNumSchedules) + ")");
      return BSI_ERR_INVALID_ARG;
    }
    p->schedule = v;
  } else if (const char* path = std::getenv("BSI_TUNE_CACHE")) {
    const int v = cache_lookup(path, p->key);
    if (v >= 0 && v < kNumSchedules) p->schedule = v;
  }
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
  hipError_t e = hipMemcpy(p->d_desc, p->host.data(), sizeof(VolDesc) * p->host.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "uploading the descriptor table");
  e = hipMemcpy(p->d_cls, p->cls_host.data(), sizeof(VolDesc) * p->cls_host.size(), hipMemcpyHostToDevice);
  return e == hipSuccess ? BSI_OK : hip_fail(e, "uploading the class descriptor table");
}

int32_t bsi_batch_config(const bsi_batch* p, int32_t* index, int32_t* count) {
  clear_error();
  if (!p || !index || !count) {
    set_error("null argument");
    return BSI_ERR_INVALID_ARG;
  }
  *index = p->schedule;
  *count = kNumSchedules;
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
    if (!parse_schedule(force, &v)) {
      set_error(std::string("BSI_FORCE_CONFIG=") + force + " is not a schedule index in [0, " +
                std::to_string(kNumSchedules) + ")");
      return BSI_ERR_INVALID_ARG;
    }
    p->schedule = v;
    drop_graph(p);
    return BSI_OK;
  }
  hipEvent_t t0, t1;
  hipError_t e;
  if ((e = hipEventCreate(&t0)) != hipSuccess) return hip_fail(e, "creating a timing event");
  if ((e = hipEventCreate(&t1)) != hipSuccess) {
    (void)hipEventDestroy(t0);
    return hip_fail(e, "creating a timing event");
  }
  const int keep = p->schedule;
  // Two sweeps over the schedules (the first also warms clocks and caches);
  // each schedule keeps the better of its two medians of 5 timed runs.
  float sched_ms[kNumSchedules];
  for (int c = 0; c < kNumSchedules; ++c) sched_ms[c] = 1e30f;
  for (int sweep = 0; sweep < 2 && rc == BSI_OK; ++sweep)
    for (int c = 0; c < kNumSchedules && rc == BSI_OK; ++c) {
      p->schedule = c;
      if ((rc = enqueue(p, stream))) break;  // warm-up
      float times[5];
      for (int r = 0; r < 5 && rc == BSI_OK; ++r) {
        if ((e = hipEventRecord(t0, stream)) != hipSuccess) {
          rc = hip_fail(e, "recording a timing event");
          break;
        }
        if ((rc = enqueue(p, stream))) break;
        if ((e = hipEventRecord(t1, stream)) != hipSuccess || (e = hipEventSynchronize(t1)) != hipSuccess ||
            (e = hipEventElapsedTime(&times[r], t0, t1)) != hipSuccess)
          rc = hip_fail(e, "timing a schedule");
      }
      if (rc) break;
      std::sort(times, times + 5);
      sched_ms[c] = std::min(sched_ms[c], times[2]);
    }
  int best = keep;
  float best_ms = 1e30f;
  for (int c = 0; c < kNumSchedules; ++c)
    if (sched_ms[c] < best_ms) {
      best_ms = sched_ms[c];
      best = c;
    }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  p->schedule = rc == BSI_OK ? best : keep;
  drop_graph(p);
  if (rc == BSI_OK)
    if (const char* path = std::getenv("BSI_TUNE_CACHE")) cache_store(path, p->key, p->schedule);
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
