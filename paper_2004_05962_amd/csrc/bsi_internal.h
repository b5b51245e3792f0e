// Host-side internals of libbsi: error reporting, device state and launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "bsi.h"
#include "bsi_device.h"

namespace bsi {

// Thread-local last-error message (returned by bsi_last_error).
void set_error(const std::string& msg);
void clear_error();
int32_t hip_fail(hipError_t e, const char* what);  // records and returns BSI_ERR_HIP

// Current device, checking that one exists (BSI_ERR_NO_DEVICE otherwise).
int32_t current_device(int* dev);

// Basis table of every spacing 1..kMaxSpacing on device `dev` (uploaded on the
// first call per device, then cached for the life of the process).
int32_t lut_device_ptr(int dev, const float** out);
// Lerp-form weights (h0, h1, g1, 0) per offset, same row layout (lut_row).
int32_t lerp_lut_device_ptr(int dev, const float** out);

// Host-side geometry helpers.
int32_t make_geom(const int32_t dims[3], const int32_t spacing[3], VolGeom* g);
int32_t check_control_plane(int32_t gx, int32_t gy);  // UNSUPPORTED at 2^31 floats or more
AdjGeom make_adj_geom(const VolGeom& g);
size_t adj_workspace_bytes(const AdjGeom& a);

// Forward launch shape (workgroups of kFwdRows waves; z split into chunks).
struct FwdLaunch {
  int nbx, nby, nbz, zchunk;
};
#ifndef BSI_FWD_BLOCKS
#define BSI_FWD_BLOCKS 2048
#endif
constexpr int kFwdTargetBlocks = BSI_FWD_BLOCKS; // z is split until this many workgroups
// width x rows: the voxels and rows one workgroup covers in x and y.
FwdLaunch make_fwd_launch(const VolGeom& g, long target = kFwdTargetBlocks, int width = kWave, int rows = kFwdRows);
// Rows per span of the span forward (fwd_span), 0 when a span of one row does not fit.
int span_rows(const VolGeom& g, int C);

hipError_t launch_forward(const float* grid, float* field, const VolGeom& g, const float* lut,
                          hipStream_t s);
hipError_t launch_forward_scalar(const float* grid, float* image, const VolGeom& g, const float* lut,
                                 hipStream_t s);
hipError_t launch_forward_lerp(const float* grid, float* field, const VolGeom& g, const float* lerp_lut,
                               hipStream_t s);
hipError_t launch_adjoint(const float* dfield, float* grad, const AdjGeom& a, const float* lut,
                          float* part, hipStream_t s);
hipError_t launch_adjoint_partials(const float* dfield, const AdjGeom& a, const float* lut, float* part,
                                  hipStream_t s);
hipError_t launch_adjoint_reduce(const float* part, float* grad, const AdjGeom& a, hipStream_t s);
hipError_t launch_warp(const float* field, const float* image, const VolGeom& g, float* out,
                       hipStream_t s);
size_t ssd_partial_count(const VolGeom& g);
hipError_t launch_ssd_grad(const float* field, const float* moving, const float* fixed,
                           const VolGeom& g, float* dfield, float* loss, float* partials,
                           hipStream_t s);
// Fixed-order sum of n floats into out[0] (one workgroup).
hipError_t launch_sum(const float* partials, long n, float* out, hipStream_t s);
// Fused BSI -> warp -> SSD -> adjoint (fused.hip).
size_t fused_workspace_bytes(const AdjGeom& a);
// descend_grid: null, or the grid to update in place by grid -= eta * grad
// after the gradient is formed (the descent step folded into the last launch).
hipError_t launch_ssd_fused(const float* grid, const float* moving, const float* fixed, float* grad, float* loss,
                            const AdjGeom& a, const float* lut, void* workspace, hipStream_t s,
                            float* descend_grid = nullptr, float eta = 0.f);
// Real spacing s and origin o per axis (general.hip): control point a at voxel
// o + (a - 1) s, n voxels, g control points.
struct GenAxis {
  float s, o;  // the caller's FP32 spacing and origin
  int n, g;
};
struct GenGeom {
  GenAxis x, y, z;
};
int32_t make_gen_geom(const int32_t dims[3], const float spacing[3], const float origin[3], GenGeom* q,
                      VolGeom* g);
hipError_t launch_forward_general(const float* grid, float* field, const VolGeom& g, const GenGeom& q,
                                  hipStream_t s);
size_t general_workspace_bytes(const GenGeom& q);
hipError_t launch_adjoint_general(const float* dfield, float* grad, const GenGeom& q, void* workspace,
                                  hipStream_t s);
hipError_t launch_descent(float* grid, const float* grad, float eta, int64_t count, hipStream_t s);

}  // namespace bsi
