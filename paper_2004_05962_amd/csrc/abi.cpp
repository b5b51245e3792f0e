// C ABI of libbsi (declared in include/bsi.h): argument validation, error
// reporting and dispatch to the kernel launchers.  Nothing here allocates.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <limits>
#include <cmath>
#include <string>

#include "bsi.h"
#include "bsi_internal.h"

namespace bsi {

namespace {
thread_local std::string t_last_error;
}

void set_error(const std::string& msg) { t_last_error = msg; }
void clear_error() { t_last_error.clear(); }
const char* last_error_cstr() { return t_last_error.c_str(); }

int32_t hip_fail(hipError_t e, const char* what) {
  set_error(std::string("HIP error while ") + what + ": " + hipGetErrorName(e) + " (" +
            hipGetErrorString(e) + ")");
  return BSI_ERR_HIP;
}

int32_t current_device(int* dev) {
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e == hipErrorNoDevice || (e == hipSuccess && n == 0)) {
    set_error("no HIP device is visible");
    return BSI_ERR_NO_DEVICE;
  }
  if (e != hipSuccess) return hip_fail(e, "counting devices");
  e = hipGetDevice(dev);
  if (e != hipSuccess) return hip_fail(e, "querying the current device");
  return BSI_OK;
}

// Offsets within one control plane (gx * gy points of 3 floats) are signed
// 32-bit in the kernels' staging maps, with -1 for "outside the window".
int32_t check_control_plane(int32_t gx, int32_t gy) {
  if ((double)gx * gy * 3 >= 2147483648.0) {
    set_error("a control plane (gx * gy) of 7.16e8 points or more");
    return BSI_ERR_UNSUPPORTED;
  }
  return BSI_OK;
}

int32_t make_geom(const int32_t dims[3], const int32_t spacing[3], VolGeom* g) {
  if (!dims || !spacing) {
    set_error("dims and spacing must be non-null");
    return BSI_ERR_INVALID_ARG;
  }
  for (int a = 0; a < 3; ++a) {
    if (dims[a] < 1 || spacing[a] < 1) {
      set_error("dims and spacing must be >= 1 on every axis");
      return BSI_ERR_INVALID_ARG;
    }
    if (spacing[a] > BSI_MAX_SPACING) {
      set_error("spacing above BSI_MAX_SPACING (64)");
      return BSI_ERR_UNSUPPORTED;
    }
    if (dims[a] > BSI_MAX_DIM) {
      set_error("a volume axis above BSI_MAX_DIM");
      return BSI_ERR_UNSUPPORTED;
    }
  }
  g->nx = dims[0];
  g->ny = dims[1];
  g->nz = dims[2];
  g->dx = spacing[0];
  g->dy = spacing[1];
  g->dz = spacing[2];
  g->gx = (dims[0] + spacing[0] - 1) / spacing[0] + 3;
  g->gy = (dims[1] + spacing[1] - 1) / spacing[1] + 3;
  g->gz = (dims[2] + spacing[2] - 1) / spacing[2] + 3;
  // Row and plane counts are carried in 32-bit ints by the launchers.
  const double rows = (double)g->ny * g->nz;
  const double voxels = rows * g->nx;
  if (rows > 2.0e9 || voxels * 3 > 9.0e18 / 16) {
    set_error("volume too large");
    return BSI_ERR_UNSUPPORTED;
  }
  // Offsets within one voxel plane of the field are 32-bit in the kernels.
  if ((double)g->nx * g->ny * 3 >= 4294967296.0) {
    set_error("a voxel plane (nx * ny) above 1.43e9 voxels");
    return BSI_ERR_UNSUPPORTED;
  }
  return check_control_plane(g->gx, g->gy);
}

}  // namespace bsi

using namespace bsi;

namespace {

// Validation order: geometry and pointers first (host-only, so every argument
// error is reported even without a device), then the device and its table.
int32_t device_lut(const float** lut) {
  int dev = 0;
  int32_t rc = current_device(&dev);
  if (rc) return rc;
  return lut_device_ptr(dev, lut);
}

int32_t device_only() {
  int dev = 0;
  return current_device(&dev);
}

int32_t image_geom(const int32_t dims[3], VolGeom* g) {
  const int32_t one[3] = {1, 1, 1};
  return make_geom(dims, one, g);
}

int32_t null_arg(const char* name) {
  set_error(std::string(name) + " must be a non-null device pointer");
  return BSI_ERR_INVALID_ARG;
}

}  // namespace

extern "C" {

int32_t bsi_version(void) { return 10000; }

const char* bsi_last_error(void) { return last_error_cstr(); }

int32_t bsi_grid_dims(const int32_t dims[3], const int32_t spacing[3], int32_t out_g[3]) {
  clear_error();
  if (!out_g) {
    set_error("out_g must be non-null");
    return BSI_ERR_INVALID_ARG;
  }
  VolGeom g;
  int32_t rc = make_geom(dims, spacing, &g);
  if (rc) return rc;
  out_g[0] = g.gx;
  out_g[1] = g.gy;
  out_g[2] = g.gz;
  return BSI_OK;
}

int32_t bsi_forward(const float* grid, const int32_t dims[3], const int32_t spacing[3], float* field,
                    hipStream_t stream) {
  clear_error();
  VolGeom g;
  int32_t rc = make_geom(dims, spacing, &g);
  if (rc) return rc;
  if (!grid) return null_arg("grid");
  if (!field) return null_arg("field");
  const float* lut = nullptr;
  if ((rc = device_lut(&lut))) return rc;
  hipError_t e = launch_forward(grid, field, g, lut, stream);
  return e == hipSuccess ? BSI_OK : hip_fail(e, "launching the forward kernel");
}

int32_t bsi_forward_lerp(const float* grid, const int32_t dims[3], const int32_t spacing[3], float* field,
                         hipStream_t stream) {
  clear_error();
  VolGeom g;
  int32_t rc = make_geom(dims, spacing, &g);
  if (rc) return rc;
  if (!grid) return null_arg("grid");
  if (!field) return null_arg("field");
  int dev = 0;
  if ((rc = current_device(&dev))) return rc;
  const float* lut = nullptr;
  if ((rc = lerp_lut_device_ptr(dev, &lut))) return rc;
  hipError_t e = launch_forward_lerp(grid, field, g, lut, stream);
  return e == hipSuccess ? BSI_OK : hip_fail(e, "launching the lerp-form forward kernel");
}

int32_t bsi_forward_scalar(const float* grid, const int32_t dims[3], const int32_t spacing[3], float* image,
                           hipStream_t stream) {
  clear_error();
  VolGeom g;
  int32_t rc = make_geom(dims, spacing, &g);
  if (rc) return rc;
  if (!grid) return null_arg("grid");
  if (!image) return null_arg("image");
  const float* lut = nullptr;
  if ((rc = device_lut(&lut))) return rc;
  hipError_t e = launch_forward_scalar(grid, image, g, lut, stream);
  return e == hipSuccess ? BSI_OK : hip_fail(e, "launching the scalar forward kernel");
}

int32_t bsi_adjoint_workspace_size(const int32_t dims[3], const int32_t spacing[3], size_t* bytes) {
  clear_error();
  if (!bytes) {
    set_error("bytes must be non-null");
    return BSI_ERR_INVALID_ARG;
  }
  VolGeom g;
  int32_t rc = make_geom(dims, spacing, &g);
  if (rc) return rc;
  *bytes = adj_workspace_bytes(make_adj_geom(g));
  return BSI_OK;
}

namespace {
// Geometry and workspace checks shared by the adjoint entry points.
int32_t adjoint_setup(const int32_t dims[3], const int32_t spacing[3], const void* workspace,
                      size_t workspace_bytes, AdjGeom* a) {
  VolGeom g;
  int32_t rc = make_geom(dims, spacing, &g);
  if (rc) return rc;
  if (!workspace) return null_arg("workspace");
  *a = make_adj_geom(g);
  const size_t need = adj_workspace_bytes(*a);
  if (workspace_bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return BSI_ERR_INVALID_ARG;
  }
  return BSI_OK;
}
}  // namespace

int32_t bsi_adjoint(const float* dfield, const int32_t dims[3], const int32_t spacing[3], float* grid_grad,
                    void* workspace, size_t workspace_bytes, hipStream_t stream) {
  clear_error();
  AdjGeom a;
  int32_t rc = adjoint_setup(dims, spacing, workspace, workspace_bytes, &a);
  if (rc) return rc;
  if (!dfield) return null_arg("dfield");
  if (!grid_grad) return null_arg("grid_grad");
  const float* lut = nullptr;
  if ((rc = device_lut(&lut))) return rc;
  hipError_t e = launch_adjoint(dfield, grid_grad, a, lut, static_cast<float*>(workspace), stream);
  return e == hipSuccess ? BSI_OK : hip_fail(e, "launching the adjoint kernels");
}

int32_t bsi_adjoint_partials(const float* dfield, const int32_t dims[3], const int32_t spacing[3],
                             void* workspace, size_t workspace_bytes, hipStream_t stream) {
  clear_error();
  AdjGeom a;
  int32_t rc = adjoint_setup(dims, spacing, workspace, workspace_bytes, &a);
  if (rc) return rc;
  if (!dfield) return null_arg("dfield");
  const float* lut = nullptr;
  if ((rc = device_lut(&lut))) return rc;
  hipError_t e = launch_adjoint_partials(dfield, a, lut, static_cast<float*>(workspace), stream);
  return e == hipSuccess ? BSI_OK : hip_fail(e, "launching the adjoint partials kernel");
}

int32_t bsi_adjoint_reduce(const void* workspace, size_t workspace_bytes, const int32_t dims[3],
                           const int32_t spacing[3], float* grid_grad, hipStream_t stream) {
  clear_error();
  AdjGeom a;
  int32_t rc = adjoint_setup(dims, spacing, workspace, workspace_bytes, &a);
  if (rc) return rc;
  if (!grid_grad) return null_arg("grid_grad");
  if ((rc = device_only())) return rc;
  hipError_t e = launch_adjoint_reduce(static_cast<const float*>(workspace), grid_grad, a, stream);
  return e == hipSuccess ? BSI_OK : hip_fail(e, "launching the adjoint reduce kernel");
}

int32_t bsi_general_grid_dims(const int32_t dims[3], const float spacing[3], const float origin[3],
                              int32_t out_g[3]) {
  clear_error();
  if (!out_g) return null_arg("out_g");
  GenGeom q;
  VolGeom g;
  int32_t rc = make_gen_geom(dims, spacing, origin, &q, &g);
  if (rc) return rc;
  out_g[0] = g.gx;
  out_g[1] = g.gy;
  out_g[2] = g.gz;
  return BSI_OK;
}

int32_t bsi_forward_general(const float* grid, const int32_t dims[3], const float spacing[3],
                            const float origin[3], float* field, hipStream_t stream) {
  clear_error();
  GenGeom q;
  VolGeom g;
  int32_t rc = make_gen_geom(dims, spacing, origin, &q, &g);
  if (rc) return rc;
  if (!grid) return null_arg("grid");
  if (!field) return null_arg("field");
  if ((rc = device_only())) return rc;
  hipError_t e = launch_forward_general(grid, field, g, q, stream);
  return e == hipSuccess ? BSI_OK : hip_fail(e, "launching the general forward kernel");
}

int32_t bsi_adjoint_general_workspace_size(const int32_t dims[3], const float spacing[3],
                                           const float origin[3], size_t* bytes) {
  clear_error();
  if (!bytes) return null_arg("bytes");
  GenGeom q;
  VolGeom g;
  int32_t rc = make_gen_geom(dims, spacing, origin, &q, &g);
  if (rc) return rc;
  *bytes = general_workspace_bytes(q);
  return BSI_OK;
}

int32_t bsi_adjoint_general(const float* dfield, const int32_t dims[3], const float spacing[3],
                            const float origin[3], float* grid_grad, void* workspace, size_t workspace_bytes,
                            hipStream_t stream) {
  clear_error();
  GenGeom q;
  VolGeom g;
  int32_t rc = make_gen_geom(dims, spacing, origin, &q, &g);
  if (rc) return rc;
  if (!dfield) return null_arg("dfield");
  if (!grid_grad) return null_arg("grid_grad");
  if (!workspace) return null_arg("workspace");
  const size_t need = general_workspace_bytes(q);
  if (workspace_bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return BSI_ERR_INVALID_ARG;
  }
  if ((rc = device_only())) return rc;
  hipError_t e = launch_adjoint_general(dfield, grid_grad, q, workspace, stream);
  return e == hipSuccess ? BSI_OK : hip_fail(e, "launching the general adjoint kernels");
}

int32_t bsi_warp(const float* field, const float* image, const int32_t dims[3], float* out,
                 hipStream_t stream) {
  clear_error();
  VolGeom g;
  int32_t rc = image_geom(dims, &g);
  if (rc) return rc;
  if (!field) return null_arg("field");
  if (!image) return null_arg("image");
  if (!out) return null_arg("out");
  if ((rc = device_only())) return rc;
  hipError_t e = launch_warp(field, image, g, out, stream);
  return e == hipSuccess ? BSI_OK : hip_fail(e, "launching the warp kernel");
}

int32_t bsi_ssd_workspace_size(const int32_t dims[3], size_t* bytes) {
  clear_error();
  if (!bytes) {
    set_error("bytes must be non-null");
    return BSI_ERR_INVALID_ARG;
  }
  VolGeom g;
  int32_t rc = image_geom(dims, &g);
  if (rc) return rc;
  *bytes = ssd_partial_count(g) * sizeof(float);
  return BSI_OK;
}

int32_t bsi_ssd_grad(const float* field, const float* moving, const float* fixed, const int32_t dims[3],
                     float* dfield, float* loss, void* workspace, size_t workspace_bytes,
                     hipStream_t stream) {
  clear_error();
  VolGeom g;
  int32_t rc = image_geom(dims, &g);
  if (rc) return rc;
  if (!field) return null_arg("field");
  if (!moving) return null_arg("moving");
  if (!fixed) return null_arg("fixed");
  if (!dfield) return null_arg("dfield");
  if (!loss) return null_arg("loss");
  if (!workspace) return null_arg("workspace");
  const size_t need = ssd_partial_count(g) * sizeof(float);
  if (workspace_bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return BSI_ERR_INVALID_ARG;
  }
  if ((rc = device_only())) return rc;
  hipError_t e = launch_ssd_grad(field, moving, fixed, g, dfield, loss, static_cast<float*>(workspace), stream);
  return e == hipSuccess ? BSI_OK : hip_fail(e, "launching the SSD kernels");
}

int32_t bsi_ssd_fused_workspace_size(const int32_t dims[3], const int32_t spacing[3], size_t* bytes) {
  clear_error();
  if (!bytes) {
    set_error("bytes must be non-null");
    return BSI_ERR_INVALID_ARG;
  }
  VolGeom g;
  int32_t rc = make_geom(dims, spacing, &g);
  if (rc) return rc;
  *bytes = fused_workspace_bytes(make_adj_geom(g));
  return BSI_OK;
}

int32_t bsi_ssd_fused(const float* grid, const float* moving, const float* fixed, const int32_t dims[3],
                      const int32_t spacing[3], float* grid_grad, float* loss, void* workspace,
                      size_t workspace_bytes, hipStream_t stream) {
  clear_error();
  VolGeom g;
  int32_t rc = make_geom(dims, spacing, &g);
  if (rc) return rc;
  if (!grid) return null_arg("grid");
  if (!moving) return null_arg("moving");
  if (!fixed) return null_arg("fixed");
  if (!grid_grad) return null_arg("grid_grad");
  if (!loss) return null_arg("loss");
  if (!workspace) return null_arg("workspace");
  const AdjGeom a = make_adj_geom(g);
  const size_t need = fused_workspace_bytes(a);
  if (workspace_bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return BSI_ERR_INVALID_ARG;
  }
  const float* lut = nullptr;
  if ((rc = device_lut(&lut))) return rc;
  hipError_t e = launch_ssd_fused(grid, moving, fixed, grid_grad, loss, a, lut, workspace, stream);
  return e == hipSuccess ? BSI_OK : hip_fail(e, "launching the fused SSD kernels");
}

int32_t bsi_ssd_fused_descent(float* grid, const float* moving, const float* fixed, const int32_t dims[3],
                              const int32_t spacing[3], float eta, float* grid_grad, float* loss, void* workspace,
                              size_t workspace_bytes, hipStream_t stream) {
  clear_error();
  VolGeom g;
  int32_t rc = make_geom(dims, spacing, &g);
  if (rc) return rc;
  if (!grid) return null_arg("grid");
  if (!moving) return null_arg("moving");
  if (!fixed) return null_arg("fixed");
  if (!grid_grad) return null_arg("grid_grad");
  if (!loss) return null_arg("loss");
  if (!workspace) return null_arg("workspace");
  if (!std::isfinite(eta)) {
    set_error("eta must be finite");
    return BSI_ERR_INVALID_ARG;
  }
  const AdjGeom a = make_adj_geom(g);
  const size_t need = fused_workspace_bytes(a);
  if (workspace_bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return BSI_ERR_INVALID_ARG;
  }
  const float* lut = nullptr;
  if ((rc = device_lut(&lut))) return rc;
  hipError_t e = launch_ssd_fused(grid, moving, fixed, grid_grad, loss, a, lut, workspace, stream, grid, eta);
  return e == hipSuccess ? BSI_OK : hip_fail(e, "launching the fused SSD step");
}

int32_t bsi_descent_step(float* grid, const float* grad, float eta, int64_t count, hipStream_t stream) {
  clear_error();
  if (!grid) return null_arg("grid");
  if (!grad) return null_arg("grad");
  if (count < 0) {
    set_error("count must be >= 0");
    return BSI_ERR_INVALID_ARG;
  }
  int32_t rc = device_only();
  if (rc) return rc;
  if (count == 0) return BSI_OK;
  hipError_t e = launch_descent(grid, grad, eta, count, stream);
  return e == hipSuccess ? BSI_OK : hip_fail(e, "launching the descent kernel");
}

}  // extern "C"
