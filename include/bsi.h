/*
 * bsi.h -- C ABI of libbsi: cubic B-spline interpolation (BSI) of a 3-D
 * free-form-deformation control grid on AMD Instinct MI355X (gfx950).
 *
 * The operation (paper: Sec. 2.1, Eq. 1).  For every voxel (x, y, z) of a volume
 * of nx x ny x nz voxels and a control grid with integer spacings dx, dy, dz
 * (in voxels, grid aligned to the voxels, Sec. 3.4):
 *
 *   T(x,y,z) = sum_{l,m,n=0..3} B_l(u) B_m(v) B_n(w) phi[k+n][j+m][i+l]
 *
 *   i = floor(x/dx), u = x/dx - floor(x/dx)      (likewise j, v and k, w)
 *   B0 = (1-u)^3/6, B1 = (3u^3-6u^2+4)/6, B2 = (-3u^3+3u^2+3u+1)/6, B3 = u^3/6
 *
 * Indices here are storage indices: the paper's control-point index plus one,
 * so that every index is >= 0.  The grid therefore has g = ceil(n/d) + 3 points
 * per axis (bsi_grid_dims).
 *
 * Layouts (row-major, component last; components are the x, y, z displacement):
 *   grid, grid_grad  : float [gz][gy][gx][3]
 *   field, dfield    : float [nz][ny][nx][3]
 *   images           : float [nz][ny][nx]
 *   dims    = {nx, ny, nz},  spacing = {dx, dy, dz}  (host int32 arrays)
 *
 * Common rules for every entry point below unless it says otherwise:
 *   - Buffer pointers are DEVICE pointers owned by the caller.  The library
 *     never frees or retains them; the buffers must not overlap.  4-byte
 *     alignment is enough.
 *   - dims/spacing/out-params are HOST pointers.
 *   - Work is enqueued asynchronously on `stream` (0 = the null stream) of the
 *     current HIP device; no call synchronises the host.
 *   - Arithmetic is FP32.  For a fixed build the result bits are a function of
 *     the inputs only (no atomics, fixed summation order): reruns, tuning
 *     choices, batched and per-volume launches give identical bits.
 *   - Return 0 on success or a negative BSI_ERR_* code; bsi_last_error() then
 *     holds a message.  No exception crosses the ABI.
 */
#ifndef BSI_H
#define BSI_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BSI_OK 0
#define BSI_ERR_INVALID_ARG (-1) /* null pointer, n < 1, d < 1, bad size     */
#define BSI_ERR_UNSUPPORTED (-2) /* d > BSI_MAX_SPACING, or a size too large
                                    (an axis above BSI_MAX_DIM, a voxel plane
                                    nx * ny of 2^32 / 3 voxels or more, or a
                                    control plane gx * gy of 2^31 / 3 points
                                    or more)                                 */
#define BSI_ERR_HIP (-3)         /* a HIP call failed; see bsi_last_error()  */
#define BSI_ERR_NO_DEVICE (-4)   /* no HIP device is visible                 */
#define BSI_ERR_NOMEM (-5)       /* allocation of a batched plan failed      */

#define BSI_MAX_SPACING 64       /* largest supported spacing, per axis      */
#define BSI_MAX_DIM (1 << 20)    /* largest supported voxel count per axis   */

/* Version of this ABI (major * 10000 + minor * 100 + patch). */
int32_t bsi_version(void);

/* Message for the last failed call on this host thread ("" if none). */
const char* bsi_last_error(void);

/* Control-grid size for a volume: out_g[a] = ceil(dims[a]/spacing[a]) + 3.
   Host-only; needs no device.  Errors: INVALID_ARG, UNSUPPORTED. */
int32_t bsi_grid_dims(const int32_t dims[3], const int32_t spacing[3], int32_t out_g[3]);

/* Forward BSI (Eq. 1): field[z][y][x][:] = T(x, y, z) for every voxel.
   grid: [gz][gy][gx][3] read-only; field: [nz][ny][nx][3] fully overwritten.
   Errors: INVALID_ARG, UNSUPPORTED, NO_DEVICE, HIP. */
int32_t bsi_forward(const float* grid, const int32_t dims[3], const int32_t spacing[3],
                    float* field, hipStream_t stream);

/* Forward BSI evaluated in the paper's lerp form (Sec. 3.3, App. B): per voxel,
   8 trilinear interpolations of the 2x2x2 sub-cubes of its 4x4x4 window with
   h0 = B1/(B0+B1), h1 = B3/(B2+B3), then one of the 8 results with
   g1 = B2+B3.  Same result as bsi_forward up to FP32 rounding, with about
   15 times its arithmetic: an ablation of the paper's evaluation against the
   sum-factorised kernel, not a faster path.  Arguments and errors as in
   bsi_forward. */
int32_t bsi_forward_lerp(const float* grid, const int32_t dims[3], const int32_t spacing[3],
                         float* field, hipStream_t stream);

/* Scalar forward BSI: Eq. 1 with one value per control point, e.g. the pixels
   of a coarse image as control points, giving its cubic B-spline upsampling by
   the integer factors `spacing` ("image zooming", the other use of BSI named
   in Sec. 8).  image[z][y][x] = sum B_l(u) B_m(v) B_n(w) grid[k+n][j+m][i+l].
   grid: float [gz][gy][gx] read-only; image: float [nz][ny][nx] fully
   overwritten.  Each value equals, bit for bit, the same component of
   bsi_forward on a grid holding these values in that component.  For a 2-D
   image use nz = 1 and spacing[2] = 1 (the grid then needs gz = 4 planes).
   Errors: INVALID_ARG, UNSUPPORTED, NO_DEVICE, HIP. */
int32_t bsi_forward_scalar(const float* grid, const int32_t dims[3], const int32_t spacing[3],
                           float* image, hipStream_t stream);

/* Scratch size in bytes that bsi_adjoint needs for this geometry (host-only). */
int32_t bsi_adjoint_workspace_size(const int32_t dims[3], const int32_t spacing[3],
                                   size_t* bytes);

/* Adjoint of Eq. 1 (its exact transpose; not in the paper): for every control
   point a,
     grid_grad[a] = sum over voxels x whose 4x4x4 window contains a of
                    B_{a_x-i}(u) B_{a_y-j}(v) B_{a_z-k}(w) * dfield[x].
   dfield: [nz][ny][nx][3] read-only; grid_grad: [gz][gy][gx][3] OVERWRITTEN
   (not accumulated).  workspace: device scratch of at least
   bsi_adjoint_workspace_size() bytes, owned by the caller, contents ignored on
   entry and undefined on exit; it must not be shared by calls that may run
   concurrently.  Deterministic gather in a fixed order, no atomics.
   Errors: INVALID_ARG (also when workspace_bytes is too small), UNSUPPORTED,
   NO_DEVICE, HIP. */
int32_t bsi_adjoint(const float* dfield, const int32_t dims[3], const int32_t spacing[3],
                    float* grid_grad, void* workspace, size_t workspace_bytes,
                    hipStream_t stream);

/* The two passes of bsi_adjoint as separate calls; bsi_adjoint is exactly
   bsi_adjoint_partials followed by bsi_adjoint_reduce on the same workspace and
   stream, with identical bits.  Splitting them lets a caller time or overlap
   the passes, or reduce partials written earlier.
   bsi_adjoint_partials: reads dfield and writes, for every brick of voxels, the
   partial sums of that brick's voxels to each control point it touches into
   workspace (layout internal to the library).
   bsi_adjoint_reduce: sums each control point's brick partials in a fixed order
   and OVERWRITES grid_grad.  The workspace must hold the output of a
   bsi_adjoint_partials call of the same geometry that is ordered before it
   (same stream, or synchronised).
   Arguments, ownership and errors as in bsi_adjoint. */
int32_t bsi_adjoint_partials(const float* dfield, const int32_t dims[3],
                             const int32_t spacing[3], void* workspace,
                             size_t workspace_bytes, hipStream_t stream);
int32_t bsi_adjoint_reduce(const void* workspace, size_t workspace_bytes,
                           const int32_t dims[3], const int32_t spacing[3],
                           float* grid_grad, hipStream_t stream);

/* The adjoint of bsi_adjoint without its workspace arguments, and without
   any allocation.  For callers that cannot allocate device memory: code
   under HIP graph capture, tight serving loops, harnesses that forbid
   hipMalloc.  Same kernels and same bits as bsi_adjoint.
   The partials live in a static device array of BSI_ADJOINT_NOALLOC_MAX_BYTES
   that each GPU the library runs on holds until the process ends; all calls on
   one GPU share it, so calls that may overlap on one GPU (other streams or
   host threads) race, and the caller must order them.  The first call on a
   device (of this or any other entry point) uploads the basis table with a
   blocking copy: make it outside graph capture.
   Arguments, layouts and ownership as in bsi_adjoint; grid_grad OVERWRITTEN.
   Errors: INVALID_ARG, UNSUPPORTED (also when this geometry's partials,
   bsi_adjoint_workspace_size(), exceed BSI_ADJOINT_NOALLOC_MAX_BYTES),
   NO_DEVICE, HIP. */
#define BSI_ADJOINT_NOALLOC_MAX_BYTES ((size_t)64 << 20) /* 64 MiB per device */
int32_t bsi_adjoint_noalloc(const float* dfield, const int32_t dims[3], const int32_t spacing[3],
                            float* grid_grad, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Control grids with real spacing and an origin offset (the paper's method
 * needs the grid aligned to the voxels with integer spacing, Sec. 3.4; Sec. 8
 * names this as its limitation).  Per axis a, with spacing[a] = s >= 1 and
 * origin[a] = o, -s < o <= 0 (host float arrays):
 *   control point (storage index) c sits at voxel o + (c - 1) s;
 *   voxel x reads c = i .. i+3, i = floor(t), weights B_l(t - i), t = (x - o)/s,
 *   where i is the exact floor of (x - o)/s for the float values of s and o
 *   (decided with FP32 error-free arithmetic) and t - i and the weights are FP32;
 *   the grid has g = floor((n - 1 - o)/s) + 4 points (ceil(n/s) + 3 for
 *   integer s and o = 0, where these calls compute the same map as
 *   bsi_forward / bsi_adjoint, up to FP32 rounding).
 * Weights are evaluated per coordinate instead of per in-tile offset.
 * ------------------------------------------------------------------------- */

/* Control-grid size out_g[a] for this geometry (host-only).
   Errors: INVALID_ARG (s < 1, o outside (-s, 0], n < 1), UNSUPPORTED. */
int32_t bsi_general_grid_dims(const int32_t dims[3], const float spacing[3], const float origin[3],
                              int32_t out_g[3]);

/* Forward (Eq. 1) on the general grid.  grid: [gz][gy][gx][3]; field:
   [nz][ny][nx][3] overwritten.  Errors as bsi_general_grid_dims, NO_DEVICE, HIP. */
int32_t bsi_forward_general(const float* grid, const int32_t dims[3], const float spacing[3],
                            const float origin[3], float* field, hipStream_t stream);

/* Scratch bytes for bsi_adjoint_general (host-only). */
int32_t bsi_adjoint_general_workspace_size(const int32_t dims[3], const float spacing[3],
                                           const float origin[3], size_t* bytes);

/* Adjoint of bsi_forward_general, grid_grad OVERWRITTEN: three separable
   gathers (x, then y, then z) in a fixed order, no atomics.  workspace as for
   bsi_adjoint, of bsi_adjoint_general_workspace_size() bytes.
   Errors as bsi_forward_general (INVALID_ARG also for a small workspace). */
int32_t bsi_adjoint_general(const float* dfield, const int32_t dims[3], const float spacing[3],
                            const float origin[3], float* grid_grad, void* workspace,
                            size_t workspace_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * SSD registration step (the FFD loop of Sec. 6 with a sum-of-squared-
 * differences similarity standing in for the paper's NiftyReg measure).
 * p(x) = x + T(x) in voxel units, formed in FP32; trilinear interpolation with
 * corners on voxel centres and p clamped to [0, n-1] per axis; at an exact
 * integer p the cell [p, p+1] is used.
 * ------------------------------------------------------------------------- */

/* out[z][y][x] = image sampled at p(x).  field: [nz][ny][nx][3]; image, out:
   [nz][ny][nx].  Errors: INVALID_ARG, UNSUPPORTED, NO_DEVICE, HIP. */
int32_t bsi_warp(const float* field, const float* image, const int32_t dims[3], float* out,
                 hipStream_t stream);

/* Scratch size in bytes that bsi_ssd_grad needs for this volume (host-only). */
int32_t bsi_ssd_workspace_size(const int32_t dims[3], size_t* bytes);

/* SSD loss and its gradient with respect to the displacement field:
     W = moving(p(x)),  r = W - fixed,  loss[0] = sum_x r^2 (FP32, fixed order),
     dfield[x][c] = 2 r dW/dp_c, and 0 where p_c <= 0 or p_c >= n_c - 1.
   field: [nz][ny][nx][3]; moving, fixed: [nz][ny][nx]; dfield: [nz][ny][nx][3]
   overwritten; loss: one device float, overwritten.  workspace as for
   bsi_adjoint, of bsi_ssd_workspace_size() bytes.
   Errors: INVALID_ARG, UNSUPPORTED, NO_DEVICE, HIP. */
int32_t bsi_ssd_grad(const float* field, const float* moving, const float* fixed,
                     const int32_t dims[3], float* dfield, float* loss, void* workspace,
                     size_t workspace_bytes, hipStream_t stream);

/* Scratch size in bytes that bsi_ssd_fused needs for this geometry (host-only). */
int32_t bsi_ssd_fused_workspace_size(const int32_t dims[3], const int32_t spacing[3],
                                     size_t* bytes);

/* The registration step's loss and control-grid gradient in one pass, without
   materialising the field or its gradient (merging FFD steps into BSI, the
   further work named in Sec. 8):
     T = Eq. 1 of grid,  W = moving(x + T(x)),  r = W - fixed,
     loss[0]   = sum_x r^2 (FP32, fixed order),
     grid_grad = B^T [2 r dW/dp]  (the adjoint of Eq. 1 applied to the
                 bsi_ssd_grad field gradient), OVERWRITTEN.
   grid_grad equals bsi_forward -> bsi_ssd_grad -> bsi_adjoint bit for bit
   (T is formed with the forward's operations, the residual and gradient with
   the SSD kernel's, and the adjoint is the same pass 1 and pass 2); the loss
   is summed in another fixed order than bsi_ssd_grad's.
   grid: [gz][gy][gx][3]; moving, fixed: [nz][ny][nx]; grid_grad as grid;
   loss: one device float.  workspace: device scratch of at least
   bsi_ssd_fused_workspace_size() bytes, owned by the caller, not shared by
   concurrent calls.  Deterministic, no atomics.
   Errors: INVALID_ARG, UNSUPPORTED, NO_DEVICE, HIP. */
int32_t bsi_ssd_fused(const float* grid, const float* moving, const float* fixed,
                      const int32_t dims[3], const int32_t spacing[3], float* grid_grad,
                      float* loss, void* workspace, size_t workspace_bytes,
                      hipStream_t stream);

/* One fused registration iteration: bsi_ssd_fused at the current grid, then
   grid -= eta * grid_grad (each float as bsi_descent_step computes it), with
   the descent update and the loss sum folded into the gradient's launch.
   grid is read and updated in place; the other arguments are those of
   bsi_ssd_fused (same workspace size).  grid_grad and loss hold the gradient
   and loss at the grid before the update.  Errors: INVALID_ARG (also a
   non-finite eta), UNSUPPORTED, NO_DEVICE, HIP. */
int32_t bsi_ssd_fused_descent(float* grid, const float* moving, const float* fixed,
                              const int32_t dims[3], const int32_t spacing[3], float eta,
                              float* grid_grad, float* loss, void* workspace,
                              size_t workspace_bytes, hipStream_t stream);

/* Gradient-descent update grid[i] -= eta * grad[i] for i < count (count = number
   of floats).  Errors: INVALID_ARG, NO_DEVICE, HIP. */
int32_t bsi_descent_step(float* grid, const float* grad, float eta, int64_t count,
                         hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batched forward + adjoint of many volumes of different sizes and spacings in
 * persistent launches (not in the paper).  A plan fixes the geometry at
 * creation, binds the per-volume buffers once, and can capture the whole
 * forward + adjoint into one HIP graph that is replayed with one launch.
 * Results are bit-identical to bsi_forward / bsi_adjoint on each volume.
 * A plan belongs to the device that was current at bsi_batch_create; every
 * call on it must run with that device current.
 * ------------------------------------------------------------------------- */
typedef struct bsi_batch bsi_batch;

/* Create a plan for `count` volumes; dims3xN / spacing3xN hold count triples
   (host).  Allocates the plan's descriptor table and adjoint scratch on the
   current device.  Errors: INVALID_ARG, UNSUPPORTED, NO_DEVICE, NOMEM, HIP. */
int32_t bsi_batch_create(int32_t count, const int32_t* dims3xN, const int32_t* spacing3xN,
                         bsi_batch** out);

/* Bind device buffers (host arrays of exactly `count` device pointers each;
   the library cannot check their length or the buffers' sizes, which must be
   those of each volume's grid and field).  grids and fields are used by the
   forward, dfields and grid_grads by the adjoint; pass NULL for a whole pass to
   leave it out.  Synchronises the plan's device first (a launch still running
   reads the tables this call rewrites), then invalidates a captured graph. */
int32_t bsi_batch_bind(bsi_batch* plan, const float* const* grids, float* const* fields,
                       const float* const* dfields, float* const* grid_grads);

/* Choose the plan's schedule by timing it on `stream` with the bound buffers
   (the outputs are written while timing).  A schedule sets nine knobs: the
   forward's workgroup shape (rows x 64-voxel strips: 4x1, 2x2, 8x1), its
   items per volume (z split target 512, 2048, 8192), the persistent grid of
   each pass in workgroups per CU (forward 0/2/4/8, pass 1 0/1/2/3, pass 2 0/8;
   0 = one workgroup per item), the number of streams the pass-1 launches
   spread over (1, 2, 4), whether the forward runs beside the adjoint or before
   it, whether the forward's stores are ordinary or non-temporal, and whether
   pass 1 runs one launch per x-spacing class or one launch for all the
   spacings 4..12 (a kernel that takes the spacing at run time).  The search
   is a coordinate descent from the current schedule, each candidate timed as
   the median of 5 runs on `stream` after a warm-up run.  Drops a captured
   graph.  The choice is stored in the JSON file named by the environment
   variable BSI_TUNE_CACHE (if set) and read back by later plans with the same
   geometry; BSI_FORCE_CONFIG=<index> skips timing, and an index outside
   [0, count) (see bsi_batch_config) is rejected with INVALID_ARG, here and in
   bsi_batch_create.  BSI_TUNE_VERBOSE (set) prints each timing to stderr.
   Synchronises the plan's device.  No schedule changes a result bit. */
int32_t bsi_batch_tune(bsi_batch* plan, hipStream_t stream);

/* Index of the schedule the plan uses, and the number of schedules. */
int32_t bsi_batch_config(const bsi_batch* plan, int32_t* index, int32_t* count);

/* The plan's schedule as text ("fwd_tile=4x1 fwd_items=2048 ..."), written
   NUL-terminated into buf (host, len bytes; truncated to fit).
   Errors: INVALID_ARG (null plan or buffer, len < 1). */
int32_t bsi_batch_describe(const bsi_batch* plan, char* buf, int32_t len);

/* Enqueue the persistent forward and adjoint kernels directly on `stream`. */
int32_t bsi_batch_run(bsi_batch* plan, hipStream_t stream);

/* Reference schedule: one bsi_forward + bsi_adjoint launch pair per volume,
   enqueued back to back on `stream` (same kernels' arithmetic, same bits). */
int32_t bsi_batch_run_separate(bsi_batch* plan, hipStream_t stream);

/* Capture bsi_batch_run into a HIP graph (stream capture on `stream`) and
   instantiate it, replacing an earlier graph (the plan's device is synchronised
   first, so no launch of that graph is still running).
   Errors: INVALID_ARG (nothing bound), HIP. */
int32_t bsi_batch_capture(bsi_batch* plan, hipStream_t stream);

/* Replay the captured graph with one hipGraphLaunch on `stream`.
   Errors: INVALID_ARG (no graph captured), HIP. */
int32_t bsi_batch_launch(bsi_batch* plan, hipStream_t stream);

/* Release the plan, its graph and its device memory (synchronises the device
   that owns it).  NULL is ignored. */
void bsi_batch_destroy(bsi_batch* plan);

#ifdef __cplusplus
}
#endif

#endif /* BSI_H */
