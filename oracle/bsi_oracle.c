/*
 * FP64 CPU oracle for cubic B-spline interpolation (BSI) of a 3-D free-form
 * deformation control grid.
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists to check the HIP library.  Only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it; the product path never does.  It shares no code, header, table
 * or helper with the GPU library.
 *
 * What it computes (paper: Sec. 2.1, Eq. 1):
 *
 *   T(x,y,z) = sum_{l=0..3} sum_{m=0..3} sum_{n=0..3}
 *                B_l(u) B_m(v) B_n(w) phi[i+l][j+m][k+n]
 *
 *   i = floor(x/dx) - 1,  u = x/dx - floor(x/dx)   (and likewise j,v / k,w)
 *
 * The paper leaves B_l to its citations; the uniform cubic B-spline basis of
 * Rueckert et al. (1999), the FFD paper it builds on, is used:
 *   B0 = (1-u)^3/6, B1 = (3u^3-6u^2+4)/6, B2 = (-3u^3+3u^2+3u+1)/6, B3 = u^3/6.
 *
 * Conventions shared with the library's public interface (not its code):
 *   - voxel coordinates are integer indices x in [0,nx), etc.; spacings are
 *     integers >= 1 given in voxels (the grid is aligned to the voxels, Sec. 3.4);
 *   - the control grid has g = ceil(n/d) + 3 points per axis, and its array
 *     index is the paper's index plus one, so voxel x reads grid columns
 *     floor(x/dx) .. floor(x/dx)+3;
 *   - layouts are row-major with the component last:
 *       grid  [gz][gy][gx][3],   field / dfield [nz][ny][nx][3].
 *   - dims = {nx, ny, nz}, spacing = {dx, dy, dz}.
 *
 * Inputs and outputs are FP64.  The Python wrapper promotes the FP32 arrays the
 * GPU receives (exactly), so input rounding is not counted as error.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the OpenMP loops that follow (n >= 1); used to time the oracle
   on one core as well as on all of them. */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Uniform cubic B-spline basis at local coordinate u in [0,1) (Eq. 1's B_l). */
void oracle_basis(double u, double B[4]) {
    double v = 1.0 - u;
    B[0] = v * v * v / 6.0;
    B[1] = (3.0 * u * u * u - 6.0 * u * u + 4.0) / 6.0;
    B[2] = (-3.0 * u * u * u + 3.0 * u * u + 3.0 * u + 1.0) / 6.0;
    B[3] = u * u * u / 6.0;
}

static int64_t grid_points(int32_t n, int32_t d) { return (int64_t)((n + d - 1) / d) + 3; }

static int check_geometry(const int32_t dims[3], const int32_t spacing[3]) {
    for (int a = 0; a < 3; ++a)
        if (dims[a] < 1 || spacing[a] < 1) return -1;
    return 0;
}

/* Tile index t = floor(x/d) (as a storage index it is the paper's i plus one)
   and local coordinate u = x/d - floor(x/d), computed in FP64. */
static void locate(int64_t x, int32_t d, int64_t* t, double* u) {
    *t = x / d;
    *u = (double)(x - *t * d) / (double)d;
}

/* Eq. 1 at one voxel, written exactly as the triple sum (l, m, n order). */
static void eval_voxel(const double* grid, int64_t gx, int64_t gy, const int32_t spacing[3],
                       int64_t x, int64_t y, int64_t z, double out[3]) {
    int64_t i, j, k;
    double u, v, w, Bu[4], Bv[4], Bw[4];
    locate(x, spacing[0], &i, &u);
    locate(y, spacing[1], &j, &v);
    locate(z, spacing[2], &k, &w);
    oracle_basis(u, Bu);
    oracle_basis(v, Bv);
    oracle_basis(w, Bw);
    for (int c = 0; c < 3; ++c) {
        double s = 0.0;
        for (int l = 0; l < 4; ++l)
            for (int m = 0; m < 4; ++m)
                for (int n = 0; n < 4; ++n) {
                    int64_t idx = (((k + n) * gy + (j + m)) * gx + (i + l)) * 3 + c;
                    s += Bu[l] * Bv[m] * Bw[n] * grid[idx];
                }
        out[c] = s;
    }
}

/* Forward BSI over the whole volume (Eq. 1).  field: [nz][ny][nx][3] FP64. */
int oracle_forward(const double* grid, const int32_t dims[3], const int32_t spacing[3],
                   double* field) {
    if (check_geometry(dims, spacing)) return -1;
    const int64_t nx = dims[0], ny = dims[1], nz = dims[2];
    const int64_t gx = grid_points(dims[0], spacing[0]);
    const int64_t gy = grid_points(dims[1], spacing[1]);
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x)
                eval_voxel(grid, gx, gy, spacing, x, y, z, field + ((z * ny + y) * nx + x) * 3);
    return 0;
}

/* Forward BSI at a list of voxels pts[k] = (x, y, z); out[k] = T(x,y,z). */
int oracle_forward_points(const double* grid, const int32_t dims[3], const int32_t spacing[3],
                          const int64_t* pts, int64_t count, double* out) {
    if (check_geometry(dims, spacing)) return -1;
    const int64_t gx = grid_points(dims[0], spacing[0]);
    const int64_t gy = grid_points(dims[1], spacing[1]);
    for (int64_t p = 0; p < count; ++p) {
        int64_t x = pts[3 * p], y = pts[3 * p + 1], z = pts[3 * p + 2];
        if (x < 0 || y < 0 || z < 0 || x >= dims[0] || y >= dims[1] || z >= dims[2]) return -2;
        eval_voxel(grid, gx, gy, spacing, x, y, z, out + 3 * p);
    }
    return 0;
}

/* Adjoint (transpose) of Eq. 1: every voxel scatters its upstream value, times
   the same basis product, onto the 64 control points it reads.  Voxels are
   visited in raster order; accumulation is FP64.  grad: [gz][gy][gx][3]. */
int oracle_adjoint(const double* dfield, const int32_t dims[3], const int32_t spacing[3],
                   double* grad) {
    if (check_geometry(dims, spacing)) return -1;
    const int64_t nx = dims[0], ny = dims[1], nz = dims[2];
    const int64_t gx = grid_points(dims[0], spacing[0]);
    const int64_t gy = grid_points(dims[1], spacing[1]);
    const int64_t gz = grid_points(dims[2], spacing[2]);
    for (int64_t q = 0; q < gx * gy * gz * 3; ++q) grad[q] = 0.0;
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t i, j, k;
                double u, v, w, Bu[4], Bv[4], Bw[4];
                locate(x, spacing[0], &i, &u);
                locate(y, spacing[1], &j, &v);
                locate(z, spacing[2], &k, &w);
                oracle_basis(u, Bu);
                oracle_basis(v, Bv);
                oracle_basis(w, Bw);
                const double* d = dfield + ((z * ny + y) * nx + x) * 3;
                for (int l = 0; l < 4; ++l)
                    for (int m = 0; m < 4; ++m)
                        for (int n = 0; n < 4; ++n) {
                            double wt = Bu[l] * Bv[m] * Bw[n];
                            double* g = grad + (((k + n) * gy + (j + m)) * gx + (i + l)) * 3;
                            g[0] += wt * d[0];
                            g[1] += wt * d[1];
                            g[2] += wt * d[2];
                        }
            }
    return 0;
}

/* One entry of the adjoint, computed as a gather: control point a = (ax,ay,az)
   collects every voxel whose 4x4x4 window contains it, i.e. floor(x/dx) in
   [ax-3, ax] (and likewise in y, z), each weighted by the basis product for
   index l = ax - floor(x/dx).  Each point is an independent literal sum over
   its support in raster order, so the points are spread over OpenMP threads;
   used for single points of large volumes and, over every point, as the
   parallel form of the whole adjoint. */
int oracle_adjoint_points(const double* dfield, const int32_t dims[3], const int32_t spacing[3],
                          const int64_t* cps, int64_t count, double* out) {
    if (check_geometry(dims, spacing)) return -1;
    const int64_t nx = dims[0], ny = dims[1];
    const int64_t g[3] = {grid_points(dims[0], spacing[0]), grid_points(dims[1], spacing[1]),
                          grid_points(dims[2], spacing[2])};
    for (int64_t p = 0; p < count; ++p)
        for (int ax = 0; ax < 3; ++ax)
            if (cps[3 * p + ax] < 0 || cps[3 * p + ax] >= g[ax]) return -2;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < count; ++p) {
        const int64_t a[3] = {cps[3 * p], cps[3 * p + 1], cps[3 * p + 2]};
        int64_t lo[3], hi[3];
        for (int ax = 0; ax < 3; ++ax) {
            lo[ax] = (a[ax] - 3) * spacing[ax];
            if (lo[ax] < 0) lo[ax] = 0;
            hi[ax] = (a[ax] + 1) * spacing[ax];
            if (hi[ax] > dims[ax]) hi[ax] = dims[ax];
        }
        double s[3] = {0.0, 0.0, 0.0};
        for (int64_t z = lo[2]; z < hi[2]; ++z)
            for (int64_t y = lo[1]; y < hi[1]; ++y)
                for (int64_t x = lo[0]; x < hi[0]; ++x) {
                    int64_t i, j, k;
                    double u, v, w, Bu[4], Bv[4], Bw[4];
                    locate(x, spacing[0], &i, &u);
                    locate(y, spacing[1], &j, &v);
                    locate(z, spacing[2], &k, &w);
                    oracle_basis(u, Bu);
                    oracle_basis(v, Bv);
                    oracle_basis(w, Bw);
                    double wt = Bu[a[0] - i] * Bv[a[1] - j] * Bw[a[2] - k];
                    const double* d = dfield + ((z * ny + y) * nx + x) * 3;
                    s[0] += wt * d[0];
                    s[1] += wt * d[1];
                    s[2] += wt * d[2];
                }
        out[3 * p] = s[0];
        out[3 * p + 1] = s[1];
        out[3 * p + 2] = s[2];
    }
    return 0;
}

/* ---- Trilinear reformulation (Sec. 3.3, App. B) -------------------------
 * Along one axis, B0 p0 + B1 p1 + B2 p2 + B3 p3 equals
 *   lerp( lerp(p0, p1, h0), lerp(p2, p3, h1), g1 )
 * with g1 = B2 + B3, h0 = B1 / (B0 + B1), h1 = B3 / (B2 + B3), because the
 * four weights sum to one.  In 3-D the 4x4x4 cube splits into eight 2x2x2
 * sub-cubes; each is one trilinear interpolation with the h-weights, and a
 * ninth trilinear interpolation of the eight results uses the g1-weights.
 * Each trilinear interpolation is seven linear interpolations a + w (b - a). */
static double lerp(double a, double b, double w) { return a + w * (b - a); }

static double trilerp(const double c[2][2][2], double wx, double wy, double wz) {
    /* c[z][y][x]; interpolate along x, then y, then z: 4 + 2 + 1 = 7 lerps. */
    double x00 = lerp(c[0][0][0], c[0][0][1], wx);
    double x01 = lerp(c[0][1][0], c[0][1][1], wx);
    double x10 = lerp(c[1][0][0], c[1][0][1], wx);
    double x11 = lerp(c[1][1][0], c[1][1][1], wx);
    double y0 = lerp(x00, x01, wy);
    double y1 = lerp(x10, x11, wy);
    return lerp(y0, y1, wz);
}

static void lerp_weights(const double B[4], double* g1, double h[2]) {
    *g1 = B[2] + B[3];
    h[0] = B[1] / (B[0] + B[1]);
    h[1] = B[3] / (B[2] + B[3]);
}

int oracle_forward_lerp(const double* grid, const int32_t dims[3], const int32_t spacing[3],
                        double* field) {
    if (check_geometry(dims, spacing)) return -1;
    const int64_t nx = dims[0], ny = dims[1], nz = dims[2];
    const int64_t gx = grid_points(dims[0], spacing[0]);
    const int64_t gy = grid_points(dims[1], spacing[1]);
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t i, j, k;
                double u, v, w, Bu[4], Bv[4], Bw[4], gu, gv, gw, hu[2], hv[2], hw[2];
                locate(x, spacing[0], &i, &u);
                locate(y, spacing[1], &j, &v);
                locate(z, spacing[2], &k, &w);
                oracle_basis(u, Bu);
                oracle_basis(v, Bv);
                oracle_basis(w, Bw);
                lerp_weights(Bu, &gu, hu);
                lerp_weights(Bv, &gv, hv);
                lerp_weights(Bw, &gw, hw);
                for (int c = 0; c < 3; ++c) {
                    double sub[2][2][2];
                    /* sub-cube (r, q, p) covers control offsets 2r..2r+1 in z,
                       2q..2q+1 in y and 2p..2p+1 in x */
                    for (int r = 0; r < 2; ++r)
                        for (int q = 0; q < 2; ++q)
                            for (int p = 0; p < 2; ++p) {
                                double cube[2][2][2];
                                for (int dz = 0; dz < 2; ++dz)
                                    for (int dy = 0; dy < 2; ++dy)
                                        for (int dx = 0; dx < 2; ++dx) {
                                            int64_t idx = (((k + 2 * r + dz) * gy + (j + 2 * q + dy)) * gx +
                                                           (i + 2 * p + dx)) * 3 + c;
                                            cube[dz][dy][dx] = grid[idx];
                                        }
                                sub[r][q][p] = trilerp(cube, hu[p], hv[q], hw[r]);
                            }
                    field[((z * ny + y) * nx + x) * 3 + c] = trilerp(sub, gu, gv, gw);
                }
            }
    return 0;
}
