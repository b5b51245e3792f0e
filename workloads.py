"""Seeded synthetic inputs for the BSI library and its oracle.

This module holds NO arithmetic of the method: it only draws random control grids,
upstream gradients and test images with the shapes of the paper's workloads
(Sec. 4, Table 1: CT/MR volumes of 8-45 M voxels, tile sizes 3^3 to 7^3).  The
clinical volumes themselves are not available; these stand in for them.  Timing of
BSI does not depend on the values (Sec. 5.2), so random values are faithful for
performance.

Every generator draws from ``numpy.random.default_rng(seed)`` in FP64 and casts to
FP32.  Conventions: dims = (nx, ny, nz), spacing = (dx, dy, dz), grid arrays
(gz, gy, gx, 3), field arrays (nz, ny, nx, 3), images (nz, ny, nx).

Named workloads (seed = 1000 + index):
  1  64^3, spacing 5, grid 16^3 x 3 ~ N(0, 2)
  2  512 x 512 x 256, spacing 3 / 5 / 8, grid ~ N(0, 3) then a 3-point box filter
  3  256^3, spacing 5, grid 55^3 x 3 ~ N(0, 2), upstream dfield ~ N(0, 1);
     plus a 12^3 finite-difference case
  4  256 x 256 x 160 registration pair: fixed = 200 Gaussian blobs, and a known
     control grid (spacing 5, ~ N(0, 2)) that warps it into the moving image
  5  32 volumes, each axis uniform in [96, 320] x [96, 320] x [64, 200], isotropic
     spacing uniform in {4..10}, grids ~ N(0, 2), dfields ~ N(0, 1)
"""
import numpy as np


def grid_shape(dims, spacing):
    """Array shape (gz, gy, gx, 3) of the control grid for a volume: g = ceil(n/d) + 3."""
    gx, gy, gz = (-(-int(n) // int(d)) + 3 for n, d in zip(dims, spacing))
    return (gz, gy, gx, 3)


def field_shape(dims):
    nx, ny, nz = (int(v) for v in dims)
    return (nz, ny, nx, 3)


def normal(rng, shape, sigma):
    """FP32 array of N(0, sigma^2) values drawn in FP64."""
    return (rng.standard_normal(shape) * sigma).astype(np.float32)


def box3(a):
    """Three-point box filter [1, 1, 1]/3 along each of the three spatial axes of a
    (gz, gy, gx, 3) array, with edge replication, in FP64 (x, then y, then z)."""
    out = np.asarray(a, dtype=np.float64)
    for axis in (2, 1, 0):
        pad = [(0, 0)] * out.ndim
        pad[axis] = (1, 1)
        p = np.pad(out, pad, mode="edge")
        n = out.shape[axis]
        sl = lambda s: tuple(slice(s, s + n) if k == axis else slice(None) for k in range(out.ndim))
        out = (p[sl(0)] + p[sl(1)] + p[sl(2)]) / 3.0
    return out


def random_grid(dims, spacing, sigma, seed):
    return normal(np.random.default_rng(seed), grid_shape(dims, spacing), sigma)


def random_field(dims, sigma, seed):
    return normal(np.random.default_rng(seed), field_shape(dims), sigma)


# ---------------------------------------------------------------- named workloads
def cfg1(seed=1001):
    dims, spacing = (64, 64, 64), (5, 5, 5)
    rng = np.random.default_rng(seed)
    return dict(dims=dims, spacing=spacing, grid=normal(rng, grid_shape(dims, spacing), 2.0))


CFG2_DIMS = (512, 512, 256)
CFG2_SPACINGS = (3, 5, 8)


def cfg2(delta=5, seed=1002):
    dims, spacing = CFG2_DIMS, (delta, delta, delta)
    rng = np.random.default_rng(seed)
    raw = rng.standard_normal(grid_shape(dims, spacing)) * 3.0
    return dict(dims=dims, spacing=spacing, grid=box3(raw).astype(np.float32))


CFG3_DIMS = (256, 256, 256)


def cfg3(seed=1003, dims=CFG3_DIMS, spacing=(5, 5, 5)):
    rng = np.random.default_rng(seed)
    grid = normal(rng, grid_shape(dims, spacing), 2.0)
    dfield = normal(rng, field_shape(dims), 1.0)
    return dict(dims=tuple(dims), spacing=tuple(spacing), grid=grid, dfield=dfield)


def cfg3_fd(seed=1013):
    """12^3 voxels, spacing 5: 6^3 control points x 3 = 648 parameters."""
    return cfg3(seed=seed, dims=(12, 12, 12), spacing=(5, 5, 5))


CFG4_DIMS = (256, 256, 160)


def blobs(dims, count, seed, sigma_range=(3.0, 12.0), amp_range=(0.5, 1.5)):
    """Sum of ``count`` isotropic Gaussian blobs a * exp(-|x - c|^2 / (2 s^2)) on the
    voxel lattice, FP64 then FP32.  Centres are uniform in [0, n) per axis, s uniform
    in sigma_range, a uniform in amp_range.  Each blob is evaluated separably and
    only within |x - c| <= 4 s per axis (beyond, it is below exp(-8))."""
    nx, ny, nz = (int(v) for v in dims)
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, 1.0, size=(count, 3)) * np.array([nx, ny, nz], np.float64)
    s = rng.uniform(sigma_range[0], sigma_range[1], size=count)
    a = rng.uniform(amp_range[0], amp_range[1], size=count)
    img = np.zeros((nz, ny, nx), np.float64)
    for k in range(count):
        r = 4.0 * s[k]
        lo = [max(0, int(np.ceil(c[k, i] - r))) for i in range(3)]
        hi = [min(n, int(np.floor(c[k, i] + r)) + 1) for i, n in enumerate((nx, ny, nz))]
        if any(h <= l for l, h in zip(lo, hi)):
            continue
        e = [np.exp(-((np.arange(lo[i], hi[i]) - c[k, i]) ** 2) / (2.0 * s[k] ** 2)) for i in range(3)]
        img[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += a[k] * (e[2][:, None, None] * e[1][None, :, None] * e[0][None, None, :])
    return img.astype(np.float32)


def cfg4(seed=1004, dims=CFG4_DIMS, spacing=(5, 5, 5), nblobs=200, sigma=2.0):
    """Fixed image and the known control grid that generates the moving image.

    The moving image is moving(x) = fixed(x + T_true(x)) with T_true = BSI of
    ``grid_true``; producing it uses the method, so it is left to the caller."""
    rng = np.random.default_rng(seed)
    blob_seed = int(rng.integers(0, 2**31 - 1))
    grid_true = normal(rng, grid_shape(dims, spacing), sigma)
    return dict(dims=tuple(dims), spacing=tuple(spacing), fixed=blobs(dims, nblobs, blob_seed),
                grid_true=grid_true)


CFG5_COUNT = 32
CFG5_LO = (96, 96, 64)
CFG5_HI = (320, 320, 200)


def cfg5_geometry(seed=1005, count=CFG5_COUNT, lo=CFG5_LO, hi=CFG5_HI, spacing_range=(4, 10)):
    """Per-volume dims (count, 3) and isotropic spacings (count, 3), int32."""
    rng = np.random.default_rng(seed)
    dims = np.stack([rng.integers(lo[i], hi[i] + 1, size=count) for i in range(3)], axis=1)
    d = rng.integers(spacing_range[0], spacing_range[1] + 1, size=count)
    return dims.astype(np.int32), np.stack([d, d, d], axis=1).astype(np.int32)


def cfg5_volume(dims, spacing, index, seed=1005):
    """Grid ~ N(0, 2) and dfield ~ N(0, 1) of volume ``index`` (own sub-seed)."""
    rng = np.random.default_rng([seed, int(index)])
    grid = normal(rng, grid_shape(dims, spacing), 2.0)
    dfield = normal(rng, field_shape(dims), 1.0)
    return grid, dfield
