"""Brute-force BSI for tiny volumes: a sum over *every* control point.

Test infrastructure only (see ``oracle/__init__.py``).

This is an independent formulation of Eq. 1 (Sec. 2.1) with no tiles, no floor and
no per-offset basis: each control point is a bump centred on its own position, and
the field is the sum of all bumps.  With the paper's index i = floor(x/d) - 1, the
control point with paper index p sits at voxel p*d, and in storage (index a = p + 1)
at voxel (a - 1)*d.  The bump is the centred cubic B-spline

    beta3(t) = 2/3 - t^2 + |t|^3/2       for |t| < 1
             = (2 - |t|)^3 / 6            for 1 <= |t| < 2
             = 0                          otherwise,

evaluated at t = x/d - (a - 1) per axis.  Pure Python loops: only for a few
thousand voxel-point pairs.
"""
from fractions import Fraction

import numpy as np


def beta3(t):
    """Centred cubic B-spline (exact for Fraction inputs)."""
    t = abs(t)
    if t < 1:
        return Fraction(2, 3) - t * t + t * t * t / 2 if isinstance(t, Fraction) else 2.0 / 3.0 - t * t + t ** 3 / 2.0
    if t < 2:
        return (2 - t) ** 3 / 6
    return 0 * t


def forward(grid, dims, spacing):
    """T(x) = sum over all control points a of phi_a * prod_axes beta3(x/d - (a-1))."""
    nx, ny, nz = (int(v) for v in dims)
    dx, dy, dz = (int(v) for v in spacing)
    g = np.asarray(grid, dtype=np.float64)
    gz, gy, gx, _ = g.shape
    out = np.zeros((nz, ny, nx, 3), np.float64)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                acc = np.zeros(3)
                for az in range(gz):
                    wz = beta3(z / dz - (az - 1))
                    if wz == 0:
                        continue
                    for ay in range(gy):
                        wy = beta3(y / dy - (ay - 1))
                        if wy == 0:
                            continue
                        for ax in range(gx):
                            wx = beta3(x / dx - (ax - 1))
                            if wx == 0:
                                continue
                            acc += wx * wy * wz * g[az, ay, ax]
                out[z, y, x] = acc
    return out


def matrix(dims, spacing):
    """Dense matrix B (one component) with field = B @ grid, built from beta3.

    Rows are voxels in raster order (x fastest), columns control points in raster
    order.  Its transpose is the adjoint."""
    nx, ny, nz = (int(v) for v in dims)
    dx, dy, dz = (int(v) for v in spacing)
    gx, gy, gz = (-(-nx // dx) + 3, -(-ny // dy) + 3, -(-nz // dz) + 3)
    M = np.zeros((nx * ny * nz, gx * gy * gz))
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                r = (z * ny + y) * nx + x
                for az in range(gz):
                    wz = beta3(z / dz - (az - 1))
                    if wz == 0:
                        continue
                    for ay in range(gy):
                        wy = beta3(y / dy - (ay - 1))
                        if wy == 0:
                            continue
                        for ax in range(gx):
                            wx = beta3(x / dx - (ax - 1))
                            if wx != 0:
                                M[r, (az * gy + ay) * gx + ax] = wx * wy * wz
    return M
