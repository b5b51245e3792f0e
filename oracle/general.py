"""FP64 BSI for a control grid with real spacing and an origin offset.

Test infrastructure only (see ``oracle/__init__.py``).

The paper's method needs the grid aligned to the voxels with integer spacing
(Sec. 3.4; its conclusion in Sec. 8 names this as the limitation).  This is Eq. 1
for the general case, per axis:

  control point a (storage index, paper index + 1) sits at voxel o + (a - 1) s,
  spacing s >= 1 (real), origin -s < o <= 0;
  voxel x:  t = (x - o) / s,  i = floor(t),  u = t - i,
            window of control points i .. i+3 with weights B_0..B_3(u);
  g = floor((n - 1 - o) / s) + 4 points per axis.

For integer s and o = 0 this is exactly the aligned case: t = x/s, g = ceil(n/s) + 3.
s and o are the FP32 values the library receives; t is their exact rational
(x - o)/s, so the window start i = floor(t) is the exact one, and u = t - i is
rounded to FP64 once.  Forward: the plain triple sum; adjoint: the raster-order
scatter of the same products.
"""
from fractions import Fraction

import numpy as np

from . import basis


def _f(v):
    return float(np.float32(v))


def _t(x, s, o):
    """t = (x - o)/s as an exact rational (s, o already FP32 values)."""
    return (Fraction(int(x)) - Fraction(o)) / Fraction(s)


def axis_table(n, s, o):
    """Window start i and weights B(u) (n, 4) of every coordinate 0..n-1."""
    s, o = _f(s), _f(o)
    i = np.empty(n, np.int64)
    w = np.empty((n, 4), np.float64)
    for x in range(n):
        t = _t(x, s, o)
        i[x] = t.numerator // t.denominator
        w[x] = basis(float(t - int(i[x])))
    return i, w


def grid_dims(dims, spacing, origin):
    """Control points per axis (gx, gy, gz): floor((n - 1 - o)/s) + 4."""
    out = []
    for n, s, o in zip(dims, spacing, origin):
        s, o = _f(s), _f(o)
        if not (s >= 1.0 and -s < o <= 0.0):
            raise ValueError("need spacing >= 1 and -spacing < origin <= 0")
        t = _t(int(n) - 1, s, o)
        out.append(t.numerator // t.denominator + 4)
    return tuple(out)


def forward(grid, dims, spacing, origin):
    """Field (nz, ny, nx, 3) of a grid (gz, gy, gx, 3), FP64."""
    nx, ny, nz = (int(v) for v in dims)
    gx, gy, gz = grid_dims(dims, spacing, origin)
    g = np.asarray(grid, dtype=np.float64)
    if g.shape != (gz, gy, gx, 3):
        raise ValueError(f"grid has shape {g.shape}, expected {(gz, gy, gx, 3)}")
    ix, wx = axis_table(nx, spacing[0], origin[0])
    iy, wy = axis_table(ny, spacing[1], origin[1])
    iz, wz = axis_table(nz, spacing[2], origin[2])
    out = np.zeros((nz, ny, nx, 3), np.float64)
    for n in range(4):
        for m in range(4):
            for l in range(4):
                w = wz[:, n][:, None, None] * wy[:, m][None, :, None] * wx[:, l][None, None, :]
                out += w[..., None] * g[(iz + n)[:, None, None], (iy + m)[None, :, None], (ix + l)[None, None, :]]
    return out


def adjoint(dfield, dims, spacing, origin):
    """Transpose of ``forward``: grad (gz, gy, gx, 3), FP64; every voxel adds its value times
    each of its 64 basis products onto the control point that product belongs to."""
    nx, ny, nz = (int(v) for v in dims)
    gx, gy, gz = grid_dims(dims, spacing, origin)
    d = np.asarray(dfield, dtype=np.float64)
    ix, wx = axis_table(nx, spacing[0], origin[0])
    iy, wy = axis_table(ny, spacing[1], origin[1])
    iz, wz = axis_table(nz, spacing[2], origin[2])
    grad = np.zeros((gz, gy, gx, 3), np.float64)
    for n in range(4):
        for m in range(4):
            for l in range(4):
                w = wz[:, n][:, None, None] * wy[:, m][None, :, None] * wx[:, l][None, None, :]
                np.add.at(grad, ((iz + n)[:, None, None], (iy + m)[None, :, None], (ix + l)[None, None, :]),
                          w[..., None] * d)
    return grad


def forward_points(grid, dims, spacing, origin, pts):
    """``forward`` at voxels pts[k] = (x, y, z) only: (k, 3), FP64."""
    g = np.asarray(grid, dtype=np.float64)
    p = np.asarray(pts, dtype=np.int64).reshape(-1, 3)
    tabs = [axis_table(int(n), s, o) for n, s, o in zip(dims, spacing, origin)]
    (ix, wx), (iy, wy), (iz, wz) = [(i[p[:, a]], w[p[:, a]]) for a, (i, w) in enumerate(tabs)]
    out = np.zeros((p.shape[0], 3), np.float64)
    for n in range(4):
        for m in range(4):
            for l in range(4):
                out += (wz[:, n] * wy[:, m] * wx[:, l])[:, None] * g[iz + n, iy + m, ix + l]
    return out
