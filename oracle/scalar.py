"""FP64 scalar BSI: Eq. 1 with one value per control point.

Test infrastructure only (see ``oracle/__init__.py``).

The same operation as the vector forward, with pixels (or voxels) of a coarse
image as the control points: the B-spline upsampling ("image zooming") that the
paper names as the other use of BSI (Sec. 8).  For every voxel,

  out[z][y][x] = sum_{n=0..3} sum_{m=0..3} sum_{l=0..3}
                 Bz_n(w) By_m(v) Bx_l(u) grid[floor(z/dz)+n][floor(y/dy)+m][floor(x/dx)+l]

with u = (x mod dx)/dx etc., the uniform cubic B-spline basis of ``oracle.basis``
and storage index = paper index + 1 (g = ceil(n/d) + 3 points per axis).  The
triple sum is written out term by term; each term is evaluated for all voxels
at once (numpy), in FP64.
"""
import numpy as np

from . import basis, grid_dims


def _axis(n, d):
    """Tile index and the four basis weights of every coordinate 0..n-1."""
    c = np.arange(n)
    t = c // d
    table = np.stack([basis((o % d) / d) for o in range(d)])  # (d, 4)
    return t, table[c % d]


def forward(grid, dims, spacing):
    """Scalar Eq. 1: grid (gz, gy, gx) -> image (nz, ny, nx), FP64."""
    nx, ny, nz = (int(v) for v in dims)
    dx, dy, dz = (int(v) for v in spacing)
    g = np.asarray(grid, dtype=np.float64)
    gx, gy, gz = grid_dims(dims, spacing)
    if g.shape != (gz, gy, gx):
        raise ValueError(f"grid has shape {g.shape}, expected {(gz, gy, gx)}")
    tx, bx = _axis(nx, dx)
    ty, by = _axis(ny, dy)
    tz, bz = _axis(nz, dz)
    out = np.zeros((nz, ny, nx), np.float64)
    for n in range(4):
        for m in range(4):
            for l in range(4):
                w = bz[:, n][:, None, None] * by[:, m][None, :, None] * bx[:, l][None, None, :]
                out += w * g[(tz + n)[:, None, None], (ty + m)[None, :, None], (tx + l)[None, None, :]]
    return out
