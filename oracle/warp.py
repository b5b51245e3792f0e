"""FP64 trilinear warp, SSD and its gradient: the registration step around BSI.

Test infrastructure only (see ``oracle/__init__.py``).

Not from the paper, which plugs BSI into NiftyReg's registration loop (Sec. 6); this
is the plain sum-of-squared-differences step that drives the adjoint:

  p(x)   = x + T(x)  per axis, in voxel units (x, y, z index order = field comps)
  W(x)   = moving sampled trilinearly at p, corners aligned, p clamped to [0, n-1]
  L      = sum_x (W(x) - fixed(x))^2
  dL/dT  = 2 (W - fixed) * dW/dp, where dW/dp is the analytic trilinear gradient;
           a coordinate that lies on or beyond the border (p <= 0 or p >= n-1)
           gets zero gradient, and at an exact integer p the cell [p, p+1] is
           used (a right-sided derivative).  This matches grid_sample's
           'border' padding with align_corners=True.

``coord_dtype`` is the precision in which x + T is formed; the GPU forms it in
FP32, so a parity check passes ``np.float32`` to take the same cell decisions.
Everything after the coordinate is FP64.
"""
import numpy as np


def _axis(coord_raw, n):
    """Cell index, fraction and gradient mask along one axis."""
    p = coord_raw.astype(np.float64)
    mask = (p > 0.0) & (p < n - 1)
    p = np.clip(p, 0.0, n - 1)
    if n >= 2:
        i0 = np.minimum(np.floor(p), n - 2).astype(np.int64)
        f = p - i0
        i1 = i0 + 1
    else:
        i0 = np.zeros(p.shape, np.int64)
        i1 = i0
        f = np.zeros(p.shape)
        mask = np.zeros(p.shape, bool)
    return i0, i1, f, mask


def _coords(field, coord_dtype):
    nz, ny, nx, _ = field.shape
    t = np.asarray(field)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    if coord_dtype == np.float32:
        t32 = t.astype(np.float32)
        px = xx.astype(np.float32) + t32[..., 0]
        py = yy.astype(np.float32) + t32[..., 1]
        pz = zz.astype(np.float32) + t32[..., 2]
    else:
        t64 = t.astype(np.float64)
        px, py, pz = xx + t64[..., 0], yy + t64[..., 1], zz + t64[..., 2]
    return px, py, pz


def _sample(image, field, coord_dtype):
    m = np.asarray(image, dtype=np.float64)
    nz, ny, nx = m.shape
    px, py, pz = _coords(field, coord_dtype)
    x0, x1, fx, mx = _axis(px, nx)
    y0, y1, fy, my = _axis(py, ny)
    z0, z1, fz, mz = _axis(pz, nz)
    c = {}
    for a, zi in (("0", z0), ("1", z1)):
        for b, yi in (("0", y0), ("1", y1)):
            for d, xi in (("0", x0), ("1", x1)):
                c[a + b + d] = m[zi, yi, xi]
    gx, gy, gz = 1.0 - fx, 1.0 - fy, 1.0 - fz
    W = (gz * (gy * (gx * c["000"] + fx * c["001"]) + fy * (gx * c["010"] + fx * c["011"]))
         + fz * (gy * (gx * c["100"] + fx * c["101"]) + fy * (gx * c["110"] + fx * c["111"])))
    dWdx = (gz * (gy * (c["001"] - c["000"]) + fy * (c["011"] - c["010"]))
            + fz * (gy * (c["101"] - c["100"]) + fy * (c["111"] - c["110"])))
    dWdy = (gz * (gx * (c["010"] - c["000"]) + fx * (c["011"] - c["001"]))
            + fz * (gx * (c["110"] - c["100"]) + fx * (c["111"] - c["101"])))
    dWdz = (gy * (gx * (c["100"] - c["000"]) + fx * (c["101"] - c["001"]))
            + fy * (gx * (c["110"] - c["010"]) + fx * (c["111"] - c["011"])))
    return W, (dWdx * mx, dWdy * my, dWdz * mz)


def warp(image, field, coord_dtype=np.float64):
    """moving(x + T(x)) with trilinear interpolation and border clamping; FP64."""
    W, _ = _sample(image, field, coord_dtype)
    return W


def ssd_grad(field, moving, fixed, coord_dtype=np.float64):
    """Return (L, dL/dT) with L = sum (W - fixed)^2 in FP64 and dL/dT (nz,ny,nx,3) FP64."""
    W, (gx, gy, gz) = _sample(moving, field, coord_dtype)
    r = W - np.asarray(fixed, dtype=np.float64)
    loss = float(np.sum(r * r))
    dT = np.stack([2.0 * r * gx, 2.0 * r * gy, 2.0 * r * gz], axis=-1)
    return loss, dT
