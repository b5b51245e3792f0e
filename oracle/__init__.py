"""FP64 CPU oracle for cubic B-spline interpolation (BSI) and the SSD registration step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code with
the HIP library in ``paper_2004_05962_amd`` and never imports it.

Contents
  * ``bsi_oracle.c`` (wrapped here): Eq. 1 of Sec. 2.1 as a literal FP64 triple
    sum, its transpose as an FP64 scatter, a per-control-point gather of the
    transpose, and the trilinear (lerp) reformulation of Sec. 3.3 / App. B.
  * ``brute.py``: the same map written as a sum over *all* control points with the
    centred cubic B-spline kernel (no tiles, no floor) for tiny cases.
  * ``warp.py``: trilinear warp, SSD and its gradient (not from the paper; the
    registration step that drives the adjoint).
  * ``registration.py``: gradient-descent loop built from the pieces above.

Array conventions: grid ``(gz, gy, gx, 3)``, field ``(nz, ny, nx, 3)``;
``dims = (nx, ny, nz)``, ``spacing = (dx, dy, dz)`` integers >= 1 in voxels;
``g = ceil(n/d) + 3`` per axis.  Inputs may be FP32 (the arrays the GPU receives,
promoted exactly) or FP64; all arithmetic and outputs are FP64.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        lib = ctypes.CDLL(path)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        lib.oracle_basis.argtypes = [ctypes.c_double, f64p]
        lib.oracle_basis.restype = None
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_num_threads.restype = None
        for name in ("oracle_forward", "oracle_forward_lerp"):
            getattr(lib, name).argtypes = [f64p, i32p, i32p, f64p]
            getattr(lib, name).restype = ctypes.c_int
        lib.oracle_adjoint.argtypes = [f64p, i32p, i32p, f64p]
        lib.oracle_adjoint.restype = ctypes.c_int
        for name in ("oracle_forward_points", "oracle_adjoint_points"):
            getattr(lib, name).argtypes = [f64p, i32p, i32p, i64p, ctypes.c_int64, f64p]
            getattr(lib, name).restype = ctypes.c_int
        _LIB = lib
    return _LIB


def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads for the oracle's later OpenMP loops."""
    _lib().oracle_set_num_threads(int(n))


def grid_dims(dims, spacing):
    """Control points per axis (gx, gy, gz) = ceil(n/d) + 3."""
    return tuple(-(-int(n) // int(d)) + 3 for n, d in zip(dims, spacing))


def basis(u: float) -> np.ndarray:
    """Uniform cubic B-spline basis (B0..B3) at local coordinate u."""
    out = np.zeros(4, np.float64)
    _lib().oracle_basis(float(u), out)
    return out


def _geom(dims, spacing):
    d = np.ascontiguousarray(dims, dtype=np.int32)
    s = np.ascontiguousarray(spacing, dtype=np.int32)
    if d.shape != (3,) or s.shape != (3,) or (d < 1).any() or (s < 1).any():
        raise ValueError("dims and spacing must be three integers >= 1")
    return d, s


def _check_grid(grid, dims, spacing):
    gx, gy, gz = grid_dims(dims, spacing)
    g = np.ascontiguousarray(grid, dtype=np.float64)
    if g.shape != (gz, gy, gx, 3):
        raise ValueError(f"grid shape {g.shape} != {(gz, gy, gx, 3)}")
    return g


def _check_field(field, dims):
    nx, ny, nz = (int(v) for v in dims)
    f = np.ascontiguousarray(field, dtype=np.float64)
    if f.shape != (nz, ny, nx, 3):
        raise ValueError(f"field shape {f.shape} != {(nz, ny, nx, 3)}")
    return f


def forward(grid, dims, spacing) -> np.ndarray:
    """Eq. 1 evaluated at every voxel: FP64 field of shape (nz, ny, nx, 3)."""
    d, s = _geom(dims, spacing)
    g = _check_grid(grid, dims, spacing)
    out = np.empty((int(d[2]), int(d[1]), int(d[0]), 3), np.float64)
    if _lib().oracle_forward(g, d, s, out) != 0:
        raise RuntimeError("oracle_forward failed")
    return out


def forward_lerp(grid, dims, spacing) -> np.ndarray:
    """Eq. 1 through the trilinear reformulation of Sec. 3.3 (9 x 7 lerps per value)."""
    d, s = _geom(dims, spacing)
    g = _check_grid(grid, dims, spacing)
    out = np.empty((int(d[2]), int(d[1]), int(d[0]), 3), np.float64)
    if _lib().oracle_forward_lerp(g, d, s, out) != 0:
        raise RuntimeError("oracle_forward_lerp failed")
    return out


def forward_points(grid, dims, spacing, pts) -> np.ndarray:
    """Eq. 1 at voxels pts[k] = (x, y, z); returns (k, 3) FP64."""
    d, s = _geom(dims, spacing)
    g = _check_grid(grid, dims, spacing)
    p = np.ascontiguousarray(pts, dtype=np.int64).reshape(-1, 3)
    out = np.empty((p.shape[0], 3), np.float64)
    if _lib().oracle_forward_points(g, d, s, p, p.shape[0], out) != 0:
        raise ValueError("voxel out of range")
    return out


def adjoint(dfield, dims, spacing) -> np.ndarray:
    """Transpose of Eq. 1 applied to dfield: FP64 gradient of shape (gz, gy, gx, 3)."""
    d, s = _geom(dims, spacing)
    f = _check_field(dfield, dims)
    gx, gy, gz = grid_dims(dims, spacing)
    out = np.empty((gz, gy, gx, 3), np.float64)
    if _lib().oracle_adjoint(f, d, s, out) != 0:
        raise RuntimeError("oracle_adjoint failed")
    return out


def adjoint_points(dfield, dims, spacing, cps) -> np.ndarray:
    """Adjoint at control points cps[k] = (cx, cy, cz), by direct gather; (k, 3) FP64."""
    d, s = _geom(dims, spacing)
    f = _check_field(dfield, dims)
    p = np.ascontiguousarray(cps, dtype=np.int64).reshape(-1, 3)
    out = np.empty((p.shape[0], 3), np.float64)
    if _lib().oracle_adjoint_points(f, d, s, p, p.shape[0], out) != 0:
        raise ValueError("control point out of range")
    return out


def adjoint_gather(dfield, dims, spacing) -> np.ndarray:
    """Transpose of Eq. 1 by the per-control-point gather (``adjoint_points`` over
    every control point, spread over OpenMP threads): the same sums as ``adjoint``
    in another order; FP64 gradient of shape (gz, gy, gx, 3)."""
    gx, gy, gz = grid_dims(dims, spacing)
    cz, cy, cx = np.meshgrid(np.arange(gz), np.arange(gy), np.arange(gx), indexing="ij")
    cps = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)
    return adjoint_points(dfield, dims, spacing, cps).reshape(gz, gy, gx, 3)


from . import brute, general, warp, registration, scalar  # noqa: E402,F401
