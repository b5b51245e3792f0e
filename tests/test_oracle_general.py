"""Pins for the oracle of BSI with real spacing and an origin offset (the
generalisation of the aligned, integer-spacing grid that Sec. 8 names as the
method's limitation).

Independent of its own sums: the aligned oracle for integer spacing and zero
origin, scipy's cubic B-spline evaluator at the coordinate (x - o)/s + 1 of
every voxel, the adjoint (dot-product) identity, and the grid-size formula."""
import numpy as np
import pytest
from scipy import ndimage

import oracle
import workloads
from oracle import general


def _grid(dims, spacing, origin, seed):
    gx, gy, gz = general.grid_dims(dims, spacing, origin)
    return np.random.default_rng(seed).standard_normal((gz, gy, gx, 3))


def test_integer_spacing_zero_origin_is_the_aligned_case():
    dims, spacing = (17, 12, 9), (4, 3, 2)
    assert general.grid_dims(dims, spacing, (0, 0, 0)) == oracle.grid_dims(dims, spacing)
    g = workloads.random_grid(dims, spacing, 2.0, seed=8).astype(np.float64)
    np.testing.assert_allclose(general.forward(g, dims, spacing, (0, 0, 0)), oracle.forward(g, dims, spacing),
                               rtol=0, atol=1e-12)
    d = np.random.default_rng(3).standard_normal((9, 12, 17, 3))
    np.testing.assert_allclose(general.adjoint(d, dims, spacing, (0, 0, 0)), oracle.adjoint(d, dims, spacing),
                               rtol=0, atol=1e-11)


@pytest.mark.parametrize("spacing,origin", [((2.5, 3.25, 1.75), (-0.5, 0.0, -1.25)),
                                            ((1.0, 4.5, 6.125), (-0.25, -4.0, -3.0)),
                                            ((3.3, 1.1, 2.2), (-1.7, -0.9, 0.0))])
def test_matches_scipy_spline(spacing, origin):
    dims = (19, 14, 11)
    g = _grid(dims, spacing, origin, seed=5)
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    s = [float(np.float32(v)) for v in spacing]
    o = [float(np.float32(v)) for v in origin]
    coords = np.stack([(z - o[2]) / s[2] + 1.0, (y - o[1]) / s[1] + 1.0, (x - o[0]) / s[0] + 1.0])
    f = general.forward(g, dims, spacing, origin)
    for c in range(3):
        ref = ndimage.map_coordinates(g[..., c], coords, order=3, prefilter=False, mode="nearest")
        np.testing.assert_allclose(f[..., c], ref, rtol=0, atol=1e-12)


def test_adjoint_identity():
    dims, spacing, origin = (13, 10, 8), (2.75, 1.5, 3.5), (-1.0, -0.5, -2.25)
    g = _grid(dims, spacing, origin, seed=7)
    d = np.random.default_rng(9).standard_normal((8, 10, 13, 3))
    lhs = float(np.sum(general.forward(g, dims, spacing, origin) * d))
    rhs = float(np.sum(g * general.adjoint(d, dims, spacing, origin)))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)


def test_grid_dims_formula_and_checks():
    # last voxel n-1 must still have its window i..i+3 inside the grid
    for n, s, o in [(100, 3.7, -1.2), (64, 1.0, 0.0), (10, 9.99, -9.5), (7, 2.0, -1.999)]:
        (g, _, _) = general.grid_dims((n, 1, 1), (s, 1, 1), (o, 0, 0))
        i_last = int(np.floor((n - 1 - np.float32(o)) / np.float32(s)))
        assert g == i_last + 4
    with pytest.raises(ValueError):
        general.grid_dims((10, 1, 1), (2.0, 1, 1), (0.5, 0, 0))
    with pytest.raises(ValueError):
        general.grid_dims((10, 1, 1), (0.5, 1, 1), (0, 0, 0))


def test_points_match_full_forward():
    dims, spacing, origin = (15, 11, 9), (2.6, 1.3, 3.9), (-2.0, -0.3, 0.0)
    g = _grid(dims, spacing, origin, seed=11)
    f = general.forward(g, dims, spacing, origin)
    rng = np.random.default_rng(1)
    pts = np.stack([rng.integers(0, n, 50) for n in dims], axis=1)
    np.testing.assert_allclose(general.forward_points(g, dims, spacing, origin, pts),
                               f[pts[:, 2], pts[:, 1], pts[:, 0]], rtol=0, atol=1e-13)
