"""Pins for the scalar oracle (Eq. 1 with one value per control point: B-spline
upsampling, the other application the paper names in Sec. 8).

Independent of its own triple sum: scipy's cubic B-spline evaluator
(``ndimage.map_coordinates``, order 3, no prefilter) on the coarse image, the
vector oracle one component at a time, the brute-force sum over all control
points, and reproduction of a linear ramp (the B-spline moments)."""
import numpy as np
import pytest
from scipy import ndimage

import oracle
import workloads
from oracle import brute, scalar


def _grid(dims, spacing, seed):
    gx, gy, gz = oracle.grid_dims(dims, spacing)
    return np.random.default_rng(seed).standard_normal((gz, gy, gx))


@pytest.mark.parametrize("dims,spacing", [((13, 9, 11), (3, 2, 4)), ((20, 7, 5), (5, 1, 2)), ((4, 4, 4), (4, 4, 4))])
def test_scalar_matches_scipy_spline(dims, spacing):
    grid = _grid(dims, spacing, seed=sum(dims))
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    coords = np.stack([z / spacing[2] + 1.0, y / spacing[1] + 1.0, x / spacing[0] + 1.0])
    ref = ndimage.map_coordinates(grid, coords, order=3, prefilter=False, mode="nearest")
    np.testing.assert_allclose(scalar.forward(grid, dims, spacing), ref, rtol=0, atol=1e-12)


def test_scalar_is_each_component_of_the_vector_oracle():
    dims, spacing = (17, 12, 9), (4, 3, 2)
    g3 = workloads.random_grid(dims, spacing, 2.0, seed=8).astype(np.float64)
    f3 = oracle.forward(g3, dims, spacing)
    for c in range(3):
        np.testing.assert_allclose(scalar.forward(g3[..., c], dims, spacing), f3[..., c], rtol=0, atol=1e-12)


def test_scalar_matches_brute_force():
    dims, spacing = (6, 5, 4), (2, 3, 2)
    grid = _grid(dims, spacing, seed=2)
    g3 = np.zeros(grid.shape + (3,))
    g3[..., 0] = grid
    ref = brute.forward(g3, dims, spacing)[..., 0]
    np.testing.assert_allclose(scalar.forward(grid, dims, spacing), ref, rtol=0, atol=1e-12)


def test_scalar_reproduces_a_linear_ramp():
    # control value a*(index-1)*d + b at each point reproduces a*x + b exactly
    dims, spacing = (23, 6, 5), (5, 2, 3)
    gx, gy, gz = oracle.grid_dims(dims, spacing)
    pos = (np.arange(gx) - 1.0) * spacing[0]
    grid = np.broadcast_to(0.75 * pos - 2.0, (gz, gy, gx))
    out = scalar.forward(grid, dims, spacing)
    np.testing.assert_allclose(out, np.broadcast_to(0.75 * np.arange(dims[0]) - 2.0, out.shape), rtol=0, atol=1e-12)
