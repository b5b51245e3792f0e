"""Pins for the oracle's forward BSI (Eq. 1, Sec. 2.1) and its lerp form (Sec. 3.3).

Independent of the oracle's own formula: polynomial reproduction fixed by the
B-spline moments, scipy's spline evaluator, the delta = 1 filter [1 4 1]/6, the
delta = 2 half-way weights (1, 23, 23, 1)/48, and a brute-force sum over all
control points with the centred kernel.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle
import workloads
from oracle import brute


def _rand_grid(dims, spacing, seed, sigma=2.0):
    return workloads.random_grid(dims, spacing, sigma, seed)


def _positions(dims, spacing):
    """Per-axis control-point positions in voxels: storage index a sits at (a-1)*d."""
    g = oracle.grid_dims(dims, spacing)
    return [(np.arange(g[i]) - 1.0) * spacing[i] for i in range(3)]


def test_constant_grid_gives_constant_field():
    dims, spacing = (13, 9, 11), (3, 2, 4)
    gshape = workloads.grid_shape(dims, spacing)
    grid = np.empty(gshape, np.float32)
    grid[...] = np.array([1.25, -3.5, 0.75], np.float32)
    f = oracle.forward(grid, dims, spacing)
    np.testing.assert_allclose(f, np.broadcast_to([1.25, -3.5, 0.75], f.shape), rtol=0, atol=1e-14)


@pytest.mark.parametrize("dims,spacing", [((17, 11, 9), (5, 3, 4)), ((8, 8, 8), (1, 1, 1)), ((10, 7, 12), (7, 2, 3))])
def test_polynomial_reproduction(dims, spacing):
    # phi_a = P(position) for P of degree <= 3 reproduces, per axis, t -> t (linear),
    # t^2 -> t^2 + d^2/3 and t^3 -> t^3 + d^2 t, where t is the voxel coordinate:
    # the moments of the cubic B-spline scaled by the spacing.
    px, py, pz = _positions(dims, spacing)
    Z, Y, X = np.meshgrid(pz, py, px, indexing="ij")
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    dx, dy, dz = spacing
    grid = np.stack([0.5 * X - 0.25 * Y + 2.0 * Z + 1.0,
                     X * X + Y * Z,
                     X ** 3 - Z * Z], axis=-1)
    f = oracle.forward(grid, dims, spacing)
    expect = np.stack([0.5 * x - 0.25 * y + 2.0 * z + 1.0,
                       x * x + dx * dx / 3.0 + y * z,
                       x ** 3 + dx * dx * x - (z * z + dz * dz / 3.0)], axis=-1)
    np.testing.assert_allclose(f, expect, rtol=1e-13, atol=1e-10)


@pytest.mark.parametrize("dims,spacing", [((19, 14, 11), (5, 4, 3)), ((16, 16, 16), (5, 5, 5)), ((7, 9, 5), (2, 3, 1))])
def test_scipy_map_coordinates(dims, spacing):
    # scipy evaluates sum_a c_a beta3(t - a) (order 3, no prefilter) at t = x/d + 1.
    grid = _rand_grid(dims, spacing, seed=11).astype(np.float64)
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    coords = np.stack([z / spacing[2] + 1.0, y / spacing[1] + 1.0, x / spacing[0] + 1.0])
    f = oracle.forward(grid, dims, spacing)
    for c in range(3):
        ref = ndimage.map_coordinates(grid[..., c], coords, order=3, prefilter=False, mode="nearest")
        np.testing.assert_allclose(f[..., c], ref, rtol=0, atol=1e-12)


def test_delta_one_is_141_filter():
    dims, spacing = (9, 7, 6), (1, 1, 1)
    grid = _rand_grid(dims, spacing, seed=3).astype(np.float64)
    k = np.array([1.0, 4.0, 1.0]) / 6.0
    ref = grid
    for axis in (0, 1, 2):  # z, y, x of the (gz, gy, gx, 3) array; voxel x reads a = x..x+3
        ref = k[0] * np.take(ref, range(0, ref.shape[axis] - 2), axis=axis) \
            + k[1] * np.take(ref, range(1, ref.shape[axis] - 1), axis=axis) \
            + k[2] * np.take(ref, range(2, ref.shape[axis]), axis=axis)
    nx, ny, nz = dims
    np.testing.assert_allclose(oracle.forward(grid, dims, spacing), ref[:nz, :ny, :nx], rtol=0, atol=1e-13)


def test_delta_two_halfway_weights():
    # 1-D along x (ny = nz = 1): odd voxels sit half-way in a tile, weights (1, 23, 23, 1)/48.
    dims, spacing = (12, 1, 1), (2, 1, 1)
    grid = _rand_grid(dims, spacing, seed=5).astype(np.float64)
    f = oracle.forward(grid, dims, spacing)
    # y and z are at node positions: weights (1, 4, 1)/6 on rows 0..2
    row = (grid[0] + 4 * grid[1] + grid[2]) / 6.0
    row = (row[0] + 4 * row[1] + row[2]) / 6.0          # (gx, 3)
    w = np.array([1.0, 23.0, 23.0, 1.0]) / 48.0
    for x in range(1, 12, 2):
        t = x // 2
        np.testing.assert_allclose(f[0, 0, x], w @ row[t:t + 4], rtol=0, atol=1e-13)


@pytest.mark.parametrize("dims,spacing", [((7, 5, 4), (3, 2, 2)), ((6, 6, 3), (4, 5, 1)), ((5, 4, 6), (2, 3, 4))])
def test_brute_force_all_control_points(dims, spacing):
    grid = _rand_grid(dims, spacing, seed=17)
    np.testing.assert_allclose(oracle.forward(grid, dims, spacing), brute.forward(grid, dims, spacing),
                               rtol=0, atol=1e-12)


@pytest.mark.parametrize("dims,spacing", [((23, 17, 12), (5, 3, 4)), ((16, 16, 16), (5, 5, 5)), ((9, 10, 11), (1, 2, 3))])
def test_lerp_form_equals_direct_sum(dims, spacing):
    grid = _rand_grid(dims, spacing, seed=23)
    np.testing.assert_allclose(oracle.forward_lerp(grid, dims, spacing), oracle.forward(grid, dims, spacing),
                               rtol=0, atol=1e-13)


def test_points_match_full_forward():
    dims, spacing = (21, 13, 9), (4, 3, 5)
    grid = _rand_grid(dims, spacing, seed=29)
    f = oracle.forward(grid, dims, spacing)
    rng = np.random.default_rng(0)
    pts = np.stack([rng.integers(0, n, 50) for n in dims], axis=1)
    got = oracle.forward_points(grid, dims, spacing, pts)
    np.testing.assert_array_equal(got, f[pts[:, 2], pts[:, 1], pts[:, 0]])


def test_rejects_bad_geometry():
    with pytest.raises(ValueError):
        oracle.forward(np.zeros((4, 4, 4, 3), np.float32), (0, 1, 1), (1, 1, 1))
    with pytest.raises(ValueError):
        oracle.forward(np.zeros((4, 4, 4, 3), np.float32), (2, 2, 2), (1, 1, 1))
