"""Pins for the oracle's adjoint (transpose of Eq. 1) and its per-point gather.

The adjoint is not in the paper; it is fixed by linear algebra: the explicit
transpose of a brute-force matrix, the dot-product identity, column sums of a
partition of unity, and the exact interior value d_x d_y d_z of B^T 1.
"""
import numpy as np
import pytest

import oracle
import workloads
from oracle import brute


@pytest.mark.parametrize("dims,spacing", [((6, 5, 4), (3, 2, 2)), ((5, 7, 3), (2, 3, 1)), ((4, 4, 4), (4, 4, 4))])
def test_matches_dense_transpose(dims, spacing):
    M = brute.matrix(dims, spacing)
    dfield = workloads.random_field(dims, 1.0, seed=41)
    g = oracle.adjoint(dfield, dims, spacing)
    ref = np.stack([M.T @ dfield[..., c].reshape(-1).astype(np.float64) for c in range(3)], axis=-1)
    np.testing.assert_allclose(g.reshape(-1, 3), ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("dims,spacing", [((23, 14, 12), (5, 3, 4)), ((12, 12, 12), (5, 5, 5))])
def test_dot_product_identity(dims, spacing):
    x = workloads.random_grid(dims, spacing, 2.0, seed=43)
    y = workloads.random_field(dims, 1.0, seed=44)
    lhs = np.sum(oracle.forward(x, dims, spacing) * y.astype(np.float64))
    rhs = np.sum(x.astype(np.float64) * oracle.adjoint(y, dims, spacing))
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(oracle.forward(x, dims, spacing) * y))


def test_column_sums_equal_total():
    # Each voxel's weights sum to one, so sum_a (B^T y)_a = sum_x y_x.
    dims, spacing = (19, 11, 8), (4, 3, 5)
    y = workloads.random_field(dims, 1.0, seed=45)
    g = oracle.adjoint(y, dims, spacing)
    np.testing.assert_allclose(g.sum(axis=(0, 1, 2)), y.astype(np.float64).sum(axis=(0, 1, 2)), rtol=1e-12)


@pytest.mark.parametrize("spacing", [(5, 5, 5), (3, 4, 2), (1, 1, 1)])
def test_interior_ones_give_cell_volume(spacing):
    # For a control point whose support lies inside the volume, (B^T 1)_a = dx dy dz:
    # the B-spline samples at the d offsets of each of its 4 tiles sum to d per axis.
    dims = tuple(8 * s for s in spacing)
    ones = np.ones(workloads.field_shape(dims), np.float32)
    g = oracle.adjoint(ones, dims, spacing)
    vol = spacing[0] * spacing[1] * spacing[2]
    # storage index a is interior when its 4 tiles a-3..a are inside [0, n/d): a in [3, n/d)
    inner = g[3:dims[2] // spacing[2], 3:dims[1] // spacing[1], 3:dims[0] // spacing[0]]
    assert inner.size > 0
    np.testing.assert_allclose(inner, vol, rtol=0, atol=1e-12 * vol)


def test_points_match_scatter():
    dims, spacing = (22, 15, 13), (5, 4, 3)
    y = workloads.random_field(dims, 1.0, seed=47)
    g = oracle.adjoint(y, dims, spacing)
    gx, gy, gz = oracle.grid_dims(dims, spacing)
    rng = np.random.default_rng(1)
    cps = np.stack([rng.integers(0, gx, 40), rng.integers(0, gy, 40), rng.integers(0, gz, 40)], axis=1)
    cps = np.concatenate([cps, [[0, 0, 0], [gx - 1, gy - 1, gz - 1]]])
    got = oracle.adjoint_points(y, dims, spacing, cps)
    np.testing.assert_allclose(got, g[cps[:, 2], cps[:, 1], cps[:, 0]], rtol=0, atol=1e-12)


def test_finite_differences_of_linear_map():
    # L(phi) = <BSI(phi), y> is linear, so central differences are exact up to rounding.
    case = workloads.cfg3_fd()
    dims, spacing, y = case["dims"], case["spacing"], case["dfield"]
    phi = case["grid"].astype(np.float64)
    g = oracle.adjoint(y, dims, spacing)
    eps = 1e-6
    rng = np.random.default_rng(2)
    idx = [tuple(rng.integers(0, s) for s in phi.shape) for _ in range(30)]
    for i in idx:
        p, m = phi.copy(), phi.copy()
        p[i] += eps
        m[i] -= eps
        fd = (np.sum(oracle.forward(p, dims, spacing) * y) - np.sum(oracle.forward(m, dims, spacing) * y)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-8 * max(1.0, abs(g[i])) + 1e-7


@pytest.mark.parametrize("dims,spacing", [((22, 15, 13), (5, 4, 3)), ((9, 30, 7), (1, 7, 2)), ((40, 3, 19), (64, 1, 5))])
def test_gather_over_every_point_matches_scatter(dims, spacing):
    # The parallel gather (every control point's literal sum over its support) is
    # the raster scatter in another order: equal to FP64 rounding, pinned at
    # every point, with the interior-volume identity checked on the scatter above.
    y = workloads.random_field(dims, 1.0, seed=48 + sum(dims))
    np.testing.assert_allclose(oracle.adjoint_gather(y, dims, spacing), oracle.adjoint(y, dims, spacing),
                               rtol=0, atol=1e-12)
