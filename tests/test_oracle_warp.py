"""Pins for the oracle's trilinear warp and SSD gradient (the registration step).

Not from the paper; pinned to torch.nn.functional.grid_sample in float64 on the
CPU (5-D 'bilinear' is trilinear; align_corners=True; padding_mode='border') and
to its autograd for dL/dT.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import warp


def _grid_sample_ref(moving, field, fixed):
    nz, ny, nx = moving.shape
    m = torch.tensor(moving, dtype=torch.float64)[None, None]
    T = torch.tensor(field, dtype=torch.float64, requires_grad=True)
    z, y, x = torch.meshgrid(torch.arange(nz, dtype=torch.float64), torch.arange(ny, dtype=torch.float64),
                             torch.arange(nx, dtype=torch.float64), indexing="ij")
    px, py, pz = x + T[..., 0], y + T[..., 1], z + T[..., 2]
    g = torch.stack([2 * px / (nx - 1) - 1, 2 * py / (ny - 1) - 1, 2 * pz / (nz - 1) - 1], dim=-1)[None]
    W = torch.nn.functional.grid_sample(m, g, mode="bilinear", padding_mode="border", align_corners=True)[0, 0]
    loss = ((W - torch.tensor(fixed, dtype=torch.float64)) ** 2).sum()
    loss.backward()
    return W.detach().numpy(), float(loss.detach()), T.grad.numpy()


@pytest.mark.parametrize("shape,sigma", [((7, 9, 11), 1.5), ((6, 5, 8), 4.0)])
def test_matches_grid_sample(shape, sigma):
    nz, ny, nx = shape
    rng = np.random.default_rng(3)
    moving = rng.standard_normal(shape)
    fixed = rng.standard_normal(shape)
    # displacements large enough that many samples fall outside and get clamped
    field = rng.standard_normal(shape + (3,)) * sigma
    W_ref, L_ref, dT_ref = _grid_sample_ref(moving, field, fixed)
    np.testing.assert_allclose(warp.warp(moving, field), W_ref, rtol=0, atol=1e-12)
    L, dT = warp.ssd_grad(field, moving, fixed)
    assert abs(L - L_ref) <= 1e-12 * L_ref
    np.testing.assert_allclose(dT, dT_ref, rtol=0, atol=1e-11)


def test_zero_field_is_identity():
    img = workloads.blobs((10, 8, 6), 5, seed=1)
    W = warp.warp(img, np.zeros(img.shape + (3,)))
    np.testing.assert_array_equal(W, img.astype(np.float64))


def test_integer_shift_moves_image():
    img = np.random.default_rng(4).standard_normal((6, 7, 9))
    field = np.zeros(img.shape + (3,))
    field[..., 0] = 2.0     # sample two voxels to the right
    field[..., 2] = -1.0    # and one plane back
    W = warp.warp(img, field)
    np.testing.assert_allclose(W[1:, :, :-2], img[:-1, :, 2:], rtol=0, atol=1e-15)


def test_fp32_coordinates_agree_away_from_cell_edges():
    rng = np.random.default_rng(5)
    img = rng.standard_normal((8, 8, 8))
    field = (rng.standard_normal((8, 8, 8, 3)) * 2.0).astype(np.float32)
    a = warp.warp(img, field, coord_dtype=np.float32)
    b = warp.warp(img, field, coord_dtype=np.float64)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-5)
