"""Parity of the scalar forward (Eq. 1 with one value per control point: cubic
B-spline upsampling) against the FP64 scalar oracle.

Bar: max |gpu - oracle| <= 1e-5 * max|grid| (as for the vector forward); the
scalar kernel and the vector kernel perform the same operations per component,
so a scalar result equals that component of bsi_forward bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import paper_2004_05962_amd as bsi
from gpu_util import dev, host, max_abs, say
from oracle import scalar as oscalar

pytestmark = pytest.mark.gpu


def _grid(dims, spacing, seed):
    gx, gy, gz = bsi.bsi_grid_dims(dims, spacing)
    return np.random.default_rng(seed).standard_normal((gz, gy, gx)).astype(np.float32)


CASES = [
    ((64, 64, 64), (4, 4, 4)),
    ((1, 1, 1), (1, 1, 1)),
    ((130, 9, 11), (5, 4, 3)),      # more than one 64-lane strip, ragged tiles
    ((65, 70, 33), (64, 7, 10)),
    ((200, 5, 6), (1, 1, 1)),
    ((96, 80, 1), (3, 5, 1)),       # a 2-D image
]


@pytest.mark.parametrize("dims,spacing", CASES)
def test_scalar_matches_oracle(dims, spacing):
    say("scalar forward", dims, spacing)
    grid = _grid(dims, spacing, seed=sum(dims) + sum(spacing))
    nx, ny, nz = dims
    out = torch.empty((nz, ny, nx), device="cuda")
    bsi.bsi_forward_scalar(dev(grid), dims, spacing, out)
    ref = oscalar.forward(grid, dims, spacing)
    assert max_abs(host(out), ref) <= 1e-5 * float(np.abs(grid).max())


@pytest.mark.parametrize("dims,spacing", [
    ((77, 45, 31), (5, 4, 6)),      # rows not 16-byte aligned: one voxel per lane
    ((300, 21, 17), (4, 5, 3)),     # 4 voxels per lane; a partial second 256-voxel strip
])
def test_scalar_equals_vector_component_bits(dims, spacing):
    say("scalar vs vector component bits", dims, spacing)
    g3 = torch.randn(bsi.grid_shape(dims, spacing), device="cuda")
    f3 = bsi.forward(g3, dims, spacing)
    for c in range(3):
        img = bsi.upsample(g3[..., c].contiguous(), spacing, dims)
        assert torch.equal(img, f3[..., c])


def test_scalar_canary_and_default_dims():
    spacing = (4, 3, 2)
    grid = torch.randn(9, 11, 13, device="cuda")  # gz, gy, gx
    dims = ((13 - 3) * 4, (11 - 3) * 3, (9 - 3) * 2)
    n = dims[0] * dims[1] * dims[2]
    buf = torch.full((n + 1024,), 1.0e30, device="cuda")
    out = buf[:n].view(dims[2], dims[1], dims[0])
    bsi.upsample(grid, spacing, out=out)
    torch.cuda.synchronize()
    assert torch.all(buf[n:] == 1.0e30) and not torch.any(out == 1.0e30)
    ref = oscalar.forward(host(grid), dims, spacing)
    assert max_abs(host(out), ref) <= 1e-5 * float(grid.abs().max())


def test_scalar_full_size_sampled():
    # 128 x 128 x 64 coarse volume upsampled by 4 (output 512 x 512 x 256, 268 MB):
    # sampled voxels against the oracle's point evaluation of the same values
    dims, spacing = (512, 512, 256), (4, 4, 4)
    say("scalar upsampling 512x512x256 sampled")
    grid = _grid(dims, spacing, seed=77)
    img = bsi.upsample(dev(grid), spacing, dims)
    rng = np.random.default_rng(5)
    pts = np.stack([rng.integers(0, n, 4000) for n in dims], axis=1).astype(np.int64)
    pts[:4] = [[0, 0, 0], [511, 511, 255], [511, 0, 255], [0, 511, 0]]
    g3 = np.zeros(grid.shape + (3,), np.float32)
    g3[..., 0] = grid
    ref = oracle.forward_points(g3, dims, spacing, pts)[:, 0]
    got = host(img)[pts[:, 2], pts[:, 1], pts[:, 0]]
    assert np.max(np.abs(got - ref)) <= 1e-5 * float(np.abs(grid).max())


def test_scalar_unaligned_output_same_bits():
    # rows of 4k voxels, but the image starts 4 bytes past a 16-byte boundary:
    # one voxel per lane, same values as the 4-voxels-per-lane path
    dims, spacing = (136, 19, 14), (5, 3, 4)
    say("scalar forward, unaligned output", dims, spacing)
    grid = dev(_grid(dims, spacing, seed=11))
    nx, ny, nz = dims
    n = nx * ny * nz
    aligned = torch.empty((nz, ny, nx), device="cuda")
    bsi.bsi_forward_scalar(grid, dims, spacing, aligned)
    buf = torch.full((n + 2,), 1.0e30, device="cuda")
    out = buf[1:1 + n].view(nz, ny, nx)
    assert out.data_ptr() % 16 == 4
    bsi.bsi_forward_scalar(grid, dims, spacing, out)
    torch.cuda.synchronize()
    assert torch.equal(out, aligned)
    assert bool(buf[0] == 1.0e30) and bool(buf[-1] == 1.0e30)  # float32 canaries untouched
