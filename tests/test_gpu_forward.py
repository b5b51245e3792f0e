"""Parity of the HIP forward BSI (Eq. 1) against the FP64 oracle.

Bar: max |gpu - oracle| <= 1e-5 * max|grid| (FP32 against FP64), on every voxel
for volumes the oracle finishes in seconds (several tiles, ragged tails, odd
spacings) and at the 512 x 512 x 256 sizes the benchmark times, plus
size-independent properties.  Reruns are bit-identical."""
import numpy as np
import pytest
import torch

import oracle
import paper_2004_05962_amd as bsi
import workloads
from gpu_util import dev, host, max_abs, say

pytestmark = pytest.mark.gpu

CASES = [
    ((64, 64, 64), (5, 5, 5)),        # workload 1
    ((1, 1, 1), (1, 1, 1)),
    ((1, 1, 1), (64, 64, 64)),
    ((7, 3, 2), (2, 3, 1)),
    ((130, 9, 11), (5, 4, 3)),        # x beyond one 64-lane strip, ragged tiles
    ((65, 70, 33), (64, 7, 10)),      # largest spacing on x
    ((200, 5, 6), (1, 1, 1)),
    ((33, 17, 129), (8, 3, 6)),
    ((96, 80, 72), (3, 5, 8)),
    ((272, 7, 9), (5, 3, 4)),         # rows of 64-byte multiples, ragged strips and rows (4 x 1)
    ((272, 7, 12), (5, 3, 5)),        # the same with 5-plane z-tiles: 2 rows x 8 strips, 5 strips idle
    ((528, 3, 13), (7, 2, 6)),        # 2 x 8, a second workgroup in x
    ((510, 6, 7), (5, 5, 5)),         # rows off 64-byte boundaries: edge stores on every strip
]


def _tol(grid):
    return 1e-5 * float(np.abs(grid).max())


@pytest.mark.parametrize("dims,spacing", CASES)
def test_forward_matches_oracle(dims, spacing):
    say("forward", dims, spacing)
    grid = workloads.random_grid(dims, spacing, 2.0, seed=100 + sum(dims) + 7 * sum(spacing))
    if dims == (64, 64, 64):
        grid = workloads.cfg1()["grid"]
    got = host(bsi.forward(dev(grid), dims, spacing))
    ref = oracle.forward(grid, dims, spacing)
    assert got.shape == ref.shape
    assert max_abs(got, ref) <= _tol(grid)


def test_forward_canary_and_rerun_bits():
    dims, spacing = (77, 45, 31), (5, 4, 6)
    say("forward canary", dims, spacing)
    grid = dev(workloads.random_grid(dims, spacing, 2.0, seed=5))
    n = int(np.prod(bsi.field_shape(dims)))
    buf = torch.full((n + 4096,), 1.0e30, dtype=torch.float32, device="cuda")
    field = buf[:n].view(bsi.field_shape(dims))
    bsi.forward(grid, dims, spacing, out=field)
    again = bsi.forward(grid, dims, spacing)
    torch.cuda.synchronize()
    assert torch.all(buf[n:] == 1.0e30), "kernel wrote past the field"
    assert not torch.any(field == 1.0e30), "kernel left voxels unwritten"
    assert torch.equal(field, again)


@pytest.mark.parametrize("shift", [1, 2, 3])
@pytest.mark.parametrize("dims", [(77, 45, 31), (128, 8, 6), (320, 6, 5)])
def test_forward_unaligned_field_pointer(shift, dims):
    """A field that starts 4, 8 or 12 bytes past a 16-byte boundary: the same
    bits as an aligned field, and nothing written outside it."""
    spacing = (5, 4, 6)
    say("forward unaligned field", dims, spacing, shift)
    grid = dev(workloads.random_grid(dims, spacing, 2.0, seed=6))
    n = int(np.prod(bsi.field_shape(dims)))
    buf = torch.full((n + 64,), 1.0e30, dtype=torch.float32, device="cuda")
    field = buf[shift:shift + n].view(bsi.field_shape(dims))
    assert field.data_ptr() % 16 == 4 * shift
    bsi.forward(grid, dims, spacing, out=field)
    aligned = bsi.forward(grid, dims, spacing)
    torch.cuda.synchronize()
    assert torch.all(buf[:shift] == 1.0e30) and torch.all(buf[shift + n:] == 1.0e30)
    assert torch.equal(field, aligned)


@pytest.mark.parametrize("delta", workloads.CFG2_SPACINGS)
def test_forward_clinical_size_every_voxel(delta):
    """The benchmark's volume (512 x 512 x 256) at spacings 3, 5 and 8, launched as
    bsi_forward launches it there, against the FP64 oracle on every voxel (the
    accuracy study of Sec. 5.4 compares whole outputs)."""
    case = workloads.cfg2(delta)
    dims, spacing, grid = case["dims"], case["spacing"], case["grid"]
    say("forward 512x512x256 delta", delta, "every voxel")
    g = dev(grid)
    field = bsi.forward(g, dims, spacing)
    got = host(field)
    ref = oracle.forward(grid, dims, spacing)
    err = max_abs(got, ref)
    mean = float(np.mean(np.abs(got - ref)))
    print(f"forward 512x512x256 d{delta}: max err {err:.3e} mean err {mean:.3e}")
    assert err <= _tol(grid)
    del ref, got
    assert bool(torch.isfinite(field).all())
    again = bsi.forward(g, dims, spacing)
    assert torch.equal(field, again)


def test_linear_grid_reproduced_at_full_size():
    # Property at any size: a grid sampled from a linear function of position
    # (control point a at voxel (a-1)*d) gives that linear function exactly.
    dims, spacing = workloads.CFG2_DIMS, (5, 5, 5)
    say("forward linear reproduction 512x512x256")
    gz, gy, gx, _ = bsi.grid_shape(dims, spacing)
    Z, Y, X = torch.meshgrid(*[(torch.arange(n, dtype=torch.float64, device="cuda") - 1) * 5 for n in (gz, gy, gx)],
                             indexing="ij")
    grid = torch.stack([0.01 * X + 0.5, -0.02 * Y + 0.003 * Z, 0.004 * X + 0.002 * Y - 0.001 * Z], -1).float()
    field = bsi.forward(grid.contiguous(), dims, spacing)
    z, y, x = torch.meshgrid(*[torch.arange(n, dtype=torch.float64, device="cuda") for n in (dims[2], dims[1], dims[0])],
                             indexing="ij")
    expect = torch.stack([0.01 * x + 0.5, -0.02 * y + 0.003 * z, 0.004 * x + 0.002 * y - 0.001 * z], -1)
    err = (field.double() - expect).abs().max().item()
    assert err <= 1e-5 * grid.abs().max().item()


def test_rejects_bad_tensors():
    say("forward argument checks")
    dims, spacing = (10, 10, 10), (5, 5, 5)
    g = torch.zeros(bsi.grid_shape(dims, spacing), device="cuda")
    with pytest.raises(ValueError):
        bsi.forward(g[:, :, :-1], dims, spacing)
    with pytest.raises(TypeError):
        bsi.forward(g.double(), dims, spacing)
    with pytest.raises(ValueError):
        bsi.forward(g.cpu(), dims, spacing)


@pytest.mark.parametrize("dims,spacing", CASES)
def test_lerp_form_matches_oracle(dims, spacing):
    """The lerp-form kernel (Sec. 3.3 / App. B) against the direct FP64 sum and
    the oracle's own lerp form, at the forward's bar."""
    say("forward lerp form", dims, spacing)
    grid = workloads.random_grid(dims, spacing, 2.0, seed=300 + sum(dims) + 7 * sum(spacing))
    out = torch.empty(bsi.field_shape(dims), device="cuda")
    bsi.bsi_forward_lerp(dev(grid), dims, spacing, out)
    got = host(out)
    assert max_abs(got, oracle.forward(grid, dims, spacing)) <= _tol(grid)
    assert max_abs(got, oracle.forward_lerp(grid, dims, spacing)) <= _tol(grid)
