"""Parity of BSI with real spacing and an origin offset (forward and its
separable adjoint) against the FP64 general oracle.

Bars as for the aligned kernels: forward max-abs <= 1e-5 * max|grid|, adjoint
max-abs <= 1e-5 * max|oracle grad|; the adjoint identity <Bx, y> = <x, B^T y>
with the GPU pair, accumulated in FP64 on the host."""
import numpy as np
import pytest
import torch

import paper_2004_05962_amd as bsi
from gpu_util import dev, host, max_abs, say
from oracle import general

pytestmark = pytest.mark.gpu

CASES = [
    ((64, 48, 40), (4.7, 5.3, 5.1), (-1.5, 0.0, -2.25)),
    ((37, 29, 23), (2.5, 3.25, 1.75), (-0.5, -3.0, -1.25)),
    ((130, 9, 11), (1.0, 2.2, 3.3), (0.0, -1.1, -0.2)),      # unit spacing in x, several strips
    ((70, 45, 20), (63.5, 7.75, 10.0), (-63.0, -2.5, -9.5)),  # very coarse x
    ((20, 20, 20), (4.0, 4.0, 4.0), (0.0, 0.0, 0.0)),         # integer and aligned
    ((192, 9, 7), (5.5, 2.0, 3.0), (-1.0, 0.0, -0.5)),        # rows of 64-byte multiples, 3 strips
]


def _grid(dims, spacing, origin, seed):
    gx, gy, gz = bsi.bsi_general_grid_dims(dims, spacing, origin)
    return np.random.default_rng(seed).standard_normal((gz, gy, gx, 3)).astype(np.float32)


@pytest.mark.parametrize("dims,spacing,origin", CASES)
def test_general_forward_matches_oracle(dims, spacing, origin):
    say("general forward", dims, spacing, origin)
    grid = _grid(dims, spacing, origin, seed=sum(dims))
    out = torch.empty(bsi.field_shape(dims), device="cuda")
    bsi.bsi_forward_general(dev(grid), dims, spacing, origin, out)
    ref = general.forward(grid, dims, spacing, origin)
    assert max_abs(host(out), ref) <= 1e-5 * float(np.abs(grid).max())


def _adjoint(d, dims, spacing, origin):
    out = torch.empty(bsi.general_grid_shape(dims, spacing, origin), device="cuda")
    ws = torch.empty(bsi.bsi_adjoint_general_workspace_size(dims, spacing, origin), dtype=torch.uint8,
                     device="cuda")
    bsi.bsi_adjoint_general(d, dims, spacing, origin, out, ws)
    return out


@pytest.mark.parametrize("dims,spacing,origin", CASES)
def test_general_adjoint_matches_oracle(dims, spacing, origin):
    say("general adjoint", dims, spacing, origin)
    nx, ny, nz = dims
    d = np.random.default_rng(7 + nx).standard_normal((nz, ny, nx, 3)).astype(np.float32)
    got = host(_adjoint(dev(d), dims, spacing, origin))
    ref = general.adjoint(d, dims, spacing, origin)
    assert max_abs(got, ref) <= 1e-5 * float(np.abs(ref).max())


def test_general_adjoint_identity_and_rerun_bits():
    dims, spacing, origin = (96, 80, 72), (4.3, 5.6, 3.1), (-2.0, -0.7, -1.0)
    say("general adjoint identity", dims)
    x = torch.from_numpy(_grid(dims, spacing, origin, seed=3)).cuda()
    y = torch.randn(bsi.field_shape(dims), device="cuda")
    bx = torch.empty(bsi.field_shape(dims), device="cuda")
    bsi.bsi_forward_general(x, dims, spacing, origin, bx)
    bty = _adjoint(y, dims, spacing, origin)
    lhs = float((bx.double() * y.double()).sum())
    rhs = float((x.double() * bty.double()).sum())
    scale = float((bx.double() * y.double()).abs().sum())
    assert abs(lhs - rhs) <= 1e-5 * scale
    assert torch.equal(bty, _adjoint(y, dims, spacing, origin))


@pytest.mark.parametrize("shift", [1, 3])
def test_general_forward_unaligned_output_same_bits(shift):
    # rows of 64-byte multiples written through a pointer 4 or 12 bytes past a
    # 64-byte boundary: the edge-store path, same bits as the aligned path
    dims, spacing, origin = (192, 9, 7), (5.5, 2.0, 3.0), (-1.0, 0.0, -0.5)
    say("general forward, unaligned output", dims, shift)
    grid = dev(_grid(dims, spacing, origin, seed=9))
    aligned = torch.empty(bsi.field_shape(dims), device="cuda")
    bsi.bsi_forward_general(grid, dims, spacing, origin, aligned)
    n = aligned.numel()
    buf = torch.full((n + 32,), 1.0e30, device="cuda")
    out = buf[shift:shift + n].view(bsi.field_shape(dims))
    assert out.data_ptr() % 64 == 4 * shift
    bsi.bsi_forward_general(grid, dims, spacing, origin, out)
    torch.cuda.synchronize()
    assert torch.equal(out, aligned)
    assert bool((buf[:shift] == 1.0e30).all()) and bool((buf[shift + n:] == 1.0e30).all())


def test_general_integer_case_agrees_with_aligned_kernels():
    dims, spacing = (77, 45, 31), (5, 4, 6)
    say("general vs aligned", dims, spacing)
    g = torch.randn(bsi.grid_shape(dims, spacing), device="cuda")
    a = bsi.forward(g, dims, spacing)
    b = torch.empty_like(a)
    bsi.bsi_forward_general(g, dims, spacing, (0.0, 0.0, 0.0), b)
    assert float((a - b).abs().max()) <= 1e-5 * float(g.abs().max())
    d = torch.randn(bsi.field_shape(dims), device="cuda")
    ga = bsi.adjoint(d, dims, spacing)
    gb = _adjoint(d, dims, spacing, (0.0, 0.0, 0.0))
    assert float((ga - gb).abs().max()) <= 1e-5 * float(ga.abs().max())


def test_general_full_size_sampled_and_errors():
    dims, spacing, origin = (512, 512, 256), (5.3, 4.7, 5.1), (-2.5, -0.25, -4.0)
    say("general forward 512x512x256 sampled")
    grid = _grid(dims, spacing, origin, seed=21)
    out = torch.empty(bsi.field_shape(dims), device="cuda")
    bsi.bsi_forward_general(dev(grid), dims, spacing, origin, out)
    rng = np.random.default_rng(4)
    pts = np.stack([rng.integers(0, n, 3000) for n in dims], axis=1)
    pts[:2] = [[0, 0, 0], [511, 511, 255]]
    ref = general.forward_points(grid, dims, spacing, origin, pts)
    got = host(out)[pts[:, 2], pts[:, 1], pts[:, 0]]
    assert np.max(np.abs(got - ref)) <= 1e-5 * float(np.abs(grid).max())
    with pytest.raises(bsi.BSIError):
        bsi.bsi_general_grid_dims(dims, (0.5, 1, 1), (0, 0, 0))
    small = torch.empty(bsi.bsi_adjoint_general_workspace_size(dims, spacing, origin) - 4, dtype=torch.uint8,
                        device="cuda")
    gg = torch.empty(bsi.general_grid_shape(dims, spacing, origin), device="cuda")
    with pytest.raises(bsi.BSIError):
        bsi.bsi_adjoint_general(out, dims, spacing, origin, gg, small)
