"""Parity of the fused SSD step (BSI -> warp -> SSD -> adjoint in one pass).

The oracle is the composition of its plain parts: FP64 forward (Eq. 1), the
FP64 warp/SSD gradient with the sample coordinate formed in FP32, and the FP64
adjoint scatter.

Bars:
  * zero grid (T = 0 exactly on both sides, so every cell decision agrees):
    gradient max-abs <= 1e-5 * max|oracle|, loss within 1e-5 relative;
  * random smooth grids: the GPU sums T in another order than the oracle, so
    a coordinate within an ulp of a cell boundary can fall in the neighbouring
    cell, where the trilinear gradient differs by the image's second
    difference.  With smooth (blob) images that moves a control-point gradient
    by far less than 1e-4 * max|grad|, the bar used, and the loss agrees to
    1e-5 relative.
  * against the unfused GPU chain (forward -> SSD gradient -> adjoint): the
    fused pass forms T, the sample, the per-voxel gradient and the adjoint's
    sums with the same operations in the same order, so the control-grid
    gradient is bit-identical; only the loss is summed in another order.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2004_05962_amd as bsi
import workloads
from gpu_util import dev, host, max_abs, say
from oracle import warp as owarp

pytestmark = pytest.mark.gpu


def _images(dims, seed, nblobs=12):
    case = workloads.cfg4(seed=seed, dims=dims, spacing=(5, 5, 5), nblobs=nblobs, sigma=2.0)
    T = oracle.forward(case["grid_true"], case["dims"], case["spacing"])
    moving = owarp.warp(case["fixed"], T).astype(np.float32)
    return case["fixed"], moving


def _oracle(grid, moving, fixed, dims, spacing):
    T = oracle.forward(grid, dims, spacing)
    L, dT = owarp.ssd_grad(T, moving, fixed, coord_dtype=np.float32)
    return L, oracle.adjoint(dT, dims, spacing)


def _fused(grid, moving, fixed, dims, spacing):
    out = torch.empty(bsi.grid_shape(dims, spacing), device="cuda")
    loss = torch.empty(1, device="cuda")
    ws = torch.empty(bsi.bsi_ssd_fused_workspace_size(dims, spacing), dtype=torch.uint8, device="cuda")
    bsi.bsi_ssd_fused(dev(grid), dev(moving), dev(fixed), dims, spacing, out, loss, ws)
    return host(out), float(host(loss)[0])


ZERO_CASES = [
    ((48, 40, 32), (5, 5, 5)),
    ((37, 29, 23), (3, 4, 6)),      # ragged tiles on every axis
    ((70, 45, 20), (1, 2, 3)),      # spacing 1 in x: direct column sums
    ((40, 70, 21), (12, 35, 7)),    # y tiles taller than a brick
    ((75, 40, 21), (17, 5, 7)),     # the generic kernel (x spacing above 12)
    ((150, 9, 11), (8, 4, 3)),      # several bricks in x
]


@pytest.mark.parametrize("dims,spacing", ZERO_CASES)
def test_fused_zero_grid_matches_oracle(dims, spacing):
    say("fused zero grid", dims, spacing)
    fixed, moving = _images(dims, seed=31 + sum(dims))
    grid = np.zeros(bsi.grid_shape(dims, spacing), np.float32)
    got, L = _fused(grid, moving, fixed, dims, spacing)
    L_ref, ref = _oracle(grid, moving, fixed, dims, spacing)
    assert abs(L - L_ref) <= 1e-5 * L_ref
    assert max_abs(got, ref) <= 1e-5 * float(np.abs(ref).max())


RANDOM_CASES = [
    ((48, 40, 32), (5, 5, 5)),
    ((37, 29, 23), (3, 4, 6)),
    ((40, 70, 21), (12, 35, 7)),
    ((64, 64, 64), (8, 8, 8)),
]


@pytest.mark.parametrize("dims,spacing", RANDOM_CASES)
def test_fused_random_grid_matches_oracle_and_unfused(dims, spacing):
    say("fused random grid", dims, spacing)
    fixed, moving = _images(dims, seed=47 + sum(dims))
    grid = workloads.random_grid(dims, spacing, 1.5, seed=9 + sum(spacing))
    got, L = _fused(grid, moving, fixed, dims, spacing)
    L_ref, ref = _oracle(grid, moving, fixed, dims, spacing)
    scale = float(np.abs(ref).max())
    err = np.abs(got.astype(np.float64) - ref)
    say(f"  loss rel {abs(L - L_ref) / L_ref:.2e}  grad max {err.max() / scale:.2e}  mean {err.mean() / scale:.2e}")
    assert abs(L - L_ref) <= 1e-5 * L_ref
    assert err.max() <= 1e-4 * scale
    assert err.mean() <= 1e-6 * scale

    # the unfused GPU chain: forward -> ssd_grad -> adjoint
    field = bsi.forward(dev(grid), dims, spacing)
    dT = torch.empty_like(field)
    loss = torch.empty(1, device="cuda")
    ws = torch.empty(bsi.bsi_ssd_workspace_size(dims), dtype=torch.uint8, device="cuda")
    bsi.bsi_ssd_grad(field, dev(moving), dev(fixed), dims, dT, loss, ws)
    unfused = host(bsi.adjoint(dT, dims, spacing))
    assert abs(float(host(loss)[0]) - L_ref) <= 1e-5 * L_ref
    assert np.array_equal(got, unfused), "fused and unfused gradients differ"


def test_fused_rerun_bits_and_workspace_check():
    dims, spacing = (77, 45, 31), (5, 4, 6)
    say("fused rerun bits", dims, spacing)
    fixed, moving = _images(dims, seed=5)
    grid = dev(workloads.random_grid(dims, spacing, 1.5, seed=3))
    M, X = dev(moving), dev(fixed)
    need = bsi.bsi_ssd_fused_workspace_size(dims, spacing)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    outs = []
    for _ in range(2):
        out = torch.empty(bsi.grid_shape(dims, spacing), device="cuda")
        loss = torch.empty(1, device="cuda")
        bsi.bsi_ssd_fused(grid, M, X, dims, spacing, out, loss, ws)
        outs.append((out, loss))
    torch.cuda.synchronize()
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    small = torch.empty(need - 4, dtype=torch.uint8, device="cuda")
    with pytest.raises(bsi.BSIError):
        bsi.bsi_ssd_fused(grid, M, X, dims, spacing, outs[0][0], outs[0][1], small)


@pytest.mark.parametrize("dims,spacing", [((77, 45, 31), (5, 4, 6)), ((130, 40, 21), (5, 5, 5))])
def test_fused_descent_equals_fused_then_descent(dims, spacing):
    """bsi_ssd_fused_descent: gradient and loss at the grid as bsi_ssd_fused gives
    them, and the grid updated exactly as bsi_descent_step updates it."""
    say("fused descent", dims, spacing)
    fixed, moving = _images(dims, seed=9)
    grid0 = dev(workloads.random_grid(dims, spacing, 1.5, seed=4))
    M, X = dev(moving), dev(fixed)
    ws = torch.empty(bsi.bsi_ssd_fused_workspace_size(dims, spacing), dtype=torch.uint8, device="cuda")
    eta = 0.37
    ref_g = torch.empty(bsi.grid_shape(dims, spacing), device="cuda")
    ref_l = torch.empty(1, device="cuda")
    bsi.bsi_ssd_fused(grid0, M, X, dims, spacing, ref_g, ref_l, ws)
    ref_grid = grid0.clone()
    bsi.bsi_descent_step(ref_grid, ref_g, eta)
    grid = grid0.clone()
    g = torch.empty_like(ref_g)
    loss = torch.empty(1, device="cuda")
    bsi.bsi_ssd_fused_descent(grid, M, X, dims, spacing, eta, g, loss, ws)
    torch.cuda.synchronize()
    assert torch.equal(g, ref_g)
    assert torch.equal(loss, ref_l)
    assert torch.equal(grid, ref_grid)
    with pytest.raises(bsi.BSIError):
        bsi.bsi_ssd_fused_descent(grid, M, X, dims, spacing, float("nan"), g, loss, ws)
