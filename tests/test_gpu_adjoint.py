"""Parity of the HIP adjoint (transpose of Eq. 1) and its autograd wrapper.

Bar: max |gpu - oracle| <= 1e-5 * max|oracle grad| on every control point
(full FP64 oracle, including the 256^3 workload), the dot-product identity
<Bx, y> = <x, B^T y> accumulated in FP64 on the host, central finite
differences on the 12^3 case, bit-identical reruns."""
import numpy as np
import pytest
import torch

import oracle
import paper_2004_05962_amd as bsi
import workloads
from gpu_util import dev, host, max_abs, say

pytestmark = pytest.mark.gpu

CASES = [
    ((64, 64, 64), (5, 5, 5)),
    ((1, 1, 1), (1, 1, 1)),
    ((3, 2, 5), (64, 64, 64)),
    ((7, 3, 2), (2, 3, 1)),
    ((130, 9, 11), (5, 4, 3)),
    ((65, 70, 33), (64, 7, 10)),
    ((200, 5, 6), (1, 1, 1)),
    ((33, 40, 129), (8, 33, 6)),      # y spacing above the 32-row brick: unaligned bricks
    ((96, 80, 72), (3, 5, 8)),
    ((61, 47, 53), (2, 2, 2)),
    ((100, 30, 20), (9, 4, 3)),       # the larger specialised x spacings, ragged
    ((130, 40, 17), (10, 5, 6)),
    ((77, 35, 29), (11, 3, 7)),
    ((200, 33, 9), (12, 12, 2)),
    ((91, 20, 12), (13, 2, 3)),       # first spacing on the generic x path
]


@pytest.mark.parametrize("dims,spacing", CASES)
def test_adjoint_matches_oracle(dims, spacing):
    say("adjoint", dims, spacing)
    dfield = workloads.random_field(dims, 1.0, seed=200 + sum(dims) + 3 * sum(spacing))
    got = host(bsi.adjoint(dev(dfield), dims, spacing))
    ref = oracle.adjoint(dfield, dims, spacing)
    assert got.shape == ref.shape
    assert max_abs(got, ref) <= 1e-5 * float(np.abs(ref).max())


@pytest.fixture(scope="module")
def cfg3():
    return workloads.cfg3()


def test_adjoint_256_full_oracle(cfg3):
    dims, spacing = cfg3["dims"], cfg3["spacing"]
    say("adjoint 256^3 delta 5 full oracle")
    d = dev(cfg3["dfield"])
    got = host(bsi.adjoint(d, dims, spacing))
    ref = oracle.adjoint(cfg3["dfield"], dims, spacing)
    err = max_abs(got, ref)
    assert err <= 1e-5 * float(np.abs(ref).max()), err
    again = host(bsi.adjoint(d, dims, spacing))
    assert np.array_equal(got, again)


def test_dot_product_identity_256(cfg3):
    dims, spacing = cfg3["dims"], cfg3["spacing"]
    say("dot product 256^3")
    x, y = dev(cfg3["grid"]), dev(cfg3["dfield"])
    Bx = bsi.forward(x, dims, spacing)
    BTy = bsi.adjoint(y, dims, spacing)
    torch.cuda.synchronize()
    lhs_terms = (Bx.double() * y.double())
    lhs = lhs_terms.sum().item()
    rhs = (x.double() * BTy.double()).sum().item()
    bound = 1e-5 * lhs_terms.abs().sum().item()
    assert abs(lhs - rhs) <= bound, (lhs, rhs, bound)


def test_finite_differences_12():
    case = workloads.cfg3_fd()
    dims, spacing = case["dims"], case["spacing"]
    say("finite differences 12^3")
    y = dev(case["dfield"])
    phi = dev(case["grid"])
    g = host(bsi.adjoint(y, dims, spacing))
    # FP64 oracle gradient of the same linear functional
    ref = oracle.adjoint(case["dfield"], dims, spacing)
    assert max_abs(g, ref) <= 1e-5 * float(np.abs(ref).max())
    # central differences through the GPU forward: L is linear, so FD is exact
    # up to FP32 rounding of L
    eps = 1e-2
    flat = phi.view(-1)
    idx = np.random.default_rng(3).choice(flat.numel(), 96, replace=False)
    L = lambda p: (bsi.forward(p.view(phi.shape), dims, spacing).double() * y.double()).sum().item()
    gflat = g.reshape(-1)
    for i in idx:
        p = flat.clone()
        m = flat.clone()
        p[i] += eps
        m[i] -= eps
        fd = (L(p) - L(m)) / (2 * eps)
        assert abs(fd - gflat[i]) <= 1e-3 * max(1.0, abs(gflat[i])), (i, fd, gflat[i])


def test_autograd_function():
    dims, spacing = (50, 37, 29), (5, 4, 3)
    say("autograd", dims, spacing)
    grid_np = workloads.random_grid(dims, spacing, 2.0, seed=9)
    w_np = workloads.random_field(dims, 1.0, seed=10)
    grid = dev(grid_np).requires_grad_(True)
    w = dev(w_np)
    field = bsi.bsi(grid, dims, spacing)
    assert max_abs(host(field), oracle.forward(grid_np, dims, spacing)) <= 1e-5 * float(np.abs(grid_np).max())
    (field * w).sum().backward()
    # the gradient autograd delivers against the FP64 transpose of Eq. 1
    ref = oracle.adjoint(w_np, dims, spacing)
    assert max_abs(host(grid.grad), ref) <= 1e-5 * float(np.abs(ref).max())
    expect = bsi.adjoint(w, dims, spacing)
    torch.cuda.synchronize()
    assert torch.equal(grid.grad, expect)
    # autograd accumulates across backward passes; the library overwrites
    field = bsi.bsi(grid, dims, spacing)
    (field * w).sum().backward()
    torch.cuda.synchronize()
    assert torch.allclose(grid.grad, 2 * expect, rtol=0, atol=0)


def test_workspace_too_small_raises():
    dims, spacing = (40, 30, 20), (5, 5, 5)
    say("adjoint workspace check")
    d = torch.zeros(bsi.field_shape(dims), device="cuda")
    out = torch.empty(bsi.grid_shape(dims, spacing), device="cuda")
    ws = torch.empty(bsi.bsi_adjoint_workspace_size(dims, spacing) - 4, dtype=torch.uint8, device="cuda")
    with pytest.raises(bsi.BSIError):
        bsi.bsi_adjoint(d, dims, spacing, out, ws)


@pytest.mark.parametrize("dims,spacing", [((64, 64, 64), (5, 5, 5)), ((33, 40, 129), (8, 33, 6))])
def test_split_passes_bit_identical(dims, spacing):
    """bsi_adjoint_partials + bsi_adjoint_reduce == bsi_adjoint, bit for bit, also
    when the reduce runs on another stream ordered by an event."""
    say("adjoint split passes", dims, spacing)
    d = dev(workloads.random_field(dims, 1.0, seed=77))
    nbytes = bsi.bsi_adjoint_workspace_size(dims, spacing)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    whole = torch.empty(bsi.grid_shape(dims, spacing), device="cuda")
    bsi.bsi_adjoint(d, dims, spacing, whole, ws)
    split = torch.full_like(whole, float("nan"))
    ws2 = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    bsi.bsi_adjoint_partials(d, dims, spacing, ws2)
    done = torch.cuda.Event()
    done.record()
    side = torch.cuda.Stream()
    side.wait_event(done)
    bsi.bsi_adjoint_reduce(ws2, dims, spacing, split, stream=side)
    torch.cuda.synchronize()
    assert torch.equal(whole, split)
    ref = oracle.adjoint(host(d), dims, spacing)
    assert max_abs(host(split), ref) <= 1e-5 * float(np.abs(ref).max())
    small = torch.empty(nbytes - 4, dtype=torch.uint8, device="cuda")
    with pytest.raises(bsi.BSIError):
        bsi.bsi_adjoint_partials(d, dims, spacing, small)
    with pytest.raises(bsi.BSIError):
        bsi.bsi_adjoint_reduce(small, dims, spacing, split)


def test_adjoint_full_size_every_point():
    """The benchmark's configuration (512 x 512 x 256, spacing 5, the same
    partials + reduce launches) against the oracle's gather on every control
    point, and bit-identical to the one-call adjoint."""
    case = workloads.cfg2(5)
    dims, spacing = case["dims"], case["spacing"]
    say("adjoint 512x512x256 delta 5 every control point")
    dfield = workloads.random_field(dims, 1.0, seed=1102)
    d = dev(dfield)
    ws = torch.empty(bsi.bsi_adjoint_workspace_size(dims, spacing), dtype=torch.uint8, device="cuda")
    grad = torch.empty(bsi.grid_shape(dims, spacing), device="cuda")
    bsi.bsi_adjoint_partials(d, dims, spacing, ws)
    bsi.bsi_adjoint_reduce(ws, dims, spacing, grad)
    got = host(grad)
    ref = oracle.adjoint_gather(dfield, dims, spacing)
    err = max_abs(got, ref)
    print(f"adjoint 512x512x256 d5: max err {err:.3e} mean err {float(np.mean(np.abs(got - ref))):.3e} "
          f"max |grad| {float(np.abs(ref).max()):.3e}")
    assert err <= 1e-5 * float(np.abs(ref).max())
    again = torch.empty_like(grad)
    bsi.bsi_adjoint(d, dims, spacing, again, ws)
    assert torch.equal(grad, again)


@pytest.mark.parametrize("dims,spacing", [((65536, 3, 2), (7, 1, 2)), ((2, 65536, 3), (1, 5, 1)),
                                          ((3, 2, 65536), (2, 1, 6))])
def test_extreme_aspect_forward_and_adjoint(dims, spacing):
    """A 65536-voxel axis with two tiny ones: many bricks along one axis, one
    along the others, partial tiles and partial strips everywhere."""
    say("extreme aspect", dims, spacing)
    grid = workloads.random_grid(dims, spacing, 2.0, seed=sum(dims))
    f = host(bsi.forward(dev(grid), dims, spacing))
    assert max_abs(f, oracle.forward(grid, dims, spacing)) <= 1e-5 * float(np.abs(grid).max())
    dfield = workloads.random_field(dims, 1.0, seed=sum(dims) + 1)
    g = host(bsi.adjoint(dev(dfield), dims, spacing))
    ref = oracle.adjoint(dfield, dims, spacing)
    assert max_abs(g, ref) <= 1e-5 * float(np.abs(ref).max())
