"""Parity of the registration step kernels (warp, SSD gradient, descent) and of a
50-step SSD registration loop against the FP64 oracle.

Warp / SSD bar: the oracle forms the sample coordinate x + T in FP32, as the
kernel does, so both take the same cell decisions; the rest is FP64.  Values
within 1e-5 of the image range, loss within 1e-5 relative.  Loop bar: the loss
of every step within 1e-3 relative of the FP64 trajectory (at 48 x 40 x 32
computed in the test, at 256 x 256 x 160 from the oracle's stored run)."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2004_05962_amd as bsi
import workloads
from gpu_util import dev, host, max_abs, say
from oracle import registration as oreg
from oracle import warp as owarp

pytestmark = pytest.mark.gpu

GOLDEN_TRAJ = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "registration_256x256x160_d5_trajectory.json")


def _pair(dims, nblobs, seed=1004, sigma=2.0):
    case = workloads.cfg4(seed=seed, dims=dims, spacing=(5, 5, 5), nblobs=nblobs, sigma=sigma)
    T = oracle.forward(case["grid_true"], case["dims"], case["spacing"])
    moving = owarp.warp(case["fixed"], T).astype(np.float32)
    return case, moving


@pytest.mark.parametrize("shape,sigma", [((32, 40, 48), 2.0), ((9, 1, 13), 4.0), ((20, 17, 2), 1.0)])
def test_warp_and_ssd_match_oracle(shape, sigma):
    nz, ny, nx = shape
    dims = (nx, ny, nz)
    say("warp/ssd", dims, sigma)
    rng = np.random.default_rng(11)
    moving = rng.standard_normal(shape).astype(np.float32)
    fixed = rng.standard_normal(shape).astype(np.float32)
    field = (rng.standard_normal(shape + (3,)) * sigma).astype(np.float32)
    field[0, 0, 0] = [0.0, 0.0, 0.0]       # exact integer coordinates
    field[-1, -1, -1] = [0.0, 0.0, 0.0]
    F, M, X = dev(field), dev(moving), dev(fixed)
    W = torch.empty(shape, device="cuda")
    bsi.bsi_warp(F, M, dims, W)
    ref_w = owarp.warp(moving, field, coord_dtype=np.float32)
    assert max_abs(host(W), ref_w) <= 1e-5 * float(np.abs(moving).max())
    dT = torch.empty_like(F)
    loss = torch.empty(1, device="cuda")
    ws = torch.empty(bsi.bsi_ssd_workspace_size(dims), dtype=torch.uint8, device="cuda")
    bsi.bsi_ssd_grad(F, M, X, dims, dT, loss, ws)
    L_ref, dT_ref = owarp.ssd_grad(field, moving, fixed, coord_dtype=np.float32)
    assert abs(float(host(loss)[0]) - L_ref) <= 1e-5 * L_ref
    assert max_abs(host(dT), dT_ref) <= 1e-5 * float(np.abs(dT_ref).max())


def test_descent_step():
    say("descent step")
    g = torch.randn(1000003, device="cuda")
    d = torch.randn(1000003, device="cuda")
    expect = g.double() - 0.37 * d.double()
    bsi.bsi_descent_step(g, d, 0.37)
    assert (g.double() - expect).abs().max().item() <= 1e-6


@pytest.mark.parametrize("fused", [True, False])
def test_registration_trajectory_matches_oracle(fused):
    dims = (48, 40, 32)
    case, moving = _pair(dims, nblobs=20)
    fixed, spacing = case["fixed"], case["spacing"]
    say("registration trajectory", dims, "fused" if fused else "unfused")
    reg = bsi.SSDRegistration(dev(fixed), dev(moving), spacing, fused=fused)
    eta = 0.5 / float(np.abs(oreg.step(np.zeros(case["grid_true"].shape), moving, fixed, spacing)[1]).max())
    reg.eta = eta
    losses = host(reg.run(50))
    ref, _ = oreg.run(np.zeros(case["grid_true"].shape), moving, fixed, spacing, eta, 50)
    rel = np.abs(losses - np.array(ref)) / np.array(ref)
    assert rel.max() <= 1e-3, rel.max()
    assert losses[-1] < losses[0]


def test_registration_full_size_loss_falls_and_resume_is_exact():
    dims = workloads.CFG4_DIMS
    case, moving = _pair(dims, nblobs=200)
    fixed, spacing = case["fixed"], case["spacing"]
    say("registration 256x256x160 first step vs oracle")
    reg = bsi.SSDRegistration(dev(fixed), dev(moving), spacing)
    L0_ref, g0_ref = oreg.step(np.zeros(case["grid_true"].shape), moving, fixed, spacing)
    reg.eta = 0.5 / float(np.abs(g0_ref).max())
    loss0 = reg.evaluate(loss_out=torch.empty(1, device="cuda"))
    assert abs(float(host(loss0)[0]) - L0_ref) <= 1e-5 * L0_ref
    # the fused step's bar: its T is summed in another order than the oracle's,
    # so a sample coordinate within rounding of a cell boundary may change cell
    # (the trilinear gradient jumps there by the image's second difference)
    diff = np.abs(host(reg.grad) - g0_ref)
    gmax = float(np.abs(g0_ref).max())
    print(f"registration first gradient: max err {diff.max():.3e} mean err {diff.mean():.3e} max |g| {gmax:.3e}")
    assert diff.max() <= 1e-4 * gmax
    assert diff.mean() <= 1e-6 * gmax

    say("registration 256x256x160 50 steps with resume at 25")
    reg.run(25)
    state = reg.state_dict()
    reg.run(25)
    losses = host(reg.losses[:50])
    assert losses[-1] < losses[0]
    assert sum(b < a for a, b in zip(losses, losses[1:])) >= 40
    other = bsi.SSDRegistration(dev(fixed), dev(moving), spacing)
    other.load_state_dict(state)
    other.run(25)
    assert torch.equal(other.grid, reg.grid)


@pytest.mark.parametrize("fused", [True, False])
def test_registration_full_size_trajectory_matches_oracle(fused):
    """50 descent steps at 256 x 256 x 160 against the FP64 oracle's trajectory
    (stored by tests/golden/make_registration_trajectory.py, which calls only the
    oracle): every step's loss within 1e-3 relative."""
    with open(GOLDEN_TRAJ) as f:
        gold = json.load(f)
    dims = tuple(gold["dims"])
    case, moving = _pair(dims, nblobs=200)
    say("registration 256x256x160 trajectory", "fused" if fused else "unfused")
    reg = bsi.SSDRegistration(dev(case["fixed"]), dev(moving), case["spacing"], fused=fused)
    reg.eta = gold["eta"]
    losses = host(reg.run(gold["steps"]))
    ref = np.array(gold["losses"])
    rel = np.abs(losses - ref) / ref
    print(f"trajectory ({'fused' if fused else 'unfused'}): max rel loss err {rel.max():.3e}")
    assert rel.max() <= 1e-3, rel.max()
