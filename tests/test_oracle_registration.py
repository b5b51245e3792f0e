"""Pins for the oracle's SSD registration step (BSI -> warp -> SSD -> adjoint).

The whole chain's gradient is checked by central finite differences of the FP64
loss; gradient descent must lower the loss.
"""
import numpy as np

import oracle
import workloads
from oracle import registration


def _small_pair(seed=1004):
    case = workloads.cfg4(seed=seed, dims=(20, 18, 12), spacing=(5, 5, 5), nblobs=12, sigma=1.0)
    dims, spacing = case["dims"], case["spacing"]
    T = oracle.forward(case["grid_true"], dims, spacing)
    moving = oracle.warp.warp(case["fixed"], T).astype(np.float32)
    return case["fixed"], moving, spacing, case["grid_true"]


def test_chain_gradient_finite_differences():
    fixed, moving, spacing, gt = _small_pair()
    rng = np.random.default_rng(9)
    phi = 0.3 * rng.standard_normal(gt.shape)
    L0, g = registration.step(phi, moving, fixed, spacing)
    eps = 1e-6
    for _ in range(25):
        i = tuple(rng.integers(0, s) for s in phi.shape)
        p, m = phi.copy(), phi.copy()
        p[i] += eps
        m[i] -= eps
        fd = (registration.step(p, moving, fixed, spacing)[0] - registration.step(m, moving, fixed, spacing)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-5 * max(1.0, abs(g[i]))


def test_descent_lowers_loss():
    fixed, moving, spacing, gt = _small_pair()
    phi0 = np.zeros(gt.shape)
    L0, g0 = registration.step(phi0, moving, fixed, spacing)
    eta = 0.5 / np.abs(g0).max()
    losses, phi = registration.run(phi0, moving, fixed, spacing, eta, 15)
    assert losses[0] == L0
    assert losses[-1] < 0.8 * losses[0]
    assert sum(b < a for a, b in zip(losses, losses[1:])) >= 12
