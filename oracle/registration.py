"""FP64 SSD registration loop: BSI -> trilinear warp -> SSD -> adjoint -> descent.

Test infrastructure only (see ``oracle/__init__.py``).

One iteration, in this order (the FFD step of Sec. 6 with SSD standing in for the
paper's NiftyReg similarity):
  T      = BSI(phi)                     (Eq. 1, ``oracle.forward``)
  L, dT  = SSD of moving(x + T) vs fixed and its gradient (``oracle.warp``)
  g      = B^T dT                       (``oracle.adjoint``)
  phi    = phi - eta * g
The loss recorded for iteration s is the loss of phi_s, before its update.
"""
import numpy as np


def step(phi, moving, fixed, spacing, coord_dtype=np.float64):
    """One loss/gradient evaluation at control grid phi; returns (L, dL/dphi)."""
    from . import adjoint, forward
    from .warp import ssd_grad

    nz, ny, nx = np.asarray(fixed).shape
    dims = (nx, ny, nz)
    T = forward(phi, dims, spacing)
    loss, dT = ssd_grad(T, moving, fixed, coord_dtype=coord_dtype)
    return loss, adjoint(dT, dims, spacing)


def run(phi0, moving, fixed, spacing, eta, steps):
    """Plain gradient descent for ``steps`` iterations.

    Returns (losses, phi) with losses[s] the SSD at phi_s (FP64) and phi the FP64
    grid after the last update."""
    phi = np.array(phi0, dtype=np.float64)
    losses = []
    for _ in range(int(steps)):
        loss, g = step(phi, moving, fixed, spacing)
        losses.append(loss)
        phi = phi - eta * g
    return losses, phi
