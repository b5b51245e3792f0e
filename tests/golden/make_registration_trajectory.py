"""Write the FP64 oracle's 50-step SSD registration trajectory at 256 x 256 x 160.

Calls only ``oracle/`` and the seeded input generators (``workloads``).  The
registration loop is the FFD step of Sec. 6 with SSD as the similarity:
BSI (Eq. 1) -> trilinear warp -> SSD -> adjoint -> descent, from a zero grid,
with eta = 0.5 / max|dL/dphi| at the zero grid (the first update moves no
control point by more than half a voxel).  Output: the JSON file next to this
script, read by the GPU trajectory test.

Run:  python tests/golden/make_registration_trajectory.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402
from oracle import registration as oreg  # noqa: E402
from oracle import warp as owarp  # noqa: E402

OUT = os.path.join(HERE, "registration_256x256x160_d5_trajectory.json")
STEPS = 50


def main():
    case = workloads.cfg4()
    dims, spacing = case["dims"], case["spacing"]
    T = oracle.forward(case["grid_true"], dims, spacing)
    moving = owarp.warp(case["fixed"], T).astype(np.float32)
    phi0 = np.zeros(case["grid_true"].shape)
    t0 = time.time()
    _, g0 = oreg.step(phi0, moving, case["fixed"], spacing)
    eta = 0.5 / float(np.abs(g0).max())
    losses, _ = oreg.run(phi0, moving, case["fixed"], spacing, eta, STEPS)
    rec = {"workload": "256x256x160, spacing 5, 200 Gaussian blobs, moving = fixed warped by BSI of an "
                       "N(0, 2) grid (seed 1004)",
           "dims": list(dims), "spacing": list(spacing), "steps": STEPS, "eta": eta,
           "losses": [float(v) for v in losses],
           "source": "oracle.registration.run (FP64), written by make_registration_trajectory.py"}
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s: loss {losses[0]:.6g} -> {losses[-1]:.6g}")


if __name__ == "__main__":
    main()
