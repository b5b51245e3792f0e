"""Helpers shared by the GPU tests (no arithmetic of the method here)."""
import sys

import numpy as np
import torch


def say(*args):
    """Name the case about to run on the GPU, flushed, so a fault can be traced."""
    print("[gpu-case]", *args, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def max_abs(a, b):
    return float(np.max(np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64)))) if np.size(a) else 0.0
