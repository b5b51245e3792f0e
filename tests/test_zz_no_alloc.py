"""The allocation-free adjoint entry point (bsi_adjoint_noalloc) against
bsi_adjoint, through the C ABI, on two calls in a row (the second on a smaller
volume, so the shared scratch holds the first call's partials when it starts)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2004_05962_amd as bsi
import workloads


def _adjoint_with_workspace(y, dims, spacing):
    out = torch.empty(bsi.grid_shape(dims, spacing), device="cuda")
    ws = torch.empty(bsi.bsi_adjoint_workspace_size(dims, spacing), dtype=torch.uint8, device="cuda")
    bsi.bsi_adjoint(y, dims, spacing, out, ws)
    return out


@pytest.mark.gpu
def test_noalloc_matches_workspace_adjoint_twice(gpu):
    cases = [((256, 256, 160), (5, 5, 5), 3101), ((97, 70, 41), (4, 6, 3), 3102)]
    for dims, spacing, seed in cases:
        print("noalloc case", dims, spacing, flush=True)
        y_np = workloads.random_field(dims, 1.0, seed=seed)
        y = torch.from_numpy(y_np).to(gpu)
        got = torch.full(bsi.grid_shape(dims, spacing), float("nan"), device=gpu)
        bsi.bsi_adjoint_noalloc(y, dims, spacing, got)
        ref = _adjoint_with_workspace(y, dims, spacing)
        torch.cuda.synchronize()
        # the same kernels on the same partial layout: identical bits
        assert torch.equal(got, ref), (dims, spacing)
        if dims[0] * dims[1] * dims[2] <= 300_000:
            exact = oracle.adjoint(y_np, dims, spacing)
            err = float(np.abs(got.cpu().numpy() - exact).max())
            assert err <= 1e-5 * float(np.abs(exact).max()), err


@pytest.mark.gpu
def test_noalloc_rejects_oversized_geometry(gpu):
    dims, spacing = (512, 512, 256), (2, 2, 2)
    assert bsi.bsi_adjoint_workspace_size(dims, spacing) > bsi._lib.BSI_ADJOINT_NOALLOC_MAX_BYTES
    y = torch.zeros(1, device=gpu)  # never read: the size check comes first
    with pytest.raises(bsi.BSIError):
        bsi._lib.lib()
        rc = bsi._lib.lib().bsi_adjoint_noalloc(bsi._lib._VP(y.data_ptr()), bsi._lib._triple(dims, "d"),
                                                bsi._lib._triple(spacing, "s"), bsi._lib._VP(y.data_ptr()),
                                                bsi._lib._VP(0))
        bsi._lib._check(rc)
