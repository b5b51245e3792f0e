"""Forward BSI as a differentiable torch op; its backward is the HIP adjoint.

``BSIFunction.apply(grid, dims, spacing)`` maps a control grid (gz, gy, gx, 3) to
the dense displacement field (nz, ny, nx, 3) with ``bsi_forward`` (Eq. 1, Sec. 2.1).
Backward computes dL/dgrid = B^T dL/dfield with ``bsi_adjoint``: a deterministic
gather without atomics; the library overwrites, autograd accumulates.
"""
import torch

from ._lib import bsi_adjoint, bsi_adjoint_workspace_size, bsi_forward, field_shape, grid_shape


def forward(grid, dims, spacing, out=None, stream=None):
    """Dense field of ``grid``; allocates ``out`` (float32, same device) if not given."""
    if out is None:
        out = torch.empty(field_shape(dims), dtype=torch.float32, device=grid.device)
    bsi_forward(grid, dims, spacing, out, stream)
    return out


def adjoint(dfield, dims, spacing, out=None, workspace=None, stream=None):
    """B^T dfield; allocates ``out`` and the scratch workspace if not given."""
    if out is None:
        out = torch.empty(grid_shape(dims, spacing), dtype=torch.float32, device=dfield.device)
    if workspace is None:
        workspace = torch.empty(bsi_adjoint_workspace_size(dims, spacing), dtype=torch.uint8,
                                device=dfield.device)
    bsi_adjoint(dfield, dims, spacing, out, workspace, stream)
    return out


class BSIFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, grid, dims, spacing):
        ctx.dims = tuple(int(v) for v in dims)
        ctx.spacing = tuple(int(v) for v in spacing)
        return forward(grid.contiguous(), ctx.dims, ctx.spacing)

    @staticmethod
    def backward(ctx, dfield):
        grad = None
        if ctx.needs_input_grad[0]:
            grad = adjoint(dfield.contiguous(), ctx.dims, ctx.spacing)
        return grad, None, None


def bsi(grid, dims, spacing):
    """Differentiable BSI: field = B(grid)."""
    return BSIFunction.apply(grid, dims, spacing)
