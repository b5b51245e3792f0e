"""MI355X-native cubic B-spline interpolation (BSI) of 3-D FFD control grids.

Hot path: forward BSI (Eq. 1 of Sec. 2.1), its adjoint behind a
``torch.autograd.Function``, the SSD registration step that drives it, and a
batched persistent launch captured in a HIP graph.  All arithmetic runs in the
hand-written HIP kernels of ``libbsi.so`` (C ABI in ``include/bsi.h``); this
package only marshals arguments.  PyTorch provides device memory and streams.
"""
from . import _lib
from ._lib import (BSIError, bsi_adjoint, bsi_adjoint_noalloc, bsi_adjoint_general, bsi_adjoint_general_workspace_size,
                   bsi_adjoint_partials, bsi_adjoint_reduce, bsi_adjoint_workspace_size, bsi_batch_bind,
                   bsi_batch_capture, bsi_batch_config, bsi_batch_create, bsi_batch_describe, bsi_batch_destroy,
                   bsi_batch_launch, bsi_batch_run, bsi_batch_run_separate, bsi_batch_tune,
                   bsi_descent_step, bsi_forward, bsi_forward_general, bsi_forward_lerp,
                   bsi_forward_scalar, bsi_general_grid_dims, bsi_grid_dims, bsi_last_error, bsi_ssd_fused,
                   bsi_ssd_fused_descent, bsi_ssd_fused_workspace_size, bsi_ssd_grad, bsi_ssd_workspace_size, bsi_version,
                   bsi_warp, field_shape, general_grid_shape, grid_shape, upsample)
from .autograd import BSIFunction, adjoint, bsi, forward
from .batch import BatchPlan
from .registration import SSDRegistration

__all__ = [n for n in dir() if not n.startswith("_")]
