"""SSD registration loop on the GPU: BSI -> trilinear warp -> SSD -> adjoint -> step.

One iteration (the FFD step of Sec. 6, with a sum-of-squared-differences
similarity standing in for the paper's NiftyReg measure):
  field = B(grid)                       bsi_forward
  loss, dL/dfield                       bsi_ssd_grad
  g = B^T dL/dfield                     bsi_adjoint
  grid -= eta * g                       bsi_descent_step
With ``fused=True`` (the default) an iteration is one call, bsi_ssd_fused_descent,
which never stores the field or dL/dfield (the merge of FFD steps into BSI that
Sec. 8 names as further work) and folds the update into its last launch; the
gradient and the updated grid equal the unfused ones bit for bit, the loss is
summed in another fixed order.
All calls run on one stream; losses are written into a device buffer, so the host
synchronises only when it reads them.  ``losses[s]`` is the loss of grid_s,
before its update.  State for checkpoint/resume is (grid, step, eta).
"""
import torch

from ._lib import (bsi_adjoint, bsi_adjoint_workspace_size, bsi_descent_step, bsi_forward, bsi_ssd_fused,
                   bsi_ssd_fused_descent, bsi_ssd_fused_workspace_size, bsi_ssd_grad, bsi_ssd_workspace_size, field_shape, grid_shape)


class SSDRegistration:
    def __init__(self, fixed, moving, spacing, grid=None, eta=None, max_steps=1024, fused=True):
        if fixed.shape != moving.shape or fixed.dim() != 3:
            raise ValueError("fixed and moving must be (nz, ny, nx) images of one shape")
        nz, ny, nx = fixed.shape
        self.dims = (int(nx), int(ny), int(nz))
        self.spacing = tuple(int(v) for v in spacing)
        dev = fixed.device
        self.fixed = fixed.contiguous()
        self.moving = moving.contiguous()
        gshape = grid_shape(self.dims, self.spacing)
        self.grid = (torch.zeros(gshape, dtype=torch.float32, device=dev) if grid is None
                     else grid.to(device=dev, dtype=torch.float32).contiguous().clone())
        self.fused = bool(fused)
        self.grad = torch.empty(gshape, dtype=torch.float32, device=dev)
        if self.fused:
            self.ws_fused = torch.empty(bsi_ssd_fused_workspace_size(self.dims, self.spacing), dtype=torch.uint8,
                                        device=dev)
        else:
            self.field = torch.empty(field_shape(self.dims), dtype=torch.float32, device=dev)
            self.dfield = torch.empty_like(self.field)
            self.ws_adj = torch.empty(bsi_adjoint_workspace_size(self.dims, self.spacing), dtype=torch.uint8,
                                      device=dev)
            self.ws_ssd = torch.empty(bsi_ssd_workspace_size(self.dims), dtype=torch.uint8, device=dev)
        self.losses = torch.zeros(max_steps, dtype=torch.float32, device=dev)
        self.step_index = 0
        self.eta = eta

    def evaluate(self, loss_out=None, stream=None):
        """Loss and gradient at the current grid (no update); gradient in self.grad."""
        loss_out = self.losses[self.step_index:self.step_index + 1] if loss_out is None else loss_out
        if self.fused:
            bsi_ssd_fused(self.grid, self.moving, self.fixed, self.dims, self.spacing, self.grad, loss_out,
                          self.ws_fused, stream)
            return loss_out
        bsi_forward(self.grid, self.dims, self.spacing, self.field, stream)
        bsi_ssd_grad(self.field, self.moving, self.fixed, self.dims, self.dfield, loss_out, self.ws_ssd, stream)
        bsi_adjoint(self.dfield, self.dims, self.spacing, self.grad, self.ws_adj, stream)
        return loss_out

    def auto_eta(self, max_move=0.5):
        """eta such that the first update moves no control point by more than max_move voxels."""
        probe = torch.zeros(1, dtype=torch.float32, device=self.grid.device)
        self.evaluate(loss_out=probe)
        gmax = float(self.grad.abs().max())
        self.eta = max_move / gmax if gmax > 0 else 0.0
        return self.eta

    def step(self, stream=None):
        if self.eta is None:
            raise ValueError("set eta (or call auto_eta) before stepping")
        if self.step_index >= self.losses.numel():
            raise RuntimeError("loss buffer full")
        if self.fused:  # evaluation and update in one call (the update folded into its last launch)
            bsi_ssd_fused_descent(self.grid, self.moving, self.fixed, self.dims, self.spacing, self.eta, self.grad,
                                  self.losses[self.step_index:self.step_index + 1], self.ws_fused, stream)
        else:
            self.evaluate(stream=stream)
            bsi_descent_step(self.grid, self.grad, self.eta, stream)
        self.step_index += 1

    def run(self, steps, stream=None):
        for _ in range(int(steps)):
            self.step(stream)
        return self.losses[:self.step_index]

    def state_dict(self):
        return {"grid": self.grid.detach().cpu().clone(), "step": self.step_index, "eta": self.eta,
                "losses": self.losses[:self.step_index].detach().cpu().clone()}

    def load_state_dict(self, state):
        self.grid.copy_(state["grid"].to(self.grid.device))
        self.step_index = int(state["step"])
        self.eta = state["eta"]
        self.losses[:self.step_index].copy_(state["losses"].to(self.losses.device))
