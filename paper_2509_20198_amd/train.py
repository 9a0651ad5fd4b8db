"""Training of the refinement network (Section 3.4) on heightmaps the method
produces itself: the inputs are reconstructions of sparse points, the
targets full-resolution textures of the same area in metres and [0, 1]
colour (the per-texel mean of dense points as the paper builds its ground
truth, with gaps as NaN, or the max-height splat), normalised inside the
loss with the input's centre height and radius.

The loss runs in the library (ls_target_loss): the paper's NaN-masked,
clipped mean squared error, heights and colours averaged, or the configured
L1.  The optimiser follows the paper's training setup: AdamW (lr 1e-4, betas
(0.9, 0.999), eps 1e-5, weight decay 1e-2) with the learning rate divided by
10 after one and two thirds of the run.
"""
from __future__ import annotations

import torch

from . import BF16, FP32, LOSS_CLIPPED_MSE, LOSS_L1, Grid, RefineFn, target_loss  # noqa: F401


class TargetLossFn(torch.autograd.Function):
    """L = loss(y, target) through ls_target_loss; the per-element gradient
    is computed with the loss and scaled by the incoming gradient."""

    @staticmethod
    def forward(ctx, y, tex, cz, grid, kind=LOSS_CLIPPED_MSE):
        loss, grad = target_loss(y.contiguous(), tex.contiguous(), cz.contiguous(), grid, kind,
                                 want_grad=ctx.needs_input_grad[0])
        ctx.save_for_backward(grad if grad is not None else torch.empty(0, device=y.device))
        return loss[0].float()

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return grad * g.to(grad.dtype), None, None, None, None


def loss_value(y: torch.Tensor, tex: torch.Tensor, cz: torch.Tensor, grid, kind: int = LOSS_CLIPPED_MSE) -> float:
    """The loss alone (no gradient), as a Python float."""
    loss, _ = target_loss(y.contiguous(), tex.contiguous(), cz.contiguous(), grid, kind, want_grad=False)
    return float(loss[0].item())


def linear_baseline(x: torch.Tensor, pad: int, res: int) -> torch.Tensor:
    """The zero-head output: the linear reconstruction on the crop."""
    return x[:, pad:pad + res, pad:pad + res][..., [0, 2, 3, 4]].contiguous()


class Trainer:
    """AdamW on the flat FP32 weight vector, gradients from RefineFn and the
    library's loss.

    save_acts=False recomputes the forward inside every backward instead of
    keeping the activations (for batches whose activations do not fit)."""

    def __init__(self, w0: torch.Tensor, grid, precision: int = BF16, save_acts: bool = True,
                 total_steps: int = 75, lr: float = 1e-4, loss_kind: int = LOSS_CLIPPED_MSE):
        self.grid = Grid.of(grid)
        self.precision = precision
        self.save_acts = save_acts
        self.loss_kind = loss_kind
        self.w = w0.detach().clone().float().requires_grad_(True)
        self.opt = torch.optim.AdamW([self.w], lr=lr, betas=(0.9, 0.999), eps=1e-5, weight_decay=1e-2,
                                     amsgrad=False)
        m = [max(1, total_steps // 3), max(2, 2 * total_steps // 3)]
        self.sched = torch.optim.lr_scheduler.MultiStepLR(self.opt, milestones=m, gamma=0.1)

    def step(self, x: torch.Tensor, tex: torch.Tensor, cz: torch.Tensor) -> torch.Tensor:
        """One AdamW step on the batch (x from recon_tiles, tex the target
        texture in metres / [0, 1], cz the batch's centre heights)."""
        self.opt.zero_grad(set_to_none=True)
        y = RefineFn.apply(x, self.w, self.grid, self.precision, self.save_acts)
        loss = TargetLossFn.apply(y, tex, cz, self.grid, self.loss_kind)
        loss.backward()
        self.opt.step()
        self.sched.step()
        return loss.detach()

    def state_dict(self) -> dict:
        """Weights, optimiser moments and schedule: everything a resumed run needs."""
        return {"w": self.w.detach().clone(), "opt": self.opt.state_dict(), "sched": self.sched.state_dict(),
                "precision": self.precision, "loss_kind": self.loss_kind}

    def load_state_dict(self, sd: dict) -> None:
        with torch.no_grad():
            self.w.copy_(sd["w"])
        self.opt.load_state_dict(sd["opt"])
        self.sched.load_state_dict(sd["sched"])
        self.precision = sd["precision"]
        self.loss_kind = sd["loss_kind"]

    def save(self, path: str) -> None:
        """Checkpoint to a file (torch.save of tensors and plain values only)."""
        torch.save(self.state_dict(), path)

    def load(self, path: str) -> None:
        self.load_state_dict(torch.load(path, weights_only=True, map_location=self.w.device))
