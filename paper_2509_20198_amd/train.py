"""Training of the refinement network (Section 3.4) on heightmaps the method
produces itself: the inputs are reconstructions of sparse points, the
targets full-resolution heightmaps of the same area (the max-height splat of
dense points), normalised with the input's centre height and radius.

The optimiser follows the paper's training setup: AdamW (lr 1e-4, betas
(0.9, 0.999), eps 1e-5, weight decay 1e-2) with the learning rate divided by
10 after one and two thirds of the run.  The loss is the configured L1:
L = 1/2 mean|y_h - t_h| + 1/2 mean|y_rgb - t_rgb| over the res x res crop,
with sign(0) = 0 in its gradient.
"""
from __future__ import annotations

import torch

from . import BF16, FP32, Grid, RefineFn  # noqa: F401


def normalise_target(tex: torch.Tensor, cz: torch.Tensor, r_m: float) -> torch.Tensor:
    """Texture [n, res, res, 4] (height in metres, colour in [0, 1]) -> the
    network's normalised output space: h' = (h - cz) / r_m, colour unchanged."""
    t = tex.clone()
    t[..., 0] = ((tex[..., 0].double() - cz.view(-1, 1, 1)) / r_m).float()
    return t


def l1_loss(y: torch.Tensor, t: torch.Tensor) -> torch.Tensor:
    return 0.5 * (y[..., 0] - t[..., 0]).abs().mean() + 0.5 * (y[..., 1:] - t[..., 1:]).abs().mean()


def linear_baseline(x: torch.Tensor, pad: int, res: int) -> torch.Tensor:
    """The zero-head output: the linear reconstruction on the crop."""
    return x[:, pad:pad + res, pad:pad + res][..., [0, 2, 3, 4]]


class Trainer:
    """AdamW on the flat FP32 weight vector, gradients from RefineFn.

    save_acts=False recomputes the forward inside every backward instead of
    keeping the activations (for batches whose activations do not fit)."""

    def __init__(self, w0: torch.Tensor, grid, precision: int = BF16, save_acts: bool = True,
                 total_steps: int = 75, lr: float = 1e-4):
        self.grid = Grid.of(grid)
        self.precision = precision
        self.save_acts = save_acts
        self.w = w0.detach().clone().float().requires_grad_(True)
        self.opt = torch.optim.AdamW([self.w], lr=lr, betas=(0.9, 0.999), eps=1e-5, weight_decay=1e-2,
                                     amsgrad=False)
        m = [max(1, total_steps // 3), max(2, 2 * total_steps // 3)]
        self.sched = torch.optim.lr_scheduler.MultiStepLR(self.opt, milestones=m, gamma=0.1)

    def step(self, x: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
        self.opt.zero_grad(set_to_none=True)
        y = RefineFn.apply(x, self.w, self.grid, self.precision, self.save_acts)
        loss = l1_loss(y, target)
        loss.backward()
        self.opt.step()
        self.sched.step()
        return loss.detach()
