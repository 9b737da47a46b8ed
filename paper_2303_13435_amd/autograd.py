"""torch.autograd bindings of the binned forward path and its adjoint.

``BinnedIntensity.apply(amp, plan, cell, mask, zoom)`` returns the mean
intensity of every |Q| bin (0 for empty bins) of the box generated from the
unit cell with atom amplitudes ``amp``; its backward calls ``ur_adjoint``,
which gives dL/d amp from dL/dI_b (the gradient of eq. 1's |F|^2 averaged per
bin, folded back through tiling and masking); when nothing else ran on the
plan since the forward call it starts from the plan's held y-pass output
(``ur_adjoint_reuse``) instead of recomputing it.  ``BinnedIntensityRho`` does
the same for a given voxel density, and ``chi2`` is the misfit of a curve
against a target with its per-bin gradient (``ur_chi2``).  All of it runs in
the HIP kernels; the Python here only moves pointers.
"""
from __future__ import annotations

import torch

from . import DeviceCell, Hist, Plan
from . import chi2 as _chi2


def _means(h: Hist) -> torch.Tensor:
    """Per-bin means written by the finalize kernel, empty bins (NaN) as 0."""
    return torch.nan_to_num(h.mean, nan=0.0)


class BinnedIntensity(torch.autograd.Function):
    @staticmethod
    def forward(ctx, amp: torch.Tensor, plan: Plan, cell: DeviceCell, mask, zoom):
        if zoom.factor != 1 or zoom.n1 != plan.n:
            raise ValueError("amplitude gradients are defined for ED-1 boxes (zoom factor 1)")
        a = amp.detach().contiguous().to(torch.float64)
        h = Hist(plan.nbins)
        plan.simulate(cell, mask, zoom, h, amp=a)
        ctx.plan, ctx.cell, ctx.mask, ctx.hist, ctx.amp = plan, cell, mask, h, a
        ctx.calls = plan.calls                  # the plan's workspace holds this forward's output
        return _means(h)

    @staticmethod
    def backward(ctx, g_mean: torch.Tensor):
        g = torch.where(ctx.hist.count > 0, g_mean.to(torch.float64), torch.zeros_like(g_mean, dtype=torch.float64))
        grad = torch.empty_like(ctx.amp)
        aligned = ctx.cell.rot is None and ctx.cell.grain_seed is None
        if ctx.plan.calls == ctx.calls and not ctx.plan.c2c and aligned:
            # nothing ran on the plan since this forward (of a lattice aligned
            # with the box): start from its held output
            ctx.plan.adjoint_reuse(ctx.hist, g.contiguous(), ctx.cell, ctx.mask, grad, amp=ctx.amp)
        else:
            ctx.plan.adjoint(ctx.hist, g.contiguous(), cell=ctx.cell, mask=ctx.mask, grad_amp=grad, amp=ctx.amp)
        return grad, None, None, None, None


class BinnedIntensityRho(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho: torch.Tensor, plan: Plan):
        r = rho.detach().contiguous()
        h = Hist(plan.nbins)
        plan.simulate_rho(r, h)
        ctx.plan, ctx.hist, ctx.rho = plan, h, r
        return _means(h)

    @staticmethod
    def backward(ctx, g_mean: torch.Tensor):
        g = torch.where(ctx.hist.count > 0, g_mean.to(torch.float64), torch.zeros_like(g_mean, dtype=torch.float64))
        grad = torch.empty_like(ctx.rho)
        ctx.plan.adjoint(ctx.hist, g.contiguous(), rho=ctx.rho, grad_rho=grad)
        return grad, None


class Chi2(torch.autograd.Function):
    """chi^2 of a binned curve against a target and its gradient per bin,
    both computed by ``ur_chi2`` on the device (fixed-order compensated sum)."""

    @staticmethod
    def forward(ctx, mean: torch.Tensor, target: torch.Tensor, count: torch.Tensor, rel_sigma: float = 0.01):
        m = mean.detach().to(torch.float64).contiguous()
        g = torch.empty_like(m)
        out = _chi2(m, count.detach().to(torch.float64).contiguous(), target.detach().to(torch.float64).contiguous(),
                    rel_sigma, g_bin=g)
        ctx.save_for_backward(g)
        return out[0].clone()

    @staticmethod
    def backward(ctx, g_out: torch.Tensor):
        (g,) = ctx.saved_tensors
        return g * g_out, None, None, None


def chi2(mean: torch.Tensor, target: torch.Tensor, count: torch.Tensor, rel_sigma: float = 0.01) -> torch.Tensor:
    """sum over populated bins of ((I_b - T_b) / (rel_sigma T_b))^2 (ur_chi2)."""
    return Chi2.apply(mean, target, count, rel_sigma)
