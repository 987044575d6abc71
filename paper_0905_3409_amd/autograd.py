"""torch.autograd wrappers of the advance and of the shape loss (2D sine
stream-function fields). Forward and backward run in the library's kernels:
the advance stores checkpoints (gals_advance_save) and the backward pass is
the library's reverse sweep (gals_adjoint), which recomputes each segment of
states from its checkpoint."""
from __future__ import annotations

import numpy as np
import torch

from . import STREAM_SIN


def stream_params(amps, modes):
    """Parameter vector (a_k, m_k, n_k) of a sine stream function."""
    modes = np.asarray(modes, dtype=np.float64).reshape(-1, 2)
    a = np.asarray(amps, dtype=np.float64).reshape(-1)
    return np.stack([a, modes[:, 0], modes[:, 1]], axis=1).ravel()


class StreamAdvance(torch.autograd.Function):
    """u_T = advance(u_0; a) on `grid` for s = sum_k a_k sin(m_k pi x)
    sin(n_k pi y) (x cos(pi t / period) if period > 0). Differentiable in the
    amplitudes `amps` (a CPU or device tensor of K values) and in the initial
    state."""

    @staticmethod
    def forward(ctx, amps, state0, grid, modes, period, t0, dt, steps, every):
        params = stream_params(amps.detach().cpu().numpy(), modes)
        grid.set_velocity(STREAM_SIN, params, period)
        st = state0.detach().clone()
        ckpt = grid.advance_save(st, t0, dt, steps, every)
        ctx.grid, ctx.ckpt, ctx.params = grid, ckpt, params
        ctx.args = (period, t0, dt, steps, every)
        ctx.modes = np.asarray(modes, dtype=np.int64).reshape(-1, 2)
        ctx.amps_meta = (amps.dtype, amps.device)
        ctx.state_dtype = state0.dtype
        return st

    @staticmethod
    def backward(ctx, grad_state):
        grid = ctx.grid
        period, t0, dt, steps, every = ctx.args
        grid.set_velocity(STREAM_SIN, ctx.params, period)
        lam = grid.empty_adjoint()
        lam.copy_(grad_state[: 3].to(torch.float64))
        dS = grid.adjoint(ctx.ckpt, t0, dt, steps, every, lam)
        idx = torch.as_tensor(4 * (ctx.modes[:, 0] - 1) + (ctx.modes[:, 1] - 1),
                              device=dS.device)
        d_amps = dS[idx].to(dtype=ctx.amps_meta[0], device=ctx.amps_meta[1])
        return d_amps, lam.to(ctx.state_dtype), None, None, None, None, None, None, None


class ShapeLoss(torch.autograd.Function):
    """prod(h) sum over nodes (H_eps(phi) - H_eps(phi_ref))^2, FP64."""

    @staticmethod
    def forward(ctx, state, ref, grid, eps):
        loss, lam = grid.shape_loss(state.detach(), ref.detach(), eps)
        ctx.save_for_backward(lam)
        ctx.state_dtype = state.dtype
        return torch.tensor(loss, dtype=torch.float64, device=state.device)

    @staticmethod
    def backward(ctx, grad_loss):
        (lam,) = ctx.saved_tensors
        return (lam * grad_loss).to(ctx.state_dtype), None, None, None
