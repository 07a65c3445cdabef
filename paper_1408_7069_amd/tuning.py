"""Differentiable tuning of the filter's knobs: the mean residual-phase
variance over T frames as a torch.autograd.Function of each instance's
(rho, r_scale, taper_c) -- inflation, noise scale of Sigma_w = s diag(r)
(Sec. 3.1.1) and Gaspari-Cohn half width of the localisation taper (Sec. 4.1).

The forward runs the frames on the GPU (letkf_step) and accumulates the loss
(letkf_residual_variance); it keeps the analysis ensemble and frame counter
every `checkpoint_every` frames.  The backward walks the segments in reverse:
it restores a checkpoint, recomputes the segment's analysis ensembles, then
applies letkf_residual_variance_adjoint and letkf_adjoint frame by frame.
Every step runs in the HIP library; this module only orders the calls.
"""
from __future__ import annotations

import torch

from . import binding as B


def _params_of(f: B.Letkf, theta):
    th = theta.detach().to("cpu", torch.float64).reshape(-1, 3)
    if th.shape[0] != f.sizes["n_instances"]:
        raise ValueError(f"theta must hold (rho, r_scale, taper_c) for each of the "
                         f"{f.sizes['n_instances']} instances")
    for i in range(th.shape[0]):
        f.set_params(i, float(th[i, 0]), float(th[i, 1]), float(th[i, 2]))


class ResidualVarianceLoss(torch.autograd.Function):
    """loss[i] = (1/T) sum_k residual variance of instance i at frame k."""

    @staticmethod
    def forward(ctx, theta, f: B.Letkf, y_seq, truth_seq, V_seq, checkpoint_every: int):
        T = len(y_seq)
        if T < 1 or len(truth_seq) != T or (V_seq is not None and len(V_seq) != T):
            raise ValueError("y_seq, truth_seq (and V_seq) need one entry per frame")
        every = max(1, int(checkpoint_every))
        _params_of(f, theta)
        dev = f"cuda:{f.device}"
        n = f.sizes["n_instances"]
        acc = torch.zeros(n, dtype=torch.float64, device=dev)
        w = torch.full((n,), 1.0 / T, dtype=torch.float64, device=dev)
        ckpts = [(0, f.get_ensemble(), f.get_frame())]
        for k in range(T):
            f.step(y_seq[k], None if V_seq is None else V_seq[k])
            f.residual_variance(truth_seq[k], acc, weights=w)
            if (k + 1) % every == 0 and k + 1 < T:
                ckpts.append((k + 1, f.get_ensemble(), f.get_frame()))
        ctx.f, ctx.y, ctx.truth, ctx.V, ctx.T = f, y_seq, truth_seq, V_seq, T
        ctx.ckpts = ckpts
        ctx.theta_meta = (theta.shape, theta.dtype, theta.device)
        return acc

    @staticmethod
    def backward(ctx, g):
        f, T = ctx.f, ctx.T
        dev = f"cuda:{f.device}"
        n = f.sizes["n_instances"]
        w = (g.detach().to(dev, torch.float64) / T).contiguous()
        x_end, frame_end = f.get_ensemble(), f.get_frame()
        xbar = torch.zeros(f.sizes["ensemble_elems"], dtype=f.dtype, device=dev)
        theta_bar = torch.zeros(3 * n, dtype=torch.float64, device=dev)
        bounds = [c[0] for c in ctx.ckpts] + [T]
        for s in range(len(ctx.ckpts) - 1, -1, -1):
            k0, x0, fr0 = ctx.ckpts[s]
            k1 = bounds[s + 1]
            f.set_ensemble(x0)
            f.set_frame(fr0)
            states = [x0]
            for k in range(k0, k1):
                f.step(ctx.y[k], None if ctx.V is None else ctx.V[k])
                states.append(f.get_ensemble())
            for k in range(k1 - 1, k0 - 1, -1):
                f.residual_variance_adjoint(ctx.truth[k], xbar, xa=states[k - k0 + 1], weights=w)
                f.adjoint(states[k - k0], ctx.y[k], xbar, theta_bar, fr0 + (k - k0),
                          V=None if ctx.V is None else ctx.V[k])
        f.set_ensemble(x_end)
        f.set_frame(frame_end)
        shape, dtype, device = ctx.theta_meta
        grad = theta_bar.view(n, 3).to(device=device, dtype=dtype).reshape(shape)
        return grad, None, None, None, None, None


def residual_variance_loss(f: B.Letkf, theta, y_seq, truth_seq, V_seq=None, checkpoint_every: int = 20):
    """Mean residual-phase variance over the frames of y_seq, per instance, as a
    differentiable function of theta = (rho, r_scale, taper_c) per instance
    ((3,) or (n_instances, 3)).  The handle is left after the last frame."""
    return ResidualVarianceLoss.apply(theta, f, y_seq, truth_seq, V_seq, checkpoint_every)


__all__ = ["ResidualVarianceLoss", "residual_variance_loss"]
