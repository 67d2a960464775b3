"""torch.autograd face of the Wiener-filter map.

``WienerFilter.apply(d, theta, plan, schedule, adjoint_schedule)`` returns the
Wiener filter s_W (Eq. 2-3) of every problem of `plan` (concatenated), with
the band amplitudes `theta` as the signal power spectrum of band problems.  Its
backward is the library's adjoint messenger solve (``mf_wiener_backward``):
implicit differentiation of the normal equations (S^-1 + N^-1) s_W = N^-1 d of
Eq. 7 gives dL/dd = N^-1 v and dL/dtheta_b = sum_{k in b} Re(v_k^* s_k)/(n^2 theta_b^2)
with v = (S^-1 + N^-1)^-1 dL/ds_W.  Torch only holds memory and records the graph.
"""
from __future__ import annotations

import torch

from ._binding import Plan, Schedule


class WienerFilter(torch.autograd.Function):
    @staticmethod
    def forward(ctx, d, theta, plan: Plan, schedule: Schedule, adjoint_schedule: Schedule):
        if theta is not None and plan.total_bands > 0:
            plan.set_band_amplitudes(theta.detach().double().cpu().numpy())
        s, info = plan.wiener(d.detach().float().contiguous(), schedule, allow_not_converged=True)
        ctx.plan = plan
        ctx.adjoint_schedule = adjoint_schedule
        ctx.theta_meta = None if theta is None else (theta.dtype, theta.device)
        ctx.save_for_backward(s)
        ctx.info = info
        return s

    @staticmethod
    def backward(ctx, grad_s):
        (s,) = ctx.saved_tensors
        want_bands = ctx.theta_meta is not None and ctx.plan.total_bands > 0
        gd, gb, _, _ = ctx.plan.wiener_backward(s, grad_s.float().contiguous(), ctx.adjoint_schedule,
                                                want_bands=want_bands, allow_not_converged=True)
        gtheta = None
        if want_bands:
            gtheta = gb.to(dtype=ctx.theta_meta[0], device=ctx.theta_meta[1])
        return gd, gtheta, None, None, None


def wiener_filter(d, theta, plan: Plan, schedule: Schedule, adjoint_schedule: Schedule):
    return WienerFilter.apply(d, theta, plan, schedule, adjoint_schedule)


class BandPosteriorLoss:
    """Loss of a band-spectrum problem at its Wiener solution s = s_W(d, theta):

        L = 1/2 s^T S^-1 s + 1/2 (d - A s)^T N^-1 (d - A s) + 1/2 sum_k ln(n P_k)
            + 1/2 ||s - s_true||^2,

    the negative log-posterior of Eq. 5-7 up to constants plus an L2 distance to
    a reference field, with the plan's own noise model and response.
    value_and_grad() runs the Wiener filter and then the library's mf_band_loss,
    which evaluates L and its gradient with respect to d and theta (explicit
    terms plus one adjoint solve through s_W) on the device."""

    def __init__(self, plan: Plan):
        if plan.total_bands <= 0:
            raise ValueError("BandPosteriorLoss needs band-spectrum problems")
        self.plan = plan

    def value_and_grad(self, d, theta, s_true, schedule: Schedule, adjoint_schedule: Schedule):
        plan = self.plan
        plan.set_band_amplitudes(theta.detach().double().cpu().numpy())
        s, _ = plan.wiener(d, schedule, allow_not_converged=True)
        loss, grad_d, grad_theta, _ = plan.band_loss(d, s, s_true, adjoint_schedule, allow_not_converged=True)
        return float(loss.sum().item()), grad_d, grad_theta, s
