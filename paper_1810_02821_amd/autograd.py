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

import numpy as np
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

        L = 1/2 s^T S^-1 s + 1/2 (d - s)^T N^-1 (d - s) + 1/2 sum_k ln(n P_k)
            + 1/2 ||s - s_true||^2,

    the negative log-posterior of Eq. 5-7 up to constants plus an L2 distance to
    a reference field.  value_and_grad() returns L and its gradient with respect
    to d and theta.  At s_W the log-posterior part is stationary in s, so only
    the L2 term sends a gradient through s_W (one adjoint solve); the rest is
    explicit.  All spectral sums come from the library's band reduction."""

    def __init__(self, plan: Plan, noise_var_concat: np.ndarray, device="cuda"):
        if plan.total_bands <= 0:
            raise ValueError("BandPosteriorLoss needs band-spectrum problems")
        self.plan = plan
        nv = np.asarray(noise_var_concat, dtype=np.float64)
        self.ninv = torch.from_numpy(np.where(np.isfinite(nv), 1.0 / nv, 0.0)).to(device)
        self.device = device
        # per-band mode counts: the band power of a unit impulse is the count
        imp = np.zeros(plan.total_pixels, dtype=np.float32)
        for i, _ in enumerate(plan.problems):
            imp[plan.offsets[i]] = 1.0
        t = torch.from_numpy(imp).to(device)
        self.counts = plan.band_power(t, t)
        self.n_per_band = torch.zeros(plan.total_bands, dtype=torch.float64, device=device)
        o = 0
        for p in plan.problems:
            if p.spectrum.kind == "bands":
                nb = len(p.spectrum.amps)
                self.n_per_band[o:o + nb] = float(p.H * p.W)
                o += nb

    def value_and_grad(self, d, theta, s_true, schedule: Schedule, adjoint_schedule: Schedule):
        plan = self.plan
        plan.set_band_amplitudes(theta.detach().double().cpu().numpy())
        s, info = plan.wiener(d, schedule, allow_not_converged=True)
        power = plan.band_power(s, s)
        n = self.n_per_band
        th = theta.detach().to(device=self.device, dtype=torch.float64)
        sd = s.double()
        r = d.double() - sd
        e = sd - s_true.double()
        L = (0.5 * torch.sum(power / (n * n * th))
             + 0.5 * torch.sum(self.ninv * r * r)
             + 0.5 * torch.sum(self.counts * torch.log(n * th))
             + 0.5 * torch.sum(e * e))
        gd_imp, gt_imp, _, _ = plan.wiener_backward(s, e.float(), adjoint_schedule, want_bands=True,
                                                    allow_not_converged=True)
        grad_d = self.ninv * r + gd_imp.double()
        grad_theta = -0.5 * power / (n * n * th * th) + 0.5 * self.counts / th + gt_imp
        return float(L), grad_d, grad_theta, s
