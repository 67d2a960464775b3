"""Gradients of the Wiener-filter map (FP64, CPU).

The Wiener filter s* solves the normal equations read off Eq. 7,
    (S^-1 + N^-1) s* = N^-1 d,
with S^-1 diagonal in Fourier space (eigenvalues 1/(n P_k)) and N^-1 diagonal in
pixel space (0 on missing pixels).  For a loss with dL/ds* = gbar, implicit
differentiation gives, with v = (S^-1 + N^-1)^-1 gbar (the matrix is symmetric):
    dL/dd       = N^-1 v
    dL/dtheta_b = -v^T (dS^-1/dtheta_b) s*
                = sum_{k in band b} Re(conj(v_hat_k) s*_hat_k) / (n^2 theta_b^2)
(numpy FFT scaling) when P_k = theta_b on band b.

v is found by the messenger iteration itself: with right-hand side b = gbar in
the pixel step t = (1 - a) v + T gbar, the fixed point satisfies
(S^-1 + T^-1 a) v = gbar and T^-1 a = N^-1, so the same sweep solves it.

The dense path builds S(theta) = sum_b theta_b C_b from per-band cosine sums
and differentiates the dense solve of Eq. 2 with torch autograd, sharing no
arithmetic with the messenger path.
"""
from __future__ import annotations

import numpy as np

from . import dense, messenger


def band_of_modes(edges, H, W):
    return messenger.band_index(edges, H, W)


def adjoint_solve(problem, gbar, schedule: messenger.Schedule, nP=None):
    """v = (S^-1 + N^-1)^-1 gbar by the messenger iteration."""
    g = np.asarray(gbar, dtype=np.float64)
    return messenger.solve(problem.noise_var, problem.spectrum, lambda c: g,
                           schedule, None, nP, messenger.response_of(problem))


def band_cross_power(x, y, edges, H, W):
    """sum over modes k in band b of Re(conj(fft2(x)_k) fft2(y)_k)."""
    idx = band_of_modes(edges, H, W)
    prod = np.real(np.conj(np.fft.fft2(x)) * np.fft.fft2(y))
    nb = len(edges) - 1
    return np.array([prod[idx == b].sum() for b in range(nb)])


def wiener_vjp(problem, s_wf, gbar, schedule: messenger.Schedule = None, solver: str = "messenger"):
    """(dL/dd, dL/dtheta) for dL/ds* = gbar.  dL/dtheta is only defined for a
    band spectrum; it is None for a power law.  `solver` picks the messenger
    iteration or conjugate gradients for v (same linear system)."""
    if solver == "cg":
        v, it = messenger.wiener_cg(problem, tol=1e-12, rhs=gbar)
        info = it
    else:
        v, info = adjoint_solve(problem, gbar, schedule)
    c = messenger.coefficients(problem.noise_var, problem.spectrum, 1.0, None, messenger.response_of(problem))
    grad_d = c.ninv * v  # A^T N^-1 v
    grad_theta = None
    if problem.spectrum.kind == "bands":
        H, W = problem.H, problem.W
        n = H * W
        theta = np.asarray(problem.spectrum.amps, dtype=np.float64)
        cross = band_cross_power(v, s_wf, problem.spectrum.edges, H, W)
        grad_theta = cross / (n * n * theta ** 2)
    return grad_d, grad_theta, v, info


# --------------------------------------------------------------------------
# Unrolled mode: the gradient of a *truncated* Wiener iteration (a fixed number
# of deterministic sweeps through cooling levels), by reverse-mode through the
# sweeps.  Sweep k maps s_{k-1} -> t_k = (1 - a_k) s_{k-1} + a_k d,
# s_k = ifft2(f_k fft2(t_k)); its transpose filters by f_k in Fourier space and
# then scales by (1 - a_k) in pixel space.
# --------------------------------------------------------------------------

def level_sequence(schedule: messenger.Schedule):
    seq = []
    for lam, k in zip(schedule.lambdas, schedule.sweeps):
        seq += [float(lam)] * int(k)
    return seq


def unrolled_vjp(problem, schedule: messenger.Schedule, gbar):
    """(s_K, dL/dd, dL/dtheta) for L with dL/ds_K = gbar, where s_K is the
    result of the schedule's sweeps from s_0 = 0 (no convergence phase)."""
    H, W = problem.H, problem.W
    n = H * W
    d = np.where(problem.mask, 0.0, problem.d)
    s = np.zeros((H, W))
    tape = []
    for lam in level_sequence(schedule):
        c = messenger.coefficients(problem.noise_var, problem.spectrum, lam, None, messenger.response_of(problem))
        s_new, t = messenger.sweep(s, c.ninv * d, c)
        tape.append((t, c))
        s = s_new
    bands = problem.spectrum.kind == "bands"
    if bands:
        idx = band_of_modes(problem.spectrum.edges, H, W)
        nb = len(problem.spectrum.amps)
        gtheta = np.zeros(nb)
    sbar = np.asarray(gbar, dtype=np.float64)
    dbar = np.zeros((H, W))
    for t, c in reversed(tape):
        F_sbar = np.fft.fft2(sbar)
        if bands:
            # dL/df = Re(conj(F sbar) F t)/n and df/dtheta_b = n T/(nP + T)^2 on band b
            contrib = np.real(np.conj(F_sbar) * np.fft.fft2(t)) * c.T / (c.nP + c.T) ** 2
            gtheta += np.array([contrib[idx == b].sum() for b in range(nb)])
        tbar = np.fft.ifft2(c.f * F_sbar).real
        dbar += c.T * c.ninv * tbar  # dt/dd = T A^T N_eff^-1 (= a when A = I)
        sbar = (1.0 - c.a) * tbar
    return s, dbar, (gtheta if bands else None)


def unrolled_vjp_torch(problem, schedule: messenger.Schedule, gbar):
    """The same gradient by torch autograd through the truncated iteration
    written directly from the sweep's definition (float64, CPU)."""
    import torch
    H, W = problem.H, problem.W
    n = H * W
    nv = problem.noise_var
    obs = np.isfinite(nv)
    tau = float(np.min(nv[obs])) if obs.any() else 1.0
    nbar = torch.from_numpy(np.where(obs, nv - tau, np.inf))
    idx = torch.from_numpy(band_of_modes(problem.spectrum.edges, H, W))
    theta = torch.tensor(np.asarray(problem.spectrum.amps, dtype=np.float64), requires_grad=True)
    d = torch.tensor(np.where(problem.mask, 0.0, problem.d), requires_grad=True)
    nP = n * theta[idx]
    s = torch.zeros((H, W), dtype=torch.float64)
    for lam in level_sequence(schedule):
        T = lam * tau
        a = torch.where(torch.isfinite(nbar), T / (T + nbar), torch.zeros_like(nbar))
        t = (1 - a) * s + a * d
        s = torch.fft.ifft2(nP / (nP + T) * torch.fft.fft2(t)).real
    L = torch.sum(s * torch.from_numpy(np.asarray(gbar, dtype=np.float64)))
    gd, gt = torch.autograd.grad(L, (d, theta))
    return s.detach().numpy(), gd.numpy(), gt.numpy()


# --------------------------------------------------------------------------
# Loss of the differentiation workload: negative log-posterior of the
# Wiener image (Eq. 5-7, up to constants) plus an L2 distance to the true field.
# --------------------------------------------------------------------------

def _likelihood_residual(problem, s_wf):
    """(d - A s) on the pixels that carry data (finite noise, A_i != 0), else 0,
    and the noise variance there (1 elsewhere)."""
    resp = messenger.response_of(problem)
    A = 1.0 if resp is None else np.asarray(resp, dtype=np.float64)
    obs = messenger.observed(problem.noise_var, resp)
    d = np.where(problem.mask, 0.0, problem.d)
    r = np.where(obs, d - A * s_wf, 0.0)
    return r, np.where(obs, problem.noise_var, 1.0)


def loss_terms(problem, s_wf, s_true):
    """L = 1/2 s^T S^-1 s + 1/2 (d - A s)^T N^-1 (d - A s) + 1/2 sum_k ln(n P_k)
           + 1/2 ||s - s_true||^2  at s = s_wf.  The likelihood term sums over
    the pixels that carry data (finite noise and, with a response, A_i != 0);
    A = I when the problem has no response."""
    c = messenger.coefficients(problem.noise_var, problem.spectrum, 1.0, None, messenger.response_of(problem))
    r, nv = _likelihood_residual(problem, s_wf)
    prior = 0.5 * float(np.sum(s_wf * messenger.apply_S_inverse(s_wf, c)))
    like = 0.5 * float(np.sum(r * r / nv))
    logdet = 0.5 * float(np.sum(np.log(c.nP)))
    l2 = 0.5 * float(np.sum((s_wf - s_true) ** 2))
    return prior + like + logdet + l2


def loss_grad(problem, s_wf, s_true, schedule: messenger.Schedule = None, solver: str = "messenger"):
    """Full gradient of loss_terms w.r.t. d and the band amplitudes.

    At the Wiener solution the prior + likelihood part is stationary in s, so
    only the L2 term sends a gradient through s*: gbar = s* - s_true.  The
    explicit part in d is N^-1 (d - A s) on the pixels that carry data."""
    H, W = problem.H, problem.W
    n = H * W
    r, nv = _likelihood_residual(problem, s_wf)
    gd_imp, gt_imp, v, info = wiener_vjp(problem, s_wf, s_wf - s_true, schedule, solver)
    grad_d = r / nv + gd_imp
    theta = np.asarray(problem.spectrum.amps, dtype=np.float64)
    edges = problem.spectrum.edges
    idx = band_of_modes(edges, H, W)
    counts = np.array([np.sum(idx == b) for b in range(len(theta))], dtype=np.float64)
    power = band_cross_power(s_wf, s_wf, edges, H, W)
    grad_theta = -0.5 * power / (n * n * theta ** 2) + 0.5 * counts / theta + gt_imp
    return grad_d, grad_theta


# --------------------------------------------------------------------------
# Dense path (torch autograd, float64, CPU).
# --------------------------------------------------------------------------

def band_basis(edges, H, W):
    """C_b[x, y] = sum_{k in band b} cos(2 pi k.(x - y)/N), shape (B, n, n)."""
    import types
    nb = len(edges) - 1
    out = []
    for b in range(nb):
        amps = np.zeros(nb)
        amps[b] = 1.0
        spec = types.SimpleNamespace(kind="bands", edges=np.asarray(edges), amps=amps)
        out.append(dense.signal_covariance(spec, H, W))
    return np.stack(out)


def dense_wiener_torch(theta, d, noise_var, basis):
    """s* = S A^T (A S A^T + N_o)^-1 d_o as a differentiable torch function."""
    import torch
    nv = np.asarray(noise_var).ravel()
    obs = torch.from_numpy(np.isfinite(nv))
    S = torch.einsum("b,bij->ij", theta, basis)
    No = torch.from_numpy(np.where(np.isfinite(nv), nv, 0.0))[obs]
    So = S[obs][:, obs] + torch.diag(No)
    x = torch.linalg.solve(So, d.reshape(-1)[obs])
    return S[:, obs] @ x


def dense_vjp(problem, gbar, basis=None):
    """(dL/dd, dL/dtheta) of L = <gbar, s*> by torch autograd on the dense solve."""
    import torch
    if basis is None:
        basis = band_basis(problem.spectrum.edges, problem.H, problem.W)
    theta = torch.tensor(np.asarray(problem.spectrum.amps, dtype=np.float64), requires_grad=True)
    d = torch.tensor(np.where(problem.mask, 0.0, problem.d), requires_grad=True)
    s = dense_wiener_torch(theta, d, problem.noise_var, torch.from_numpy(basis))
    L = torch.dot(s, torch.from_numpy(np.asarray(gbar, dtype=np.float64).ravel()))
    gd, gt = torch.autograd.grad(L, (d, theta))
    return gd.numpy(), gt.numpy(), s.detach().numpy().reshape(problem.H, problem.W)
