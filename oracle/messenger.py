"""Messenger-field Wiener filter and Wiener-posterior sampler (FP64, CPU).

Algorithm 1 (Sec. 2.2) with A = I, written step by step in numpy:

  1. pixel space, per pixel i:   t_i = mu_i^t + sigma_i^t G(0,1) with
         mu_i^t      = T/(T + Nbar_i) d_i + Nbar_i/(T + Nbar_i) s_i
         (sigma_i^t)^2 = T Nbar_i / (T + Nbar_i)
  2. t_hat = F_2D(t)
  3. harmonic space, per mode k: s_hat_k = mu_k + sigma_k G(0,1) with
         mu_k = S_k/(S_k + T_k) t_hat_k,  sigma_k^2 = S_k T_k/(S_k + T_k)
  4. s = F_2D^{-1}(s_hat); return s; repeat.

with T = tau I, tau = min_i N_i over observed pixels and Nbar = N - T
(definitions under Algorithm 1).  Missing pixels have infinite noise
(Sec. 1.1), so Nbar_i = inf and the update reduces to t_i = s_i + sqrt(T) G.
Replacing the variates by zero gives the Wiener filter (Sec. 2.2).

Readings of the paper used here (listed with reasons in the design notes):
* power spectrum in the synthesis convention: in the unitary Fourier basis the
  signal covariance S has eigenvalue n P(|k|) on mode k, and T_k = T;
* numpy FFT conventions: T_hat = fft2(t), S_hat = f T_hat + w eta,
  s = ifft2(S_hat), with f = nP/(nP+T) and w = sqrt(n * nP T/(nP+T)), which
  is step 3 in the unitary basis scaled by sqrt(n);
* two real chains ride in one complex field (real and imaginary parts); the
  complex variate eta = z0 + i z1 then gives each of them an independent exact
  conditional draw, since f and w are real and even in k;
* cooling: T = lambda tau with Nbar kept fixed, whose fixed point is the
  Wiener filter for noise N + (lambda - 1) tau;
* the pixel step is written t = (1 - a) s + T b + sigma_t xi with
  a = T/(T + Nbar) and b = N_eff^{-1} d (N_eff = Nbar + T); this is exactly
  mu_i^t above, and it lets a general right-hand side b drive the same sweep
  (the adjoint solve uses b = g);
* convergence residual r = ||t_k - t_{k+1}|| / (T ||b||), which equals
  ||(S^-1 + N_eff^-1) s_k - b|| / ||b|| exactly.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

from . import philox

__all__ = [
    "wavenumbers", "power_spectrum", "Coefficients", "coefficients",
    "pixel_step", "harmonic_step", "sweep", "Schedule", "WienerInfo",
    "wiener", "sample", "initial_state", "apply_S_inverse",
]


def wavenumbers(H: int, W: int) -> np.ndarray:
    """|k| on the unshifted FFT grid, integer indices in grid units."""
    ky = np.fft.fftfreq(H) * H
    kx = np.fft.fftfreq(W) * W
    return np.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)


def power_spectrum(spectrum, H: int, W: int) -> np.ndarray:
    """P(|k|) per mode (Eq. 9), from the spectrum's parameters."""
    k = wavenumbers(H, W)
    if spectrum.kind == "powerlaw":
        return float(spectrum.amp) * (k + float(spectrum.k0)) ** (-float(spectrum.n))
    if spectrum.kind == "bands":
        edges = np.asarray(spectrum.edges, dtype=np.float64)
        amps = np.asarray(spectrum.amps, dtype=np.float64)
        out = np.zeros_like(k)  # a mode outside every band has no signal power
        for b in range(len(amps)):
            lo, hi = edges[b], edges[b + 1]
            sel = (k >= lo) & ((k < hi) | ((b == len(amps) - 1) & (k <= hi)))
            out[sel] = amps[b]
        return out
    raise ValueError(spectrum.kind)


def band_index(edges, H: int, W: int) -> np.ndarray:
    """Band of each mode: edges[b] <= |k| < edges[b+1], last band closed."""
    k = wavenumbers(H, W)
    edges = np.asarray(edges, dtype=np.float64)
    nb = len(edges) - 1
    idx = np.full(k.shape, -1, dtype=np.int64)
    for b in range(nb):
        sel = (k >= edges[b]) & ((k < edges[b + 1]) | ((b == nb - 1) & (k <= edges[b + 1])))
        idx[sel] = b
    return idx


@dataclasses.dataclass
class Coefficients:
    """Diagonal coefficients of one sweep at one cooling level."""
    tau: float
    T: float
    a: np.ndarray        # T/(T+Nbar), 0 where masked
    sig_t: np.ndarray    # sqrt(T Nbar/(T+Nbar)) = sqrt(T (1-a))
    ninv: np.ndarray     # 1/(Nbar+T) = a/T, 0 where masked
    nP: np.ndarray       # n P(|k|), eigenvalues of S in the unitary basis
    f: np.ndarray        # nP/(nP+T)
    w: np.ndarray        # sqrt(n * nP T/(nP+T)) (numpy FFT scaling)
    vk: np.ndarray       # nP T/(nP+T), eigenvalues of (S^-1 + T^-1)^-1


def observed(noise_var: np.ndarray, response: Optional[np.ndarray] = None) -> np.ndarray:
    """Pixels that carry data: finite noise and, with a response A, A_i != 0."""
    obs = np.isfinite(noise_var)
    if response is not None:
        obs = obs & (np.asarray(response) != 0)
    return obs


def messenger_tau(noise_var: np.ndarray, response: Optional[np.ndarray] = None) -> float:
    """tau = min over observed pixels of N_i / A_i^2, the diagonal of
    (A^-1)^dagger N A^-1 (T = tau I under Algorithm 1); 1.0 when every pixel
    is missing (any T works then: the chain samples the prior)."""
    obs = observed(noise_var, response)
    if not obs.any():
        return 1.0
    A2 = 1.0 if response is None else np.asarray(response, dtype=np.float64)[obs] ** 2
    return float(np.min(noise_var[obs] / A2))


def coefficients(noise_var: np.ndarray, spectrum, lam: float = 1.0,
                 nP: Optional[np.ndarray] = None,
                 response: Optional[np.ndarray] = None) -> Coefficients:
    """Coefficients of Algorithm 1's definitions with a diagonal A (identity
    when `response` is None): Nbar_i = N_i - tau A_i^2, and on observed pixels
        mu_i^t = T A_i d_i / (T A_i^2 + Nbar_i) + Nbar_i s_i / (T A_i^2 + Nbar_i),
        (sigma_i^t)^2 = T Nbar_i / (T A_i^2 + Nbar_i),
    i.e. a = T A^2 / (T A^2 + Nbar), mu = (1 - a) s + T b with
    b = A d / (T A^2 + Nbar) = A^T N_eff^-1 d, sigma_t^2 = T (1 - a)."""
    H, W = noise_var.shape
    n = H * W
    obs = observed(noise_var, response)
    A = np.ones((H, W)) if response is None else np.asarray(response, dtype=np.float64)
    tau = messenger_tau(noise_var, response)
    T = float(lam) * tau
    with np.errstate(invalid="ignore", divide="ignore"):
        # Nbar >= 0 by the choice of tau; the clamp removes the rounding of (N/A^2) A^2
        nbar = np.where(obs, np.maximum(noise_var - tau * A * A, 0.0), np.inf)
        den = np.where(obs, T * A * A + nbar, np.inf)
        a = np.where(obs, T * A * A / den, 0.0)
        ninv = np.where(obs, A / den, 0.0)
    sig_t = np.sqrt(T * (1.0 - a))
    if nP is None:
        nP = n * power_spectrum(spectrum, H, W)
    f = nP / (nP + T)
    vk = nP * T / (nP + T)
    w = np.sqrt(n * vk)
    return Coefficients(tau=tau, T=T, a=a, sig_t=sig_t, ninv=ninv, nP=nP,
                        f=f, w=w, vk=vk)


def response_of(problem) -> Optional[np.ndarray]:
    return getattr(problem, "response", None)


def pixel_step(s, b, c: Coefficients, xi=None):
    """Step 1: t = (1 - a) s + T b (+ sigma_t xi).  For a complex chain pair
    the real right-hand side b drives both chains."""
    src = c.T * b
    if np.iscomplexobj(s):
        src = src * (1.0 + 1.0j)
    t = (1.0 - c.a) * s + src
    if xi is not None:
        t = t + c.sig_t * xi
    return t


def harmonic_step(t_hat, c: Coefficients, eta=None):
    """Step 3 in numpy FFT scaling: S_hat = f T_hat (+ w eta)."""
    s_hat = c.f * t_hat
    if eta is not None:
        s_hat = s_hat + c.w * eta
    return s_hat


def sweep(s, b, c: Coefficients, xi=None, eta=None):
    """One pass of Algorithm 1.  Returns (s_new, t)."""
    t = pixel_step(s, b, c, xi)
    t_hat = np.fft.fft2(t)
    s_hat = harmonic_step(t_hat, c, eta)
    s_new = np.fft.ifft2(s_hat)
    if not np.iscomplexobj(s):
        s_new = s_new.real
    return s_new, t


def apply_S_inverse(x: np.ndarray, c: Coefficients) -> np.ndarray:
    """S^{-1} x (S diagonal in Fourier space with eigenvalues nP)."""
    return np.fft.ifft2(np.fft.fft2(x) / c.nP).real


# --------------------------------------------------------------------------
# Wiener filter: variates set to zero, cooling levels, residual stopping.
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Schedule:
    """Cooling schedule: run sweeps[j] sweeps at lambda[j] for each level j,
    then (if tol > 0) keep sweeping at the last lambda, testing the residual
    every `check_every` sweeps, until it is <= tol or `max_sweeps` sweeps
    have been done in total."""
    lambdas: Sequence[float] = (1.0,)
    sweeps: Sequence[int] = (0,)
    tol: float = 0.0
    max_sweeps: int = 0
    check_every: int = 10

    @staticmethod
    def geometric(lam_start: float, lam_end: float, levels: int,
                  sweeps_per_level: int, tol: float = 0.0,
                  max_sweeps: int = 0, check_every: int = 10) -> "Schedule":
        lams = np.geomspace(lam_start, lam_end, levels) if levels > 1 else [lam_end]
        return Schedule(tuple(float(x) for x in lams), (int(sweeps_per_level),) * levels,
                        tol, max_sweeps, check_every)

    @staticmethod
    def fixed(n_sweeps: int, lam: float = 1.0) -> "Schedule":
        return Schedule((float(lam),), (int(n_sweeps),), 0.0, 0, 10)


@dataclasses.dataclass
class WienerInfo:
    sweeps: int
    residual: float
    converged: bool


def _norm(x) -> float:
    return float(np.sqrt(np.sum(np.abs(x) ** 2)))


def solve(noise_var, spectrum, rhs_of, schedule: Schedule, s0=None,
          nP: Optional[np.ndarray] = None, response: Optional[np.ndarray] = None):
    """Deterministic messenger iteration with right-hand side b = rhs_of(c)
    at each cooling level.  Returns (s, WienerInfo)."""
    H, W = noise_var.shape
    s = np.zeros((H, W)) if s0 is None else np.array(s0, dtype=np.float64)
    total = 0
    c = None
    for lam, k in zip(schedule.lambdas, schedule.sweeps):
        c = coefficients(noise_var, spectrum, lam, nP, response)
        b = rhs_of(c)
        for _ in range(int(k)):
            s, _ = sweep(s, b, c)
            total += 1
    residual = float("nan")
    converged = schedule.tol <= 0
    if schedule.tol > 0:
        c = coefficients(noise_var, spectrum, schedule.lambdas[-1], nP, response)
        b = rhs_of(c)
        bnorm = _norm(b)
        t_prev = None
        while total < schedule.max_sweeps:
            s, t = sweep(s, b, c)
            total += 1
            if total % schedule.check_every == 0 and t_prev is not None:
                residual = _norm(t - t_prev) / (c.T * bnorm) if bnorm > 0 else 0.0
                if residual <= schedule.tol:
                    converged = True
                    break
            # the messenger of the next sweep is compared with this one
            t_prev = t if (total + 1) % schedule.check_every == 0 else None
    return s, WienerInfo(total, residual, converged)


def wiener(problem, schedule: Schedule, s0=None, nP=None):
    """Wiener filter of one problem by the messenger iteration."""
    d = np.where(problem.mask, 0.0, problem.d)
    return solve(problem.noise_var, problem.spectrum, lambda c: c.ninv * d,
                 schedule, s0, nP, response_of(problem))


def residual(problem, s, lam: float = 1.0) -> float:
    """Relative residual ||(S^-1 + N_eff^-1) s - N_eff^-1 d|| / ||N_eff^-1 d||
    of the normal equations (Eq. 7) at cooling level lam, by definition."""
    c = coefficients(problem.noise_var, problem.spectrum, lam, None, response_of(problem))
    d = np.where(problem.mask, 0.0, problem.d)
    b = c.ninv * d
    A = 1.0 if response_of(problem) is None else response_of(problem)
    r = apply_S_inverse(s, c) + c.ninv * A * s - b
    return _norm(r) / _norm(b)


def wiener_cg(problem, tol: float = 1e-12, max_iter: int = 20000, lam: float = 1.0, rhs=None):
    """The Wiener filter as the exact solution of its normal equations (Eq. 7),
    (S^-1 + N_eff^-1) s = b with b = N_eff^-1 d (or a given rhs), by conjugate
    gradients on the S-preconditioned form (I + S^1/2 N^-1 S^1/2) x = S^1/2 b,
    s = S^1/2 x.  A second, independent route to the same fixed point for images
    too large for dense algebra; S^1/2 is diagonal in Fourier space."""
    c = coefficients(problem.noise_var, problem.spectrum, lam, None, response_of(problem))
    d = np.where(problem.mask, 0.0, problem.d)
    b = c.ninv * d if rhs is None else np.asarray(rhs, dtype=np.float64)
    A = 1.0 if response_of(problem) is None else response_of(problem)
    prec = c.ninv * A  # A^T N_eff^-1 A
    sq = np.sqrt(c.nP)

    def half(x):  # S^1/2 x
        return np.fft.ifft2(sq * np.fft.fft2(x)).real

    def op(x):
        return x + half(prec * half(x))

    rhs_x = half(b)
    x = np.zeros_like(rhs_x)
    r = rhs_x - op(x)
    p = r.copy()
    rr = float(np.sum(r * r))
    r0 = np.sqrt(rr)
    it = 0
    while np.sqrt(rr) > tol * r0 and it < max_iter:
        Ap = op(p)
        alpha = rr / float(np.sum(p * Ap))
        x += alpha * p
        r -= alpha * Ap
        rr_new = float(np.sum(r * r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return half(x), it


# --------------------------------------------------------------------------
# Sampler (Algorithm 1 with the counter-based normal stream).
# --------------------------------------------------------------------------

def initial_state(seed: int, problem_index: int, pair: int, H: int, W: int,
                  scale: float = 0.0) -> np.ndarray:
    """Chain-pair start: 0, or scale * (z0 + i z1) from the init stream."""
    if scale == 0.0:
        return np.zeros((H, W), dtype=np.complex128)
    z0, z1 = philox.stream_normals(seed, philox.STAGE_INIT, 0, problem_index,
                                   pair, H * W)
    return scale * (z0 + 1j * z1).reshape(H, W)


def pair_normals(seed: int, stage: int, sweep_index: int, problem_index: int,
                 pair: int, H: int, W: int) -> np.ndarray:
    z0, z1 = philox.stream_normals(seed, stage, sweep_index, problem_index,
                                   pair, H * W)
    return (z0 + 1j * z1).reshape(H, W)


def sample_pair(problem, seed: int, problem_index: int, pair: int,
                burn_in: int, n_samples: int, thin: int = 1,
                s0: Optional[np.ndarray] = None, sweep_offset: int = 0,
                c: Optional[Coefficients] = None, cooling: Sequence = ()):
    """Run one chain pair; returns (samples [2, n_samples, H, W], last state).

    Sweep k (global index sweep_offset + k) draws xi from stage 0 and eta from
    stage 1 of the stream.  A sample is the state after sweep k when
    k >= burn_in and (k - burn_in + 1) is a multiple of thin.  `cooling`
    levels (lambda, sweeps) run first, each sweep drawn at T = lambda tau
    (so it samples the posterior for noise N + (lambda - 1) tau), taking the
    global sweep indices before the burn-in's."""
    H, W = problem.H, problem.W
    if c is None:
        c = coefficients(problem.noise_var, problem.spectrum, 1.0, None, response_of(problem))
    d = np.where(problem.mask, 0.0, problem.d)
    s = np.zeros((H, W), dtype=np.complex128) if s0 is None else np.array(s0, dtype=np.complex128)
    for lam, n_lev in cooling:
        cl = coefficients(problem.noise_var, problem.spectrum, float(lam), None, response_of(problem))
        for _ in range(int(n_lev)):
            xi = pair_normals(seed, philox.STAGE_PIXEL, sweep_offset, problem_index, pair, H, W)
            eta = pair_normals(seed, philox.STAGE_HARMONIC, sweep_offset, problem_index, pair, H, W)
            s, _ = sweep(s, cl.ninv * d, cl, xi, eta)
            sweep_offset += 1
    b = c.ninv * d
    out = np.empty((2, n_samples, H, W))
    emitted = 0
    total = burn_in + n_samples * thin
    for k in range(total):
        g = sweep_offset + k
        xi = pair_normals(seed, philox.STAGE_PIXEL, g, problem_index, pair, H, W)
        eta = pair_normals(seed, philox.STAGE_HARMONIC, g, problem_index, pair, H, W)
        s, _ = sweep(s, b, c, xi, eta)
        if k >= burn_in and (k - burn_in + 1) % thin == 0:
            out[0, emitted] = s.real
            out[1, emitted] = s.imag
            emitted += 1
    return out, s


def sample(problem, seed: int, problem_index: int, n_chains: int,
           burn_in: int, n_samples: int, thin: int = 1, init_scale: float = 0.0,
           pairs: Optional[List[int]] = None):
    """Samples [n_chains, n_samples, H, W]; chain 2p / 2p+1 = Re / Im of pair p."""
    H, W = problem.H, problem.W
    n_pairs = (n_chains + 1) // 2
    c = coefficients(problem.noise_var, problem.spectrum, 1.0, None, response_of(problem))
    out = np.empty((n_chains, n_samples, H, W))
    for p in (range(n_pairs) if pairs is None else pairs):
        s0 = initial_state(seed, problem_index, p, H, W, init_scale)
        smp, _ = sample_pair(problem, seed, problem_index, p, burn_in, n_samples,
                             thin, s0, 0, c)
        out[2 * p] = smp[0]
        if 2 * p + 1 < n_chains:
            out[2 * p + 1] = smp[1]
    return out
