"""Mass mapping from shear (Sec. 5): the messenger Wiener filter and sampler
for a spin-2 operator A, FP64, CPU.

The data are the complex shear gamma = gamma_1 + i gamma_2 per pixel, the
signal the complex convergence kappa = kappa_E + i kappa_B (two real
Gaussian random fields, E with spectrum P_E, B with P_B = r P_E), and
gamma = A kappa + n with A = F^-1 D F, D_k = (k_1 + i k_2)^2 / |k|^2 (the
Kaiser-Squires relation between convergence and shear; D_0 = 0: the mean
convergence is not measured), n of variance N_i per component.

The messenger field lives in shear space (T = tau I, tau = min N, Nbar = N - T):
    t | kappa, gamma   = (1 - a) A kappa + a gamma + sqrt(T (1 - a)) (xi_1 + i xi_2),
    kappa | t          per mode: u = conj(D) fft2(t); its E and B parts
                       u_E = (u(k) + conj u(-k)) / 2,  u_B = (u(k) - conj u(-k)) / (2i)
                       (the spectra of the real fields Re and Im of ifft2(u)) get the
                       Wiener-sampler step of each real field,
    kappa_E = ifft2(f_E fft2(z_E)).real + ifft2(w_E eta).real,   z = ifft2(u),
    kappa_B = ifft2(f_B fft2(z_B)).real + ifft2(w_B eta).imag,
with f = nP/(nP + T), w = sqrt(n nP T/(nP + T)) per field (|D| = 1 for k != 0),
and at k = 0 (D = 0, no data) f = 0, w = sqrt(n nP): the prior.  The sweep's
state is the model shear A kappa; kappa itself is F^-1 of the mode values.
The variates: xi from stage 0 (pixel), eta from stage 1 (mode) of the stream,
one chain per stream "pair" index.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import messenger, philox


def ks_kernel(H: int, W: int) -> np.ndarray:
    """D_k on the unshifted FFT grid (k_1 along x, k_2 along y); D_0 = 0."""
    k2 = (np.fft.fftfreq(H) * H)[:, None]
    k1 = (np.fft.fftfreq(W) * W)[None, :]
    den = k1 ** 2 + k2 ** 2
    with np.errstate(invalid="ignore", divide="ignore"):
        D = ((k1 ** 2 - k2 ** 2) + 2j * k1 * k2) / den
    D[0, 0] = 0.0
    return D


def apply_A(kappa: np.ndarray) -> np.ndarray:
    H, W = kappa.shape
    return np.fft.ifft2(ks_kernel(H, W) * np.fft.fft2(kappa))


class ShearCoefficients:
    def __init__(self, problem, b_ratio: float, lam: float = 1.0):
        H, W = problem.H, problem.W
        n = H * W
        c = messenger.coefficients(problem.noise_var, problem.spectrum, lam)
        self.T, self.a, self.sig_t = c.T, c.a, c.sig_t
        self.D = ks_kernel(H, W)
        nPE = c.nP
        nPB = float(b_ratio) * nPE
        self.fE, self.wE = nPE / (nPE + c.T), np.sqrt(n * nPE * c.T / (nPE + c.T))
        self.fB, self.wB = nPB / (nPB + c.T), np.sqrt(n * nPB * c.T / (nPB + c.T))
        # no data at k = 0: the prior
        self.fE[0, 0] = self.fB[0, 0] = 0.0
        self.wE[0, 0] = np.sqrt(n * nPE[0, 0])
        self.wB[0, 0] = np.sqrt(n * nPB[0, 0])


def shear_sweep(s_gamma, gamma, c: ShearCoefficients, xi=None, eta=None):
    """One sweep: returns (new model shear A kappa, kappa)."""
    t = (1.0 - c.a) * s_gamma + c.a * gamma
    if xi is not None:
        t = t + c.sig_t * xi
    z = np.fft.ifft2(np.conj(c.D) * np.fft.fft2(t))
    kE = np.fft.ifft2(c.fE * np.fft.fft2(z.real)).real
    kB = np.fft.ifft2(c.fB * np.fft.fft2(z.imag)).real
    if eta is not None:
        kE = kE + np.fft.ifft2(c.wE * eta).real
        kB = kB + np.fft.ifft2(c.wB * eta).imag
    kappa = kE + 1j * kB
    return apply_A(kappa), kappa


def shear_data(problem) -> np.ndarray:
    return np.where(problem.mask, 0.0, problem.gamma)


def wiener_shear(problem, schedule: messenger.Schedule, b_ratio: float = 0.0):
    """Wiener filter of kappa by the deterministic sweeps of the schedule
    (fixed sweep counts) from kappa = 0."""
    g = shear_data(problem)
    s = np.zeros((problem.H, problem.W), dtype=np.complex128)
    kappa = s
    for lam, k in zip(schedule.lambdas, schedule.sweeps):
        c = ShearCoefficients(problem, b_ratio, lam)
        for _ in range(int(k)):
            s, kappa = shear_sweep(s, g, c)
    return kappa


def sample_shear_chain(problem, seed: int, problem_index: int, chain: int, burn_in: int,
                       n_samples: int, thin: int = 1, b_ratio: float = 0.0,
                       s0: Optional[np.ndarray] = None, sweep_offset: int = 0):
    """Samples of kappa [n_samples, H, W] (complex) and the final model shear."""
    H, W = problem.H, problem.W
    c = ShearCoefficients(problem, b_ratio)
    g = shear_data(problem)
    s = np.zeros((H, W), dtype=np.complex128) if s0 is None else np.array(s0, dtype=np.complex128)
    out = np.empty((n_samples, H, W), dtype=np.complex128)
    emitted = 0
    for k in range(burn_in + n_samples * thin):
        sw = sweep_offset + k
        xi = messenger.pair_normals(seed, philox.STAGE_PIXEL, sw, problem_index, chain, H, W)
        eta = messenger.pair_normals(seed, philox.STAGE_HARMONIC, sw, problem_index, chain, H, W)
        s, kappa = shear_sweep(s, g, c, xi, eta)
        if k >= burn_in and (k - burn_in + 1) % thin == 0:
            out[emitted] = kappa
            emitted += 1
    return out, s
