"""Dense linear-algebra definitions the messenger method converges to.

For images small enough to hold n x n matrices (n <= a few thousand pixels):

* signal covariance S_xy = <s_x s_y> for a statistically homogeneous field
  with power spectrum P(|k|) (Eq. 9, synthesis convention):
      S_xy = sum_k P(|k|) cos(2 pi (k_x dx / W + k_y dy / H)),
  summed directly over the integer modes k in [-N/2, N/2) -- no FFT;
* Wiener filter, Eq. 2-3, with A the selector of the observed pixels so that
  missing pixels (infinite noise, Sec. 1.1) simply drop out:
      s_W = S A^T (A S A^T + N_o)^{-1} d_o;
* posterior covariance of Eq. 7, (S^-1 + A^T N_o^-1 A)^-1, in the equivalent
  Woodbury form S - S A^T (A S A^T + N_o)^-1 A S, which needs no S^-1;
* the mass-mapping posterior (Sec. 5): gamma = A kappa + n with A built from
  explicit sums over the modes (no FFT) and kappa = kappa_E + i kappa_B two
  independent fields with spectra P and b_ratio P, as one real Gaussian
  linear model in [kappa_E; kappa_B];
* the exact stationary law of the Gibbs chain: one sampler sweep is an affine
  map s' = M s + c + B z of the state and of the unit normals z, so the chain
  is a discrete Lyapunov system whose stationary mean solves (I - M) m = c and
  whose covariance solves Sigma = M Sigma M^T + B B^T.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def _mode_grid(N: int) -> np.ndarray:
    return np.arange(-(N // 2), N - N // 2, dtype=np.float64)


def spectrum_on_modes(spectrum, H: int, W: int):
    """(ky, kx, P) on the integer mode grid [-H/2, H/2) x [-W/2, W/2)."""
    ky, kx = np.meshgrid(_mode_grid(H), _mode_grid(W), indexing="ij")
    k = np.hypot(ky, kx)
    if spectrum.kind == "powerlaw":
        P = float(spectrum.amp) * (k + float(spectrum.k0)) ** (-float(spectrum.n))
    elif spectrum.kind == "bands":
        edges = np.asarray(spectrum.edges, dtype=np.float64)
        amps = np.asarray(spectrum.amps, dtype=np.float64)
        P = np.zeros_like(k)
        nb = len(amps)
        for b in range(nb):
            sel = (k >= edges[b]) & ((k < edges[b + 1]) | ((b == nb - 1) & (k <= edges[b + 1])))
            P[sel] = amps[b]
    else:
        raise ValueError(spectrum.kind)
    return ky.ravel(), kx.ravel(), P.ravel()


def autocorrelation(spectrum, H: int, W: int, lam_noise: float = 0.0) -> np.ndarray:
    """c[dy, dx] = sum_k P(|k|) cos(2 pi (k_x dx/W + k_y dy/H))."""
    ky, kx, P = spectrum_on_modes(spectrum, H, W)
    dy, dx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                         indexing="ij")
    phase = 2.0 * np.pi * (np.outer(dy.ravel(), ky) / H + np.outer(dx.ravel(), kx) / W)
    return (np.cos(phase) @ P).reshape(H, W)


def signal_covariance(spectrum, H: int, W: int) -> np.ndarray:
    """Dense S (n x n), pixels in row-major order."""
    c = autocorrelation(spectrum, H, W)
    yy, xx = np.divmod(np.arange(H * W), W)
    dy = (yy[:, None] - yy[None, :]) % H
    dx = (xx[:, None] - xx[None, :]) % W
    return c[dy, dx]


def _observed_rows(noise_var, response):
    nv = noise_var.ravel()
    obs = np.isfinite(nv)
    A = np.ones_like(nv) if response is None else np.asarray(response, dtype=np.float64).ravel()
    obs = obs & (A != 0)
    return nv, obs, A


def effective_noise(noise_var: np.ndarray, lam: float = 1.0, tau: float = None,
                    response=None) -> np.ndarray:
    """N + (lam - 1) tau A^2 on observed pixels (the noise a cooling level sees,
    tau = min N / A^2)."""
    nv, obs, A = _observed_rows(noise_var, response)
    obs = obs.reshape(noise_var.shape)
    A = A.reshape(noise_var.shape)
    if tau is None:
        tau = float(np.min(noise_var[obs] / A[obs] ** 2)) if obs.any() else 1.0
    return np.where(obs, noise_var + (lam - 1.0) * tau * A * A, np.inf)


def wiener_dense(S: np.ndarray, noise_var: np.ndarray, d: np.ndarray, response=None) -> np.ndarray:
    """Eq. 2-3, s_W = S A^T (A S A^T + N)^-1 d over the observed rows of the
    diagonal response A (identity when None; missing pixels drop out)."""
    nv, obs, A = _observed_rows(noise_var, response)
    Ao = A[obs]
    So = Ao[:, None] * S[np.ix_(obs, obs)] * Ao[None, :] + np.diag(nv[obs])
    x = scipy.linalg.solve(So, d.ravel()[obs], assume_a="pos")
    return (S[:, obs] @ (Ao * x)).reshape(noise_var.shape)


def posterior_covariance(S: np.ndarray, noise_var: np.ndarray, response=None) -> np.ndarray:
    """(S^-1 + A^T N_o^-1 A)^-1 = S - S A^T (A S A^T + N_o)^-1 A S  (Eq. 7)."""
    nv, obs, A = _observed_rows(noise_var, response)
    Ao = A[obs]
    So = Ao[:, None] * S[np.ix_(obs, obs)] * Ao[None, :] + np.diag(nv[obs])
    SA = S[:, obs] * Ao[None, :]
    X = scipy.linalg.solve(So, SA.T, assume_a="pos")
    C = S - SA @ X
    return 0.5 * (C + C.T)


def chain_transition(sweep_fn, H: int, W: int):
    """Extract (M, c, B) of a real-chain sweep s' = M s + c + B z by probing
    `sweep_fn(s, xi, eta) -> s'` (complex pair fields; only the real chain is
    read) with unit vectors.  z stacks the pixel draw xi (n), and the real and
    imaginary parts of the harmonic draw eta (2n)."""
    n = H * W
    zero = np.zeros((H, W), dtype=np.complex128)
    c = sweep_fn(zero, zero, zero).real.ravel()
    M = np.empty((n, n))
    B = np.empty((n, 3 * n))
    for i in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[i] = 1.0
        e = e.reshape(H, W)
        M[:, i] = sweep_fn(e, zero, zero).real.ravel() - c
        B[:, i] = sweep_fn(zero, e, zero).real.ravel() - c
        B[:, n + i] = sweep_fn(zero, zero, e).real.ravel() - c
        B[:, 2 * n + i] = sweep_fn(zero, zero, 1j * e).real.ravel() - c
    return M, c, B


def stationary_law(M: np.ndarray, c: np.ndarray, B: np.ndarray):
    """Mean and covariance of the stationary distribution of s' = M s + c + B z."""
    n = M.shape[0]
    mean = np.linalg.solve(np.eye(n) - M, c)
    Q = B @ B.T
    Sigma = scipy.linalg.solve_discrete_lyapunov(M, Q)
    return mean, 0.5 * (Sigma + Sigma.T)


def spin2_operator(H: int, W: int) -> np.ndarray:
    """Complex n x n matrix of gamma = A kappa for the spin-2 shear operator:
    A_xy = (1/n) sum_k D_k e^{2 pi i k.(x - y)}, D_k = (k_1 + i k_2)^2/|k|^2
    (k_1 along x), D_0 = 0, summed over the integer modes directly."""
    ky = _mode_grid(H)
    kx = _mode_grid(W)
    KY, KX = np.meshgrid(ky, kx, indexing="ij")
    den = KX ** 2 + KY ** 2
    D = np.where(den > 0, ((KX ** 2 - KY ** 2) + 2j * KX * KY) / np.where(den > 0, den, 1.0), 0.0)
    yy, xx = np.divmod(np.arange(H * W), W)
    ph = 2j * np.pi * (np.outer(yy, KY.ravel()) / H + np.outer(xx, KX.ravel()) / W)
    E = np.exp(ph)
    return (E * D.ravel()[None, :]) @ np.conj(E).T / (H * W)


def shear_posterior(problem, b_ratio: float):
    """Mean and covariance of [kappa_E; kappa_B] (2n) given the shear data of
    a mass-mapping problem (missing pixels drop out of both components)."""
    H, W = problem.H, problem.W
    n = H * W
    Ac = spin2_operator(H, W)
    A = np.block([[Ac.real, -Ac.imag], [Ac.imag, Ac.real]])
    SE = signal_covariance(problem.spectrum, H, W)
    S = np.block([[SE, np.zeros((n, n))], [np.zeros((n, n)), b_ratio * SE]])
    nv = np.concatenate([problem.noise_var.ravel(), problem.noise_var.ravel()])
    obs = np.isfinite(nv)
    g = np.concatenate([problem.gamma.real.ravel(), problem.gamma.imag.ravel()])
    Ao = A[obs]
    K = Ao @ S @ Ao.T + np.diag(nv[obs])
    SA = S @ Ao.T
    mean = SA @ np.linalg.solve(K, g[obs])
    cov = S - SA @ np.linalg.solve(K, SA.T)
    return mean, 0.5 * (cov + cov.T)
