"""Power-spectrum Gibbs step and the hierarchical sampler (FP64, CPU).

Sec. 5 extends the sampler to infer the power spectrum itself: draw P(k)
given the current signal, then the signal given P(k), and repeat.  For a
spectrum that is constant, theta_b, on each band b of |k| the conditional is
closed-form.  With S = U^dagger diag(n P_k) U (synthesis convention, see
``messenger``) and numpy's unnormalised s_hat = fft2(s),

    -2 log p(s | theta) = sum_k |s_hat_k|^2 / (n^2 P_k) + sum_k log(n P_k) + const,

so with m_b modes in band b and band power sigma_b = sum_{k in b} |s_hat_k|^2,
p(theta_b | s) is proportional to theta_b^(-m_b/2) exp(-sigma_b / (2 n^2 theta_b)).
An inverse-gamma prior with nu_0/2 shape and beta_0 scale (nu_0 = beta_0 = 0
is Jeffreys' 1/theta) keeps it inverse-gamma:

    theta_b | s ~ IG((m_b + nu_0)/2, beta_0 + sigma_b/(2 n^2)),

drawn exactly as theta_b = (2 beta_0 + sigma_b/n^2) / x_b with x_b a
chi-square variate of nu_b = m_b + nu_0 degrees of freedom, made as the sum of
nu_b squared unit normals from stage 3 of the stream.  Bands with nu_b <= 0 (or
a zero chi-square sum) keep their amplitude.

Each chain of a pair has its own band amplitudes, so the two chains of a pair
no longer share the harmonic coefficients f and w.  The sweep is written here
per chain, on real fields: chain A takes the real parts of the pixel and mode
variates of the pair's stream, chain B the imaginary parts,

    t_X   = (1 - a) s_X + a d + sigma_t xi_X
    s_A   = ifft2(f_A fft2(t_A)).real + ifft2(w_A eta).real
    s_B   = ifft2(f_B fft2(t_B)).real + ifft2(w_B eta).imag

which is the pair sweep of ``messenger`` when f_A = f_B and w_A = w_B.

Iteration i (global index g = iteration_offset + i) runs `sweeps` messenger
sweeps (global sweep indices g*sweeps + k) with theta^(i) and then draws
theta^(i+1) from the new signal with the stage-3 stream at counter word 1 = g.
The chi-square normals of band b are the flat elements prefix_b .. prefix_b +
nu_b - 1 (prefix over the bands in order); chain A sums their z0, chain B their z1.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from . import messenger, philox


def band_counts(edges, H: int, W: int) -> np.ndarray:
    """m_b: number of modes of the H x W grid in each band."""
    idx = messenger.band_index(edges, H, W)
    nb = len(edges) - 1
    return np.array([np.sum(idx == b) for b in range(nb)], dtype=np.int64)


def band_power(x: np.ndarray, edges, H: int, W: int) -> np.ndarray:
    """sigma_b = sum over the modes of band b of |fft2(x)_k|^2."""
    idx = messenger.band_index(edges, H, W)
    p = np.abs(np.fft.fft2(x)) ** 2
    return np.array([p[idx == b].sum() for b in range(len(edges) - 1)])


def degrees_of_freedom(counts: np.ndarray, prior_dof: int) -> np.ndarray:
    return np.maximum(np.asarray(counts, dtype=np.int64) + int(prior_dof), 0)


def chi2_normals(seed: int, iteration: int, problem_index: int, pair: int, total: int):
    """(z0, z1): the stage-3 normals of one chain pair for one iteration."""
    n = total + (total % 2)
    if n == 0:
        return np.zeros(0), np.zeros(0)
    z0, z1 = philox.stream_normals(seed, philox.STAGE_SPECTRUM, iteration, problem_index, pair, n)
    return z0[:total], z1[:total]


def draw_theta(theta: np.ndarray, sigma: np.ndarray, dof: np.ndarray, z: np.ndarray,
               n: int, prior_beta: float) -> np.ndarray:
    """theta_b = (2 beta_0 + sigma_b / n^2) / sum of dof_b squared normals."""
    out = np.array(theta, dtype=np.float64)
    start = 0
    for b in range(len(dof)):
        k = int(dof[b])
        if k > 0:
            x = float(np.sum(z[start:start + k] ** 2))
            if x > 0.0:
                out[b] = (2.0 * prior_beta + sigma[b] / float(n) ** 2) / x
        start += k
    return out


def chain_coefficients(problem, theta: np.ndarray) -> messenger.Coefficients:
    """Sweep coefficients at lambda = 1 for band amplitudes theta."""
    H, W = problem.H, problem.W
    spec = type("S", (), {"kind": "bands", "edges": np.asarray(problem.spectrum.edges),
                          "amps": np.asarray(theta, dtype=np.float64)})()
    return messenger.coefficients(problem.noise_var, spec, 1.0, None, messenger.response_of(problem))


def chain_sweep(sA, sB, d, cA: messenger.Coefficients, cB: messenger.Coefficients, xi, eta):
    """One messenger sweep of the two chains of a pair with their own spectra."""
    b = cA.ninv * d  # the pixel coefficients do not depend on the spectrum
    tA = (1.0 - cA.a) * sA + cA.T * b + cA.sig_t * xi.real
    tB = (1.0 - cA.a) * sB + cA.T * b + cA.sig_t * xi.imag
    nA = np.fft.ifft2(cA.w * eta)
    nB = np.fft.ifft2(cB.w * eta)
    sA = np.fft.ifft2(cA.f * np.fft.fft2(tA)).real + nA.real
    sB = np.fft.ifft2(cB.f * np.fft.fft2(tB)).real + nB.imag
    return sA, sB


def sample_pair_hierarchical(problem, seed: int, problem_index: int, pair: int,
                             burn_in: int, n_samples: int, thin: int = 1, sweeps: int = 1,
                             prior_dof: int = 0, prior_beta: float = 0.0,
                             theta0: Optional[Sequence[np.ndarray]] = None,
                             s0: Optional[np.ndarray] = None, iteration_offset: int = 0):
    """Gibbs chain pair over (s, theta).  Returns
    (theta samples [2, n_samples, n_bands], s samples [2, n_samples, H, W],
     final pair state (complex), final theta [2, n_bands]).
    A sample is (s^(i), theta^(i+1)) after iteration i when i >= burn_in and
    (i - burn_in + 1) is a multiple of thin."""
    H, W = problem.H, problem.W
    n = H * W
    edges = np.asarray(problem.spectrum.edges)
    nb = len(edges) - 1
    counts = band_counts(edges, H, W)
    dof = degrees_of_freedom(counts, prior_dof)
    total = int(dof.sum())
    base = np.asarray(problem.spectrum.amps, dtype=np.float64)
    thA = np.array(base if theta0 is None else theta0[0], dtype=np.float64)
    thB = np.array(base if theta0 is None else theta0[1], dtype=np.float64)
    d = np.where(problem.mask, 0.0, problem.d)
    s = np.zeros((H, W), dtype=np.complex128) if s0 is None else np.array(s0, dtype=np.complex128)
    sA, sB = s.real.copy(), s.imag.copy()
    th_out = np.empty((2, n_samples, nb))
    s_out = np.empty((2, n_samples, H, W))
    emitted = 0
    iters = burn_in + n_samples * thin
    for i in range(iters):
        g = iteration_offset + i
        cA = chain_coefficients(problem, thA)
        cB = chain_coefficients(problem, thB)
        for k in range(sweeps):
            sw = g * sweeps + k
            xi = messenger.pair_normals(seed, philox.STAGE_PIXEL, sw, problem_index, pair, H, W)
            eta = messenger.pair_normals(seed, philox.STAGE_HARMONIC, sw, problem_index, pair, H, W)
            sA, sB = chain_sweep(sA, sB, d, cA, cB, xi, eta)
        z0, z1 = chi2_normals(seed, g, problem_index, pair, total)
        thA = draw_theta(thA, band_power(sA, edges, H, W), dof, z0, n, prior_beta)
        thB = draw_theta(thB, band_power(sB, edges, H, W), dof, z1, n, prior_beta)
        if i >= burn_in and (i - burn_in + 1) % thin == 0:
            th_out[0, emitted], th_out[1, emitted] = thA, thB
            s_out[0, emitted], s_out[1, emitted] = sA, sB
            emitted += 1
    return th_out, s_out, sA + 1j * sB, np.stack([thA, thB])
