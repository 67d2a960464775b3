"""Pins of the dense definitions (Eq. 2-3, Eq. 7, Eq. 9) the oracle uses."""
import numpy as np
import pytest

from oracle import dense
from paper_1810_02821_amd import synth


def _spec():
    return synth.spectrum_powerlaw(1.0, 1.0, 2.0)


def test_signal_covariance_is_circulant_with_spectrum_eigenvalues():
    H = W = 8
    S = dense.signal_covariance(_spec(), H, W)
    assert np.allclose(S, S.T, atol=1e-13)
    # eigenvalues of a 2D-circulant matrix are the 2D DFT of its first row;
    # under the synthesis convention they must be n P(|k|)
    row = S[0].reshape(H, W)
    eig = np.fft.fft2(row).real
    ky = np.fft.fftfreq(H) * H
    kx = np.fft.fftfreq(W) * W
    k = np.hypot(ky[:, None], kx[None, :])
    assert np.allclose(eig, H * W * (k + 1.0) ** -2.0, rtol=1e-12)
    # pixel variance is the sum of the spectrum
    assert np.isclose(S[0, 0], np.sum((k + 1.0) ** -2.0))


def test_generator_field_has_covariance_S():
    H = W = 6
    spec = _spec()
    S = dense.signal_covariance(spec, H, W)
    rng = np.random.default_rng(0)
    X = np.stack([synth.grf(H, W, spec, rng).ravel() for _ in range(40000)])
    emp = X.T @ X / X.shape[0]
    assert np.max(np.abs(emp - S)) < 0.05 * S[0, 0]


def test_wiener_homoscedastic_unmasked_is_fourier_filter():
    # textbook special case: N = sigma^2 I => s_W = F^-1[nP/(nP+sigma^2) F d]
    H = W = 8
    sig2 = 0.7
    spec = _spec()
    S = dense.signal_covariance(spec, H, W)
    rng = np.random.default_rng(1)
    d = rng.standard_normal((H, W))
    nv = np.full((H, W), sig2)
    sw = dense.wiener_dense(S, nv, d)
    ky = np.fft.fftfreq(H) * H
    kx = np.fft.fftfreq(W) * W
    nP = H * W * (np.hypot(ky[:, None], kx[None, :]) + 1.0) ** -2.0
    ref = np.fft.ifft2(nP / (nP + sig2) * np.fft.fft2(d)).real
    assert np.allclose(sw, ref, atol=1e-12)


def test_all_masked_gives_zero_filter_and_prior_covariance():
    H = W = 4
    S = dense.signal_covariance(_spec(), H, W)
    nv = np.full((H, W), np.inf)
    assert np.all(dense.wiener_dense(S, nv, np.zeros((H, W))) == 0)
    assert np.allclose(dense.posterior_covariance(S, nv), S)


def test_posterior_covariance_equals_precision_inverse():
    # Woodbury form against (S^-1 + N^-1)^-1 when nothing is masked
    p = synth.config_small(3, 8)
    nv = np.where(np.isfinite(p.noise_var), p.noise_var, 1.3)
    S = dense.signal_covariance(p.spectrum, 8, 8)
    C = dense.posterior_covariance(S, nv)
    ref = np.linalg.inv(np.linalg.inv(S) + np.diag(1.0 / nv.ravel()))
    assert np.allclose(C, ref, rtol=1e-8, atol=1e-10)


def test_wiener_is_the_posterior_mode():
    # the Wiener filter minimises the negative log-posterior of Eq. 7
    p = synth.config_small(4, 8)
    S = dense.signal_covariance(p.spectrum, 8, 8)
    sw = dense.wiener_dense(S, p.noise_var, p.d).ravel()
    Sinv = np.linalg.inv(S)
    ninv = np.where(np.isfinite(p.noise_var), 1.0 / p.noise_var, 0.0).ravel()
    grad = Sinv @ sw - ninv * (p.d.ravel() - sw)
    assert np.linalg.norm(grad) < 1e-8 * np.linalg.norm(ninv * p.d.ravel())
