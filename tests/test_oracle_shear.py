"""Pins of the mass-mapping oracle (spin-2 operator A) against dense Gaussian
algebra built without FFTs: A from explicit sums over the modes, S from the
cosine sums of ``dense.signal_covariance``."""
import numpy as np
import pytest

from oracle import dense, messenger as om, shear as osh
from paper_1810_02821_amd import synth


_dense_A = dense.spin2_operator
_dense_posterior = dense.shear_posterior


def test_kernel_is_unitary_off_zero_and_matches_the_generator():
    D = osh.ks_kernel(16, 16)
    m = np.abs(D)
    assert D[0, 0] == 0 and np.allclose(m.ravel()[1:], 1.0)
    # D(-k) = D(k) off the Nyquist lines (there -k aliases to the same index)
    mirror = np.roll(np.flip(D), 1, axis=(0, 1))
    inner = np.ones((16, 16), dtype=bool)
    inner[8, :] = inner[:, 8] = False
    assert np.allclose(D[inner], mirror[inner])
    kappa = np.random.default_rng(0).standard_normal((16, 16))
    assert np.allclose(osh.apply_A(kappa), synth.shear_from_convergence(kappa))
    assert np.allclose(osh.apply_A(kappa).ravel(), _dense_A(16, 16) @ kappa.ravel())


@pytest.mark.parametrize("b_ratio", [0.0, 0.5])
def test_shear_wiener_filter_equals_dense(b_ratio):
    p = synth.config_shear(1, 16, b_ratio)
    mean, _ = _dense_posterior(p, b_ratio)
    sch = om.Schedule(tuple(np.geomspace(100.0, 1.0, 20)) + (1.0,), (20,) * 20 + (20000,))
    kappa = osh.wiener_shear(p, sch, b_ratio)
    ref = mean[:256] + 1j * mean[256:]
    assert np.max(np.abs(kappa.ravel() - ref)) < 1e-7 * np.max(np.abs(ref))


@pytest.mark.parametrize("b_ratio", [0.0, 0.7])
def test_shear_sampler_has_the_exact_posterior(b_ratio):
    """The sweep is affine in (kappa, xi, eta); its stationary law is the dense
    Gaussian posterior of gamma = A kappa + n."""
    p = synth.config_shear(2, 8, b_ratio)
    H = W = 8
    n = 64
    c = osh.ShearCoefficients(p, b_ratio)
    g = osh.shear_data(p)

    def step(x, xi, eta):
        kappa = x[:n].reshape(H, W) + 1j * x[n:].reshape(H, W)
        _, k1 = osh.shear_sweep(osh.apply_A(kappa), g, c, xi, eta)
        return np.concatenate([k1.real.ravel(), k1.imag.ravel()])

    zero_c = np.zeros((H, W), dtype=np.complex128)
    x0 = np.zeros(2 * n)
    c0 = step(x0, zero_c, zero_c)
    M = np.empty((2 * n, 2 * n))
    for i in range(2 * n):
        e = np.zeros(2 * n)
        e[i] = 1.0
        M[:, i] = step(e, zero_c, zero_c) - c0
    B = []
    for part in range(4):  # xi real, xi imag, eta real, eta imag
        for i in range(n):
            e = np.zeros(n)
            e[i] = 1.0
            v = e.reshape(H, W) * (1j if part % 2 else 1.0)
            xi, eta = (v, zero_c) if part < 2 else (zero_c, v)
            B.append(step(x0, xi, eta) - c0)
    B = np.array(B).T
    mean, cov = dense.stationary_law(M, c0, B)
    ref_mean, ref_cov = _dense_posterior(p, b_ratio)
    assert np.allclose(mean, ref_mean, atol=1e-9 * np.max(np.abs(ref_mean)))
    assert np.allclose(cov, ref_cov, atol=1e-9 * np.max(np.abs(ref_cov)))
