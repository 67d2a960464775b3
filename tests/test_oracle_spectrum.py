"""Pins of the power-spectrum Gibbs step and the hierarchical sampler oracle."""
import numpy as np
import pytest
from scipy import special, stats

from oracle import messenger as om, philox, spectrum as osp
from paper_1810_02821_amd import synth


def _band_problem(seed=0, size=16, n_bands=6, masked=None):
    p = synth.config_bands(seed, size, n_bands)
    if masked is not None:
        p.noise_var = np.where(masked, np.inf, p.noise_var)
        p.mask = masked.copy()
        p.d = np.where(masked, 0.0, p.d)
    return p


def test_band_counts_and_parseval():
    p = _band_problem(1, 16, 6)
    edges = p.spectrum.edges
    m = osp.band_counts(edges, 16, 16)
    assert m.sum() == 256 and np.all(m[1:] > 0) and m[0] == 1
    x = np.random.default_rng(0).standard_normal((16, 16))
    sig = osp.band_power(x, edges, 16, 16)
    # Parseval with numpy's unnormalised DFT: sum_k |x_k|^2 = n sum_x x^2
    assert np.isclose(sig.sum(), 256 * np.sum(x * x), rtol=1e-12)
    # a single Fourier mode puts all its power in its own band
    ky, kx = 1, 2
    y, xx = np.mgrid[0:16, 0:16]
    wave = np.cos(2 * np.pi * (ky * y + kx * xx) / 16)
    sig = osp.band_power(wave, edges, 16, 16)
    b = om.band_index(edges, 16, 16)[ky, kx]
    assert np.isclose(sig[b], sig.sum()) and np.isclose(sig.sum(), 256 * np.sum(wave ** 2))


def test_chain_sweep_with_equal_spectra_is_the_pair_sweep():
    p = _band_problem(2, 16, 6)
    c = om.coefficients(p.noise_var, p.spectrum, 1.0)
    cc = osp.chain_coefficients(p, p.spectrum.amps)
    rng = np.random.default_rng(1)
    s = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    xi = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    eta = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    d = np.where(p.mask, 0.0, p.d)
    ref, _ = om.sweep(s, c.ninv * d, c, xi, eta)
    a, b = osp.chain_sweep(s.real, s.imag, d, cc, cc, xi, eta)
    assert np.allclose(a, ref.real, atol=1e-12) and np.allclose(b, ref.imag, atol=1e-12)


def test_chain_sweep_keeps_chains_separate():
    """Changing chain B's spectrum leaves chain A's update untouched, and each
    chain's harmonic step is its own real Fourier filter plus noise."""
    p = _band_problem(3, 16, 6)
    rng = np.random.default_rng(2)
    thA = np.asarray(p.spectrum.amps)
    thB = thA * rng.uniform(0.2, 5.0, size=thA.shape)
    cA, cB = osp.chain_coefficients(p, thA), osp.chain_coefficients(p, thB)
    s = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    xi = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    eta = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    d = np.where(p.mask, 0.0, p.d)
    a1, b1 = osp.chain_sweep(s.real, s.imag, d, cA, cB, xi, eta)
    a2, _ = osp.chain_sweep(s.real, s.imag, d, cA, cA, xi, eta)
    assert np.array_equal(a1, a2)
    # chain B alone, written as a real-field Wiener-sampler step
    tB = (1 - cB.a) * s.imag + cB.a * d + cB.sig_t * xi.imag
    noise = np.fft.ifft2(cB.w * eta).imag
    assert np.allclose(b1, np.fft.ifft2(cB.f * np.fft.fft2(tB)).real + noise, atol=1e-12)


@pytest.mark.parametrize("prior_dof,prior_beta", [(0, 0.0), (4, 0.7)])
def test_theta_draw_is_inverse_gamma(prior_dof, prior_beta):
    """For a fixed signal the draw follows IG((m_b + nu_0)/2, beta_0 + sigma_b/(2 n^2))
    (Kolmogorov-Smirnov over 3000 independent iterations of the stream)."""
    p = _band_problem(4, 16, 6)
    edges = p.spectrum.edges
    s = p.s_true
    m = osp.band_counts(edges, 16, 16)
    dof = osp.degrees_of_freedom(m, prior_dof)
    sig = osp.band_power(s, edges, 16, 16)
    total = int(dof.sum())
    draws = []
    for g in range(3000):
        z0, _ = osp.chi2_normals(77, g, 0, 0, total)
        draws.append(osp.draw_theta(np.ones(6), sig, dof, z0, 256, prior_beta))
    draws = np.array(draws)
    for b in (1, 3, 5):
        alpha = dof[b] / 2.0
        beta = prior_beta + sig[b] / (2.0 * 256 ** 2)
        ks = stats.kstest(draws[:, b], stats.invgamma(alpha, scale=beta).cdf)
        assert ks.pvalue > 1e-3, (b, ks)


def test_theta_draw_keeps_bands_without_freedom():
    theta = np.array([1.5, 2.5, 3.5])
    out = osp.draw_theta(theta, np.array([1.0, 2.0, 3.0]), np.array([0, 2, 0]),
                         np.array([0.5, 1.0]), 16, 0.0)
    assert out[0] == 1.5 and out[2] == 3.5
    assert np.isclose(out[1], (2.0 / 256) / 1.25)


def test_chi2_normals_are_stage_three_of_the_stream():
    z0, z1 = osp.chi2_normals(5, 7, 2, 3, 9)
    r0, r1 = philox.stream_normals(5, philox.STAGE_SPECTRUM, 7, 2, 3, 10)
    assert np.array_equal(z0, r0[:9]) and np.array_equal(z1, r1[:9])
    a, b = philox.stream_normals_scalar(5, 3, 7, 2, 3, 8)
    assert np.isclose(z0[8], a, rtol=1e-14) and np.isclose(z1[8], b, rtol=1e-14)


def test_resume_by_iteration_offset_is_exact():
    p = _band_problem(5, 16, 6)
    th_all, s_all, st_all, thf_all = osp.sample_pair_hierarchical(p, 11, 0, 1, 0, 5, sweeps=2)
    th_a, s_a, st_a, thf_a = osp.sample_pair_hierarchical(p, 11, 0, 1, 0, 2, sweeps=2)
    th_b, s_b, st_b, thf_b = osp.sample_pair_hierarchical(p, 11, 0, 1, 0, 3, sweeps=2, theta0=thf_a,
                                                          s0=st_a, iteration_offset=2)
    assert np.array_equal(th_all[:, 2:], th_b) and np.array_equal(s_all[:, 2:], s_b)
    assert np.array_equal(st_all, st_b) and np.array_equal(thf_all, thf_b)


def test_prior_is_recovered_without_data():
    """Every pixel missing: the joint (s, theta) chain has the prior
    IG(nu_0/2, beta_0) as its theta marginal.  E[log theta] = log beta_0 -
    digamma(nu_0/2) is checked with a batch-means standard error."""
    masked = np.ones((8, 8), dtype=bool)
    p = synth.config_bands(6, 8, 4)
    p.noise_var = np.full((8, 8), np.inf)
    p.mask = masked
    p.d = np.zeros((8, 8))
    nu0, beta0 = 6, 0.02
    p.spectrum = synth.spectrum_bands(p.spectrum.edges, np.full(4, beta0 / 2.0))
    th, _, _, _ = osp.sample_pair_hierarchical(p, 3, 0, 0, 50, 6000, sweeps=3, prior_dof=nu0,
                                               prior_beta=beta0)
    target = np.log(beta0) - special.digamma(nu0 / 2.0)
    for chain in range(2):
        for b in range(4):
            x = np.log(th[chain, :, b])
            batches = x.reshape(60, 100).mean(axis=1)
            se = batches.std(ddof=1) / np.sqrt(len(batches))
            assert abs(x.mean() - target) < 4.5 * se + 1e-3, (chain, b, x.mean(), target, se)
