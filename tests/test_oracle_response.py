"""Pins of the oracle with a diagonal response A (Algorithm 1's A_i terms):
the messenger filter and sampler against the dense Eq. 2 / Eq. 7 with A."""
import numpy as np

from oracle import adjoint as oa, dense, messenger as om
from paper_1810_02821_amd import synth


def _problem(seed=0, size=16):
    return synth.config_response(seed, size, dead=0.03)


def test_response_problem_has_dead_and_masked_pixels():
    p = _problem(0, 16)
    assert np.any(p.response == 0) and np.any(np.isinf(p.noise_var))
    assert np.all(p.mask[p.response == 0]) and np.all(p.d[p.mask] == 0)


def test_tau_is_min_of_noise_over_squared_response():
    p = _problem(1, 16)
    obs = np.isfinite(p.noise_var) & (p.response != 0)
    c = om.coefficients(p.noise_var, p.spectrum, 1.0, None, p.response)
    assert np.isclose(c.tau, np.min(p.noise_var[obs] / p.response[obs] ** 2))
    # the pixel with the smallest N/A^2 gets Nbar = 0: a = 1 and no messenger noise
    i = np.unravel_index(np.argmin(np.where(obs, p.noise_var / np.where(obs, p.response, 1) ** 2, np.inf)),
                         p.noise_var.shape)
    assert np.isclose(c.a[i], 1.0) and np.isclose(c.sig_t[i], 0.0)
    assert np.all(c.a[~obs] == 0) and np.all(c.ninv[~obs] == 0)


def test_messenger_wiener_with_response_equals_dense():
    p = _problem(2, 16)
    S = dense.signal_covariance(p.spectrum, 16, 16)
    ref = dense.wiener_dense(S, p.noise_var, p.d, p.response)
    s, info = om.wiener(p, om.Schedule.geometric(1e3, 1.0, 30, 20, tol=1e-12, max_sweeps=200000))
    assert info.converged
    assert np.max(np.abs(s - ref)) < 1e-8 * np.max(np.abs(ref))
    # the CG route solves the same normal equations
    s2, _ = om.wiener_cg(p, tol=1e-13)
    assert np.max(np.abs(s2 - ref)) < 1e-9 * np.max(np.abs(ref))


def test_cooled_fixed_point_with_response():
    """Level lambda: Wiener filter for noise N + (lambda - 1) tau A^2."""
    p = _problem(3, 16)
    S = dense.signal_covariance(p.spectrum, 16, 16)
    lam = 7.0
    ref = dense.wiener_dense(S, dense.effective_noise(p.noise_var, lam, None, p.response), p.d, p.response)
    s, _ = om.wiener(p, om.Schedule((lam,), (0,), 1e-12, 200000, 10))
    assert np.max(np.abs(s - ref)) < 1e-8 * np.max(np.abs(ref))


def test_residual_identity_with_response():
    """||t_{k+1} - t_k|| / (T ||b||) equals the residual of the normal equations
    (S^-1 + A^T N^-1 A) s_k = A^T N^-1 d, evaluated by definition."""
    p = _problem(4, 16)
    c = om.coefficients(p.noise_var, p.spectrum, 1.0, None, p.response)
    d = np.where(p.mask, 0.0, p.d)
    b = c.ninv * d
    s = np.random.default_rng(0).standard_normal((16, 16))
    s1, t1 = om.sweep(s, b, c)
    _, t2 = om.sweep(s1, b, c)
    lhs = np.linalg.norm(t2 - t1) / (c.T * np.linalg.norm(b))
    assert np.isclose(lhs, om.residual(p, s1), rtol=1e-10)


def test_sampler_with_response_has_the_exact_posterior():
    """The sweep with A is affine in (s, xi, eta); its stationary law is
    (s_W, (S^-1 + A^T N^-1 A)^-1) of Eq. 7 with A."""
    p = _problem(5, 8)
    H = W = 8
    c = om.coefficients(p.noise_var, p.spectrum, 1.0, None, p.response)
    d = np.where(p.mask, 0.0, p.d)
    b = c.ninv * d

    def sweep(s, xi, eta):
        return om.sweep(s, b, c, xi, eta)[0]

    M, c0, B = dense.chain_transition(sweep, H, W)
    mean, cov = dense.stationary_law(M, c0, B)
    S = dense.signal_covariance(p.spectrum, H, W)
    assert np.allclose(mean.reshape(H, W), dense.wiener_dense(S, p.noise_var, p.d, p.response), atol=1e-10)
    assert np.allclose(cov, dense.posterior_covariance(S, p.noise_var, p.response), atol=1e-10)


def test_response_equals_identity_problem_with_scaled_data():
    """A diagonal A is the A = I problem for d/A and N/A^2 (A_i = 0 missing):
    the coefficients of the two agree and so do the filters."""
    p = _problem(6, 16)
    A = p.response
    obs = np.isfinite(p.noise_var) & (A != 0)
    q = synth.Problem(H=16, W=16, d=np.where(obs, p.d / np.where(obs, A, 1.0), 0.0),
                      noise_var=np.where(obs, p.noise_var / np.where(obs, A, 1.0) ** 2, np.inf),
                      mask=~obs, spectrum=p.spectrum, s_true=p.s_true)
    cp = om.coefficients(p.noise_var, p.spectrum, 2.0, None, A)
    cq = om.coefficients(q.noise_var, q.spectrum, 2.0)
    assert np.isclose(cp.tau, cq.tau) and np.allclose(cp.a, cq.a) and np.allclose(cp.sig_t, cq.sig_t)
    sch = om.Schedule((10.0, 1.0), (5, 40))
    assert np.allclose(om.wiener(p, sch)[0], om.wiener(q, sch)[0], atol=1e-12)


def test_vjp_with_response_equals_dense_gradient():
    """d<g, s_W>/dd on observed pixels = (A S A^T + N)^-1 A S g (Eq. 2 with A)."""
    p = _problem(7, 16)
    g = np.random.default_rng(1).standard_normal((16, 16))
    S = dense.signal_covariance(p.spectrum, 16, 16)
    obs = (np.isfinite(p.noise_var) & (p.response != 0)).ravel()
    Ao = p.response.ravel()[obs]
    K = Ao[:, None] * S[np.ix_(obs, obs)] * Ao[None, :] + np.diag(p.noise_var.ravel()[obs])
    ref = np.zeros(256)
    ref[obs] = np.linalg.solve(K, Ao * (S[obs, :] @ g.ravel()))
    gd, _, _, _ = oa.wiener_vjp(p, None, g, om.Schedule((1.0,), (0,), 1e-13, 200000, 10))
    assert np.max(np.abs(gd.ravel() - ref)) < 1e-8 * np.max(np.abs(ref))


def test_unrolled_vjp_with_response_matches_finite_differences():
    """The truncated iteration is affine in d, so central differences are exact
    up to rounding."""
    p = _problem(8, 16)
    sch = om.Schedule((20.0, 3.0, 1.0), (3, 3, 4))
    g = np.random.default_rng(2).standard_normal((16, 16))
    _, dbar, _ = oa.unrolled_vjp(p, sch, g)
    rng = np.random.default_rng(3)
    obs = ~p.mask
    for _ in range(5):
        idx = tuple(rng.choice(np.argwhere(obs)))
        h = 1e-3
        pp, pm = _problem(8, 16), _problem(8, 16)
        pp.d[idx] += h
        pm.d[idx] -= h
        fp = np.sum(g * oa.unrolled_vjp(pp, sch, g)[0])
        fm = np.sum(g * oa.unrolled_vjp(pm, sch, g)[0])
        assert np.isclose((fp - fm) / (2 * h), dbar[idx], rtol=1e-6, atol=1e-10)


def _band_problem_with_response(seed=2, size=16):
    """A band-spectrum problem seen through a diagonal response with a few
    pixels of zero response (the differentiation loss needs band amplitudes)."""
    p = synth.config_bands(seed, size, 8)
    rng = np.random.default_rng(seed + 100)
    A = rng.uniform(0.5, 1.5, (size, size))
    A.flat[rng.choice(size * size, 5, replace=False)] = 0.0
    p.response = A
    p.mask = p.mask | (A == 0)
    p.d = np.where(p.mask, 0.0, A * p.s_true + rng.standard_normal((size, size)) * np.sqrt(
        np.where(np.isfinite(p.noise_var), p.noise_var, 1.0)))
    return p


def _loss_with_response(p, theta=None, d=None):
    spec = p.spectrum if theta is None else synth.spectrum_bands(p.spectrum.edges, theta)
    q = synth.Problem(p.H, p.W, p.d if d is None else d, p.noise_var, p.mask, spec, p.s_true, response=p.response)
    S = dense.signal_covariance(spec, p.H, p.W)
    sw = dense.wiener_dense(S, p.noise_var, q.d, response=p.response)
    return oa.loss_terms(q, sw, p.s_true)


def test_loss_gradient_with_response_matches_central_differences():
    """L = 1/2 s^T S^-1 s + 1/2 (d - A s)^T N^-1 (d - A s) + 1/2 sum ln(n P)
    + 1/2 ||s - s_true||^2 at the Wiener filter with A (Eq. 2 with A, dense):
    the oracle's gradient (explicit terms plus the implicit VJP) against
    central differences of the dense loss, in d and in the band amplitudes."""
    p = _band_problem_with_response()
    S = dense.signal_covariance(p.spectrum, 16, 16)
    sw = dense.wiener_dense(S, p.noise_var, p.d, response=p.response)
    gd, gt = oa.loss_grad(p, sw, p.s_true, om.Schedule((1.0,), (0,), 1e-13, 400000, 10))
    theta = np.asarray(p.spectrum.amps)
    h = 1e-4
    for b in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[b] *= 1 + h
        tm[b] *= 1 - h
        fd = (_loss_with_response(p, theta=tp) - _loss_with_response(p, theta=tm)) / (2 * h * theta[b])
        assert abs(fd - gt[b]) < 5e-7 * max(1.0, abs(gt[b]))
    rng = np.random.default_rng(0)
    obs = np.flatnonzero((np.isfinite(p.noise_var) & (p.response != 0)).ravel())
    for i in rng.choice(obs, 6, replace=False):
        dp, dm = p.d.copy(), p.d.copy()
        dp.flat[i] += 1e-3
        dm.flat[i] -= 1e-3
        fd = (_loss_with_response(p, d=dp) - _loss_with_response(p, d=dm)) / 2e-3
        assert abs(fd - gd.flat[i]) < 1e-6 * max(1.0, abs(fd))
    assert np.all(gd[p.response == 0] == 0)
