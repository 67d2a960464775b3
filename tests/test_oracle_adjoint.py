"""Pins of the oracle's gradients: dense torch autograd, finite differences and
the stationarity of the log-posterior at the Wiener solution."""
import numpy as np
import pytest

from oracle import adjoint as A, dense, messenger as M
from paper_1810_02821_amd import synth

SCHED = M.Schedule((1.0,), (0,), 1e-13, 400000, 10)


@pytest.mark.parametrize("size,n_bands", [(16, 8), (24, 32)])
def test_vjp_matches_dense_autograd(size, n_bands):
    p = synth.config_bands(0, size, n_bands)
    S = dense.signal_covariance(p.spectrum, size, size)
    sw = dense.wiener_dense(S, p.noise_var, p.d)
    g = np.random.default_rng(1).standard_normal((size, size))
    gd, gt, _, info = A.wiener_vjp(p, sw, g, SCHED)
    gd2, gt2, s2 = A.dense_vjp(p, g)
    assert info.converged
    assert np.allclose(s2, sw, atol=1e-10)
    assert np.linalg.norm(gd - gd2.reshape(size, size)) < 1e-9 * np.linalg.norm(gd2)
    assert np.max(np.abs(gt - gt2)) < 1e-9 * np.max(np.abs(gt2))
    assert np.all(gd[p.mask] == 0)


def test_band_edges_cover_every_mode():
    for N in (16, 24, 256):
        e = synth.log_band_edges(N, N, 32)
        idx = M.band_index(e, N, N)
        assert idx.min() == 0 and np.all(idx >= 0)
        assert np.sum(idx == 0) == 1          # band 0 is the k = 0 mode


def _loss_at(p, theta=None, d=None):
    spec = p.spectrum if theta is None else synth.spectrum_bands(p.spectrum.edges, theta)
    q = synth.Problem(p.H, p.W, p.d if d is None else d, p.noise_var, p.mask, spec, p.s_true)
    S = dense.signal_covariance(spec, p.H, p.W)
    sw = dense.wiener_dense(S, p.noise_var, q.d)
    return A.loss_terms(q, sw, p.s_true)


def test_loss_gradient_matches_central_differences():
    p = synth.config_bands(2, 16, 8)
    S = dense.signal_covariance(p.spectrum, 16, 16)
    sw = dense.wiener_dense(S, p.noise_var, p.d)
    gd, gt = A.loss_grad(p, sw, p.s_true, SCHED)
    theta = np.asarray(p.spectrum.amps)
    # relative steps in theta; central differences carry an O(h^2) error, so
    # the bound shrinks 100x with h (h = 1e-3 is the workload's step)
    for h, tol in ((1e-3, 5e-5), (1e-4, 5e-7)):
        for b in range(len(theta)):
            tp, tm = theta.copy(), theta.copy()
            tp[b] *= 1 + h
            tm[b] *= 1 - h
            fd = (_loss_at(p, theta=tp) - _loss_at(p, theta=tm)) / (2 * h * theta[b])
            assert abs(fd - gt[b]) < tol * max(1.0, abs(gt[b]))
    h = 1e-3
    rng = np.random.default_rng(0)
    obs = np.flatnonzero(~p.mask.ravel())
    for i in rng.choice(obs, 6, replace=False):
        dp, dm = p.d.copy(), p.d.copy()
        dp.flat[i] += h
        dm.flat[i] -= h
        fd = (_loss_at(p, d=dp) - _loss_at(p, d=dm)) / (2 * h)
        assert abs(fd - gd.flat[i]) < 1e-6 * max(1.0, abs(fd))


def test_log_posterior_part_has_no_implicit_term():
    """At s* the prior + likelihood part of the loss is stationary in s, so its
    total derivative equals its explicit derivative (envelope property)."""
    p = synth.config_bands(3, 16, 8)
    c = M.coefficients(p.noise_var, p.spectrum)
    S = dense.signal_covariance(p.spectrum, 16, 16)
    sw = dense.wiener_dense(S, p.noise_var, p.d)
    dJ = M.apply_S_inverse(sw, c) - c.ninv * (p.d - sw)
    assert np.linalg.norm(dJ) < 1e-8 * np.linalg.norm(c.ninv * p.d)


def test_unrolled_vjp_matches_autograd_through_truncated_iteration():
    """Reverse-mode through a cooling schedule of deterministic sweeps equals
    torch autograd through the same truncated iteration."""
    p = synth.config_bands(4, 16, 8)
    sched = M.Schedule((40.0, 8.0, 1.0), (7, 6, 11))
    g = np.random.default_rng(5).standard_normal((16, 16))
    s, gd, gt = A.unrolled_vjp(p, sched, g)
    s2, gd2, gt2 = A.unrolled_vjp_torch(p, sched, g)
    assert np.allclose(s, s2, atol=1e-12)
    assert np.linalg.norm(gd - gd2) < 1e-10 * np.linalg.norm(gd2)
    assert np.max(np.abs(gt - gt2)) < 1e-10 * np.max(np.abs(gt2))
    ref, _ = M.wiener(p, sched)
    assert np.allclose(s, ref, atol=1e-12)


def test_unrolled_gradient_tends_to_implicit_gradient():
    """With enough sweeps the truncated iteration is at its fixed point and the
    unrolled gradient equals the implicit one."""
    p = synth.config_bands(6, 16, 8)
    g = np.random.default_rng(6).standard_normal((16, 16))
    s, gd, gt = A.unrolled_vjp(p, M.Schedule((1.0,), (6000,)), g)
    gd_i, gt_i, _, _ = A.wiener_vjp(p, s, g, solver="cg")
    assert np.linalg.norm(gd - gd_i) < 1e-8 * np.linalg.norm(gd_i)
    assert np.max(np.abs(gt - gt_i)) < 1e-8 * np.max(np.abs(gt_i))
