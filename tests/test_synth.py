"""The seeded input generators produce the workloads they describe."""
import numpy as np

from paper_1810_02821_amd import synth


def test_small_config_shape_mask_and_noise():
    p = synth.config_small(0)
    assert (p.H, p.W) == (32, 32)
    assert p.mask.sum() == 13 * 16                   # round(0.2 * 64) tiles
    m = p.mask.reshape(8, 4, 8, 4)                    # tile aligned
    assert np.all(m.all(axis=(1, 3)) | ~m.any(axis=(1, 3)))
    s = np.sqrt(p.noise_var[~p.mask])
    assert s.min() >= 0.5 and s.max() <= 2.0
    assert np.all(np.isinf(p.noise_var[p.mask])) and np.all(p.d[p.mask] == 0)


def test_128_config():
    p = synth.config_128(0)
    assert p.mask.sum() == 256 * 16
    s = np.sqrt(p.noise_var[~p.mask])
    assert s.min() >= 0.3 and s.max() <= 3.0
    # pixel variance of the field ~ sum_k P(k) (about 4.6 for (k+2)^-2.5)
    assert 2.0 < p.s_true.var() < 8.0


def test_seeds_are_reproducible():
    a, b = synth.config_small(5), synth.config_small(5)
    assert np.array_equal(a.d, b.d) and np.array_equal(a.mask, b.mask)
    c = synth.config_small(6)
    assert not np.array_equal(a.d, c.d)


def test_uneven_batch_mix():
    probs = synth.config_uneven(0, n_problems=200, sizes=(8, 16, 32, 64))
    sizes = np.array([p.H for p in probs])
    frac = [np.mean(sizes == s) for s in (8, 16, 32, 64)]
    assert abs(frac[0] - 0.4) < 0.1 and abs(frac[3] - 0.1) < 0.07


def test_large_config_mask_geometry():
    p = synth.config_large(0, size=256)
    N = 256
    y, x = np.mgrid[0:N, 0:N]
    c = (N - 1) / 2
    disk = (x - c) ** 2 + (y - c) ** 2 <= (0.45 * N) ** 2
    assert np.all(p.mask[~disk])
    holes = (p.mask & disk).sum() / disk.sum()
    assert 0.05 <= holes < 0.06
    s = np.sqrt(p.noise_var[~p.mask])
    assert s.min() >= 0.5 - 1e-12 and s.max() <= 2.0 + 1e-12


def test_band_config():
    p = synth.config_bands(0, size=64)
    assert p.spectrum.kind == "bands" and len(p.spectrum.amps) == 32
    assert abs(p.mask.mean() - 0.30) < 0.01
