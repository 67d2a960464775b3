"""Pins of the oracle's normal stream (Philox4x32-10 + Box-Muller)."""
import math
import os

import numpy as np
import pytest
import scipy.stats

from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((tuple(w[0:4]), tuple(w[4:6]), tuple(w[6:10])))
    return rows


@pytest.mark.parametrize("row", _kat_rows())
def test_known_answers_scalar(row):
    ctr, key, expect = row
    assert philox.philox4x32_scalar(ctr, key) == expect


@pytest.mark.parametrize("row", _kat_rows())
def test_known_answers_vectorised(row):
    ctr, key, expect = row
    out = philox.philox4x32([np.array([c]) for c in ctr], key)
    assert tuple(int(o[0]) for o in out) == expect


def test_vectorised_matches_scalar_on_random_counters():
    rng = np.random.default_rng(5)
    ctr = [rng.integers(0, 2 ** 32, size=64, dtype=np.uint64) for _ in range(4)]
    key = (0x12345678, 0x9abcdef0)
    vec = philox.philox4x32(ctr, key)
    for i in range(64):
        sc = philox.philox4x32_scalar([int(c[i]) for c in ctr], key)
        assert tuple(int(v[i]) for v in vec) == sc


def test_uniforms_are_exact_24_bit_and_in_range():
    x = np.array([0, 255, 256, 2 ** 32 - 1, 2 ** 31], dtype=np.uint64)
    u1, u2 = philox.uniforms(x, x)
    assert u1.min() > 0 and u1.max() <= 1.0
    assert u2.min() >= 0 and u2.max() < 1.0
    assert u1[0] == 2.0 ** -24 and u2[0] == 0.0
    assert u1[3] == 1.0 and u2[3] == 1.0 - 2.0 ** -24
    # every uniform is a multiple of 2^-24 below 2^24, so it is exact in FP32
    for u in (u1, u2):
        assert np.all(u.astype(np.float32).astype(np.float64) == u)


def test_stream_layout_matches_scalar_definition():
    seed = (7 << 32) | 11
    z0, z1 = philox.stream_normals(seed, philox.STAGE_HARMONIC, 17, 3, 5, 64)
    for e in (0, 1, 2, 31, 62, 63):
        a, b = philox.stream_normals_scalar(seed, philox.STAGE_HARMONIC, 17, 3, 5, e)
        assert abs(a - z0[e]) < 1e-15 and abs(b - z1[e]) < 1e-15


def test_normals_are_standard_gaussian():
    z0, z1 = philox.stream_normals(1000, 0, 0, 0, 0, 1 << 18)
    z = np.concatenate([z0, z1])
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / z.size)
    assert abs(scipy.stats.kurtosis(z, fisher=False) - 3.0) < 0.05
    ks = scipy.stats.kstest(z, "norm")
    assert ks.pvalue > 1e-3
    # the two normals of a Box-Muller pair are uncorrelated
    assert abs(np.corrcoef(z0, z1)[0, 1]) < 5 / math.sqrt(z0.size)


@pytest.mark.parametrize("other", [
    dict(stage=1), dict(sweep=1), dict(problem=1), dict(pair=1), dict(seed=1001)])
def test_streams_differ_and_are_uncorrelated(other):
    base = dict(seed=1000, stage=0, sweep=0, problem=0, pair=0)
    alt = dict(base, **other)
    a = philox.stream_normals(base["seed"], base["stage"], base["sweep"], base["problem"], base["pair"], 1 << 14)[0]
    b = philox.stream_normals(alt["seed"], alt["stage"], alt["sweep"], alt["problem"], alt["pair"], 1 << 14)[0]
    assert not np.allclose(a, b)
    assert abs(np.corrcoef(a, b)[0, 1]) < 5 / math.sqrt(a.size)


def test_rejects_odd_lengths_and_oversized_problem_index():
    with pytest.raises(ValueError):
        philox.stream_normals(0, 0, 0, 0, 0, 3)
    with pytest.raises(ValueError):
        philox.stream_normals(0, 0, 0, 1 << 24, 0, 4)
