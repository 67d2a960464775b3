"""Pins of the reduced-precision storage model (oracle/storage.py): the two
rounding functions against the formats' definitions, and the split sweep
without rounding against Algorithm 1."""
import numpy as np
import pytest

from oracle import messenger as om
from oracle import storage as ost
from paper_1810_02821_amd import synth


def test_fp16_rounding_follows_binary16():
    # 10 fraction bits: spacing 2^-10 at 1; ties go to the even neighbour
    r = ost.round_fp16(np.array([1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11, 1 + 2.0 ** -11 + 2.0 ** -20,
                                 65504.0, 65519.0, 65520.0, 2.0 ** -24, 2.0 ** -26, -0.0]))
    assert r[0] == 1.0 and r[1] == 1 + 2.0 ** -9 and r[2] == 1 + 2.0 ** -10
    assert r[3] == 65504.0 and r[4] == 65504.0 and np.isinf(r[5])
    assert r[6] == 2.0 ** -24 and r[7] == 0.0 and r[8] == 0.0


def _bf16_by_search(x: float) -> float:
    """Nearest value with at most 8 significant bits and an FP32 exponent,
    ties to an even last bit, found from the binade of x (no bit tricks)."""
    if x == 0.0:
        return 0.0
    s = np.sign(x)
    a = abs(float(np.float32(x)))
    e = int(np.floor(np.log2(a)))
    ulp = 2.0 ** (e - 7)
    lo = np.floor(a / ulp) * ulp
    hi = lo + ulp
    if a - lo < hi - a:
        return s * lo
    if hi - a < a - lo:
        return s * hi
    return s * (lo if int(round(lo / ulp)) % 2 == 0 else hi)


def test_bf16_rounding_follows_the_format():
    r = ost.round_bf16(np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -20, 3.0e38, -2.5]))
    assert r[0] == 1.0 and r[1] == 1 + 2.0 ** -6 and r[2] == 1 + 2.0 ** -7
    assert abs(r[3] - 3.0e38) <= 2.0 ** -8 * 3.0e38 and r[4] == -2.5
    x = np.random.default_rng(0).standard_normal(2000) * 10.0 ** np.random.default_rng(1).uniform(-6, 6, 2000)
    ref = np.array([_bf16_by_search(v) for v in x])
    assert np.array_equal(ost.round_bf16(x), ref)


@pytest.mark.parametrize("storage,u", [("fp16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_rounding_is_idempotent_and_within_unit_roundoff(storage, u):
    rnd = ost.ROUNDERS[storage]
    x = np.random.default_rng(2).standard_normal(4096) * 3.0 + 1j * np.random.default_rng(3).standard_normal(4096)
    r = rnd(x)
    assert np.array_equal(rnd(r), r)
    big = np.abs(x.real) > 1e-3
    assert np.all(np.abs(r.real - x.real)[big] <= u * np.abs(x.real)[big])


def test_split_sweep_without_rounding_is_algorithm_1():
    p = synth.config_small(4, 32)
    c = om.coefficients(p.noise_var, p.spectrum, 1.0)
    b = c.ninv * np.where(p.mask, 0.0, p.d)
    rng = np.random.default_rng(5)
    s = rng.standard_normal((32, 32)) + 1j * rng.standard_normal((32, 32))
    xi = rng.standard_normal((32, 32)) + 1j * rng.standard_normal((32, 32))
    eta = rng.standard_normal((32, 32)) + 1j * rng.standard_normal((32, 32))
    ref, _ = om.sweep(s, b, c, xi, eta)
    got = ost.stored_sweep(s, b, c, lambda v: v, xi, eta)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("storage,u", [("fp16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_stored_chain_stays_near_the_exact_chain(storage, u):
    """A few sweeps with storage rounding stay within a few unit roundoffs of
    the unrounded chain (the sweep is a contraction, so each sweep adds at most
    its own two roundings)."""
    p = synth.config_small(6, 32)
    K = 4
    ref, _ = om.sample_pair(p, 9, 0, 0, 0, K)
    got, _ = ost.sample_pair_stored(p, 9, 0, 0, 0, K, storage=storage)
    for k in range(K):
        e = np.linalg.norm(got[:, k] - ref[:, k]) / np.linalg.norm(ref[:, k])
        assert 0.0 < e < 2 * (k + 1) * 8 * u
