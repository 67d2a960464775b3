"""Run-to-run determinism of the persistent kernels, whose LDS exchanges rely on
ordering arguments instead of block barriers in some steps (a thread that
overwrites only the addresses it has just read): a race there would show up as
outputs that differ between two identical calls.  Each workload runs twice in
the launch configuration the benchmarks use and must agree bit for bit (the
hierarchical sampler's FP64 band amplitudes to FP64 rounding)."""
import numpy as np
import pytest

from gpu_common import banner
from paper_1810_02821_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf_torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1810_02821_amd as mf
    mf.lib()
    return mf, torch


def test_sampler_128_is_deterministic(mf_torch):
    mf, torch = mf_torch
    banner("determinism: 128^2 sampler, 1024 chains")
    prob = synth.config_128(0)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    runs = []
    for _ in range(2):
        st = plan.state_buffer(1024)
        out, _ = plan.sample(d, 1000, chains=1024, burn_in=200, n_samples=98, state_out=st, form="persistent")
        runs.append((out, st))
    assert torch.equal(runs[0][0], runs[1][0]) and torch.equal(runs[0][1], runs[1][1])


def test_solve_batch_is_deterministic(mf_torch):
    mf, torch = mf_torch
    banner("determinism: persistent solves 32/64/128")
    probs = [synth.config_small(0, 32), synth.config_128(1, 64), synth.config_128(2), synth.config_128(3)]
    plan = mf.Plan(probs)
    d = plan.concat([p.d for p in probs])
    sch = mf.Schedule(list(np.geomspace(1e3, 1.0, 20)) + [1.0], [10] * 20 + [300])
    a, _ = plan.wiener(d, sch)
    b, _ = plan.wiener(d, sch)
    assert torch.equal(a, b)


def test_hierarchical_and_shear_are_deterministic(mf_torch):
    mf, torch = mf_torch
    banner("determinism: hierarchical 128^2 and mass mapping 128^2")
    bands = synth.config_bands(0, 128, 32)
    plan = mf.Plan([bands])
    d = plan.concat([bands.d])
    r = [plan.sample_spectrum(d, 7, 256, 20, 10, 1, 1, samples=True) for _ in range(2)]
    # the band powers are FP64 sums built with LDS atomics, whose order varies
    # from run to run: the amplitudes agree to FP64 rounding (about 3e-15
    # relative) and, entering the sweep through FP32 coefficients, leave the
    # signal samples bit for bit the same
    dt = ((r[0][0] - r[1][0]).abs() / r[0][0].abs()).max().item()
    print(f"amplitudes max rel diff {dt:.2e}")
    assert dt < 1e-13 and torch.equal(r[0][1], r[1][1])
    sh = synth.config_shear(1, 128, 0.3)
    splan = mf.Plan([sh])
    g = splan.concat_complex([sh.gamma])
    s = [splan.shear_sample(g, 11, 256, 20, 10, 1, b_ratio=0.3)[0] for _ in range(2)]
    assert torch.equal(s[0], s[1])
