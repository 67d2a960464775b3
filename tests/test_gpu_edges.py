"""Degenerate and empty cases on the GPU against the oracle: every pixel
missing (the filter is zero and the chains sample the prior), homoscedastic
unmasked noise (one sweep reaches the Fourier Wiener filter exactly), and
calls that run no sweep."""
import copy

import numpy as np
import pytest

from gpu_common import REL_TOL, banner, rel
from oracle import messenger as om
from paper_1810_02821_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1810_02821_amd as mf
    mf.lib()
    return torch


def _mf():
    import paper_1810_02821_amd as mf
    return mf


def _all_missing(size):
    p = copy.deepcopy(synth.config_small(3, size))
    p.noise_var = np.full((size, size), np.inf)
    p.mask = np.ones((size, size), dtype=bool)
    p.d = np.zeros((size, size))
    return p


@pytest.mark.parametrize("size,form", [(32, "persistent"), (32, "streamed"), (256, "streamed")])
def test_every_pixel_missing(torch_cuda, size, form):
    torch = torch_cuda
    mf = _mf()
    banner(f"every pixel missing {size} {form}")
    p = _all_missing(size)
    plan = mf.Plan([p], streamed_solve=form == "streamed")
    assert plan.tau(0) == 1.0
    d = plan.concat([p.d])
    s, _ = plan.wiener(d, mf.Schedule.fixed(20))
    assert torch.count_nonzero(s).item() == 0
    flat, _ = plan.sample(d, 4, chains=2, burn_in=2, n_samples=3, form=form, init_scale=2.0)
    got = plan.sample_view(flat, 0, 2, 3).cpu().numpy()
    s0 = om.initial_state(4, 0, 0, size, size, 2.0)
    ref, _ = om.sample_pair(p, 4, 0, 0, 2, 3, s0=s0)
    worst = max(rel(got[h, k], ref[h, k]) for h in range(2) for k in range(3))
    print(f"worst {worst:.2e}")
    assert worst < REL_TOL


@pytest.mark.parametrize("size,solve", [(64, "persistent"), (64, "streamed"), (512, "streamed")])
def test_homoscedastic_unmasked_one_sweep(torch_cuda, size, solve):
    """N = sigma^2 I with no missing pixel: tau = sigma^2, a = 1 everywhere, and
    one sweep of the filter lands on the Fourier Wiener filter; the GPU's one
    sweep matches the oracle's, and a second sweep does not move it."""
    mf = _mf()
    banner(f"homoscedastic one sweep {size} {solve}")
    p = copy.deepcopy(synth.config_128(2, size))
    p.noise_var = np.full((size, size), 0.7)
    p.mask = np.zeros((size, size), dtype=bool)
    plan = mf.Plan([p], streamed_solve=solve == "streamed")
    d = plan.concat([p.d])
    s1, _ = plan.wiener(d, mf.Schedule.fixed(1))
    s2, _ = plan.wiener(d, mf.Schedule.fixed(2))
    ref, _ = om.wiener(p, om.Schedule.fixed(1))
    r1 = rel(plan.split(s1)[0], ref)
    r2 = rel(plan.split(s2)[0], ref)
    print(f"one sweep {r1:.2e}, two sweeps {r2:.2e}")
    assert r1 < REL_TOL and r2 < REL_TOL


@pytest.mark.parametrize("form,chains", [("persistent", 4), ("streamed", 4), ("streamed", 1), ("plain", 2)])
def test_calls_with_no_sweep(torch_cuda, form, chains):
    """burn_in = n_samples = 0: the state comes back as it went in (or as the
    dispersed start), and nothing else is written."""
    torch = torch_cuda
    mf = _mf()
    banner(f"no sweep {form} chains {chains}")
    probs = [synth.config_small(1, 32), synth.config_small(2, 32)]
    plan = mf.Plan(probs)
    d = plan.concat([p.d for p in probs])
    st_in = torch.randn(2 * ((chains + 1) // 2) * plan.total_pixels, device="cuda")
    if chains == 1:  # single-chain states carry no imaginary part
        st_in.view(-1, 2)[:, 1] = 0
    st = torch.full_like(st_in, float("nan"))
    plan.sample(d, 3, chains=chains, burn_in=0, n_samples=0, form=form, state_in=st_in, state_out=st,
                samples=False)
    assert torch.equal(st, st_in)
    st2 = torch.full_like(st_in, float("nan"))
    plan.sample(d, 3, chains=chains, burn_in=0, n_samples=0, form=form, init_scale=3.0, state_out=st2,
                samples=False)
    for i, p in enumerate(probs):
        got = plan.state_view(st2, i, chains).cpu().numpy()[0]
        ref = om.initial_state(3, i, 0, 32, 32, 3.0)
        assert rel(got.real, ref.real) < 1e-6
        if chains > 1:
            assert rel(got.imag, ref.imag) < 1e-6


def test_wiener_with_no_sweep_returns_the_start(torch_cuda):
    torch = torch_cuda
    mf = _mf()
    banner("wiener with no sweep")
    probs = [synth.config_small(1, 32), synth.config_128(2, 256)]
    for solve in ("persistent", "streamed"):
        plan = mf.Plan(probs, streamed_solve=solve == "streamed")
        d = plan.concat([p.d for p in probs])
        s0 = torch.randn_like(d)
        s, info = plan.wiener(d, mf.Schedule.fixed(0), s_init=s0)
        assert torch.equal(s, s0) and all(i.sweeps == 0 for i in info)
        z, _ = plan.wiener(d, mf.Schedule.fixed(0))
        assert torch.count_nonzero(z).item() == 0
