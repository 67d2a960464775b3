"""The C-ABI conventions on the GPU: calls that allocate nothing after
mf_plan_reserve, capture into a caller-owned HIP graph, and the samplers'
non-finite check."""
import ctypes as C

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


@pytest.mark.parametrize("size,streamed", [(64, False), (256, True)])
def test_capture_sample_and_wiener_into_caller_graph(torch_cuda, size, streamed):
    """mf_sample and mf_wiener (fixed schedule, no info) recorded into a torch
    CUDA graph on its side stream after mf_plan_reserve: three replays, with
    eager work and synchronisation between them, each equal bit for bit to the
    eager calls; the eager calls match the oracle."""
    torch = torch_cuda
    mf = _mf()
    banner(f"caller graph capture {size} ({'streamed' if streamed else 'persistent'})")
    prob = synth.config_128(5, size)
    plan = mf.Plan([prob], streamed_solve=streamed)
    plan.reserve(["sample", "solve"], chains=4)
    d = plan.concat([prob.d])
    form = "streamed" if streamed else "persistent"
    sch = mf.Schedule([20.0, 3.0, 1.0], [4, 4, 12])
    kw = dict(seed=31, chains=4, burn_in=3, n_samples=2, form=form, check_finite=False)
    ref_smp, _ = plan.sample(d, **kw)
    ref_wf, _ = plan.wiener(d, sch, want_info=False)
    torch.cuda.synchronize()
    out_smp = torch.full_like(ref_smp, float("nan"))
    out_wf = torch.full_like(ref_wf, float("nan"))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.sample(d, out=out_smp, **kw)
        plan.wiener(d, sch, out=out_wf, want_info=False)
    for rep in range(3):
        out_smp.fill_(float("nan"))
        out_wf.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out_smp, ref_smp), f"samples, replay {rep}"
        assert torch.equal(out_wf, ref_wf), f"filter, replay {rep}"
        torch.randn(1 << 20, device="cuda").sum().item()  # eager work between replays
        torch.cuda.synchronize()
    x = plan.sample_view(ref_smp, 0, 4, 2).cpu().numpy()
    smp, _ = om.sample_pair(prob, 31, 0, 1, 3, 2)
    assert max(rel(x[2 + h, k], smp[h, k]) for h in range(2) for k in range(2)) < REL_TOL
    wf, _ = om.wiener(prob, om.Schedule((20.0, 3.0, 1.0), (4, 4, 12)))
    assert rel(plan.split(ref_wf)[0], wf) < REL_TOL


def test_reserved_calls_leave_device_memory_unchanged(torch_cuda):
    """After mf_plan_reserve the entry points allocate nothing: device free
    memory is the same before and after repeated calls of every reserved kind."""
    torch = torch_cuda
    mf = _mf()
    banner("reserved calls, device memory")
    probs = [synth.config_bands(1, 64, 16), synth.config_bands(2, 256, 16)]
    plan = mf.Plan(probs)
    plan.reserve(["sample", "solve", "spectrum", "unrolled", "moments"], chains=4, unrolled_sweeps=30,
                 checkpoint_every=7)
    d = plan.concat([p.d for p in probs])
    s_true = plan.concat([p.s_true for p in probs])
    g = plan.concat([np.ones((p.H, p.W)) for p in probs])
    sch = mf.Schedule([10.0, 1.0], [5, 10])
    smp = plan.samples_buffer(4, 2)
    wf = torch.empty_like(d)
    gd = torch.empty_like(d)
    loss = torch.empty(2, dtype=torch.float64, device="cuda")
    gb = torch.empty(plan.total_bands, dtype=torch.float64, device="cuda")
    mean = torch.empty(plan.total_pixels, dtype=torch.float64, device="cuda")
    L = mf.lib()

    def calls():
        plan.sample(d, 3, chains=4, burn_in=2, n_samples=2, out=smp, check_finite=False)
        plan.wiener(d, sch, out=wf, want_info=False)
        sc = sch._c()
        mf._binding._check(L.mf_band_loss(plan._h, C.c_void_p(d.data_ptr()), C.c_void_p(wf.data_ptr()),
                                          C.c_void_p(s_true.data_ptr()), C.byref(sc),
                                          C.c_void_p(loss.data_ptr()), C.c_void_p(gd.data_ptr()),
                                          C.c_void_p(gb.data_ptr()), None, mf._binding._stream()), True)
        plan.wiener_backward_unrolled(d, g, mf.Schedule([5.0, 1.0], [10, 20]), checkpoint_every=7)
        plan.sample_spectrum(d, 4, chains=4, burn_in=1, n_samples=1, check_finite=False)
        mf._binding._check(L.mf_sample_moments(plan._h, C.c_void_p(smp.data_ptr()), 4, 2,
                                               C.c_void_p(mean.data_ptr()), None, mf._binding._stream()))

    calls()  # torch's own allocations for the binding's outputs settle here
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(3):
        calls()
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    print(f"free before {free0}, after {free1}")
    assert free1 == free0


def test_unreserved_call_on_a_capturing_stream_is_refused(torch_cuda):
    """Without mf_plan_reserve a call that needs a workspace does not allocate
    during capture: it fails with MF_ERR_INVALID_ARG."""
    torch = torch_cuda
    mf = _mf()
    banner("unreserved capture is refused")
    prob = synth.config_128(6, 64)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    out = plan.samples_buffer(2, 1)
    g = torch.cuda.CUDAGraph()
    with pytest.raises(mf.MFError) as e:
        with torch.cuda.graph(g):
            plan.sample(d, 3, chains=2, burn_in=1, n_samples=1, out=out, check_finite=False)
    assert e.value.status == 1 and "reserve" in str(e.value)
    torch.cuda.synchronize()
    # the plan still works afterwards
    plan.sample(d, 3, chains=2, burn_in=1, n_samples=1, out=out)


@pytest.mark.parametrize("form", ["persistent", "streamed", "plain"])
def test_sampler_reports_nonfinite_data(torch_cuda, form):
    """NaN in the data of an observed pixel: the sampler's kernels run to the
    end, the call returns MF_ERR_NONFINITE naming the problem, and a clean
    problem of the same plan still matches the oracle."""
    torch = torch_cuda
    mf = _mf()
    banner(f"sampler non-finite data, {form}")
    probs = [synth.config_small(3, 32), synth.config_small(4, 32)]
    plan = mf.Plan(probs)
    bad = probs[1].d.copy()
    y, x = np.argwhere(~probs[1].mask)[7]
    bad[y, x] = np.nan
    d = plan.concat([probs[0].d, bad])
    out = plan.samples_buffer(2, 3)
    with pytest.raises(mf.MFError) as e:
        plan.sample(d, 5, chains=2, burn_in=2, n_samples=3, form=form, out=out)
    assert e.value.status == 6 and "problem 1" in str(e.value)
    got = plan.sample_view(out, 0, 2, 3).cpu().numpy()
    ref, _ = om.sample_pair(probs[0], 5, 0, 0, 2, 3)
    assert max(rel(got[c, k], ref[c, k]) for c in range(2) for k in range(3)) < REL_TOL
    # the clean data pass the check
    plan.sample(d=plan.concat([probs[0].d, probs[1].d]), seed=5, chains=2, burn_in=2, n_samples=3, form=form)


def test_hierarchical_and_shear_samplers_report_nonfinite_data(torch_cuda):
    torch = torch_cuda
    mf = _mf()
    banner("hierarchical / mass-mapping non-finite data")
    prob = synth.config_bands(2, 64, 8)
    plan = mf.Plan([prob])
    bad = prob.d.copy()
    bad[np.argwhere(~prob.mask)[3][0], np.argwhere(~prob.mask)[3][1]] = np.inf
    with pytest.raises(mf.MFError) as e:
        plan.sample_spectrum(plan.concat([bad]), 3, chains=2, burn_in=1, n_samples=2)
    assert e.value.status == 6
    plan.sample_spectrum(plan.concat([prob.d]), 3, chains=2, burn_in=1, n_samples=2)
    for size in (64, 256):  # persistent and streamed mass-mapping kernels
        sp = synth.config_shear(1, size, b_ratio=0.3)
        splan = mf.Plan([sp])
        gamma = np.array(sp.gamma, dtype=np.complex64)
        obs = np.argwhere(np.isfinite(sp.noise_var))[5]
        gamma[obs[0], obs[1]] = np.nan
        with pytest.raises(mf.MFError) as e:
            splan.shear_sample(splan.concat_complex([gamma]), 3, chains=2, burn_in=1, n_samples=1, b_ratio=0.3)
        assert e.value.status == 6
