"""GPU path vs the FP64 CPU oracle, element by element, through the C ABI."""
import numpy as np
import pytest

from gpu_common import REL_TOL, banner, rel
from oracle import adjoint as oa, dense, messenger as om
from paper_1810_02821_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1810_02821_amd as mf
    mf.lib()  # fail loudly if the library is missing
    return torch


def _mf():
    import paper_1810_02821_amd as mf
    return mf


def _check_samples(plan, flat, prob, pid, chains, n_samples, seed, burn_in, thin=1, pairs=None):
    got = plan.sample_view(flat, pid, chains, n_samples).cpu().numpy()
    for q in (pairs if pairs is not None else range((chains + 1) // 2)):
        ref, _ = om.sample_pair(prob, seed, pid, q, burn_in, n_samples, thin)
        for c in (2 * q, 2 * q + 1):
            if c >= chains:
                continue
            for k in range(n_samples):
                r = rel(got[c, k], ref[c - 2 * q, k])
                assert r < REL_TOL, f"problem {pid} chain {c} sample {k}: rel {r:.2e}"


@pytest.mark.parametrize("size,form", [(16, "streamed"), (32, "streamed"), (64, "streamed"),
                                       (128, "streamed"), (256, "streamed"), (32, "persistent"),
                                       (64, "persistent"), (128, "persistent")])
def test_samples_match_oracle(torch_cuda, size, form):
    mf = _mf()
    banner(f"samples {form} {size}x{size}")
    prob = synth.config_128(3, size) if size >= 64 else synth.config_small(3, size)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    seed = synth.philox_seed(3)
    n = 12 if size <= 128 else 4
    flat, _ = plan.sample(d, seed, chains=4, burn_in=2, n_samples=n, form=form)
    torch_cuda.cuda.synchronize()
    _check_samples(plan, flat, prob, 0, 4, n, seed, 2)


@pytest.mark.parametrize("H,W", [(512, 512), (1024, 32), (512, 64), (2048, 16), (64, 1024), (16, 2048),
                                 (256, 32), (32, 256)])
def test_long_axis_samples_match_oracle(torch_cuda, H, W):
    """Columns or rows of 256 and more (the streamed kernels that read their
    first transform pass from HBM, keep the last pass of one transform, the
    update and the first pass of the next in registers, and write their last
    pass to HBM), square and rectangular, every chain of every sample against
    the oracle."""
    mf = _mf()
    banner(f"samples streamed {H}x{W}")
    prob = synth.config_128(4, H) if H == W else synth.config_bands(4, H, 8, width=W)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    seed = synth.philox_seed(4)
    flat, _ = plan.sample(d, seed, chains=3, burn_in=2, n_samples=3, form="streamed")
    torch_cuda.cuda.synchronize()
    _check_samples(plan, flat, prob, 0, 3, 3, seed, 2)


@pytest.mark.parametrize("form", ["streamed", "persistent"])
def test_thousand_sweeps_per_sample_parity(torch_cuda, form):
    """Samples after 1, 10, 100 and 1000 sweeps on the same Philox stream."""
    mf = _mf()
    banner(f"1000 sweeps 32x32 {form}")
    prob = synth.config_small(0, 32)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    seed = synth.philox_seed(0)
    flat, _ = plan.sample(d, seed, chains=2, burn_in=0, n_samples=1000, form=form)
    got = plan.sample_view(flat, 0, 2, 1000).cpu().numpy()
    ref, _ = om.sample_pair(prob, seed, 0, 0, 0, 1000)
    worst = 0.0
    for k in (0, 9, 99, 499, 999):
        for c in range(2):
            worst = max(worst, rel(got[c, k], ref[c, k]))
    print(f"worst rel after up to 1000 sweeps: {worst:.2e}")
    assert worst < REL_TOL


@pytest.mark.parametrize("size,solve", [(32, "persistent"), (32, "streamed"), (64, "persistent"),
                                        (128, "persistent"), (128, "streamed"), (512, "streamed")])
def test_wiener_fixed_schedule_matches_oracle(torch_cuda, size, solve):
    mf = _mf()
    banner(f"wiener fixed schedule {size} {solve}")
    prob = synth.config_128(1, size) if size >= 64 else synth.config_small(1, size)
    plan = mf.Plan([prob], streamed_solve=solve == "streamed")
    d = plan.concat([prob.d])
    levels = [(30.0, 5), (5.0, 5), (1.0, 40)]
    sch = mf.Schedule([l for l, _ in levels], [k for _, k in levels])
    s, _ = plan.wiener(d, sch)
    ref, _ = om.wiener(prob, om.Schedule(tuple(l for l, _ in levels), tuple(k for _, k in levels)))
    r = rel(plan.split(s)[0], ref)
    print(f"rel {r:.2e}")
    assert r < REL_TOL


@pytest.mark.parametrize("solve", ["persistent", "streamed"])
def test_wiener_converges_to_dense_solve_32(torch_cuda, solve):
    """Cooling 1e4 -> 1 over 100 levels, then sweeps at lambda = 1 down to the
    FP32 floor of the residual (about 3e-6 here; the Wiener error is ~100x the
    residual, so a residual tolerance cannot certify 1e-4 in FP32); the result
    is compared with the dense solve of Eq. 2."""
    mf = _mf()
    banner(f"wiener converged vs dense 32 {solve}")
    prob = synth.config_small(0, 32)
    plan = mf.Plan([prob], streamed_solve=solve == "streamed")
    d = plan.concat([prob.d])
    sch = mf.Schedule.geometric(1e4, 1.0, 100, 10, tol=1e-8, max_sweeps=6000, check_every=10)
    s, info = plan.wiener(d, sch, allow_not_converged=True)
    S = dense.signal_covariance(prob.spectrum, 32, 32)
    ref = dense.wiener_dense(S, prob.noise_var, prob.d)
    r = rel(plan.split(s)[0], ref)
    print(f"info {info[0]} rel vs dense {r:.2e}")
    assert info[0].sweeps == 6000 and info[0].residual < 1e-5
    assert r < REL_TOL


@pytest.mark.parametrize("solve,size", [("persistent", 32), ("streamed", 32), ("streamed", 512)])
def test_residual_tracks_oracle(torch_cuda, solve, size):
    """Residual test sweeps and the returned residual agree with the oracle."""
    mf = _mf()
    banner(f"residual parity {solve} {size}")
    prob = synth.config_small(2, size)
    plan = mf.Plan([prob], streamed_solve=solve == "streamed")
    d = plan.concat([prob.d])
    s, info = plan.wiener(d, mf.Schedule([1.0], [0], 1e-3, 5000, 10))
    ref, rinfo = om.wiener(prob, om.Schedule((1.0,), (0,), 1e-3, 5000, 10))
    print(info[0], rinfo)
    assert info[0].sweeps == rinfo.sweeps
    assert abs(info[0].residual - rinfo.residual) < 1e-3 * rinfo.residual + 1e-6
    assert rel(plan.split(s)[0], ref) < REL_TOL


def test_uneven_batch_each_problem_matches(torch_cuda):
    mf = _mf()
    banner("uneven batch")
    probs = synth.config_uneven(5, n_problems=6, sizes=(16, 32, 64), weights=(0.3, 0.4, 0.3))
    plan = mf.Plan(probs)
    d = plan.concat([p.d for p in probs])
    seed = 77
    flat, _ = plan.sample(d, seed, chains=2, burn_in=1, n_samples=5, form="streamed")
    for i, p in enumerate(probs):
        _check_samples(plan, flat, p, i, 2, 5, seed, 1)
    s, _ = plan.wiener(d, mf.Schedule.fixed(30))
    for i, p in enumerate(probs):
        ref, _ = om.wiener(p, om.Schedule.fixed(30))
        assert rel(plan.split(s)[i], ref) < REL_TOL


def test_plain_form_equals_streamed(torch_cuda):
    mf = _mf()
    banner("plain == streamed")
    prob = synth.config_small(4, 32)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    a, _ = plan.sample(d, 5, chains=6, burn_in=3, n_samples=7, form="streamed")
    b, _ = plan.sample(d, 5, chains=6, burn_in=3, n_samples=7, form="plain")
    assert torch_cuda.equal(a, b)


@pytest.mark.parametrize("size", [32, 256, 512])
def test_resume_is_exact_and_odd_chain_count(torch_cuda, size):
    """A run split at sweep 8 and resumed from its state equals the
    uninterrupted run bit for bit (its first sweep takes the plain row kernel,
    the uninterrupted run the fused one at 256 and up)."""
    mf = _mf()
    banner(f"resume {size}")
    prob = synth.config_small(6, size)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    full, _ = plan.sample(d, 9, chains=3, burn_in=0, n_samples=20, form="streamed")
    st = plan.state_buffer(3)
    plan.sample(d, 9, chains=3, burn_in=8, n_samples=0, form="streamed", state_out=st, samples=False)
    rest, _ = plan.sample(d, 9, chains=3, burn_in=0, n_samples=12, sweep_offset=8, form="streamed",
                          state_in=st.clone())
    f = plan.sample_view(full, 0, 3, 20)
    r = plan.sample_view(rest, 0, 3, 12)
    assert torch_cuda.equal(f[:, 8:], r)
    _check_samples(plan, full, prob, 0, 3, 20, 9, 0, pairs=[1])


def test_dispersed_init_matches_oracle(torch_cuda):
    mf = _mf()
    banner("dispersed init")
    prob = synth.config_small(7, 32)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    flat, _ = plan.sample(d, 3, chains=2, burn_in=0, n_samples=3, init_scale=10.0, form="streamed")
    got = plan.sample_view(flat, 0, 2, 3).cpu().numpy()
    s0 = om.initial_state(3, 0, 0, 32, 32, 10.0)
    ref, _ = om.sample_pair(prob, 3, 0, 0, 0, 3, s0=s0)
    for k in range(3):
        assert rel(got[0, k], ref[0, k]) < REL_TOL and rel(got[1, k], ref[1, k]) < REL_TOL


@pytest.mark.parametrize("size,solve", [(32, "persistent"), (32, "streamed"), (64, "persistent"),
                                        (64, "streamed")])
def test_backward_matches_oracle_vjp(torch_cuda, size, solve):
    mf = _mf()
    banner(f"backward {size} {solve}")
    prob = synth.config_bands(1, size, 32)
    plan = mf.Plan([prob], streamed_solve=solve == "streamed")
    d = plan.concat([prob.d])
    sch_o = om.Schedule((1.0,), (0,), 1e-10, 100000, 10)
    s_ref, _ = om.wiener(prob, sch_o)
    g = np.random.default_rng(2).standard_normal((size, size))
    gd_ref, gt_ref, v_ref, _ = oa.wiener_vjp(prob, s_ref, g, sch_o)
    s_wf = plan.concat([s_ref])
    gs = plan.concat([g])
    gd, gb, v, info = plan.wiener_backward(s_wf, gs, mf.Schedule([1.0], [0], 1e-8, 6000, 10),
                                           want_v=True, allow_not_converged=True)
    rv = rel(plan.split(v)[0], v_ref)
    rd = rel(plan.split(gd)[0], gd_ref)
    gb = gb.cpu().numpy()
    rb = float(np.linalg.norm(gb - gt_ref) / np.linalg.norm(gt_ref))
    print(f"info {info[0]} rel v {rv:.2e} grad_d {rd:.2e} bands {rb:.2e}")
    assert rv < REL_TOL and rd < REL_TOL and rb < REL_TOL


def test_persistent_solve_batch_levels_and_residuals(torch_cuda):
    """Many problems of the persistent sizes (and one streamed size) in one plan,
    a cooling schedule with a convergence phase: every problem's sweep count,
    residual and image agree with the oracle's, so the per-problem stopping rule
    runs independently in each workgroup."""
    mf = _mf()
    banner("persistent solve batch")
    probs = synth.config_uneven(9, n_problems=10, sizes=(16, 32, 64, 128), weights=(0.1, 0.3, 0.3, 0.3))
    plan = mf.Plan(probs)
    d = plan.concat([p.d for p in probs])
    levels = ((20.0, 3), (4.0, 3), (1.0, 4))
    sch = mf.Schedule([l for l, _ in levels], [k for _, k in levels], 2e-3, 3000, 5)
    s, info = plan.wiener(d, sch)
    for i, p in enumerate(probs):
        ref, rinfo = om.wiener(p, om.Schedule(tuple(l for l, _ in levels), tuple(k for _, k in levels),
                                              2e-3, 3000, 5))
        r = rel(plan.split(s)[i], ref)
        print(f"problem {i} {p.H}: sweeps {info[i].sweeps}/{rinfo.sweeps} "
              f"residual {info[i].residual:.4e}/{rinfo.residual:.4e} rel {r:.2e}")
        assert info[i].converged and info[i].sweeps == rinfo.sweeps
        assert abs(info[i].residual - rinfo.residual) < 1e-3 * rinfo.residual + 1e-6
        assert r < REL_TOL


@pytest.mark.parametrize("solve", ["persistent", "streamed"])
def test_wiener_in_place_resume(torch_cuda, solve):
    """s_init may be the output array: 20 sweeps, then 25 more started from
    the first result, equal 45 sweeps of the oracle."""
    mf = _mf()
    banner(f"wiener resume in place {solve}")
    prob = synth.config_128(4, 128)
    plan = mf.Plan([prob], streamed_solve=solve == "streamed")
    d = plan.concat([prob.d])
    s, _ = plan.wiener(d, mf.Schedule.fixed(20))
    s2, _ = plan.wiener(d, mf.Schedule.fixed(25), s_init=s, out=s)
    ref, _ = om.wiener(prob, om.Schedule.fixed(45))
    r = rel(plan.split(s2)[0], ref)
    print(f"rel {r:.2e}")
    assert s2.data_ptr() == s.data_ptr() and r < REL_TOL


@pytest.mark.parametrize("solve", ["persistent", "streamed"])
def test_nonfinite_data_is_reported(torch_cuda, solve):
    """NaN in the data of an observed pixel: the residual test stops that
    problem and the call returns MF_ERR_NONFINITE; a clean problem in the same
    batch still converges to the oracle's result."""
    mf = _mf()
    banner(f"non-finite data {solve}")
    probs = [synth.config_small(3, 32), synth.config_small(4, 32)]
    plan = mf.Plan(probs, streamed_solve=solve == "streamed")
    bad = probs[0].d.copy()
    y, x = np.argwhere(~probs[0].mask)[5]
    bad[y, x] = np.nan
    d = plan.concat([bad, probs[1].d])
    sch = mf.Schedule([1.0], [0], 1e-3, 2000, 10)
    out = torch_cuda.empty_like(d)
    with pytest.raises(mf.MFError) as e:
        plan.wiener(d, sch, out=out)
    assert e.value.status == 6
    ref, _ = om.wiener(probs[1], om.Schedule((1.0,), (0,), 1e-3, 2000, 10))
    assert rel(plan.split(out)[1], ref) < REL_TOL


def test_sample_moments_match_numpy(torch_cuda):
    """Per-pixel mean and variance over chains and samples of a two-size batch,
    against numpy on the same samples (FP64 both sides)."""
    mf = _mf()
    banner("sample moments")
    probs = [synth.config_small(1, 32), synth.config_128(2, 64)]
    plan = mf.Plan(probs)
    d = plan.concat([p.d for p in probs])
    chains, n_samples = 5, 40
    flat, _ = plan.sample(d, 3, chains=chains, burn_in=5, n_samples=n_samples)
    mean, var = plan.sample_moments(flat, chains, n_samples)
    for i, p in enumerate(probs):
        x = plan.sample_view(flat, i, chains, n_samples).cpu().numpy().astype(np.float64)
        x = x.reshape(chains * n_samples, p.H, p.W)
        m_ref, v_ref = x.mean(axis=0), x.var(axis=0, ddof=1)
        m = plan.split(mean)[i]
        v = plan.split(var)[i]
        assert np.max(np.abs(m - m_ref)) < 1e-12 * np.max(np.abs(m_ref)) + 1e-12
        assert np.max(np.abs(v - v_ref) / v_ref) < 1e-10


def test_band_power_matches_numpy(torch_cuda):
    mf = _mf()
    prob = synth.config_bands(2, 64, 32)
    plan = mf.Plan([prob])
    rng = np.random.default_rng(0)
    x, y = rng.standard_normal((64, 64)), rng.standard_normal((64, 64))
    out = plan.band_power(plan.concat([x]), plan.concat([y])).cpu().numpy()
    ref = oa.band_cross_power(x, y, prob.spectrum.edges, 64, 64)
    assert np.max(np.abs(out - ref)) < 1e-4 * np.max(np.abs(ref))


def test_persistent_agrees_with_streamed_128_batch(torch_cuda):
    """The paper-size image with many chains: both forms draw the same samples
    (different FFT factorisations, so agreement is to FP32 rounding)."""
    mf = _mf()
    banner("persistent vs streamed 128, 64 chains")
    prob = synth.config_128(0)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    seed = synth.philox_seed(0)
    a, _ = plan.sample(d, seed, chains=64, burn_in=20, n_samples=5, form="persistent")
    b, _ = plan.sample(d, seed, chains=64, burn_in=20, n_samples=5, form="streamed")
    va = plan.sample_view(a, 0, 64, 5).cpu().numpy()
    vb = plan.sample_view(b, 0, 64, 5).cpu().numpy()
    worst = max(rel(va[c, k], vb[c, k]) for c in range(64) for k in range(5))
    print(f"worst persistent/streamed rel {worst:.2e}")
    assert worst < 1e-5
    _check_samples(plan, a, prob, 0, 64, 5, seed, 20, pairs=[0, 31])


def test_persistent_multi_problem_and_state(torch_cuda):
    mf = _mf()
    banner("persistent multi-problem")
    probs = [synth.config_small(i, 32) for i in range(3)] + [synth.config_128(3, 64)]
    plan = mf.Plan(probs)
    d = plan.concat([p.d for p in probs])
    st = plan.state_buffer(4)
    flat, _ = plan.sample(d, 11, chains=4, burn_in=3, n_samples=4, thin=2, form="persistent", state_out=st)
    for i, p in enumerate(probs):
        _check_samples(plan, flat, p, i, 4, 4, 11, 3, thin=2)
    # resume from the persistent state with the streamed form
    more, _ = plan.sample(d, 11, chains=4, burn_in=0, n_samples=2, sweep_offset=11, form="streamed",
                          state_in=st)
    full, _ = plan.sample(d, 11, chains=4, burn_in=11, n_samples=2, form="persistent")
    worst = max(rel(plan.sample_view(more, i, 4, 2).cpu().numpy()[c, k],
                    plan.sample_view(full, i, 4, 2).cpu().numpy()[c, k])
                for i in range(4) for c in range(4) for k in range(2))
    assert worst < 1e-5


@pytest.mark.parametrize("solve", ["persistent", "streamed"])
def test_inf_as_1e8_flag_matches_the_finite_noise_problem(torch_cuda, solve):
    """MF_FLAG_INF_AS_1E8 gives missing pixels the noise variance 1e8: the
    filter and the samples equal the oracle's on the problem with 1e8 written
    in, and the plan equals one made from that problem without the flag."""
    import copy
    torch = torch_cuda
    mf = _mf()
    banner(f"inf as 1e8, {solve}")
    prob = synth.config_small(5, 64)
    fin = copy.copy(prob)
    fin.noise_var = np.where(np.isfinite(prob.noise_var), prob.noise_var, 1e8)
    plan = mf.Plan([prob], streamed_solve=solve == "streamed", inf_as_1e8=True)
    ref_plan = mf.Plan([fin], streamed_solve=solve == "streamed")
    d = plan.concat([prob.d])
    levels = [(30.0, 5), (1.0, 40)]
    sch = mf.Schedule([l for l, _ in levels], [k for _, k in levels])
    s, _ = plan.wiener(d, sch)
    s2, _ = ref_plan.wiener(d, sch)
    assert torch.equal(s, s2)
    ref, _ = om.wiener(fin, om.Schedule(tuple(l for l, _ in levels), tuple(k for _, k in levels)))
    r = rel(plan.split(s)[0], ref)
    form = "persistent" if solve == "persistent" else "streamed"
    flat, _ = plan.sample(d, 12, chains=2, burn_in=3, n_samples=2, form=form)
    x = plan.sample_view(flat, 0, 2, 2).cpu().numpy()
    smp, _ = om.sample_pair(fin, 12, 0, 0, 3, 2)
    rs = max(rel(x[h, k], smp[h, k]) for h in range(2) for k in range(2))
    print(f"filter rel {r:.2e}, samples rel {rs:.2e}")
    assert r < REL_TOL and rs < REL_TOL
    with pytest.raises(mf.MFError):
        from paper_1810_02821_amd import _binding
        import ctypes as C
        h = C.c_void_p()
        arr = (_binding._Problem * 1)()
        nv = np.ascontiguousarray(prob.noise_var, dtype=np.float32)
        spec, keep = _binding._spectrum_c(prob.spectrum)
        arr[0] = _binding._Problem(64, 64, nv.ctypes.data_as(C.POINTER(C.c_float)), spec, None)
        _binding._check(_binding.lib().mf_plan_create(C.byref(h), 1, arr, 1 << 20, None))


@pytest.mark.parametrize("size,form", [(64, "persistent"), (64, "streamed"), (32, "plain"), (256, "auto")])
def test_sampler_with_cooling_levels_matches_oracle(torch_cuda, size, form):
    """Cooling levels before the burn-in (run on the streamed kernels for every
    form, then the form's own sampling phase from the cooled state)."""
    mf = _mf()
    banner(f"sampler with cooling {size} {form}")
    prob = synth.config_small(6, size)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    levels = [(20.0, 3), (4.0, 2)]
    cool = mf.Schedule([l for l, _ in levels], [k for _, k in levels])
    chains, burn_in, n_samples = 3, 2, 3
    st = plan.state_buffer(chains)
    flat, _ = plan.sample(d, 17, chains=chains, burn_in=burn_in, n_samples=n_samples, form=form, cooling=cool,
                          state_out=st)
    x = plan.sample_view(flat, 0, chains, n_samples).cpu().numpy()
    worst = 0.0
    for q in range(2):
        ref, s_ref = om.sample_pair(prob, 17, 0, q, burn_in, n_samples, cooling=levels)
        for h in range(2):
            if 2 * q + h >= chains:
                continue
            for k in range(n_samples):
                worst = max(worst, rel(x[2 * q + h, k], ref[h, k]))
        pair = st.view(-1, 2)[q * size * size:(q + 1) * size * size].cpu().numpy()
        worst = max(worst, rel(pair[:, 0] + 1j * pair[:, 1], s_ref.ravel()))
    print(f"worst rel {worst:.2e}")
    assert worst < REL_TOL


@pytest.mark.parametrize("size,form", [(128, "persistent"), (256, "streamed"), (512, "streamed")])
def test_thousand_sweeps_per_sample_parity_large(torch_cuda, size, form):
    """Per-sample parity every 100th sweep up to 1000 on the same Philox stream:
    the persistent kernel at the paper's image size, and the fused streamed
    kernels (first pass from HBM, update in registers, last pass to HBM) at
    256^2 and 512^2."""
    mf = _mf()
    banner(f"1000 sweeps {size}x{size} {form}")
    prob = synth.config_128(8, size)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    seed = synth.philox_seed(8)
    chains = 4 if size <= 128 else 2
    flat, _ = plan.sample(d, seed, chains=chains, burn_in=0, n_samples=10, thin=100, form=form)
    got = plan.sample_view(flat, 0, chains, 10).cpu().numpy()
    worst = 0.0
    for q in range(chains // 2):
        ref, _ = om.sample_pair(prob, seed, 0, q, 0, 10, 100)
        for h in range(2):
            for k in range(10):
                worst = max(worst, rel(got[2 * q + h, k], ref[h, k]))
    print(f"worst rel over sweeps 100..1000: {worst:.2e}")
    assert worst < REL_TOL


def _golden_wiener_1024():
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "wiener_cg_1024.txt")
    idx, val, norm = [], [], None
    with open(path) as f:
        for line in f:
            if line.startswith("# norm"):
                norm = float(line.split()[2])
            elif not line.startswith("#"):
                i, v = line.split()
                idx.append(int(i))
                val.append(float(v))
    return np.array(idx), np.array(val), norm


@pytest.mark.parametrize("solve_form", ["streamed"])
def test_converged_wiener_1024_matches_cg(torch_cuda, solve_form):
    """The converged messenger filter at 1024^2 (the paper-size recipe scaled
    up; 30 cooling levels 1e3 -> 1, then 6000 sweeps at lambda = 1) against the
    oracle's conjugate-gradient solution of Eq. 2-3 (pinned against the dense
    solve), stored at 2048 seeded pixels with the solution's norm by
    tests/golden/make_wiener_cg_1024.py."""
    mf = _mf()
    banner("converged Wiener filter 1024 vs CG")
    idx, val, norm = _golden_wiener_1024()
    prob = synth.config_128(0, 1024)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    sch = mf.Schedule(list(np.geomspace(1e3, 1.0, 30)) + [1.0], [10] * 30 + [6000])
    s, _ = plan.wiener(d, sch)
    x = plan.split(s)[0].astype(np.float64)
    r_pix = float(np.linalg.norm(x.ravel()[idx] - val) / np.linalg.norm(val))
    r_norm = abs(np.linalg.norm(x) - norm) / norm
    print(f"sampled pixels rel {r_pix:.2e}, norm rel {r_norm:.2e}")
    assert r_pix < REL_TOL and r_norm < REL_TOL
