"""Hierarchical sampler (signal + band amplitudes) on the GPU vs the FP64 oracle,
on the same seeded inputs and the same random stream.

Band amplitudes are compared per band as |theta - theta_ref| <= 1e-4 (theta_ref
+ theta_start): a band amplitude is a band power over a chi-square variate,
and the FP32 signal fixes the power only up to its own rounding.  A band with
few modes can draw an amplitude far below its scale (band 0 holds the single
mode k = 0), where a relative test would measure the signal's rounding, not
the draw; theta_start, the band's starting amplitude, is that scale.  Band
sums are FP64 atomics in LDS, so amplitudes agree between runs to FP64
rounding, not bit for bit."""
import numpy as np
import pytest

from gpu_common import REL_TOL, banner, rel
from oracle import spectrum as osp
from paper_1810_02821_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1810_02821_amd as mf
    mf.lib()
    return torch


def _check(plan, ts, smp, probs, pid, chains, n_samples, seed, burn_in, thin, sweeps, prior_dof, prior_beta):
    th = plan.theta_view(ts, pid, chains, n_samples).cpu().numpy()
    scale = np.asarray(probs[pid].spectrum.amps)
    sv = plan.sample_view(smp, pid, chains, n_samples).cpu().numpy() if smp is not None else None
    worst_t = worst_s = 0.0
    for q in range((chains + 1) // 2):
        t_ref, s_ref, _, _ = osp.sample_pair_hierarchical(probs[pid], seed, pid, q, burn_in, n_samples, thin,
                                                          sweeps, prior_dof, prior_beta)
        for h in range(2):
            c = 2 * q + h
            if c >= chains:
                continue
            worst_t = max(worst_t, float(np.max(np.abs(th[c] - t_ref[h]) / (np.abs(t_ref[h]) + scale))))
            if sv is not None:
                for k in range(n_samples):
                    worst_s = max(worst_s, rel(sv[c, k], s_ref[h, k]))
    return worst_t, worst_s


@pytest.mark.parametrize("size,prior", [(32, (0, 0.0)), (64, (4, 0.5)), (128, (0, 0.0))])
def test_hierarchical_samples_match_oracle(torch_cuda, size, prior):
    import paper_1810_02821_amd as mf
    banner(f"hierarchical sampler {size} prior {prior}")
    prob = synth.config_bands(2, size, 16)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    seed, chains, burn_in, n_samples, thin, sweeps = 21, 3, 2, 3, 2, 2
    ts, smp, _, _ = plan.sample_spectrum(d, seed, chains, burn_in, n_samples, thin, sweeps, prior[0], prior[1],
                                         samples=True)
    wt, ws = _check(plan, ts, smp, [prob], 0, chains, n_samples, seed, burn_in, thin, sweeps, *prior)
    print(f"worst theta rel {wt:.2e}, worst sample rel {ws:.2e}")
    assert wt < REL_TOL and ws < REL_TOL


def test_hierarchical_long_chain_128(torch_cuda):
    """60 iterations of one sweep each: the amplitudes stay on the oracle's path."""
    import paper_1810_02821_amd as mf
    banner("hierarchical sampler 128, 60 iterations")
    prob = synth.config_bands(3, 128, 32)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    ts, _, _, _ = plan.sample_spectrum(d, 5, 2, 0, 60, 1, 1)
    wt, _ = _check(plan, ts, None, [prob], 0, 2, 60, 5, 0, 1, 1, 0, 0.0)
    print(f"worst theta rel {wt:.2e}")
    assert wt < REL_TOL


def test_hierarchical_batch_and_resume(torch_cuda):
    """Two problems of different sizes in one plan, each against the oracle
    with its own problem index; a run split in two by iteration_offset (state
    and amplitudes carried over) equals the uninterrupted run up to the FP64
    rounding of the band sums."""
    torch = torch_cuda
    import paper_1810_02821_amd as mf
    banner("hierarchical batch + resume")
    probs = [synth.config_bands(4, 32, 8), synth.config_bands(5, 64, 12)]
    plan = mf.Plan(probs)
    d = plan.concat([p.d for p in probs])
    chains = 2
    st_full = plan.state_buffer(chains)
    ts_full, _, _, th_full = plan.sample_spectrum(d, 9, chains, 0, 6, 1, 2, state_out=st_full)
    for pid in range(2):
        wt, _ = _check(plan, ts_full, None, probs, pid, chains, 6, 9, 0, 1, 2, 0, 0.0)
        print(f"problem {pid}: worst theta rel {wt:.2e}")
        assert wt < REL_TOL
    st_a = plan.state_buffer(chains)
    ts_a, _, _, th_a = plan.sample_spectrum(d, 9, chains, 0, 2, 1, 2, state_out=st_a)
    st_b = plan.state_buffer(chains)
    ts_b, _, _, th_b = plan.sample_spectrum(d, 9, chains, 0, 4, 1, 2, iteration_offset=2, state_in=st_a,
                                            theta_in=th_a, state_out=st_b)
    assert rel(st_b.cpu().numpy(), st_full.cpu().numpy()) < 1e-6
    assert torch.allclose(th_b, th_full, rtol=1e-9, atol=0)
    for pid in range(2):
        full = plan.theta_view(ts_full, pid, chains, 6)
        assert torch.allclose(plan.theta_view(ts_b, pid, chains, 4), full[:, 2:], rtol=1e-9, atol=0)


@pytest.mark.parametrize("H,W,prior", [(256, 256, (4, 0.5)), (64, 128, (0, 0.0)), (128, 64, (2, 0.1)),
                                         (2048, 16, (0, 0.0)), (16, 1024, (0, 0.0)), (512, 32, (3, 0.2)),
                                         (1024, 16, (2, 0.3))])
def test_streamed_hierarchical_samples_match_oracle(torch_cuda, H, W, prior):
    """Size classes outside the persistent kernel (256^2 and more, or H != W)
    run on the streamed kernels with mirror-paired column tiles; the long
    thin shapes reach the 2048- and 1024-point column transforms at a size
    the oracle runs quickly."""
    import paper_1810_02821_amd as mf
    banner(f"streamed hierarchical sampler {H}x{W} prior {prior}")
    prob = synth.config_bands(6, H, 16, width=W)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    seed, chains, burn_in, n_samples, thin, sweeps = 23, 3, 1, 2, 2, 2
    ts, smp, _, _ = plan.sample_spectrum(d, seed, chains, burn_in, n_samples, thin, sweeps, prior[0], prior[1],
                                         samples=True)
    wt, ws = _check(plan, ts, smp, [prob], 0, chains, n_samples, seed, burn_in, thin, sweeps, *prior)
    print(f"worst theta rel {wt:.2e}, worst sample rel {ws:.2e}")
    assert wt < REL_TOL and ws < REL_TOL


def test_streamed_hierarchical_batch_and_resume(torch_cuda):
    """A persistent (32^2) and two streamed (64 x 128, 256^2) size classes in
    one plan, each against the oracle; the streamed run split by
    iteration_offset, resumed in place, equals the uninterrupted run."""
    torch = torch_cuda
    import paper_1810_02821_amd as mf
    banner("streamed hierarchical batch + resume")
    probs = [synth.config_bands(7, 32, 8), synth.config_bands(8, 64, 12, width=128),
             synth.config_bands(9, 256, 20)]
    plan = mf.Plan(probs)
    d = plan.concat([p.d for p in probs])
    chains = 2
    st_full = plan.state_buffer(chains)
    ts_full, _, _, th_full = plan.sample_spectrum(d, 13, chains, 0, 5, 1, 2, 2, 0.3, state_out=st_full)
    for pid in range(3):
        wt, _ = _check(plan, ts_full, None, probs, pid, chains, 5, 13, 0, 1, 2, 2, 0.3)
        print(f"problem {pid}: worst theta rel {wt:.2e}")
        assert wt < REL_TOL
    st = plan.state_buffer(chains)
    _, _, _, th_a = plan.sample_spectrum(d, 13, chains, 0, 2, 1, 2, 2, 0.3, state_out=st)
    ts_b, _, _, th_b = plan.sample_spectrum(d, 13, chains, 0, 3, 1, 2, 2, 0.3, iteration_offset=2, state_in=st,
                                            theta_in=th_a, state_out=st)
    assert rel(st.cpu().numpy(), st_full.cpu().numpy()) < 1e-6
    assert torch.allclose(th_b, th_full, rtol=1e-9, atol=0)
    for pid in range(3):
        full = plan.theta_view(ts_full, pid, chains, 5)
        assert torch.allclose(plan.theta_view(ts_b, pid, chains, 3), full[:, 2:], rtol=1e-9, atol=0)


def test_streamed_hierarchical_without_iterations_keeps_inputs(torch_cuda):
    """No iterations: the state is the start state and theta_out the amplitudes it was given."""
    torch = torch_cuda
    import paper_1810_02821_amd as mf
    banner("streamed hierarchical, zero iterations")
    prob = synth.config_bands(10, 256, 8)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    st_in = torch.randn(2 * plan.total_pixels, dtype=torch.float32, device="cuda")
    th_in = torch.rand(2 * 8, dtype=torch.float64, device="cuda") + 0.5
    st = plan.state_buffer(2)
    _, _, _, th = plan.sample_spectrum(d, 1, 2, 0, 0, state_in=st_in, theta_in=th_in, state_out=st)
    assert torch.equal(st, st_in)
    assert torch.equal(th, th_in)


def test_hierarchical_rejects_unsupported_problems(torch_cuda):
    import paper_1810_02821_amd as mf
    banner("hierarchical sampler errors")
    plan = mf.Plan([synth.config_small(0, 32)])
    d = plan.concat([synth.config_small(0, 32).d])
    with pytest.raises(mf.MFError) as e:
        plan.sample_spectrum(d, 1, 2, 0, 1)
    assert e.value.status == 1


def test_streamed_hierarchical_single_chain(torch_cuda):
    """One chain (the imaginary chain of the pair is neither emitted nor
    reported) on a streamed size class."""
    import paper_1810_02821_amd as mf
    banner("streamed hierarchical, one chain, 64x128")
    prob = synth.config_bands(11, 64, 10, width=128)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    ts, smp, _, _ = plan.sample_spectrum(d, 5, 1, 1, 2, 1, 2, samples=True)
    wt, ws = _check(plan, ts, smp, [prob], 0, 1, 2, 5, 1, 1, 2, 0, 0.0)
    print(f"worst theta rel {wt:.2e}, worst sample rel {ws:.2e}")
    assert wt < REL_TOL and ws < REL_TOL


def test_streamed_hierarchical_graph_replays_match_eager(torch_cuda):
    """MF_FLAG_GRAPH captures the streamed hierarchical loop; replays with
    eager work in between agree with the eager run (band sums are FP64
    atomics, so amplitudes agree to FP64 rounding and samples to FP32)."""
    torch = torch_cuda
    import paper_1810_02821_amd as mf
    banner("streamed hierarchical graph replays")
    prob = synth.config_bands(13, 256, 12)
    eager = mf.Plan([prob])
    graph = mf.Plan([prob], graph=True)
    d = eager.concat([prob.d])
    ts0, sm0, _, th0 = eager.sample_spectrum(d, 4, 2, 1, 2, 1, 2, samples=True)
    for _ in range(3):
        ts, sm, _, th = graph.sample_spectrum(d, 4, 2, 1, 2, 1, 2, samples=True)
        torch.cuda.synchronize()
        assert torch.allclose(ts, ts0, rtol=1e-9, atol=0) and torch.allclose(th, th0, rtol=1e-9, atol=0)
        assert rel(sm.cpu().numpy(), sm0.cpu().numpy()) < 1e-6
        eager.sample_spectrum(d, 5, 2, 0, 1, 1, 1)
        torch.cuda.synchronize()
