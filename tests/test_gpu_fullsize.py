"""The measured workloads at their full sizes, in the launch configurations the
benchmarks time, checked on outputs the FP64 oracle can compute one by one:

* 128^2 sampler: 1024 chains, 200 burn-in + 98 samples, persistent form; every
  sample of chains {0, 1, 510, 511, 1022, 1023} and their sample mean;
* uneven batch: 4096 problems of sizes {64, 128, 256, 512}^2, one chain each,
  500 sweeps, autotuned tiles and graph-captured sweep loops; the final state of
  the first problem of every size class and of the last 64^2 problem;
* large map: 2048^2 with 32 band amplitudes, the unrolled gradient with a
  checkpoint every 20 sweeps (24 sweeps, so the last segment is ragged);
* the large map in the launch configurations of the hierarchical (64 chains,
  32 bands), 16-bit storage (64 chains) and mass-mapping (32 chains, shear
  recipe) benchmarks, for a few sweeps; the last chain pair (or chain)
  against the oracle.
"""
import numpy as np
import pytest

from gpu_common import REL_TOL, banner, rel
from oracle import adjoint as oa, messenger as om
from oracle import shear as osh, spectrum as osp, storage as ost
from paper_1810_02821_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1810_02821_amd as mf
    mf.lib()
    return torch


def test_sampler_128_full_workload(torch_cuda):
    import paper_1810_02821_amd as mf
    banner("128^2 sampler, 1024 chains x (200 + 98)")
    chains, burn_in, n_samples = 1024, 200, 98
    prob = synth.config_128(0, 128)
    seed = synth.philox_seed(0)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    out = plan.samples_buffer(chains, n_samples)
    state = plan.state_buffer(chains)
    plan.sample(d, seed, chains=chains, burn_in=burn_in, n_samples=n_samples, form="persistent",
                state_out=state, out=out)
    view = plan.sample_view(out, 0, chains, n_samples)
    got_mean, ref_mean = np.zeros((128, 128)), np.zeros((128, 128))
    worst = 0.0
    for pair in (0, 255, 511):
        ref, _ = om.sample_pair(prob, seed, 0, pair, burn_in, n_samples)
        for q in range(2):
            got = view[2 * pair + q].cpu().numpy()
            for k in range(n_samples):
                worst = max(worst, rel(got[k], ref[q, k]))
            got_mean += got.mean(axis=0)
            ref_mean += ref[q].mean(axis=0)
        print(f"pair {pair}: worst sample rel so far {worst:.2e}", flush=True)
    rm = rel(got_mean, ref_mean)
    print(f"worst sample rel {worst:.2e}; mean of 6 chains rel {rm:.2e}")
    assert worst < REL_TOL and rm < REL_TOL


def test_uneven_batch_full_workload(torch_cuda):
    import paper_1810_02821_amd as mf
    banner("uneven batch, 4096 problems, 500 sweeps, autotune + graph")
    probs = synth.config_uneven(0, n_problems=4096)
    plan = mf.Plan(probs, autotune=True, graph=True)
    d = plan.concat([p.d for p in probs])
    st = plan.state_buffer(1)
    sweeps = 500
    plan.sample(d, 1000, chains=1, burn_in=sweeps, n_samples=0, form="auto", state_out=st, samples=False)
    picks = {}
    for i, p in enumerate(probs):
        picks.setdefault(p.H, i)
    picks["last64"] = max(i for i, p in enumerate(probs) if p.H == 64)
    for name, pid in picks.items():
        p = probs[pid]
        _, s_ref = om.sample_pair(p, 1000, pid, 0, sweeps, 0)
        got = plan.state_view(st, pid, 1).cpu().numpy()
        r = rel(got[0].real, s_ref.real)
        print(f"problem {pid} ({p.H}^2, {name}): rel {r:.2e}", flush=True)
        assert r < REL_TOL


def test_large_map_unrolled_gradient_2048(torch_cuda):
    import paper_1810_02821_amd as mf
    banner("large map 2048^2, unrolled gradient, 32 bands, checkpoint every 20")
    prob = synth.config_large(0, 2048, n_bands=32)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    levels = ((10.0, 12), (1.0, 12))
    g = np.random.default_rng(8).standard_normal((2048, 2048))
    s, gd, gb = plan.wiener_backward_unrolled(d, plan.concat([g]),
                                              mf.Schedule([l for l, _ in levels], [k for _, k in levels]), 20)
    s_ref, gd_ref, gt_ref = oa.unrolled_vjp(prob, om.Schedule(tuple(l for l, _ in levels),
                                                              tuple(k for _, k in levels)), g)
    rs = rel(plan.split(s)[0], s_ref)
    rd = rel(plan.split(gd)[0], gd_ref)
    gb = gb.cpu().numpy()
    rt = float(np.max(np.abs(gb - gt_ref)) / np.max(np.abs(gt_ref)))
    print(f"s {rs:.2e} grad_d {rd:.2e} grad_bands {rt:.2e}")
    assert rs < REL_TOL and rd < REL_TOL and rt < REL_TOL


def test_hierarchical_2048_streamed_launch(torch_cuda):
    import paper_1810_02821_amd as mf
    banner("2048^2 hierarchical, 64 chains, 1 iteration x 2 sweeps")
    prob = synth.config_large(0, 2048, n_bands=32)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    chains = 64
    ts, smp, _, _ = plan.sample_spectrum(d, 1000, chains, 0, 1, 1, 2, samples=True)
    th = plan.theta_view(ts, 0, chains, 1).cpu().numpy()
    sv = plan.sample_view(smp, 0, chains, 1).cpu().numpy()
    t_ref, s_ref, _, _ = osp.sample_pair_hierarchical(prob, 1000, 0, 31, 0, 1, 1, 2)
    scale = np.asarray(prob.spectrum.amps)
    for h in range(2):
        wt = float(np.max(np.abs(th[62 + h, 0] - t_ref[h, 0]) / (np.abs(t_ref[h, 0]) + scale)))
        ws = rel(sv[62 + h, 0], s_ref[h, 0])
        print(f"chain {62 + h}: theta {wt:.2e}, sample {ws:.2e}")
        assert wt < REL_TOL and ws < REL_TOL


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_storage_2048_launch(torch_cuda, storage):
    import paper_1810_02821_amd as mf
    banner(f"2048^2 sampler, 64 chains, {storage} storage, 2 sweeps")
    prob = synth.config_large(0, 2048)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    chains = 64
    flat, _ = plan.sample(d, 1000, chains=chains, burn_in=1, n_samples=1, form="streamed", storage=storage)
    x = plan.sample_view(flat, 0, chains, 1).cpu().numpy()
    ref, _ = ost.sample_pair_stored(prob, 1000, 0, 31, 1, 1, 1, storage)
    u = {"fp16": 2.0 ** -11, "bf16": 2.0 ** -8}[storage]
    tol = REL_TOL + np.sqrt(2) * 2 * np.sqrt(2 * 1e-6 / u) * 2 * u
    for h in range(2):
        e = rel(x[62 + h, 0], ref[h, 0])
        print(f"chain {62 + h}: {e:.2e} (tol {tol:.2e})")
        assert e < tol


def test_shear_2048_streamed_launch(torch_cuda):
    import paper_1810_02821_amd as mf
    banner("2048^2 mass mapping, 32 chains, 1 sweep")
    prob = synth.config_shear(0, 2048, 0.3)
    plan = mf.Plan([prob])
    g = plan.concat_complex([prob.gamma])
    chains = 32
    out, _ = plan.shear_sample(g, 1000, chains, 0, 1, 1, b_ratio=0.3)
    got = out.view(chains, 1, 2048, 2048)[31, 0].cpu().numpy()
    ref, _ = osh.sample_shear_chain(prob, 1000, 0, 31, 0, 1, 1, 0.3)
    e = rel(np.concatenate([got.real.ravel(), got.imag.ravel()]),
            np.concatenate([ref[0].real.ravel(), ref[0].imag.ravel()]))
    print(f"chain 31: {e:.2e}")
    assert e < REL_TOL
