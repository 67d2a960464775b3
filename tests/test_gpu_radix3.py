"""Image sides 2^a 3^b (even) on the GPU: the streamed kernels with radix-3
passes and ragged column tiles, against the FP64 oracle (whose library FFT is
pinned to the naive DFT of Eq. 8 at 24^2 and 12 x 18)."""
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
    mf.lib()
    return torch


def _mf():
    import paper_1810_02821_amd as mf
    return mf


def _problem(seed, H, W):
    return synth.config_128(seed, H) if H == W else synth.config_bands(seed, H, 8, width=W)


@pytest.mark.parametrize("H,W,form", [(24, 24, "streamed"), (48, 48, "streamed"), (96, 96, "streamed"),
                                      (384, 384, "streamed"), (18, 36, "streamed"), (24, 96, "plain"),
                                      (162, 54, "streamed"), (1944, 16, "streamed"), (16, 1458, "streamed"),
                                      (1536, 24, "streamed")])
def test_samples_match_oracle(torch_cuda, H, W, form):
    mf = _mf()
    banner(f"samples {form} {H}x{W}")
    prob = _problem(11, H, W)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    seed = synth.philox_seed(11)
    flat, _ = plan.sample(d, seed, chains=3, burn_in=2, n_samples=3, form=form)
    got = plan.sample_view(flat, 0, 3, 3).cpu().numpy()
    worst = 0.0
    for q in range(2):
        ref, _ = om.sample_pair(prob, seed, 0, q, 2, 3)
        for h in range(2):
            if 2 * q + h < 3:
                for k in range(3):
                    worst = max(worst, rel(got[2 * q + h, k], ref[h, k]))
    print(f"worst {worst:.2e}")
    assert worst < REL_TOL


def test_auto_form_mixed_batch_and_persistent_refused(torch_cuda):
    """A plan mixing 24^2, 32^2 (persistent) and 48 x 96: the automatic form
    runs each class on its kernels; the persistent form refuses 24^2."""
    mf = _mf()
    banner("mixed 2^a 3^b batch")
    probs = [_problem(1, 24, 24), synth.config_small(2, 32), _problem(3, 48, 96)]
    plan = mf.Plan(probs)
    d = plan.concat([p.d for p in probs])
    flat, _ = plan.sample(d, 9, chains=2, burn_in=1, n_samples=2)
    for i, p in enumerate(probs):
        got = plan.sample_view(flat, i, 2, 2).cpu().numpy()
        ref, _ = om.sample_pair(p, 9, i, 0, 1, 2)
        assert max(rel(got[h, k], ref[h, k]) for h in range(2) for k in range(2)) < REL_TOL
    with pytest.raises(mf.MFError) as e:
        plan.sample(d, 9, chains=2, burn_in=1, n_samples=2, form="persistent")
    assert e.value.status == 2


@pytest.mark.parametrize("size", [24, 96, 192])
def test_wiener_matches_oracle(torch_cuda, size):
    mf = _mf()
    banner(f"wiener {size}")
    prob = synth.config_128(4, size)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    levels = [(30.0, 5), (5.0, 5), (1.0, 40)]
    s, _ = plan.wiener(d, mf.Schedule([l for l, _ in levels], [k for _, k in levels]))
    ref, _ = om.wiener(prob, om.Schedule(tuple(l for l, _ in levels), tuple(k for _, k in levels)))
    r = rel(plan.split(s)[0], ref)
    print(f"rel {r:.2e}")
    assert r < REL_TOL


def test_gradient_24_matches_dense_fp64(torch_cuda):
    """The differentiation workload's dense check: at 24 x 24 (32 bands) the
    implicit VJP of the GPU messenger solve against the dense FP64 gradient
    (torch autograd through Eq. 2 solved densely), for a random cotangent."""
    mf = _mf()
    banner("gradient 24x24 vs dense FP64")
    prob = synth.config_bands(0, 24, 32)
    plan = mf.Plan([prob])
    S = dense.signal_covariance(prob.spectrum, 24, 24)
    s_ref = dense.wiener_dense(S, prob.noise_var, prob.d)
    g = np.random.default_rng(1).standard_normal((24, 24))
    gd_ref, gt_ref, _ = oa.dense_vjp(prob, g)
    adj = mf.Schedule(list(np.geomspace(1e3, 1.0, 30)) + [1.0], [10] * 30 + [6000])
    gd, gb, _, info = plan.wiener_backward(plan.concat([s_ref]), plan.concat([g]), adj, allow_not_converged=True)
    rd = rel(plan.split(gd)[0], gd_ref.reshape(24, 24))
    gb = gb.cpu().numpy()
    nz = np.abs(gt_ref) > 0  # empty bands have a zero gradient on both sides
    rb = float(np.linalg.norm(gb - gt_ref) / np.linalg.norm(gt_ref))
    print(f"grad_d {rd:.2e} bands {rb:.2e} ({int(nz.sum())} non-empty bands)")
    assert rd < REL_TOL and rb < REL_TOL
    assert np.all(gb[~nz] == 0)


@pytest.mark.parametrize("size,ckpt", [(48, 7), (96, 20)])
def test_unrolled_gradient_matches_oracle(torch_cuda, size, ckpt):
    """Reverse mode through a truncated schedule on the plain kernels with
    stored transforms and band slots over ragged column tiles."""
    mf = _mf()
    banner(f"unrolled gradient {size}")
    prob = synth.config_bands(7, size, 16)
    plan = mf.Plan([prob])
    lams, sweeps = (50.0, 5.0, 1.0), (20, 20, 40)
    g = np.random.default_rng(8).standard_normal((size, size))
    sK, gd, gb = plan.wiener_backward_unrolled(plan.concat([prob.d]), plan.concat([g]),
                                               mf.Schedule(list(lams), list(sweeps)), checkpoint_every=ckpt)
    s_ref, gd_ref, gt_ref = oa.unrolled_vjp(prob, om.Schedule(lams, sweeps), g)
    rs, rd = rel(plan.split(sK)[0], s_ref), rel(plan.split(gd)[0], gd_ref)
    rt = float(np.linalg.norm(gb.cpu().numpy() - gt_ref) / np.linalg.norm(gt_ref))
    print(f"s {rs:.2e} grad_d {rd:.2e} grad_theta {rt:.2e}")
    assert rs < REL_TOL and rd < REL_TOL and rt < REL_TOL


def test_band_power_matches_numpy(torch_cuda):
    mf = _mf()
    prob = synth.config_bands(2, 48, 8, width=72)
    plan = mf.Plan([prob])
    rng = np.random.default_rng(0)
    x, y = rng.standard_normal((48, 72)), rng.standard_normal((48, 72))
    out = plan.band_power(plan.concat([x]), plan.concat([y])).cpu().numpy()
    ref = oa.band_cross_power(x, y, prob.spectrum.edges, 48, 72)
    assert np.max(np.abs(out - ref)) < 1e-4 * np.max(np.abs(ref))


@pytest.mark.parametrize("H,W", [(20, 20), (27, 27), (4096, 16), (24, 30)])
def test_other_sides_are_refused(torch_cuda, H, W):
    mf = _mf()
    prob = synth.config_small(0, 16)
    prob.H, prob.W = H, W
    prob.noise_var = np.ones((H, W))
    with pytest.raises(mf.MFError) as e:
        mf.Plan([prob])
    assert e.value.status == 2


def test_hierarchical_and_shear_refuse_factor_three(torch_cuda):
    mf = _mf()
    plan = mf.Plan([synth.config_bands(1, 24, 8)])
    with pytest.raises(mf.MFError) as e:
        plan.sample_spectrum(plan.concat([plan.problems[0].d]), 1, chains=2, burn_in=1, n_samples=1)
    assert e.value.status == 2
