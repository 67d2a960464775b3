"""Problems with a diagonal response A (d = A s + n; gain variation and pixels
without response) on the GPU vs the FP64 oracle, which applies Algorithm 1's
A_i definitions directly."""
import numpy as np
import pytest

from gpu_common import REL_TOL, banner, rel
from oracle import adjoint as oa, messenger as om
from paper_1810_02821_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1810_02821_amd as mf
    mf.lib()
    return torch


@pytest.mark.parametrize("size,solve", [(64, "persistent"), (128, "streamed"), (256, "streamed")])
def test_wiener_with_response_matches_oracle(torch_cuda, size, solve):
    import paper_1810_02821_amd as mf
    banner(f"wiener with response {size} {solve}")
    probs = [synth.config_response(1, size), synth.config_128(2, size)]
    plan = mf.Plan(probs, streamed_solve=solve == "streamed")
    d = plan.concat([p.d for p in probs])
    levels = ((30.0, 5), (5.0, 5), (1.0, 40))
    s, _ = plan.wiener(d, mf.Schedule([l for l, _ in levels], [k for _, k in levels]))
    for i, p in enumerate(probs):
        ref, _ = om.wiener(p, om.Schedule(tuple(l for l, _ in levels), tuple(k for _, k in levels)))
        r = rel(plan.split(s)[i], ref)
        print(f"problem {i}: rel {r:.2e}")
        assert r < REL_TOL


def test_residual_stopping_with_response(torch_cuda):
    import paper_1810_02821_amd as mf
    banner("residual with response")
    prob = synth.config_response(3, 64)
    plan = mf.Plan([prob])
    s, info = plan.wiener(plan.concat([prob.d]), mf.Schedule([1.0], [0], 1e-3, 5000, 10))
    ref, rinfo = om.wiener(prob, om.Schedule((1.0,), (0,), 1e-3, 5000, 10))
    print(info[0], rinfo)
    assert info[0].sweeps == rinfo.sweeps
    assert abs(info[0].residual - rinfo.residual) < 1e-3 * rinfo.residual
    assert rel(plan.split(s)[0], ref) < REL_TOL


@pytest.mark.parametrize("size,form", [(64, "persistent"), (256, "streamed")])
def test_samples_with_response_match_oracle(torch_cuda, size, form):
    import paper_1810_02821_amd as mf
    banner(f"samples with response {size} {form}")
    prob = synth.config_response(4, size)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    flat, _ = plan.sample(d, 17, chains=2, burn_in=3, n_samples=4, form=form)
    got = plan.sample_view(flat, 0, 2, 4).cpu().numpy()
    ref, _ = om.sample_pair(prob, 17, 0, 0, 3, 4)
    worst = max(rel(got[c, k], ref[c, k]) for c in range(2) for k in range(4))
    print(f"worst {worst:.2e}")
    assert worst < REL_TOL


@pytest.mark.parametrize("solve", ["persistent", "streamed"])
def test_backward_with_response_matches_oracle(torch_cuda, solve):
    import paper_1810_02821_amd as mf
    banner(f"backward with response {solve}")
    prob = synth.config_response(5, 64)
    plan = mf.Plan([prob], streamed_solve=solve == "streamed")
    sch_o = om.Schedule((1.0,), (0,), 1e-10, 100000, 10)
    s_ref, _ = om.wiener(prob, sch_o)
    g = np.random.default_rng(6).standard_normal((64, 64))
    gd_ref, _, v_ref, _ = oa.wiener_vjp(prob, s_ref, g, sch_o)
    # cooling levels first, then lambda = 1 until the residual reaches the
    # FP32 floor (the residual test stops there, well inside the sweep cap)
    adj = mf.Schedule(list(np.geomspace(1e3, 1.0, 30)) + [1.0], [10] * 30 + [0], 3e-6, 20000, 10)
    gd, _, v, info = plan.wiener_backward(plan.concat([s_ref]), plan.concat([g]), adj, want_v=True,
                                          allow_not_converged=True)
    rv, rd = rel(plan.split(v)[0], v_ref), rel(plan.split(gd)[0], gd_ref)
    print(f"info {info[0]} rel v {rv:.2e} grad_d {rd:.2e}")
    assert rv < REL_TOL and rd < REL_TOL


def test_unrolled_gradient_with_response_matches_oracle(torch_cuda):
    import paper_1810_02821_amd as mf
    banner("unrolled gradient with response 128")
    prob = synth.config_response(7, 128)
    plan = mf.Plan([prob])
    levels = ((20.0, 4), (4.0, 4), (1.0, 12))
    g = np.random.default_rng(9).standard_normal((128, 128))
    sK, gd, _ = plan.wiener_backward_unrolled(plan.concat([prob.d]), plan.concat([g]),
                                              mf.Schedule([l for l, _ in levels], [k for _, k in levels]), 7)
    s_ref, gd_ref, _ = oa.unrolled_vjp(prob, om.Schedule(tuple(l for l, _ in levels),
                                                         tuple(k for _, k in levels)), g)
    rs, rd = rel(plan.split(sK)[0], s_ref), rel(plan.split(gd)[0], gd_ref)
    print(f"s {rs:.2e} grad_d {rd:.2e}")
    assert rs < REL_TOL and rd < REL_TOL
