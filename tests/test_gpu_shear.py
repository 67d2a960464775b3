"""Mass mapping (spin-2 shear operator) on the GPU vs the FP64 oracle, on
the same seeded inputs and the same random stream."""
import numpy as np
import pytest

from gpu_common import REL_TOL, banner, rel
from oracle import messenger as om, shear as osh
from paper_1810_02821_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1810_02821_amd as mf
    mf.lib()
    return torch


def crel(a, b):
    return rel(np.concatenate([a.real.ravel(), a.imag.ravel()]), np.concatenate([b.real.ravel(), b.imag.ravel()]))


@pytest.mark.parametrize("size,b_ratio", [(32, 0.0), (64, 0.5), (128, 0.0)])
def test_shear_wiener_matches_oracle(torch_cuda, size, b_ratio):
    import paper_1810_02821_amd as mf
    banner(f"shear wiener {size} b {b_ratio}")
    probs = [synth.config_shear(1, size, b_ratio), synth.config_shear(2, size, b_ratio)]
    plan = mf.Plan(probs)
    g = plan.concat_complex([p.gamma for p in probs])
    levels = ((50.0, 5), (5.0, 5), (1.0, 30))
    k = plan.shear_wiener(g, mf.Schedule([l for l, _ in levels], [n for _, n in levels]), b_ratio)
    for i, p in enumerate(probs):
        ref = osh.wiener_shear(p, om.Schedule(tuple(l for l, _ in levels), tuple(n for _, n in levels)), b_ratio)
        r = crel(plan.split_complex(k)[i], ref)
        print(f"problem {i}: rel {r:.2e}")
        assert r < REL_TOL


@pytest.mark.parametrize("size,b_ratio", [(32, 0.3), (128, 0.0)])
def test_shear_samples_match_oracle(torch_cuda, size, b_ratio):
    import paper_1810_02821_amd as mf
    banner(f"shear samples {size} b {b_ratio}")
    prob = synth.config_shear(3, size, b_ratio)
    plan = mf.Plan([prob])
    g = plan.concat_complex([prob.gamma])
    chains, burn_in, n_samples, thin = 3, 3, 4, 2
    out, _ = plan.shear_sample(g, 29, chains, burn_in, n_samples, thin, b_ratio=b_ratio)
    got = out.view(chains, n_samples, size, size).cpu().numpy()
    worst = 0.0
    for c in range(chains):
        ref, _ = osh.sample_shear_chain(prob, 29, 0, c, burn_in, n_samples, thin, b_ratio)
        for s in range(n_samples):
            worst = max(worst, crel(got[c, s], ref[s]))
    print(f"worst {worst:.2e}")
    assert worst < REL_TOL


def test_shear_resume_and_errors(torch_cuda):
    torch = torch_cuda
    import paper_1810_02821_amd as mf
    banner("shear resume + errors")
    prob = synth.config_shear(4, 64, 0.2)
    plan = mf.Plan([prob])
    g = plan.concat_complex([prob.gamma])
    st_full = plan.shear_state_buffer(2)
    full, _ = plan.shear_sample(g, 5, 2, 0, 6, 1, b_ratio=0.2, state_out=st_full)
    # the first part emits on every sweep too: emission sweeps take kappa through
    # pixel space and back, so the state is bit-identical only along the same path
    st_a = plan.shear_state_buffer(2)
    plan.shear_sample(g, 5, 2, 0, 2, 1, b_ratio=0.2, state_out=st_a)
    st_b = plan.shear_state_buffer(2)
    rest, _ = plan.shear_sample(g, 5, 2, 0, 4, 1, sweep_offset=2, b_ratio=0.2, state_in=st_a, state_out=st_b)
    assert torch.equal(st_b, st_full)
    assert torch.equal(rest.view(2, 4, -1), full.view(2, 6, -1)[:, 2:])
    with pytest.raises(mf.MFError) as e:
        plan.shear_wiener(g, mf.Schedule([1.0], [0], 1e-3, 100, 10))
    assert e.value.status == 1


@pytest.mark.parametrize("H,W,b_ratio", [(256, 256, 0.0), (64, 128, 0.5), (2048, 16, 0.3), (16, 512, 0.0)])
def test_streamed_shear_wiener_matches_oracle(torch_cuda, H, W, b_ratio):
    """Size classes outside the persistent kernel run on the streamed kernels
    with mirror-paired column tiles (a persistent 32^2 problem rides along)."""
    import paper_1810_02821_amd as mf
    banner(f"streamed shear wiener {H}x{W} b {b_ratio}")
    probs = [synth.config_shear(5, H, b_ratio, width=W), synth.config_shear(6, 32, b_ratio)]
    plan = mf.Plan(probs)
    g = plan.concat_complex([p.gamma for p in probs])
    levels = ((50.0, 5), (5.0, 5), (1.0, 20))
    k = plan.shear_wiener(g, mf.Schedule([l for l, _ in levels], [n for _, n in levels]), b_ratio)
    for i, p in enumerate(probs):
        ref = osh.wiener_shear(p, om.Schedule(tuple(l for l, _ in levels), tuple(n for _, n in levels)), b_ratio)
        r = crel(plan.split_complex(k)[i], ref)
        print(f"problem {i}: rel {r:.2e}")
        assert r < REL_TOL


@pytest.mark.parametrize("H,W,b_ratio", [(256, 256, 0.3), (128, 64, 0.0), (2048, 16, 0.5), (16, 1024, 0.3),
                                         (1024, 16, 0.2), (512, 32, 0.4)])
def test_streamed_shear_samples_match_oracle(torch_cuda, H, W, b_ratio):
    import paper_1810_02821_amd as mf
    banner(f"streamed shear samples {H}x{W} b {b_ratio}")
    prob = synth.config_shear(7, H, b_ratio, width=W)
    plan = mf.Plan([prob])
    g = plan.concat_complex([prob.gamma])
    chains, burn_in, n_samples, thin = 2, 2, 3, 2
    st = plan.shear_state_buffer(chains)
    out, _ = plan.shear_sample(g, 41, chains, burn_in, n_samples, thin, b_ratio=b_ratio, state_out=st)
    got = out.view(chains, n_samples, H, W).cpu().numpy()
    sv = st.view(chains, H, W).cpu().numpy()
    worst = 0.0
    for c in range(chains):
        ref, s_ref = osh.sample_shear_chain(prob, 41, 0, c, burn_in, n_samples, thin, b_ratio)
        for s in range(n_samples):
            worst = max(worst, crel(got[c, s], ref[s]))
        worst = max(worst, crel(sv[c], s_ref))
    print(f"worst {worst:.2e}")
    assert worst < REL_TOL


def test_streamed_shear_resume(torch_cuda):
    """A streamed run split by sweep_offset (state carried) equals the
    uninterrupted run along the same emission pattern."""
    torch = torch_cuda
    import paper_1810_02821_amd as mf
    banner("streamed shear resume")
    prob = synth.config_shear(8, 256, 0.2)
    plan = mf.Plan([prob])
    g = plan.concat_complex([prob.gamma])
    st_full = plan.shear_state_buffer(2)
    full, _ = plan.shear_sample(g, 5, 2, 0, 5, 1, b_ratio=0.2, state_out=st_full)
    st = plan.shear_state_buffer(2)
    plan.shear_sample(g, 5, 2, 0, 2, 1, b_ratio=0.2, state_out=st)
    rest, _ = plan.shear_sample(g, 5, 2, 0, 3, 1, sweep_offset=2, b_ratio=0.2, state_in=st, state_out=st)
    assert torch.equal(st, st_full)
    assert torch.equal(rest.view(2, 3, -1), full.view(2, 5, -1)[:, 2:])


def test_streamed_shear_graph_replays_match_eager(torch_cuda):
    """MF_FLAG_GRAPH captures the streamed mass-mapping loops; replays with
    eager work in between equal the eager runs bit for bit."""
    torch = torch_cuda
    import paper_1810_02821_amd as mf
    banner("streamed shear graph replays")
    prob = synth.config_shear(12, 256, 0.4)
    eager = mf.Plan([prob])
    graph = mf.Plan([prob], graph=True)
    g = eager.concat_complex([prob.gamma])
    sch = mf.Schedule([10.0, 1.0], [3, 4])
    ref_k = eager.shear_wiener(g, sch, 0.4)
    ref_s, _ = eager.shear_sample(g, 9, 2, 1, 2, 1, b_ratio=0.4)
    for _ in range(3):
        k = graph.shear_wiener(g, sch, 0.4)
        smp, _ = graph.shear_sample(g, 9, 2, 1, 2, 1, b_ratio=0.4)
        torch.cuda.synchronize()
        assert torch.equal(k, ref_k) and torch.equal(smp, ref_s)
        eager.shear_sample(g, 10, 1, 1, 1, 1, b_ratio=0.4)
        torch.cuda.synchronize()
