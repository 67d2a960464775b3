"""Single-chain problems on the streamed kernels run two to a complex field
(problem A's chain in the real part, problem B's in the imaginary part, each
with its own tables and random stream): every chain against the oracle's
chain 0 of that problem, states, resumes, dispersed starts and the
non-finite check."""
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


def _batch():
    # odd counts per class: the last problem of a class has no partner
    probs = synth.config_uneven(21, n_problems=7, sizes=(64, 256), weights=(0.6, 0.4))
    return probs


@pytest.mark.parametrize("graph", [False, True])
def test_packed_chains_match_oracle(torch_cuda, graph):
    torch = torch_cuda
    mf = _mf()
    banner(f"packed single chains (graph={graph})")
    probs = _batch()
    sizes = sorted({p.H for p in probs})
    print("sizes", [p.H for p in probs], sizes)
    plan = mf.Plan(probs, graph=graph)
    d = plan.concat([p.d for p in probs])
    st = plan.state_buffer(1)
    flat, _ = plan.sample(d, 55, chains=1, burn_in=3, n_samples=4, form="streamed", state_out=st)
    worst = 0.0
    for i, p in enumerate(probs):
        got = plan.sample_view(flat, i, 1, 4).cpu().numpy()
        ref, s_ref = om.sample_pair(p, 55, i, 0, 3, 4)
        for k in range(4):
            worst = max(worst, rel(got[0, k], ref[0, k]))
        sv = plan.state_view(st, i, 1).cpu().numpy()[0]
        worst = max(worst, rel(sv.real, s_ref.real))
        assert np.all(sv.imag == 0)
    print(f"worst {worst:.2e}")
    assert worst < REL_TOL


@pytest.mark.parametrize("size,count", [(1024, 3), (2048, 2)])
def test_packed_long_columns_match_oracle(torch_cuda, size, count):
    """The packed column step at 1024 and 2048 rows (padded LDS layouts; at
    1024 an odd count leaves one problem alone in its field)."""
    mf = _mf()
    banner(f"packed single chains {size}^2 x {count}")
    probs = synth.config_uneven(22 + size // 1024, n_problems=count, sizes=(size,), weights=(1.0,))
    plan = mf.Plan(probs)
    d = plan.concat([p.d for p in probs])
    st = plan.state_buffer(1)
    flat, _ = plan.sample(d, 57, chains=1, burn_in=1, n_samples=1, form="streamed", state_out=st)
    worst = 0.0
    for i, p in enumerate(probs):
        got = plan.sample_view(flat, i, 1, 1).cpu().numpy()
        ref, s_ref = om.sample_pair(p, 57, i, 0, 1, 1)
        worst = max(worst, rel(got[0, 0], ref[0, 0]))
        sv = plan.state_view(st, i, 1).cpu().numpy()[0]
        worst = max(worst, rel(sv.real, s_ref.real))
        assert np.all(sv.imag == 0)
    print(f"worst {worst:.2e}")
    assert worst < REL_TOL


def test_packed_resume_and_dispersed_start(torch_cuda):
    """A packed run split at sweep 5 and resumed from its states equals the
    uninterrupted packed run bit for bit; dispersed starts match the oracle."""
    torch = torch_cuda
    mf = _mf()
    banner("packed resume and dispersed starts")
    probs = _batch()
    plan = mf.Plan(probs)
    d = plan.concat([p.d for p in probs])
    full, _ = plan.sample(d, 8, chains=1, burn_in=0, n_samples=9, form="streamed", init_scale=5.0)
    st = plan.state_buffer(1)
    plan.sample(d, 8, chains=1, burn_in=5, n_samples=0, form="streamed", init_scale=5.0, state_out=st, samples=False)
    rest, _ = plan.sample(d, 8, chains=1, burn_in=0, n_samples=4, sweep_offset=5, form="streamed", state_in=st.clone())
    for i, p in enumerate(probs):
        f = plan.sample_view(full, i, 1, 9)
        r = plan.sample_view(rest, i, 1, 4)
        assert torch.equal(f[:, 5:], r), f"problem {i}"
    i = len(probs) - 1
    p = probs[i]
    s0 = om.initial_state(8, i, 0, p.H, p.W, 5.0)
    ref, _ = om.sample_pair(p, 8, i, 0, 0, 2, s0=s0)
    got = plan.sample_view(full, i, 1, 9).cpu().numpy()
    assert max(rel(got[0, k], ref[0, k]) for k in range(2)) < REL_TOL


def test_packed_nonfinite_names_the_problem(torch_cuda):
    """NaN in the data of the imaginary-part problem of a packed field: the
    shared transforms carry it into the partner's chain too, so the check names
    the lower of the two indices; problems in other fields are unaffected."""
    torch = torch_cuda
    mf = _mf()
    banner("packed non-finite check")
    probs = _batch()
    plan = mf.Plan(probs)
    big = [i for i, p in enumerate(probs) if p.H == 256]  # packed as (big[0], big[1]), (big[2], big[3]), ...
    bad_i, partner = big[1], big[0]
    ds = [p.d.copy() for p in probs]
    y, x = np.argwhere(~probs[bad_i].mask)[11]
    ds[bad_i][y, x] = np.nan
    out = plan.samples_buffer(1, 1)
    with pytest.raises(mf.MFError) as e:
        plan.sample(plan.concat(ds), 3, chains=1, burn_in=1, n_samples=1, form="streamed", out=out)
    assert e.value.status == 6 and f"problem {min(bad_i, partner)}:" in str(e.value)
    for i in big[2:]:
        got = plan.sample_view(out, i, 1, 1).cpu().numpy()
        ref, _ = om.sample_pair(probs[i], 3, i, 0, 1, 1)
        assert rel(got[0, 0], ref[0, 0]) < REL_TOL
