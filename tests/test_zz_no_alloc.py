"""mf_sample_noalloc, the sampler entry point for callers that cannot
allocate: its workspaces live in a static device array.  Called through the
C ABI and checked against mf_sample (the same kernels, so bit for bit) on two
calls in a row, the second with a smaller input; device memory is unchanged."""
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


def _noalloc(plan, d, seed, chains, burn_in, n_samples, form, state_out, out, storage="fp32"):
    from paper_1810_02821_amd import _binding as B
    args = B._SampleArgs(int(seed), int(chains), int(burn_in), int(n_samples), 1, 0, 0.0, B.FORMS[form],
                         B.STORAGES[storage], 1, None)
    return B.lib().mf_sample_noalloc(plan._h, B._ptr(d), C.byref(args), None, B._ptr(state_out), B._ptr(out),
                                     B._stream())


def _case(torch, mf, prob, chains, form, storage="fp32"):
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    ref = plan.samples_buffer(chains, 3)
    ref_state = plan.state_buffer(chains)
    plan.sample(d, 41, chains=chains, burn_in=2, n_samples=3, form=form, storage=storage, out=ref,
                state_out=ref_state)
    out = torch.full_like(ref, float("nan"))
    state = torch.full_like(ref_state, float("nan"))
    return plan, d, ref, ref_state, out, state


def test_noalloc_equals_sample_on_two_calls(torch_cuda):
    torch = torch_cuda
    import paper_1810_02821_amd as mf
    banner("mf_sample_noalloc vs mf_sample")
    cases = [(synth.config_128(0, 128), 16, "persistent", "fp32"),   # first call: the paper's image size
             (synth.config_small(1, 32), 2, "persistent", "fp32"),   # second call: a smaller input
             (synth.config_128(2, 256), 2, "streamed", "fp16")]      # streamed, 16-bit field in the scratch
    prepared = [_case(torch, mf, *c) for c in cases]
    torch.cuda.synchronize()
    # the calls in a row, device free memory read around them only (the
    # comparisons below let torch's caching allocator take memory)
    free0, _ = torch.cuda.mem_get_info()
    status = []
    for (prob, chains, form, storage), (plan, d, ref, ref_state, out, state) in zip(cases, prepared):
        status.append(_noalloc(plan, d, 41, chains, 2, 3, form, state, out, storage))
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    print(f"status {status}; free before {free0}, after {free1}")
    assert status == [0, 0, 0] and free1 == free0
    for (prob, chains, form, storage), (plan, d, ref, ref_state, out, state) in zip(cases, prepared):
        assert torch.equal(out, ref) and torch.equal(state, ref_state), f"{prob.H}^2 {form}"
        got = plan.sample_view(out, 0, chains, 3).cpu().numpy()
        smp, _ = om.sample_pair(prob, 41, 0, 0, 2, 3)
        if storage == "fp32":
            assert max(rel(got[h, k], smp[h, k]) for h in range(2) for k in range(3)) < REL_TOL


def test_noalloc_refuses_what_does_not_fit(torch_cuda):
    torch = torch_cuda
    import paper_1810_02821_amd as mf
    banner("mf_sample_noalloc limits")
    probs = [synth.config_128(i, 128) for i in range(64)]  # 1 Mi pixels of persistent tables: 20 MiB
    plan = mf.Plan(probs)
    d = plan.concat([p.d for p in probs])
    state = plan.state_buffer(2)
    out = plan.samples_buffer(2, 1)
    st = _noalloc(plan, d, 1, 2, 1, 1, "persistent", state, out)
    assert st == 1 and b"static scratch holds" in mf._binding.lib().mf_last_error()
    small = mf.Plan([synth.config_small(0, 32)])
    st = _noalloc(small, small.concat([small.problems[0].d]), 1, 2, 1, 1, "persistent", None,
                  small.samples_buffer(2, 1))
    assert st == 1 and b"state_out" in mf._binding.lib().mf_last_error()
