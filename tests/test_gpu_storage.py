"""Streamed sampler with its field stored as FP16 or BF16 between the row and
column kernels, against the storage oracle (oracle/storage.py) on the same
seeded inputs and stream.

Both sides round at the same two points per sweep; the oracle computes in FP64
and the GPU in FP32.  Where the FP32 value and the FP64 value of a stored
element fall on opposite sides of a rounding boundary the stored values differ
by one unit (2u relative); that happens to a fraction of about eps/u of the
elements (eps ~ 1e-6, the FP32 error of a transformed value at these sizes).
The tolerance is therefore the FP32 one plus sqrt(K) * 2 * sqrt(2 eps/u) * 2u
after K sweeps.  The same runs sit several times farther from the unrounded
chain (the rounding itself is seen)."""
import math

import numpy as np
import pytest

from gpu_common import REL_TOL, banner, rel
from oracle import messenger as om
from oracle import storage as ost
from paper_1810_02821_amd import synth

pytestmark = pytest.mark.gpu

UNIT = {"fp16": 2.0 ** -11, "bf16": 2.0 ** -8}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1810_02821_amd as mf
    mf.lib()
    return torch


def _tol(storage, k):
    u = UNIT[storage]
    return REL_TOL + math.sqrt(k) * 2 * math.sqrt(2 * 1e-6 / u) * 2 * u


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
@pytest.mark.parametrize("H,W,form", [(64, 64, "streamed"), (256, 256, "streamed"), (32, 512, "plain"),
                                      (2048, 16, "streamed")])
def test_stored_field_matches_storage_oracle(torch_cuda, storage, H, W, form):
    import paper_1810_02821_amd as mf
    banner(f"{storage} storage {H}x{W} {form}")
    prob = synth.config_small(3, H) if H == W else synth.config_bands(3, H, 8, width=W)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    seed, chains, burn_in, n_samples, thin = 31, 3, 1, 3, 1
    st = plan.state_buffer(chains)
    flat, _ = plan.sample(d, seed, chains=chains, burn_in=burn_in, n_samples=n_samples, thin=thin, form=form,
                          storage=storage, state_out=st)
    x = plan.sample_view(flat, 0, chains, n_samples).cpu().numpy()
    worst = worst_exact = 0.0
    for q in range((chains + 1) // 2):
        ref, s_ref = ost.sample_pair_stored(prob, seed, 0, q, burn_in, n_samples, thin, storage)
        exact, _ = om.sample_pair(prob, seed, 0, q, burn_in, n_samples, thin)
        for h in range(2):
            c = 2 * q + h
            if c >= chains:
                continue
            for k in range(n_samples):
                e = rel(x[c, k], ref[h, k])
                assert e < _tol(storage, burn_in + k + 1), (c, k, e)
                worst = max(worst, e)
                worst_exact = max(worst_exact, rel(x[c, k], exact[h, k]))
        # returned state: the stored (rounded) field of the last sweep, widened
        pair = st.view(-1, 2)[q * H * W:(q + 1) * H * W].cpu().numpy()
        got_state = pair[:, 0] + 1j * pair[:, 1]
        assert rel(got_state, s_ref.ravel()) < _tol(storage, burn_in + n_samples)
    print(f"worst vs storage oracle {worst:.2e} (tol {_tol(storage, burn_in + n_samples):.2e}), "
          f"vs unrounded chain {worst_exact:.2e}")
    assert worst_exact > 2 * worst


def test_fp32_storage_is_the_default(torch_cuda):
    torch = torch_cuda
    import paper_1810_02821_amd as mf
    banner("fp32 storage = default")
    prob = synth.config_small(1, 64)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    a, _ = plan.sample(d, 5, chains=4, burn_in=3, n_samples=2, form="streamed")
    b, _ = plan.sample(d, 5, chains=4, burn_in=3, n_samples=2, form="streamed", storage="fp32")
    assert torch.equal(a, b)


def test_persistent_form_ignores_storage(torch_cuda):
    torch = torch_cuda
    import paper_1810_02821_amd as mf
    banner("persistent form ignores storage")
    prob = synth.config_small(2, 32)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    a, _ = plan.sample(d, 6, chains=2, burn_in=3, n_samples=2, form="persistent")
    b, _ = plan.sample(d, 6, chains=2, burn_in=3, n_samples=2, form="persistent", storage="bf16")
    assert torch.equal(a, b)


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_stored_field_resume_matches_oracle(torch_cuda, storage):
    """A call resumed from the returned state (sweep_offset, state_in) follows
    the oracle started from that state: the state a call returns is the stored
    field, so a split run rounds once more than an uninterrupted one."""
    import paper_1810_02821_amd as mf
    banner(f"{storage} storage resume")
    prob = synth.config_small(4, 256)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    st = plan.state_buffer(2)
    plan.sample(d, 8, chains=2, burn_in=2, n_samples=0, form="streamed", storage=storage, state_out=st,
                samples=False)
    s0 = st.view(-1, 2).cpu().numpy()
    s0 = (s0[:, 0] + 1j * s0[:, 1]).reshape(256, 256)
    flat, _ = plan.sample(d, 8, chains=2, burn_in=0, n_samples=2, sweep_offset=2, form="streamed",
                          storage=storage, state_in=st, state_out=st)
    x = plan.sample_view(flat, 0, 2, 2).cpu().numpy()
    ref, _ = ost.sample_pair_stored(prob, 8, 0, 0, 0, 2, 1, storage, s0=s0, sweep_offset=2)
    for h in range(2):
        for k in range(2):
            assert rel(x[h, k], ref[h, k]) < _tol(storage, 2 + k + 1)


def test_unknown_storage_is_rejected(torch_cuda):
    import ctypes as C
    import paper_1810_02821_amd as mf
    from paper_1810_02821_amd import _binding
    banner("storage validation")
    prob = synth.config_small(0, 32)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    args = _binding._SampleArgs(1, 2, 1, 0, 1, 0, 0.0, 2, 7)  # valid but for storage = 7
    st = _binding.lib().mf_sample(plan._h, _binding._ptr(d), C.byref(args), None, None, None, _binding._stream())
    assert st == 1


def test_graph_replays_match_eager_with_16_bit_storage(torch_cuda):
    """The captured sweep loop (MF_FLAG_GRAPH) with FP16 storage, replayed
    several times with eager work in between, equals the eager run bit for bit."""
    torch = torch_cuda
    import paper_1810_02821_amd as mf
    banner("graph replays with fp16 storage")
    prob = synth.config_small(9, 256)
    eager = mf.Plan([prob])
    graph = mf.Plan([prob], graph=True)
    d = eager.concat([prob.d])
    ref, _ = eager.sample(d, 3, chains=4, burn_in=3, n_samples=2, form="streamed", storage="fp16")
    for _ in range(3):
        got, _ = graph.sample(d, 3, chains=4, burn_in=3, n_samples=2, form="streamed", storage="fp16")
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        eager.sample(d, 4, chains=2, burn_in=1, n_samples=1, form="streamed")
        torch.cuda.synchronize()
