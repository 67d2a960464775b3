"""GPU workloads beyond the paper-size sampler: differentiation through the
Wiener filter and the large-map streamed path, against the FP64 oracle."""
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


def _wf_schedules(mf, sweeps=4000):
    fwd = mf.Schedule(list(np.geomspace(1e3, 1.0, 30)) + [1.0], [10] * 30 + [sweeps])
    adj = mf.Schedule(list(np.geomspace(1e3, 1.0, 30)) + [1.0], [10] * 30 + [sweeps])
    return fwd, adj


def test_autograd_function_vjp_matches_oracle(torch_cuda):
    """torch.autograd through WienerFilter: grads of <w, s_W> w.r.t. d and the
    band amplitudes vs the oracle's implicit-differentiation VJP (CG solves)."""
    torch = torch_cuda
    import paper_1810_02821_amd as mf
    from paper_1810_02821_amd.autograd import wiener_filter
    banner("autograd VJP 64")
    prob = synth.config_bands(5, 64, 32)
    plan = mf.Plan([prob])
    fwd, adj = _wf_schedules(mf)
    d = plan.concat([prob.d]).requires_grad_(True)
    theta = torch.tensor(np.asarray(prob.spectrum.amps), dtype=torch.float64, device="cuda", requires_grad=True)
    w = np.random.default_rng(3).standard_normal((64, 64))
    s = wiener_filter(d, theta, plan, fwd, adj)
    L = torch.sum(s * plan.concat([w]))
    L.backward()
    s_ref, _ = om.wiener_cg(prob, tol=1e-12)
    gd_ref, gt_ref, _, _ = oa.wiener_vjp(prob, s_ref, w, solver="cg")
    rs = rel(plan.split(s.detach())[0], s_ref)
    rd = rel(plan.split(d.grad)[0], gd_ref)
    rt = float(np.max(np.abs(theta.grad.cpu().numpy() - gt_ref)) / np.max(np.abs(gt_ref)))
    print(f"s {rs:.2e} grad_d {rd:.2e} grad_theta {rt:.2e}")
    assert rs < REL_TOL and rd < REL_TOL and rt < REL_TOL


def _band_rel(got, ref):
    """Relative L2 distance over the band vector."""
    got, ref = np.asarray(got, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def test_band_loss_gradient_256_matches_oracle(torch_cuda):
    """The differentiation workload at 256^2 (32 bands, 30% mask): loss and
    gradient w.r.t. d and theta vs the oracle (CG-converged FP64 solves)."""
    torch = torch_cuda
    import paper_1810_02821_amd as mf
    from paper_1810_02821_amd.autograd import BandPosteriorLoss
    banner("band loss gradient 256")
    prob = synth.config_bands(0, 256, 32)
    plan = mf.Plan([prob])
    # 10000 sweeps at lambda = 1 after the cooling levels: the FP64 messenger
    # iteration is then within 1e-7 of the exact filter here, so what is left
    # is the FP32 floor of the GPU solve
    fwd, adj = _wf_schedules(mf, 10000)
    loss = BandPosteriorLoss(plan)
    d = plan.concat([prob.d])
    theta = torch.tensor(np.asarray(prob.spectrum.amps), dtype=torch.float64, device="cuda")
    L, gd, gt, s = loss.value_and_grad(d, theta, plan.concat([prob.s_true]), fwd, adj)
    s_ref, _ = om.wiener_cg(prob, tol=1e-12)
    L_ref = oa.loss_terms(prob, s_ref, prob.s_true)
    gd_ref, gt_ref = oa.loss_grad(prob, s_ref, prob.s_true, solver="cg")
    rs = rel(plan.split(s)[0], s_ref)
    rd = rel(gd.cpu().numpy().reshape(256, 256), gd_ref)
    rt = _band_rel(gt.cpu().numpy(), gt_ref)
    worst_band = float(np.max(np.abs(gt.cpu().numpy() - gt_ref) / np.max(np.abs(gt_ref))))
    print(f"L {L:.9e} ref {L_ref:.9e} rel {abs(L - L_ref) / abs(L_ref):.2e}; s {rs:.2e} grad_d {rd:.2e} "
          f"grad_theta {rt:.2e} (worst band / max band {worst_band:.2e})")
    assert abs(L - L_ref) < 1e-5 * abs(L_ref)
    assert rs < REL_TOL and rd < REL_TOL and rt < REL_TOL


def test_band_loss_with_response_matches_oracle(torch_cuda):
    """mf_band_loss with a diagonal response (and pixels of zero response):
    the likelihood term (d - A s)^T N^-1 (d - A s) uses the plan's own A and N,
    against the oracle's loss and gradient at the oracle's converged filter."""
    torch = torch_cuda
    import paper_1810_02821_amd as mf
    banner("band loss with response 64")
    prob = synth.config_bands(3, 64, 16)
    rng = np.random.default_rng(103)
    A = rng.uniform(0.5, 1.5, (64, 64))
    A.flat[rng.choice(64 * 64, 40, replace=False)] = 0.0
    prob.response = A
    prob.mask = prob.mask | (A == 0)
    nv = np.where(np.isfinite(prob.noise_var), prob.noise_var, 1.0)
    prob.d = np.where(prob.mask, 0.0, A * prob.s_true + rng.standard_normal((64, 64)) * np.sqrt(nv))
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    s_ref, _ = om.wiener_cg(prob, tol=1e-12)
    fwd, adj = _wf_schedules(mf, 6000)
    s, _ = plan.wiener(d, fwd, allow_not_converged=True)
    loss, gd, gt, _ = plan.band_loss(d, s, plan.concat([prob.s_true]), adj, allow_not_converged=True)
    L_ref = oa.loss_terms(prob, s_ref, prob.s_true)
    gd_ref, gt_ref = oa.loss_grad(prob, s_ref, prob.s_true, solver="cg")
    L = float(loss.sum())
    rd = rel(plan.split(gd)[0], gd_ref)
    rt = _band_rel(gt.cpu().numpy(), gt_ref)
    print(f"L {L:.9e} ref {L_ref:.9e}; s {rel(plan.split(s)[0], s_ref):.2e} grad_d {rd:.2e} grad_theta {rt:.2e}")
    assert abs(L - L_ref) < 1e-5 * abs(L_ref)
    assert rd < REL_TOL and rt < REL_TOL
    assert np.all(plan.split(gd)[0][A == 0] == 0)


def test_large_map_samples_2048(torch_cuda):
    """The large-map workload on the streamed path: one chain pair, two sweeps,
    every pixel against the oracle on the same stream."""
    import paper_1810_02821_amd as mf
    banner("large map 2048 samples")
    prob = synth.config_large(0, 2048)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    flat, _ = plan.sample(d, 1000, chains=2, burn_in=0, n_samples=2, form="streamed")
    got = plan.sample_view(flat, 0, 2, 2).cpu().numpy()
    ref, _ = om.sample_pair(prob, 1000, 0, 0, 0, 2)
    worst = max(rel(got[c, k], ref[c, k]) for c in range(2) for k in range(2))
    print(f"worst {worst:.2e}")
    assert worst < REL_TOL


def test_large_map_wiener_1024(torch_cuda):
    import paper_1810_02821_amd as mf
    banner("large map 1024 wiener")
    prob = synth.config_large(0, 1024)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    s, _ = plan.wiener(d, mf.Schedule([10.0, 1.0], [5, 10]))
    ref, _ = om.wiener(prob, om.Schedule((10.0, 1.0), (5, 10)))
    r = rel(plan.split(s)[0], ref)
    print(f"rel {r:.2e}")
    assert r < REL_TOL


def test_graph_replays_match_eager(torch_cuda):
    """The streamed sweep loop captured as a HIP graph: several replays, with
    eager work and synchronisation between them, each equal to the eager run."""
    torch = torch_cuda
    import paper_1810_02821_amd as mf
    banner("hipGraph replays 256")
    prob = synth.config_128(2, 256)
    eager = mf.Plan([prob])
    graph = mf.Plan([prob], graph=True)
    d = eager.concat([prob.d])
    ref, _ = eager.sample(d, 21, chains=4, burn_in=5, n_samples=3, form="streamed")
    out = graph.samples_buffer(4, 3)
    for rep in range(3):
        out.fill_(float("nan"))
        graph.sample(d, 21, chains=4, burn_in=5, n_samples=3, form="streamed", out=out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {rep}"
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
    ref2, _ = eager.sample(d, 22, chains=4, burn_in=5, n_samples=3, form="streamed")
    got2, _ = graph.sample(d, 22, chains=4, burn_in=5, n_samples=3, form="streamed")
    assert torch.equal(got2, ref2)
    _check = om.sample_pair(prob, 22, 0, 1, 5, 3)[0]
    assert rel(graph.sample_view(got2, 0, 4, 3).cpu().numpy()[2, 2], _check[0, 2]) < REL_TOL


def test_autotuned_shapes_give_identical_samples(torch_cuda):
    torch = torch_cuda
    import paper_1810_02821_amd as mf
    banner("autotune 256/512/1024/2048")
    probs = [synth.config_128(1, 256), synth.config_128(2, 512), synth.config_large(0, 1024),
             synth.config_large(1, 2048)]
    base = mf.Plan(probs)
    tuned = mf.Plan(probs, autotune=True)
    d = base.concat([p.d for p in probs])
    a, _ = base.sample(d, 5, chains=2, burn_in=1, n_samples=2, form="streamed")
    b, _ = tuned.sample(d, 5, chains=2, burn_in=1, n_samples=2, form="streamed")
    shapes = {p.H: (base.tile_shape(p.H, p.W), tuned.tile_shape(p.H, p.W)) for p in probs}
    rows = {p.H: (base.row_shape(p.H, p.W), tuned.row_shape(p.H, p.W)) for p in probs}
    print("default / tuned column tiles:", shapes, "fused row rows:", rows)
    defaults = {256: (8, 256), 512: (8, 256), 1024: (4, 256), 2048: (4, 256)}
    row_defaults = {256: 8, 512: 8, 1024: 2, 2048: 1}
    row_choices = {256: (8, 4, 16), 512: (8, 4, 2), 1024: (2, 1, 4), 2048: (1, 2)}
    # launches too small to fill the GPU: the shapes with the most workgroups
    narrow_defaults = {256: (4, 128, 4), 512: (4, 256, 2), 1024: (4, 256, 1), 2048: (4, 256, 1)}
    narrow = {p.H: (base.narrow_shape(p.H, p.W), tuned.narrow_shape(p.H, p.W)) for p in probs}
    print("default / tuned narrow shapes:", narrow)
    for H, (dflt, tuned_shape) in shapes.items():
        assert dflt == defaults[H]
        assert tuned_shape[0] in (4, 8, 16) and tuned_shape[1] in (128, 256, 512, 1024)
        assert rows[H][0] == row_defaults[H] and rows[H][1] in row_choices[H]
        assert narrow[H][0] == narrow_defaults[H]
        assert narrow[H][1][0] in (4, 8, 16) and narrow[H][1][2] in row_choices[H]
    assert torch.equal(a, b)


def test_every_fused_row_shape_gives_identical_samples(torch_cuda, tmp_path, monkeypatch):
    """Each rows-per-workgroup choice of the fused row kernel (forced through
    the tuning cache file) draws the default shape's samples bit for bit."""
    torch = torch_cuda
    import paper_1810_02821_amd as mf
    banner("fused row shapes 256/512/1024/2048")
    probs = [synth.config_128(1, 256), synth.config_128(2, 512), synth.config_large(0, 1024),
             synth.config_large(1, 2048)]
    base = mf.Plan(probs)
    d = base.concat([p.d for p in probs])
    ref, _ = base.sample(d, 5, chains=2, burn_in=2, n_samples=2, form="streamed")
    alts = {256: (4, 16), 512: (4,), 1024: (1, 4), 2048: (2,)}
    for k in range(2):
        cache = tmp_path / f"tune{k}.txt"
        lines = []
        for p in probs:
            c = alts[p.H]
            lines.append(f"gfx950 {p.H} {p.W} {base.tile_shape(p.H, p.W)[0]} {base.tile_shape(p.H, p.W)[1]}")
            lines.append(f"gfx950-rows {p.H} {p.W} {c[k % len(c)]}")
        cache.write_text("\n".join(lines) + "\n")
        monkeypatch.setenv("MF_TUNE_CACHE", str(cache))
        plan = mf.Plan(probs, autotune=True)
        got = {p.H: plan.row_shape(p.H, p.W) for p in probs}
        assert got == {p.H: alts[p.H][k % len(alts[p.H])] for p in probs}
        out, _ = plan.sample(d, 5, chains=2, burn_in=2, n_samples=2, form="streamed")
        assert torch.equal(out, ref), f"row shapes {got}"
        plan.close()


COL_TILES = {256: ((16, 256), (8, 256), (16, 512), (8, 512), (4, 128), (4, 256)),
             512: ((16, 512), (8, 512), (16, 256), (16, 1024), (8, 256), (4, 256)),
             1024: ((8, 512), (16, 1024), (8, 1024), (16, 512), (4, 256)),
             2048: ((4, 256), (8, 512), (8, 1024), (4, 512))}


def test_every_column_tile_gives_identical_samples(torch_cuda, tmp_path, monkeypatch):
    """Each column tile of the streamed kernels, forced through the tuning
    cache for both the wide and the narrow regime (one chain pair per problem
    runs narrow at 256^2 and 512^2), draws the default shape's samples bit
    for bit."""
    torch = torch_cuda
    import paper_1810_02821_amd as mf
    banner("column tiles 256/512/1024/2048")
    probs = [synth.config_128(1, 256), synth.config_128(2, 512), synth.config_large(0, 1024),
             synth.config_large(1, 2048)]
    base = mf.Plan(probs)
    d = base.concat([p.d for p in probs])
    ref, _ = base.sample(d, 9, chains=2, burn_in=2, n_samples=2, form="streamed")
    for k in range(6):
        cache = tmp_path / f"tiles{k}.txt"
        lines = []
        for p in probs:
            tc, nth = COL_TILES[p.H][k % len(COL_TILES[p.H])]
            lines.append(f"gfx950 {p.H} {p.W} {tc} {nth}")
            lines.append(f"gfx950-rows {p.H} {p.W} {base.row_shape(p.H, p.W)}")
            lines.append(f"gfx950-narrow {p.H} {p.W} {tc} {nth} {base.narrow_shape(p.H, p.W)[2]}")
        cache.write_text("\n".join(lines) + "\n")
        monkeypatch.setenv("MF_TUNE_CACHE", str(cache))
        plan = mf.Plan(probs, autotune=True)
        for p in probs:
            assert plan.tile_shape(p.H, p.W) == COL_TILES[p.H][k % len(COL_TILES[p.H])]
            assert plan.narrow_shape(p.H, p.W)[:2] == COL_TILES[p.H][k % len(COL_TILES[p.H])]
        out, _ = plan.sample(d, 9, chains=2, burn_in=2, n_samples=2, form="streamed")
        assert torch.equal(out, ref), f"tiles {k}"
        plan.close()


def test_narrow_solve_matches_wide_shapes(torch_cuda, tmp_path, monkeypatch):
    """A single 256^2 Wiener solve runs in the narrow shapes (its default grid
    would leave most CUs idle); forcing the wide shapes into the narrow regime
    gives the same filter bit for bit, and both match the oracle."""
    torch = torch_cuda
    import paper_1810_02821_amd as mf
    banner("narrow solve 256")
    prob = synth.config_bands(3, 256, 32)
    sch = mf.Schedule([100.0, 10.0, 1.0], [10, 10, 40])
    base = mf.Plan([prob])
    assert base.narrow_shape(256, 256) == (4, 128, 4)
    d = base.concat([prob.d])
    s_n, _ = base.wiener(d, sch, allow_not_converged=True)
    cache = tmp_path / "wide.txt"
    cache.write_text("gfx950 256 256 16 256\ngfx950-rows 256 256 8\ngfx950-narrow 256 256 16 256 8\n")
    monkeypatch.setenv("MF_TUNE_CACHE", str(cache))
    wide = mf.Plan([prob], autotune=True)
    s_w, _ = wide.wiener(d, sch, allow_not_converged=True)
    assert torch.equal(s_n, s_w)
    ref = om.wiener(prob, om.Schedule((100.0, 10.0, 1.0), (10, 10, 40)))[0]
    r = rel(base.split(s_n)[0], ref)
    print(f"narrow solve vs oracle {r:.2e}")
    assert r < REL_TOL


@pytest.mark.parametrize("size,ckpt", [(64, 7), (64, 500), (256, 20)])
def test_unrolled_gradient_matches_oracle(torch_cuda, size, ckpt):
    """Reverse-mode through a truncated cooling schedule with checkpoints every
    `ckpt` sweeps (7 does not divide the sweep count; 500 is one segment)."""
    import paper_1810_02821_amd as mf
    banner(f"unrolled gradient {size} ckpt {ckpt}")
    prob = synth.config_bands(7, size, 32)
    plan = mf.Plan([prob])
    lams, sweeps = (50.0, 5.0, 1.0), (30, 30, 60) if size <= 64 else (20, 20, 60)
    g = np.random.default_rng(8).standard_normal((size, size))
    sK, gd, gb = plan.wiener_backward_unrolled(plan.concat([prob.d]), plan.concat([g]),
                                               mf.Schedule(list(lams), list(sweeps)), checkpoint_every=ckpt)
    s_ref, gd_ref, gt_ref = oa.unrolled_vjp(prob, om.Schedule(lams, sweeps), g)
    rs = rel(plan.split(sK)[0], s_ref)
    rd = rel(plan.split(gd)[0], gd_ref)
    rt = float(np.max(np.abs(gb.cpu().numpy() - gt_ref)) / np.max(np.abs(gt_ref)))
    print(f"s {rs:.2e} grad_d {rd:.2e} grad_theta {rt:.2e}")
    assert rs < REL_TOL and rd < 1e-4 and rt < 1e-4
