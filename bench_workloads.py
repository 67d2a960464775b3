"""Secondary measured workloads of bench.py (each prints one JSON line).

large  : 2048x2048 map (P=(k+1)^-2.2, smooth noise, disk footprint with 5%
         holes), 64 chains x 200 sweeps on the streamed path, every 20th state
         emitted; reports chain-sweeps/s and HBM GB/s of the sweep kernels.
         Then the same map with the spectrum as 32 log bands: the unrolled
         gradient of a 200-sweep cooled Wiener iteration (10 levels x 20) with
         respect to d and the bands, a checkpoint every 20 sweeps, timed against
         the forward iteration alone.
uneven : 4096 problems of sizes {64,128,256,512}^2 at weights {.4,.3,.2,.1},
         per-problem spectra, noise and masks; one chain (pair) per problem,
         500 sweeps, final states written, column tiles picked by the
         autotuner and the streamed sweep loops replayed as HIP graphs;
         reports pixel-sweeps/s, and per size class when run alone.
grad   : 256x256 band-spectrum Wiener filter (32 bands) and its gradient
         (one adjoint solve); reports the gradient/forward time ratio.
spectrum: the hierarchical sampler (signal + 32 band amplitudes) on the
         128x128 band-spectrum recipe: 1024 chains, 100 iterations of one
         messenger sweep and one amplitude draw each; reports chain-iterations/s
         next to the fixed-spectrum sampler's chain-sweeps/s on the same image;
         then the streamed form on the 2048^2 large map with 32 log bands (64
         chains, 20 iterations of 5 sweeps) against the streamed fixed-spectrum
         sampler over the same 100 sweeps.
storage: the large-map sampling loop with the streamed field stored as FP32,
         FP16 and BF16 (chain-sweeps/s each); then a drift study: 2048 chains
         on a 64x64 image (6000 burn-in sweeps, 24 samples 8 apart) per
         storage, the shift of their per-pixel posterior mean and standard
         deviation from the FP32 run on the same stream, in posterior standard
         deviations.
shear  : the mass-mapping sampler (b_ratio 0.3): 1024 chains x 200 sweeps at
         128x128 (persistent) and 32 chains x 100 sweeps at 2048x2048
         (streamed, mirror-paired column tiles), every 10th / 20th convergence
         map emitted.
solve  : Wiener filters of 256 independent 128x128 images (the paper-size
         recipe, one seed each): 20 cooling levels x 10 sweeps, then sweeps at
         lambda = 1 to a residual of 1e-5 tested every 10 sweeps; the persistent
         solve kernel against the streamed kernels (host-side residual test).
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np


def _timed(fn, reps=1):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def large(args):
    import torch
    import paper_1810_02821_amd as mf
    from paper_1810_02821_amd import synth
    N, chains, sweeps, thin = 2048, 64, 200, 20
    print("[bench] large: generating 2048^2 problem", file=sys.stderr, flush=True)
    prob = synth.config_large(0, N)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    n_samples = sweeps // thin
    out = plan.samples_buffer(chains, n_samples)
    st = plan.state_buffer(chains)
    run = lambda: plan.sample(d, 1000, chains=chains, burn_in=0, n_samples=n_samples, thin=thin,
                              form="streamed", state_out=st, out=out)
    run()
    print("[bench] large: timing", file=sys.stderr, flush=True)
    t = _timed(run, max(1, args.steps // 2))
    pairs = chains // 2
    pair_sweeps = pairs * sweeps
    n = N * N
    # compulsory field traffic per pair-sweep: each of the two kernels reads and
    # writes the complex pair field (4 x 8 B/px); samples: 8 B/px per pair per emission
    field_bytes = pair_sweeps * 4 * 8 * n
    sample_bytes = pairs * n_samples * 8 * n
    table_bytes = 12 * n
    gbps = (field_bytes + sample_bytes + table_bytes) / t / 1e9
    del out, st, plan
    print("[bench] large: unrolled gradient, 32 bands", file=sys.stderr, flush=True)
    bprob = synth.config_large(0, N, n_bands=32)
    bplan = mf.Plan([bprob])
    bd = bplan.concat([bprob.d])
    sch = mf.Schedule(list(np.geomspace(100.0, 1.0, 10)), [20] * 10)
    g = bplan.concat([np.random.default_rng(8).standard_normal((N, N))])
    s_out = torch.empty_like(bd)
    fwd = lambda: bplan.wiener(bd, sch, out=s_out)
    bwd = lambda: bplan.wiener_backward_unrolled(bd, g, sch, 20)
    fwd()
    bwd()
    t_f = _timed(fwd, 2)
    t_b = _timed(bwd, 2)
    print(json.dumps({"workload": "large", "metric": "chain-sweeps/s at 2048^2 (streamed, 64 chains)",
                      "value": chains * sweeps / t, "unit": "chain-sweeps/s", "seconds": t,
                      "hbm_algorithmic_GBps": gbps, "hbm_frac": gbps / 8000.0,
                      "samples_per_s": chains * n_samples / t,
                      "unrolled_gradient": {"sweeps": 200, "checkpoint_every": 20, "bands": 32,
                                            "forward_s": t_f, "gradient_s": t_b,
                                            "ratio": t_b / t_f}}), flush=True)


def uneven(args):
    import paper_1810_02821_amd as mf
    from paper_1810_02821_amd import synth
    print("[bench] uneven: generating 4096 problems", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    probs = synth.config_uneven(0, n_problems=4096)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    plan = mf.Plan(probs, autotune=True, graph=True)
    t_plan = time.perf_counter() - t0
    d = plan.concat([p.d for p in probs])
    st = plan.state_buffer(1)
    sweeps = 500
    run = lambda: plan.sample(d, 1000, chains=1, burn_in=sweeps, n_samples=0, form="auto",
                              state_out=st, samples=False)
    run()
    print("[bench] uneven: timing", file=sys.stderr, flush=True)
    t = _timed(run, 1)
    sizes = np.array([p.H for p in probs])
    px = {int(s): int(np.sum(sizes == s)) * int(s) * int(s) for s in np.unique(sizes)}
    total_px = sum(px.values())
    # each size class alone (its own plan, same problems, same launch forms)
    per_class = {}
    for sz in np.unique(sizes):
        sub = [p for p in probs if p.H == sz]
        cplan = mf.Plan(sub, autotune=True, graph=True)
        cd = cplan.concat([p.d for p in sub])
        cst = cplan.state_buffer(1)
        crun = lambda: cplan.sample(cd, 1000, chains=1, burn_in=sweeps, n_samples=0, form="auto",
                                    state_out=cst, samples=False)
        crun()
        tc = _timed(crun, 1)
        per_class[f"{int(sz)}x{int(sz)}"] = {"problems": len(sub), "seconds": tc,
                                             "pixel_sweeps_per_s": px[int(sz)] * sweeps / tc,
                                             "form": "persistent" if sz <= 128 else "streamed"}
        del cplan, cd, cst
    # the same batch on the default shapes (autotuner off)
    print("[bench] uneven: default shapes", file=sys.stderr, flush=True)
    dplan = mf.Plan(probs, autotune=False, graph=True)
    dd = dplan.concat([p.d for p in probs])
    dst = dplan.state_buffer(1)
    drun = lambda: dplan.sample(dd, 1000, chains=1, burn_in=sweeps, n_samples=0, form="auto",
                                state_out=dst, samples=False)
    drun()
    td = _timed(drun, 1)
    default_shapes = {"seconds": td, "pixel_sweeps_per_s": total_px * sweeps / td,
                      "tile_shapes": {f"{s}x{s}": list(dplan.tile_shape(int(s), int(s)))
                                      for s in np.unique(sizes) if s >= 256},
                      "row_shapes": {f"{s}x{s}": dplan.row_shape(int(s), int(s))
                                     for s in np.unique(sizes) if s >= 256}}
    del dplan, dd, dst
    print(json.dumps({"workload": "uneven", "metric": "pixel-sweeps/s, 4096 uneven problems, 500 sweeps",
                      "value": total_px * sweeps / t, "unit": "pixel-sweeps/s (one chain per problem)",
                      "seconds": t, "problems_per_size": {int(s): int(np.sum(sizes == s)) for s in np.unique(sizes)},
                      "per_class": per_class,
                      "plan_seconds": t_plan, "generate_seconds": t_gen,
                      "graph": True, "autotune": True,
                      "tile_shapes": {f"{s}x{s}": list(plan.tile_shape(int(s), int(s)))
                                      for s in np.unique(sizes) if s >= 256},
                      "row_shapes": {f"{s}x{s}": plan.row_shape(int(s), int(s))
                                     for s in np.unique(sizes) if s >= 256},
                      "default_shapes": default_shapes, "autotune_speedup": td / t}), flush=True)


def grad(args):
    import torch
    import paper_1810_02821_amd as mf
    from paper_1810_02821_amd import synth
    from paper_1810_02821_amd.autograd import BandPosteriorLoss
    prob = synth.config_bands(0, 256, 32)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    sch = mf.Schedule(list(np.geomspace(1e3, 1.0, 30)) + [1.0], [10] * 30 + [3000])
    loss = BandPosteriorLoss(plan)
    theta = torch.tensor(np.asarray(prob.spectrum.amps), dtype=torch.float64, device="cuda")
    s_true = plan.concat([prob.s_true])
    fwd = lambda: plan.wiener(d, sch, allow_not_converged=True)
    fwd()
    t_f = _timed(fwd, 2)
    s, _ = plan.wiener(d, sch, allow_not_converged=True)
    g = (s - s_true).contiguous()
    bwd = lambda: plan.wiener_backward(s, g, sch, allow_not_converged=True)
    t_b = _timed(bwd, 2)
    t_all = _timed(lambda: loss.value_and_grad(d, theta, s_true, sch, sch), 1)
    print(json.dumps({"workload": "grad", "metric": "gradient time / forward Wiener time, 256^2, 32 bands",
                      "value": t_b / t_f, "unit": "ratio", "forward_s": t_f, "backward_s": t_b,
                      "loss_and_grad_s": t_all, "sweeps_per_solve": 3300}), flush=True)


def solve(args):
    import torch
    import paper_1810_02821_amd as mf
    from paper_1810_02821_amd import synth
    n_problems = 256
    print("[bench] solve: generating 256 problems", file=sys.stderr, flush=True)
    probs = [synth.config_128(i, 128) for i in range(n_problems)]
    sch = mf.Schedule(list(np.geomspace(1e3, 1.0, 20)) + [1.0], [10] * 20 + [0], tol=1e-5, max_sweeps=4000,
                      check_every=10)
    res = {}
    for form in ("persistent", "streamed"):
        plan = mf.Plan(probs, streamed_solve=form == "streamed")
        d = plan.concat([p.d for p in probs])
        out = torch.empty_like(d)
        run = lambda: plan.wiener(d, sch, out=out, allow_not_converged=True)
        _, info = run()
        print(f"[bench] solve: timing {form}", file=sys.stderr, flush=True)
        t = _timed(run, 2)
        sweeps = sum(i.sweeps for i in info)
        res[form] = {"seconds": t, "problem_sweeps": sweeps, "pixel_sweeps_per_s": sweeps * 128 * 128 / t,
                     "converged": sum(i.converged for i in info), "mean_sweeps": sweeps / n_problems}
        del plan
    print(json.dumps({"workload": "solve", "metric": "Wiener-filter pixel-sweeps/s, 256 x 128^2, to residual 1e-5",
                      "value": res["persistent"]["pixel_sweeps_per_s"], "unit": "pixel-sweeps/s",
                      "persistent": res["persistent"], "streamed": res["streamed"],
                      "speedup_vs_streamed": res["streamed"]["seconds"] / res["persistent"]["seconds"]}),
          flush=True)


def spectrum(args):
    import torch
    import paper_1810_02821_amd as mf
    from paper_1810_02821_amd import synth
    prob = synth.config_bands(0, 128, 32)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    chains, iters = 1024, 100
    st = plan.state_buffer(chains)
    run_h = lambda: plan.sample_spectrum(d, 1000, chains, 0, iters, 1, 1, state_out=st)
    run_s = lambda: plan.sample(d, 1000, chains=chains, burn_in=iters, n_samples=0, form="persistent",
                                state_out=st, samples=False)
    run_h()
    run_s()
    print("[bench] spectrum: timing", file=sys.stderr, flush=True)
    t_h = _timed(run_h, max(1, args.steps // 2))
    t_s = _timed(run_s, max(1, args.steps // 2))
    del st, plan
    # streamed form: the 2048^2 large map with its spectrum as 32 log bands
    print("[bench] spectrum: 2048^2 streamed", file=sys.stderr, flush=True)
    N, lchains, liters, lsweeps = 2048, 64, 20, 5
    lprob = synth.config_large(0, N, n_bands=32)
    lplan = mf.Plan([lprob])
    ld = lplan.concat([lprob.d])
    lst = lplan.state_buffer(lchains)
    run_lh = lambda: lplan.sample_spectrum(ld, 1000, lchains, 0, liters, 1, lsweeps, state_out=lst)
    run_ls = lambda: lplan.sample(ld, 1000, chains=lchains, burn_in=liters * lsweeps, n_samples=0,
                                  form="streamed", state_out=lst, samples=False)
    run_lh()
    run_ls()
    t_lh = _timed(run_lh, 2)
    t_ls = _timed(run_ls, 2)
    print(json.dumps({"workload": "spectrum",
                      "metric": "chain-iterations/s, hierarchical sampler at 128^2 (32 bands, 1024 chains)",
                      "value": chains * iters / t_h, "unit": "chain-iterations/s", "seconds": t_h,
                      "fixed_spectrum_chain_sweeps_per_s": chains * iters / t_s,
                      "cost_ratio_vs_fixed_spectrum": t_h / t_s,
                      "streamed_2048": {"chains": lchains, "iterations": liters, "sweeps_per_draw": lsweeps,
                                        "chain_sweeps_per_s": lchains * liters * lsweeps / t_lh,
                                        "fixed_spectrum_chain_sweeps_per_s": lchains * liters * lsweeps / t_ls,
                                        "cost_ratio_vs_fixed_spectrum": t_lh / t_ls}}), flush=True)


def storage(args):
    import torch
    import paper_1810_02821_amd as mf
    from paper_1810_02821_amd import synth
    # speed: the large-map sampling loop with the field stored in FP32, FP16, BF16
    N, chains, sweeps, thin = 2048, 64, 200, 20
    print("[bench] storage: generating 2048^2 problem", file=sys.stderr, flush=True)
    prob = synth.config_large(0, N)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    n_samples = sweeps // thin
    out = plan.samples_buffer(chains, n_samples)
    st = plan.state_buffer(chains)
    speed = {}
    for stg in ("fp32", "fp16", "bf16"):
        run = lambda: plan.sample(d, 1000, chains=chains, burn_in=0, n_samples=n_samples, thin=thin,
                                  form="streamed", state_out=st, out=out, storage=stg)
        run()
        print(f"[bench] storage: timing {stg}", file=sys.stderr, flush=True)
        t = _timed(run, max(1, args.steps // 2))
        speed[stg] = {"chain_sweeps_per_s": chains * sweeps / t, "seconds": t}
    del out, st, plan
    # drift: per-pixel posterior mean and standard deviation of many chains on a
    # 64^2 image, FP16 / BF16 storage against the FP32 run on the same stream,
    # in units of the posterior standard deviation (the exact-posterior checks
    # of the same samplers are GPU tests)
    print("[bench] storage: drift study 64^2", file=sys.stderr, flush=True)
    sp = synth.config_small(0, 64)
    splan = mf.Plan([sp])
    sd_d = splan.concat([sp.d])
    dchains, burn, ns, dthin = 2048, 6000, 24, 8
    moments = {}
    for stg in ("fp32", "fp16", "bf16"):
        flat, _ = splan.sample(sd_d, 4242, chains=dchains, burn_in=burn, n_samples=ns, thin=dthin,
                               form="streamed", storage=stg)
        m, v = splan.sample_moments(flat, dchains, ns)
        moments[stg] = (m.cpu().numpy(), v.cpu().numpy())
    m32, v32 = moments["fp32"]
    sd32 = np.sqrt(v32)
    drift = {}
    for stg in ("fp16", "bf16"):
        m, v = moments[stg]
        dm = np.abs(m - m32) / sd32
        drift[stg] = {"max_mean_shift_over_sd": float(dm.max()), "mean_mean_shift_over_sd": float(dm.mean()),
                      "max_sd_ratio_minus_1": float(np.max(np.abs(np.sqrt(v / v32) - 1)))}
    print(json.dumps({"workload": "storage",
                      "metric": "chain-sweeps/s at 2048^2 (streamed, 64 chains) by field storage",
                      "value": speed["fp16"]["chain_sweeps_per_s"], "unit": "chain-sweeps/s (fp16 storage)",
                      "speed": speed,
                      "speedup_fp16": speed["fp32"]["seconds"] / speed["fp16"]["seconds"],
                      "speedup_bf16": speed["fp32"]["seconds"] / speed["bf16"]["seconds"],
                      "drift_64": {"chains": dchains, "burn_in": burn, "samples": ns, "thin": dthin,
                                   "mc_standard_error_over_sd": float(1.0 / np.sqrt(dchains * ns)),
                                   "vs_fp32_same_stream": drift}}), flush=True)


def shear(args):
    import torch
    import paper_1810_02821_amd as mf
    from paper_1810_02821_amd import synth
    res = {}
    # one chain per complex field; 128^2 runs the persistent kernel, 2048^2 the streamed kernels
    for N, chains, sweeps, thin in ((128, 1024, 200, 10), (2048, 32, 100, 20)):
        print(f"[bench] shear: {N}^2", file=sys.stderr, flush=True)
        prob = synth.config_shear(0, N, 0.3)
        plan = mf.Plan([prob])
        g = plan.concat_complex([prob.gamma])
        st = plan.shear_state_buffer(chains)
        n_samples = sweeps // thin
        run = lambda: plan.shear_sample(g, 1000, chains, 0, n_samples, thin, b_ratio=0.3, state_out=st)
        run()
        t = _timed(run, max(1, args.steps // 2))
        res[str(N)] = {"chains": chains, "sweeps": sweeps, "samples_per_chain": n_samples,
                       "form": "persistent" if N <= 128 else "streamed",
                       "chain_sweeps_per_s": chains * sweeps / t, "seconds": t}
        del st, plan, g
        torch.cuda.empty_cache()
    print(json.dumps({"workload": "shear",
                      "metric": "chain-sweeps/s, mass-mapping sampler (complex convergence, b_ratio 0.3)",
                      "value": res["128"]["chain_sweeps_per_s"], "unit": "chain-sweeps/s (128^2, persistent)",
                      "by_size": res}), flush=True)


def run(args):
    {"large": large, "uneven": uneven, "grad": grad, "solve": solve, "spectrum": spectrum,
     "storage": storage, "shear": shear}[args.workload](args)
