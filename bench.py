"""Throughput of the messenger-field Wiener-posterior sampler on one MI355X.

Workload (the paper's benchmark image size): a 128x128 image, power spectrum
P(k) = (k+2)^-2.5, noise sigma ~ U[0.3, 3], 25% of pixels missing in 4x4
tiles; 1024 chains (512 complex pairs), 200 burn-in sweeps then 98 samples per
chain = 100,352 posterior samples per step.  Synthetic data (seed 0).

One step = one mf_sample call over every chain, inputs already in HBM, output
samples written to HBM.  Prints ONE JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-plain]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N = 128
CHAINS = 1024
BURN_IN = 200
N_SAMPLES = 98
DATA_SEED = 0

# MI355X peaks
PEAK_HBM_GBPS = 8000.0
# Published FP32 vector peak: 256 CUs x 2.4 GHz x 256 FLOP/clk/CU, which needs
# packed FP32 (two FP32 values per lane per instruction).  Every HIP source
# here is built without packed FP32 instructions, so the ceiling of this
# build is the single-issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP (FMA)
# x 2.4 GHz = 78.6 TFLOP/s, i.e. 39.3e12 VALU lane-instructions/s (one wave64
# instruction per SIMD every 4 clocks).
PEAK_FP32_TFLOPS_PUBLISHED = 157.3
PEAK_FP32_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
PEAK_VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9

# HBM traffic of resident_sample_kernel<128> on this workload, from rocprofv3
# FETCH_SIZE / WRITE_SIZE runs scaled by the same counters on a 1 GiB copy, and
# the hash of the kernel sources it was measured on (traffic is reported only
# while the sources are unchanged).
TRAFFIC_BYTES = int((180924.27 * 2.0 + 6493822.31 * 1.0) * 1024)  # FETCH x2.0 + WRITE x1.0 (copy-calibrated)
TRAFFIC_SOURCES_SHA = "44634bfa8470990b"
# VALU wave-instructions per launch of the same kernel (rocprofv3 SQ_INSTS_VALU,
# summed over the shader engines), and the source hash they were taken on.
VALU_WAVE_INSTS = 6124336128
VALU_SOURCES_SHA = "44634bfa8470990b"


def kernel_sources_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("mf_resident.hip", "mf_resident_fft.hpp", "mf_device.hpp", "mf_resident.hpp"):
        with open(os.path.join(ROOT, "paper_1810_02821_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_flops_per_pixel_pair_sweep(n_pixels: int) -> float:
    """Floating-point operations one chain pair needs per pixel per sweep:
    two complex 2D FFTs (forward and inverse) at the conventional 5 log2(n)
    per point each (140 at 128^2), plus the two diagonal updates at about 10
    FLOP per pixel each (the pixel step and the Fourier step with their
    scalings): 160 at 128^2.  The normal variates (two per pixel per chain:
    Philox integer rounds and Box-Muller transcendentals) are not floating-point
    arithmetic and are not counted here; flop_equivalents_per_pixel_pair_sweep
    counts them too."""
    return 2 * 5 * math.log2(n_pixels) + 2 * 10


def flop_equivalents_per_pixel_pair_sweep(n_pixels: int) -> float:
    """The same with every integer or transcendental instruction of the
    variates counted as one operation (FMA = 2): the FFTs (140 at 128^2), the
    updates as issued (pixel step 2 FMA per chain: 8; Fourier step FMA + mul
    per component: 6), and per pixel and per mode half a Philox4x32-10 call
    (10 rounds x [two 32x32->64 products + two 3-input XORs] = 40 ops per call)
    plus one Box-Muller pair (14 ops): 2 x (20 + 14) = 68; 222 at 128^2."""
    return 2 * 5 * math.log2(n_pixels) + 8 + 6 + 2 * (40 / 2 + 14)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--workload", default="paper", choices=["paper", "large", "uneven", "grad", "solve", "spectrum", "storage", "shear"],
                    help="paper (default, the headline line) or one of the other measured workloads")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (to scale HBM counters)")
    return ap.parse_args()


def calibrate_copy():
    """A plain copy of known size: 1 GiB read + 1 GiB written per launch."""
    import torch
    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))


# ----------------------------------------------------------------- oracle leg
def _oracle_worker(args):
    os.environ["OMP_NUM_THREADS"] = "1"
    pair, n_sweeps = args
    from oracle import messenger as om
    from paper_1810_02821_amd import synth
    prob = synth.config_128(DATA_SEED, N)
    t0 = time.perf_counter()
    om.sample_pair(prob, synth.philox_seed(DATA_SEED), 0, pair, burn_in=0, n_samples=n_sweeps)
    return time.perf_counter() - t0


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(budget_s: float):
    """The FP64 oracle sampler on the host cores, one chain pair per process.
    The pool takes the CPU share one GPU has on a shared host (16 cores, as
    OMP_NUM_THREADS states there), or every core of a smaller host."""
    import multiprocessing as mp
    cores = min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "16") or 16), 16)
    cores = max(cores, 1)
    # calibrate one sweep on one core, then spread ~budget_s CPU-seconds over the cores
    t_one = _oracle_worker((0, 3)) / 3.0
    sweeps = max(2, min(2000, int(budget_s / cores / max(t_one, 1e-4))))
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_worker, [(p, sweeps) for p in range(cores)])
    wall = time.perf_counter() - t0
    samples = cores * 2 * sweeps  # two chains per pair, one sample per sweep
    return {"value": samples / wall, "unit": "posterior samples/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{cores} chain pairs x {sweeps} sweeps of the 128x128 workload "
                      f"(FP64 numpy, one process per pair and core, samples counted without burn-in; "
                      f"{wall:.1f} s wall)"}


# ----------------------------------------------------------------- GPU leg
def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.workload != "paper":
        import bench_workloads
        bench_workloads.run(args)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU: the sampler's chains are independent and this build "
              f"runs on a single MI355X (asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1810_02821_amd as mf
    from paper_1810_02821_amd import synth

    torch.cuda.set_device(0)
    prob = synth.config_128(DATA_SEED, N)
    seed = synth.philox_seed(DATA_SEED)
    plan = mf.Plan([prob])
    d = plan.concat([prob.d])
    out = plan.samples_buffer(CHAINS, N_SAMPLES)
    state = plan.state_buffer(CHAINS)
    n_pix = N * N
    pairs = CHAINS // 2
    sweeps = BURN_IN + N_SAMPLES
    samples_per_step = CHAINS * N_SAMPLES

    def step(form="persistent", chains=CHAINS, o=out, s=state):
        plan.sample(d, seed, chains=chains, burn_in=BURN_IN, n_samples=N_SAMPLES, form=form,
                    state_out=s, out=o)

    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        step()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_call_ms = [a.elapsed_time(b) for a, b in ev]
    ms_per_step = wall * 1000.0 / args.steps
    value = samples_per_step / (ms_per_step / 1000.0)
    kern_ms = float(np.mean(per_call_ms))

    flops = algorithmic_flops_per_pixel_pair_sweep(n_pix) * n_pix * pairs * sweeps
    achieved_tflops = flops / (kern_ms / 1000.0) / 1e12
    # compulsory HBM bytes: samples out, final pair states out, problem tables in
    hbm_bytes = samples_per_step * n_pix * 4 + pairs * n_pix * 8 + 20 * n_pix
    hbm_gbps = hbm_bytes / (kern_ms / 1000.0) / 1e9
    traffic = TRAFFIC_BYTES if TRAFFIC_SOURCES_SHA == kernel_sources_sha() else None

    extra = {"chain_sweeps_per_s": CHAINS * sweeps / (ms_per_step / 1000.0)}
    # per-pixel mean and variance of the step's samples (the maps of Fig. 3)
    plan.sample_moments(out, CHAINS, N_SAMPLES)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    plan.sample_moments(out, CHAINS, N_SAMPLES)
    e1.record(stream)
    torch.cuda.synchronize()
    mom_ms = e0.elapsed_time(e1)
    extra["sample_moments"] = {"ms": mom_ms, "GBps": samples_per_step * n_pix * 4 / (mom_ms / 1000.0) / 1e9}
    if not args.no_plain:
        # plain form: one chain pair per launch sequence, field in HBM between kernels
        sub_chains = 8
        o2 = plan.samples_buffer(sub_chains, N_SAMPLES)
        s2 = plan.state_buffer(sub_chains)
        print("[bench] plain form (8 chains)", file=sys.stderr, flush=True)
        step("plain", sub_chains, o2, s2)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        step("plain", sub_chains, o2, s2)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t1
        plain = sub_chains * N_SAMPLES / tp
        print("[bench] streamed form (all chains)", file=sys.stderr, flush=True)
        step("streamed")
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        step("streamed")
        torch.cuda.synchronize()
        ts = time.perf_counter() - t2
        extra["plain_form"] = {"value": plain, "unit": "posterior samples/s",
                               "sample": f"{sub_chains} chains x ({BURN_IN}+{N_SAMPLES}) sweeps, one pair per launch sequence"}
        extra["streamed_form"] = {"value": samples_per_step / ts, "unit": "posterior samples/s"}
        extra["speedup_vs_plain"] = value / plain

    result = {
        "metric": "posterior samples/sec at 128^2 (batched chains) vs plain form; % HBM roofline",
        "value": value,
        "unit": "posterior samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "128x128 Gaussian-random-field image, P=(k+2)^-2.5, sigma~U[0.3,3], "
                               "25% masked 4x4 tiles; 1024 chains, 200 burn-in + 98 samples each",
                   "chains": CHAINS, "burn_in": BURN_IN, "samples_per_chain": N_SAMPLES,
                   "samples_per_step": samples_per_step, "form": "persistent"},
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tflops / PEAK_FP32_TFLOPS, "traffic": traffic,
                     "peak_note": "single-issue FP32 FMA rate (no packed FP32 in this build); "
                                  "published packed peak 157.3",
                     "frac_of_published_peak": achieved_tflops / PEAK_FP32_TFLOPS_PUBLISHED,
                     "valu_instructions_per_launch": VALU_WAVE_INSTS * 64 if VALU_SOURCES_SHA == kernel_sources_sha()
                                                     else None,
                     "valu_issue_frac": (VALU_WAVE_INSTS * 64 / (kern_ms / 1000.0) / PEAK_VALU_LANE_OPS
                                         if VALU_SOURCES_SHA == kernel_sources_sha() else None),
                     "kernel": "resident_sample_kernel<128>", "kernel_ms": kern_ms,
                     "kernel_ms_sd": float(np.std(per_call_ms, ddof=1)) if len(per_call_ms) > 1 else 0.0,
                     "flops_per_pixel_pair_sweep": algorithmic_flops_per_pixel_pair_sweep(n_pix),
                     "flop_equivalents_per_pixel_pair_sweep": flop_equivalents_per_pixel_pair_sweep(n_pix),
                     "flop_equivalent_TFLOPs": flop_equivalents_per_pixel_pair_sweep(n_pix) * n_pix * pairs * sweeps
                                               / (kern_ms / 1000.0) / 1e12,
                     "hbm_algorithmic_bytes": hbm_bytes,
                     "hbm_achieved_GBps": hbm_gbps, "hbm_frac": hbm_gbps / PEAK_HBM_GBPS},
    }
    result.update(extra)
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
