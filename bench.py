"""Benchmark of the CIL hot path on one MI355X.

One step = one pass of the whole hot path over one batch of synthetic input:
  500 Gierer-Meinhardt (source form) solves on 64x64 grids from randomised
  initial states (+-1% multiplicative noise) to stationarity (FP64 residual
  < 1e-8; FP32 stepping with FP64 polish), then the CIL statistic of the two
  250-pattern halves: canonical distance range, 13 power-law radii fitted to
  it, per-pair radius bins (62 500 pairs, d = 8192), 200 bootstrap resamples
  (Alg. 2bst halves), FP64 mean/covariance/Cholesky and the Gaussian
  log-likelihood of the full-halves vector.
Initial states are resident on the device before the timed region.

Prints one JSON line.  `value` is stationary patterns/s of the whole step.
Also reported: CIL pairs/s, the plain FP64 GPU path (one kernel per stage,
host-driven loop, FP64 distances) timed the same way, the dominant kernel's
roofline (its durations taken with HIP events on its own stream inside the
timed region), and the FP64 CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "gm_source64_stationary"
VALU_FP32_PEAK_TFLOPS = 157.3   # MI355X published FP32 vector peak


def line_dct_flops(N: int, inverse: bool) -> int:
    """Real floating-point operations of one length-N line transform as
    implemented (Makhoul reduction + radix-2 FFT of length N/2)."""
    M = N // 2
    fft = 0
    m = 2
    while m <= M:
        h = m // 2
        per_block = 0
        for j in range(h):
            trivial = (j == 0) or (4 * j == m)
            per_block += 4 if trivial else 10
        fft += (M // m) * per_block
        m *= 2
    if not inverse:
        return fft + 18 * (M + 1) - 6
    return fft + 6 * (M + 1) + 12 * M


def fused_step_flops(n: int, reaction_flops: int) -> int:
    """Algorithmic flops of one IMEX step of one solve on the fused path."""
    per_species = n * (2 * line_dct_flops(n, False) + 2 * line_dct_flops(n, True)) + n * n
    return 2 * per_species + n * n * reaction_flops


REACTION_FLOPS = {0: 12, 1: 13, 2: 13, 3: 13, 4: 4}   # kinetics + the explicit update, per point


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--cpu-sample-solves", type=int, default=32)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(solves and pair tiles would shard by index with no communication but one all-reduce "
              "of integer counts); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import cil_synth as cs
    import paper_2203_14742_amd as cil

    w = cs.WORKLOADS[WORKLOAD]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    B, n = w["count"], w["n"]
    half = B // 2
    d = 2 * n * n
    M, n_boot = w["M"], w["n_boot"]
    base = cil.cil_homogeneous_state(w["model"], w["params"])
    ics_host = cs.initial_conditions(base, n, B, seed=w["seeds"][0], law=w["ic_law"])
    ics32 = torch.tensor(ics_host, dtype=torch.float32, device=dev)
    ics64 = torch.tensor(ics_host, dtype=torch.float64, device=dev)
    probs = cil.make_problems(n, w["L"], w["nu"], w["params"], count=B)
    ia, ib = cs.resample_halves(half, half, half, half, n_boot, seed=6)
    idxA = torch.from_numpy(ia).to(dev)
    idxB = torch.from_numpy(ib).to(dev)
    bins = torch.empty((half, half), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)

    def one_step(state, ics, path):
        state.copy_(ics)
        rep = cil.cil_simulate_patterns(w["model"], state, probs, w["dt"], w["max_steps"], tol=w["tol"],
                                        check_every=w["check_every"], path=path, polish=1)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        A = state[:half].reshape(half, d)
        Bs = state[half:].reshape(half, d)
        lo, hi = cil.cil_distance_range(A, Bs)
        radii = cil.cil_radii(lo, hi, M)
        _, counts = cil.cil_pair_bins(A, Bs, radii, bins=bins)
        _, Y = cil.cil_bootstrap_features(bins, idxA, idxB, M, want_counts=False)
        y_obs = torch.tensor(counts / float(half * half), dtype=torch.float64, device=dev)
        f, ll, me, st = cil.cil_gaussian_loglik(Y, y_obs)
        ev1.record(stream)
        return rep, counts, ev0, ev1, (f, ll, me, st)

    def timed(state, ics, path, steps, warmup, profile=False):
        for _ in range(warmup):
            one_step(state, ics, path)
        torch.cuda.synchronize()
        if profile:
            cil.cil_profile(True)
        t0 = time.perf_counter()
        cil_ms = 0.0
        reps = []
        for _ in range(steps):
            rep, counts, e0, e1, out = one_step(state, ics, path)
            reps.append(rep)
            torch.cuda.synchronize()
            cil_ms += e0.elapsed_time(e1)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = {}
        if profile:
            for name in cil.cil_profile_names():
                prof[name] = cil.cil_profile_read(name)
            cil.cil_profile(False)
        return el, cil_ms / 1e3, reps, counts, out, prof

    state32 = torch.empty_like(ics32)
    el, cil_s, reps, counts, out, prof = timed(state32, ics32, cil.CIL_PATH_AUTO, args.steps, args.warmup,
                                               profile=True)
    K = args.steps
    ms_per_step = 1e3 * el / K
    patterns_per_s = B * K / el
    pairs = half * half
    pairs_per_s = pairs * K / cil_s if cil_s > 0 else None
    rep = reps[-1]
    steps_total = int(rep["steps_taken"].sum())
    steps_fp64 = int(rep["steps_fp64"].sum())
    status_ok = bool(np.all(rep["status"] == 0))

    # dominant kernel: the fused FP32 stepper (most of the step's time)
    kname = "k_fused_f32_n64"
    cnt, tot_ms = prof.get(kname, (0, 0.0))
    roof = None
    if cnt:
        # solve-steps run by the FP32 stepper over the timed region
        solve_steps_fp32 = sum(int((r["steps_taken"] - r["steps_fp64"]).sum()) for r in reps)
        flops = solve_steps_fp32 * fused_step_flops(n, REACTION_FLOPS[w["model"]])
        avg_ms = tot_ms / cnt
        flops_per_launch = flops / cnt
        achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
        roof = {"kernel": kname, "bound": "alu", "achieved": round(achieved, 3),
                "peak": VALU_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / VALU_FP32_PEAK_TFLOPS, 4), "traffic": None,
                "launches": cnt, "avg_launch_ms": round(avg_ms, 4),
                "flops_per_solve_step": fused_step_flops(n, REACTION_FLOPS[w["model"]])}
    kernels = {k: {"launches": v[0], "total_ms": round(v[1], 3)} for k, v in sorted(prof.items())}

    plain = None
    if not args.no_plain:
        state64 = torch.empty_like(ics64)
        pel, pcil_s, preps, pcounts, _, _ = timed(state64, ics64, cil.CIL_PATH_PLAIN, 1, 0)
        plain = {"patterns_per_s": round(B / pel, 3), "pairs_per_s": round(pairs / pcil_s, 1),
                 "ms_per_step": round(1e3 * pel, 2),
                 "speedup_patterns": round(patterns_per_s / (B / pel), 2),
                 "speedup_pairs": round(pairs_per_s / (pairs / pcil_s), 2) if pairs_per_s else None,
                 "mean_steps": float(preps[-1]["steps_taken"].mean())}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, ics_host, base, args.cpu_sample_solves, half, d)

    line = {
        "metric": "stationary patterns/s + CIL distance pairs/s, batched FP32 vs plain FP64",
        "value": round(patterns_per_s, 3), "unit": "patterns/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD, "model": "gierer_meinhardt_source", "solves": B, "grid": n,
                   "dt": w["dt"], "tol": w["tol"], "radii": M, "bootstrap": n_boot,
                   "pairs_per_step": pairs, "parallelism": "none (1 GPU)"},
        "pairs_per_s": round(pairs_per_s, 1) if pairs_per_s else None,
        "solve_steps": steps_total, "solve_steps_fp64_polish": steps_fp64, "all_converged": status_ok,
        "roofline": roof, "kernels": kernels, "plain_fp64": plain, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def cpu_baseline(w, ics_host, base, n_solves, half, d):
    """The FP64 oracle on host cores, on a bounded sample of the same step:
    `n_solves` solves to stationarity, and the canonical distances of a block
    of pairs of the resulting patterns; scaled to patterns/s of the full step
    (solve time per pattern + pairs-per-pattern x time per pair)."""
    import numpy as np

    import oracle

    oracle.build()
    threads = os.cpu_count() or 1
    ics = ics_host[:n_solves].copy()
    t0 = time.perf_counter()
    out, steps, res, status = oracle.imex_run(w["model"], w["params"], w["nu"], w["n"], w["L"], w["dt"],
                                              w["max_steps"], w["tol"], w["check_every"], state=ics,
                                              nthreads=threads)
    t_sim = time.perf_counter() - t0
    k = n_solves // 2
    A = out[:k].reshape(k, -1)
    Bm = out[k:2 * k].reshape(k, -1)
    t1 = time.perf_counter()
    D = oracle.pair_d2(A, Bm, nthreads=threads)
    t_pairs = time.perf_counter() - t1
    sec_per_pattern = t_sim / n_solves + (half * half / (2 * half)) * (t_pairs / D.size)
    return {"value": round(1.0 / sec_per_pattern, 4), "unit": "patterns/s", "cores": threads, "kind": "oracle",
            "sample": "%d solves to residual < %g (%.1f s) + %d canonical pair distances (%.1f s), scaled to "
                      "the full step" % (n_solves, w["tol"], t_sim, D.size, t_pairs),
            "pairs_per_s": round(D.size / t_pairs, 1), "mean_steps": float(steps.mean())}


if __name__ == "__main__":
    main()
