"""Benchmark of the CIL hot path on one MI355X.

One step = one pass of the whole hot path over one batch of synthetic input:
  500 Gierer-Meinhardt (source form) solves on 64x64 grids from randomised
  initial states (+-1% multiplicative noise) to stationarity (FP64 residual
  < 1e-8), stepped by the persistent fused kernel in FP32, each solve going
  on in FP64 from its FP32 floor to the tolerance within the same launch,
  then the CIL statistic of the two 250-pattern halves (FP32): canonical distance
  range, 13 power-law radii fitted to it and per-pair radius bins from one
  fast pass over the pairs (62 500 pairs,
  d = 8192, split-bf16x3 Gram + canonical re-check), 200 bootstrap resamples
  (Alg. 2bst halves), FP64 mean/covariance/Cholesky and the Gaussian
  log-likelihood of the full-halves vector.
Initial states are resident on the device before the timed region.

Prints one JSON line.  `value` is stationary patterns/s of the whole step.
Also reported: CIL pairs/s, the same step with FP64 fused stepping throughout,
the plain FP64 GPU path (one kernel per stage, host-driven loop, FP64
distances) timed the same way, the dominant kernel's roofline (durations
from HIP events the library records on the kernel's own stream inside the
timed region), the Gram's MFMA rate, and the FP64 CPU oracle timed on a
bounded sample.
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
VALU_FP64_PEAK_TFLOPS = 78.6    # MI355X published FP64 vector peak
MFMA_BF16_PEAK_TFLOPS = 2500.0  # MI355X dense bf16 matrix peak


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


def copy_calibration(args, dev):
    """One plain device copy of --copy-calibration-mib MiB before the timed
    work: the HBM counters' reading for a copy of known size, against which
    a kernel's FETCH_SIZE and WRITE_SIZE are scaled."""
    import torch
    if args.copy_calibration_mib > 0:
        src = torch.ones((args.copy_calibration_mib << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst


def fused_step_flops(n: int, reaction_flops: int) -> int:
    """Algorithmic flops of one IMEX step of one solve on the fused path."""
    per_species = n * (2 * line_dct_flops(n, False) + 2 * line_dct_flops(n, True)) + n * n
    return 2 * per_species + n * n * reaction_flops


REACTION_FLOPS = {0: 12, 1: 13, 2: 13, 3: 13, 4: 4}   # kinetics + the explicit update, per point


# Sources that define the fused stepper kernels (device code, launch shape).
STEPPER_SOURCES = ["stepper.hip", "stepper_common.hpp", "stepper_quad.hpp", "stepper_quad_f32.hip",
                   "stepper_quad_f64.hip", "stepper_quad_mixed.hip", "dct_quad.hpp", "cil_internal.hpp"]
TRAFFIC_PROFILES = os.path.join(ROOT, "profiles", "*_hbm_bytes.md")


def stepper_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in STEPPER_SOURCES:
        with open(os.path.join(ROOT, "paper_2203_14742_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kname: str):
    """HBM bytes per launch of `kname` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the copy-kernel calibration),
    or None when there is none or the stepper sources changed since."""
    import glob
    lines = []
    for path in sorted(glob.glob(TRAFFIC_PROFILES)):
        try:
            with open(path) as fh:
                lines += [ln.split() for ln in fh if ln.startswith("traffic ")]
        except OSError:
            pass
    for ln in lines:
        kv = dict(x.split("=", 1) for x in ln[2:])
        if ln[1] == kname and kv.get("sources") == stepper_sources_sha256():
            return int(round(1024.0 * (float(kv["fetch_kib"]) * float(kv["fetch_scale"]) +
                                       float(kv["write_kib"]) * float(kv["write_scale"]))))
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default=WORKLOAD,
                    choices=[WORKLOAD, "fhn32_fixed5000", "features4096", "mcil_stripes64", "bz_uneven2048",
                             "fhn128_mcmc", "fhn128_de", "fhn32_sbdf2", "gm_source64_lone"],
                    help="the default is the benchmarked configuration; features4096 times the CIL "
                         "statistic alone on 4096 x 32768 FP32 patterns")
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-fp64-fused", "--no-fp32-stepping", dest="no_secondary", action="store_true",
                    help="skip the secondary leg (the same step with FP64 fused stepping throughout)")
    ap.add_argument("--plain-steps", type=int, default=3,
                    help="timed steps of the plain FP64 comparison leg (after one warm-up step)")
    ap.add_argument("--cpu-sample-solves", type=int, default=500,
                    help="solves the CPU oracle runs to stationarity for the cpu_baseline leg (the whole batch "
                         "at the default: about 12 s on 16 threads)")
    ap.add_argument("--cpu-single-solves", type=int, default=12,
                    help="solves the CPU oracle runs on one thread for the single-thread figure")
    ap.add_argument("--gram-flush", type=int, default=64, choices=[32, 64, 128, 256],
                    help="features4096: FP32 -> FP64 promotion interval of the Gram")
    ap.add_argument("--gram-pipeline", type=int, default=2, choices=[0, 1, 2],
                    help="features4096: Gram staging variant (CIL_OPT_GRAM_PIPELINE)")
    ap.add_argument("--scaled", action="store_true", help="mcil_stripes64: min-max scale the patterns first")
    ap.add_argument("--tune-steps", type=int, default=100,
                    help="bz_uneven2048: steps per autotuning trial (0 = the plan's own stepping)")
    ap.add_argument("--sources-sha256", action="store_true",
                    help="print the hash of the stepper sources (recorded beside the HBM counters) and exit")
    ap.add_argument("--polish", type=int, default=2, choices=[1, 2],
                    help="continuation of each solve from its FP32 floor to the tolerance: 1 = FP64 steps, "
                         "2 = the refinement form (FP64 state, FP32 correction steps)")
    ap.add_argument("--polish-separate", action="store_true",
                    help="run the FP64 polish as a second launch over the promoted solves (CIL_OPT_POLISH_SEPARATE), "
                         "so that counters separate the FP32 and FP64 phases")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB (a known-size kernel "
                         "that scales HBM byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.sources_sha256:
        print(stepper_sources_sha256())
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(solves and pair tiles would shard by index with no communication but one all-reduce "
              "of integer counts); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.workload == "features4096":
        features_main(args)
        return
    if args.workload == "bz_uneven2048":
        uneven_main(args)
        return
    if args.workload == "mcil_stripes64":
        mcil_main(args)
        return
    if args.workload == "fhn32_fixed5000":
        fhn32_main(args)
        return
    if args.workload == "fhn128_mcmc":
        mcmc_main(args)
        return
    if args.workload == "fhn128_de":
        de_main(args)
        return
    if args.workload == "fhn32_sbdf2":
        sbdf2_main(args)
        return
    if args.workload == "gm_source64_lone":
        lone_main(args)
        return

    import cil_synth as cs
    import paper_2203_14742_amd as cil

    w = cs.WORKLOADS[WORKLOAD]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.polish_separate:
        cil.cil_set_option(cil.CIL_OPT_POLISH_SEPARATE, 1)
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
    pat32 = torch.empty((B, d), dtype=torch.float32, device=dev)
    y_obs = torch.empty(M, dtype=torch.float64, device=dev)
    Ybuf = torch.empty((n_boot, M), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    copy_calibration(args, dev)

    def one_step(state, ics, path, stat_fp32):
        """Whole hot path; stat_fp32: statistic on FP32 patterns (split-bf16x3 Gram)."""
        state.copy_(ics)
        rep = cil.cil_simulate_patterns(w["model"], state, probs, w["dt"], w["max_steps"], tol=w["tol"],
                                        check_every=w["check_every"], path=path, polish=args.polish)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        if stat_fp32 and state.dtype != torch.float32:
            pat32.copy_(state.reshape(B, d))          # patterns stored as FP32
            pats = pat32
        else:
            pats = state.reshape(B, d)
        A, Bs = pats[:half], pats[half:]
        # range, radii, bins, bootstrap, observed vector and likelihood in one
        # call (two host round trips: the radii, and the checks at the end)
        lo, hi, radii, counts, _, Y, _, out = cil.cil_statistic_adaptive(A, Bs, M, idxA, idxB, bins=bins,
                                                                         Y=Ybuf, y_obs=y_obs)
        ev1.record(stream)
        return rep, counts, ev0, ev1, out

    def timed(state, ics, path, stat_fp32, steps, warmup, profile=0):
        """profile 2: events around the stepper launches only (the timed
        headline); 1: around every hot kernel (a separate pass for the
        statistic's kernel table)."""
        for _ in range(warmup):
            one_step(state, ics, path, stat_fp32)
        torch.cuda.synchronize()
        if profile:
            cil.cil_profile(profile)
        t0 = time.perf_counter()
        cil_ms = 0.0
        reps = []
        each.clear()
        stat_each.clear()
        for _ in range(steps):
            t1 = time.perf_counter()
            rep, counts, e0, e1, out = one_step(state, ics, path, stat_fp32)
            reps.append(rep)
            torch.cuda.synchronize()
            each.append(time.perf_counter() - t1)
            stat_each.append(e0.elapsed_time(e1))
            cil_ms += stat_each[-1]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = {}
        if profile:
            for name in cil.cil_profile_names():
                prof[name] = cil.cil_profile_read(name)
            cil.cil_profile(False)
        return el, cil_ms / 1e3, reps, counts, out, prof

    each = []
    stat_each = []

    state32 = torch.empty_like(ics32)
    # batched path: persistent fused FP32 stepping, each solve continuing
    # from its FP32 floor to the tolerance in the same launch; statistic on
    # the FP32 patterns
    el, cil_s, reps, counts, out, prof = timed(state32, ics32, cil.CIL_PATH_AUTO, True, args.steps, args.warmup,
                                               profile=2)
    head_each = [round(1e3 * t, 3) for t in each]
    head_stat_each = [round(t, 4) for t in stat_each]
    # the statistic's kernels timed in a pass of their own after the timed
    # region (events around its short launches would slow the timed one)
    _, _, _, _, _, prof_stat = timed(state32, ics32, cil.CIL_PATH_AUTO, True, 2, 0, profile=1)
    K = args.steps
    ms_per_step = 1e3 * el / K
    patterns_per_s = B * K / el
    pairs = half * half
    pairs_per_s = pairs * K / cil_s if cil_s > 0 else None
    rep = reps[-1]
    status_ok = bool(np.all(rep["status"] == 0))
    solve_steps = sum(int(r["steps_taken"].sum()) for r in reps)
    fp64_steps = sum(int(r["steps_fp64"].sum()) for r in reps)

    kernels = {k: {"launches": v[0], "total_ms": round(v[1], 3)} for k, v in sorted(prof.items())}
    kernels_stat = {k: {"launches": v[0], "avg_us": round(1e3 * v[1] / v[0], 2)}
                    for k, v in sorted(prof_stat.items()) if not k.startswith("k_fused")}
    kname = max(prof, key=lambda k: prof[k][1]) if prof else None
    roof = None
    if kname and kname.startswith("k_fused"):
        cnt, tot_ms = prof[kname]
        per = fused_step_flops(n, REACTION_FLOPS[w["model"]])
        # the refinement form's polish steps transform in FP32 (its FP64 work,
        # the residual at each re-basing, is not counted as algorithmic)
        f64_steps = fp64_steps if args.polish == 1 else 0
        f32_flops = (solve_steps - f64_steps) * per
        f64_flops = f64_steps * per
        avg_ms = tot_ms / cnt
        achieved = (f32_flops + f64_flops) / cnt / (avg_ms * 1e-3) / 1e12
        # the vector ALU peak for this mix of FP32 and FP64 steps: the time the
        # work takes at the two published peaks
        peak = (f32_flops + f64_flops) / (f32_flops / VALU_FP32_PEAK_TFLOPS + f64_flops / VALU_FP64_PEAK_TFLOPS)
        roof = {"kernel": kname, "bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 2),
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": measured_traffic(kname),
                "launches": cnt, "avg_launch_ms": round(avg_ms, 4), "flops_per_solve_step": per,
                "solve_steps": solve_steps, "polish_solve_steps": fp64_steps,
                "polish": "FP64 steps" if args.polish == 1 else "refinement form (FP64 state, FP32 correction steps)",
                "peak_note": "weighted by the FP32 (157.3) and FP64 (78.6 TFLOP/s) steps of the launch"}
        # the launch lasts as long as its slowest solve: mean over maximum
        # steps per solve is the fraction a balanced batch would reach
        st = rep["steps_taken"]
        roof["tail_ceiling"] = round(float(st.mean()) / float(st.max()), 4)
        roof["frac_over_tail_ceiling"] = round(roof["frac"] / roof["tail_ceiling"], 4)
    gram = None
    gk = "k_gram_dma" if "k_gram_dma" in prof_stat else "k_gram_bf16x3"
    if gk in prof_stat:
        cnt, tot_ms = prof_stat[gk]
        executed = 6.0 * d * pairs * cnt             # three bf16 products per element pair
        gram = {"kernel": gk, "bound": "mfma", "achieved": round(executed / (tot_ms * 1e-3) / 1e12, 3),
                "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(executed / (tot_ms * 1e-3) / 1e12 / MFMA_BF16_PEAK_TFLOPS, 5),
                "avg_launch_ms": round(tot_ms / cnt, 4)}

    fp64_fused = None
    if not args.no_secondary:
        state64 = torch.empty_like(ics64)
        e64, c64, r64, _, _, _ = timed(state64, ics64, cil.CIL_PATH_AUTO, True, 1, 1)
        fp64_fused = {"patterns_per_s": round(B / e64, 3), "ms_per_step": round(1e3 * e64, 2),
                      "max_steps": int(r64[-1]["steps_taken"].max()),
                      "all_converged": bool(np.all(r64[-1]["status"] == 0)),
                      "what": "the same step with FP64 fused stepping throughout"}

    plain = None
    if not args.no_plain:
        # the plain FP64 GPU path timed like the batched one: one warm-up step,
        # then --plain-steps timed steps
        statep = torch.empty_like(ics64)
        ps_ = max(1, args.plain_steps)
        pel, pcil_s, preps, pcounts, _, _ = timed(statep, ics64, cil.CIL_PATH_PLAIN, False, ps_, 1)
        plain = {"patterns_per_s": round(B * ps_ / pel, 3), "pairs_per_s": round(pairs * ps_ / pcil_s, 1),
                 "ms_per_step": round(1e3 * pel / ps_, 2), "steps": ps_, "warmup": 1,
                 "ms_per_step_each": [round(1e3 * t, 2) for t in each],
                 "speedup_patterns": round(patterns_per_s / (B * ps_ / pel), 2),
                 "speedup_pairs": round(pairs_per_s / (pairs * ps_ / pcil_s), 2) if pairs_per_s else None,
                 "max_steps": int(preps[-1]["steps_taken"].max())}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, ics_host, base, args.cpu_sample_solves, half, d, args.cpu_single_solves)

    line = {
        "metric": "stationary patterns/s + CIL distance pairs/s, batched FP32 vs plain FP64",
        "value": round(patterns_per_s, 3), "unit": "patterns/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": WORKLOAD, "model": "gierer_meinhardt_source", "solves": B, "grid": n,
                   "dt": w["dt"], "tol": w["tol"], "radii": M, "bootstrap": n_boot,
                   "pairs_per_step": pairs,
                   "stepping": "fp32 fused persistent (quad-lane DCT); from each solve's fp32 floor to tol in the "
                               "same launch " + ("fp64 steps" if args.polish == 1 else
                                                 "in refinement form (fp64 state, fp32 correction steps)") +
                               "; fp64 residual",
                   "statistic": "fp32 patterns, split-bf16x3 MFMA Gram + canonical re-check",
                   "parallelism": "none (1 GPU)"},
        "pairs_per_s": round(pairs_per_s, 1) if pairs_per_s else None,
        "ms_per_step_each": head_each, "statistic_ms_each": head_stat_each,
        "solve_steps": solve_steps // K, "polish_solve_steps": fp64_steps // K,
        "max_solve_steps": int(rep["steps_taken"].max()), "all_converged": status_ok,
        "roofline": roof, "roofline_gram": gram, "kernels": kernels,
        "statistic_kernels": {"what": "average launch times from 2 further profiled steps", "kernels": kernels_stat},
        "fp64_fused": fp64_fused,
        "plain_fp64": plain, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def features_main(args):
    """CIL statistic alone: 4096 stand-in patterns of dimension 32768 (FP32),
    cross pairs of the two 2048-pattern halves, canonical range, 32 power-law
    radii, bins (split-bf16x3 Gram + canonical re-check), 200 bootstrap
    resamples, likelihood.  `value` is distance pairs/s."""
    import numpy as np
    import torch

    import cil_synth as cs
    import paper_2203_14742_amd as cil

    w = cs.WORKLOADS["features4096"]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    count, n, M, n_boot = w["count"], w["n"], w["M"], w["n_boot"]
    half, d = count // 2, 2 * n * n
    cil.cil_set_option(cil.CIL_OPT_GRAM_FLUSH, args.gram_flush)
    cil.cil_set_option(cil.CIL_OPT_GRAM_PIPELINE, args.gram_pipeline)
    host = cs.stripe_patterns(count, n, seed=w["seeds"][0]).reshape(count, d)
    pats = torch.from_numpy(host).to(dev)
    A, Bs = pats[:half], pats[half:]
    ia, ib = cs.resample_halves(half, half, half, half, n_boot, seed=w["boot_seed"])
    idxA = torch.from_numpy(ia).to(dev)
    idxB = torch.from_numpy(ib).to(dev)
    bins = torch.empty((half, half), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    pairs = half * half
    y_obs = torch.empty(M, dtype=torch.float64, device=dev)
    Ybuf = torch.empty((n_boot, M), dtype=torch.float64, device=dev)

    def one_step():
        lo, hi, radii, counts, _, Y, _, out = cil.cil_statistic_adaptive(A, Bs, M, idxA, idxB, bins=bins, Y=Ybuf,
                                                                         y_obs=y_obs)
        return out, counts

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    cil.cil_profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out, counts = one_step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = {k: cil.cil_profile_read(k) for k in cil.cil_profile_names()}
    cil.cil_profile(False)
    stats = cil.cil_last_distance_stats()
    K = args.steps
    plain = None
    if not args.no_plain:
        # the plain FP64 GPU path on the same pairs: FP64 patterns, direct
        # FP64 differences (split-K), the same adaptive range, radii and bins
        A64, B64 = A.double(), Bs.double()
        bins64 = torch.empty_like(bins)
        cil.cil_pair_bins_adaptive(A64, B64, M, bins=bins64)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, _, _, _, counts64 = cil.cil_pair_bins_adaptive(A64, B64, M, bins=bins64)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t1
        plain = {"value": round(pairs / tp, 1), "unit": "pairs/s", "ms": round(1e3 * tp, 3),
                 "what": "range + radii + bins of the same pairs from FP64 patterns, direct FP64 differences",
                 "same_counts": bool(np.array_equal(counts64, counts)),
                 "same_bins": bool(torch.equal(bins64, bins))}
        del A64, B64, bins64
    roof = None
    gk = "k_gram_dma" if "k_gram_dma" in prof else "k_gram_bf16x3"
    if gk in prof:
        cnt, tot_ms = prof[gk]
        executed = 6.0 * d * pairs * cnt        # one Gram per step (range and bins share it)
        ach = executed / (tot_ms * 1e-3) / 1e12
        roof = {"kernel": gk, "bound": "mfma", "achieved": round(ach, 2), "peak": MFMA_BF16_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / MFMA_BF16_PEAK_TFLOPS, 4), "traffic": None,
                "launches": cnt, "avg_launch_ms": round(tot_ms / cnt, 4),
                "flops_per_pair_executed": 6 * d, "algorithmic_flops_per_pair": 2 * d}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build()
        threads = cpu_threads()
        k = 768                                          # about 10 s on 16 threads
        t1 = time.perf_counter()
        D = oracle.pair_d2(host[:k], host[half:half + k], nthreads=threads)
        tp = time.perf_counter() - t1
        cpu = {"value": round(D.size / tp, 1), "unit": "pairs/s", "cores": threads, "host_cpus": os.cpu_count(),
               "kind": "oracle",
               "sample": "%d x %d canonical pair distances of the same sets (%.1f s)" % (k, k, tp)}
    line = {
        "metric": "stationary patterns/s + CIL distance pairs/s, batched FP32 vs plain FP64",
        "value": round(pairs * K / el, 1), "unit": "pairs/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": round(1e3 * el / K, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "features4096", "patterns": count, "dim": d, "pairs_per_step": pairs, "radii": M,
                   "bootstrap": n_boot, "statistic": "fp32 patterns, split-bf16x3 MFMA Gram + canonical re-check",
                   "parallelism": "none (1 GPU)"},
        "rechecked_pairs": stats["rechecked"], "exact_fallbacks": stats["exact_fallbacks"],
        "gram_flush": args.gram_flush, "gram_pipeline": args.gram_pipeline,
        "plain_fp64": plain,
        "speedup_vs_plain_fp64": None if plain is None else round(pairs * K / el / plain["value"], 2),
        "counts": [int(c) for c in counts],
        "loglik_status": int(out[3].cpu()[0]),
        "roofline": roof,
        "kernels": {k: {"launches": v[0], "total_ms": round(v[1], 3)} for k, v in sorted(prof.items())},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def uneven_main(args):
    """Uneven batch alone: 2048 Brusselator solves of sides 32, 64, 128 with
    per-solve parameters around a Turing point, 2000 FP32 steps (T = 100), as
    one simulate plan: a HIP graph holding one persistent kernel per side
    (forked streams, joined), code shape per side chosen by the plan's
    autotuner before timing.  A step = restore the initial states + one graph
    launch.  `value` is stationary patterns/s."""
    import numpy as np
    import torch

    import cil_synth as cs
    import paper_2203_14742_amd as cil

    w = cs.WORKLOADS["bz_uneven2048"]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ns, ps, nus = cs.brusselator_uneven(w["count"], w["seed"], sides=w["sides"], rel=w["rel"])
    bases = [cil.cil_homogeneous_state(w["model"], p) for p in ps]
    flat = cs.uneven_initial_states(bases, ns, seed=w["ic_seed"])
    probs = cil.make_problems(ns, w["L"], nus, ps)
    ics = torch.tensor(flat, dtype=torch.float32, device=dev)
    st = ics.clone()
    t0 = time.perf_counter()
    plan = cil.SimPlan(w["model"], st, probs, w["dt"], w["max_steps"], check_every=w["check_every"])
    t_plan = time.perf_counter() - t0
    t0 = time.perf_counter()
    info = plan.tune(steps=args.tune_steps)
    t_tune = time.perf_counter() - t0

    def one_step():
        st.copy_(ics)
        plan.launch()

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    cil.cil_profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = {k: cil.cil_profile_read(k) for k in cil.cil_profile_names()}
    cil.cil_profile(False)
    rep = plan.report()
    plan.close()
    K, B = args.steps, len(ns)
    cnt, tot_ms = prof["sim_plan_graph"]
    total_flops = sum(w["max_steps"] * fused_step_flops(n, REACTION_FLOPS[w["model"]]) for n in ns)
    ach = total_flops / (tot_ms / cnt * 1e-3) / 1e12
    roof = {"kernel": "sim_plan_graph (one persistent kernel per side)", "bound": "alu", "achieved": round(ach, 3),
            "peak": VALU_FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(ach / VALU_FP32_PEAK_TFLOPS, 4),
            "traffic": None, "launches": cnt, "avg_launch_ms": round(tot_ms / cnt, 3),
            "flops_per_solve_step": {str(n): fused_step_flops(n, REACTION_FLOPS[w["model"]]) for n in w["sides"]}}
    line = {
        "metric": "stationary patterns/s + CIL distance pairs/s, batched FP32 vs plain FP64",
        "value": round(B * K / el, 2), "unit": "patterns/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": round(1e3 * el / K, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "bz_uneven2048", "solves": B, "sides": list(w["sides"]), "dt": w["dt"],
                   "steps_per_solve": w["max_steps"], "stepping": "fp32 fused persistent, one HIP graph launch "
                   "(one kernel per side on forked streams)", "parallelism": "none (1 GPU)"},
        "autotune": {"trial_steps": args.tune_steps, "seconds": round(t_tune, 3), "plan_seconds": round(t_plan, 3),
                     "sides": [{"n": g["n"], "solves": g["count"], "shape": g["shape"],
                                "trial_ms": [round(m, 3) for m in g["tuned_ms"]]} for g in info]},
        "all_ok": bool(np.all(rep["status"] == 0) and np.all(rep["steps_taken"] == w["max_steps"])),
        "roofline": roof,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def fhn32_main(args):
    """The plain FP64 method's configuration: 128 FitzHugh-Nagumo solves on
    32x32 (two 64-pattern sets), 5000 fixed steps of dt = 0.01, then the
    correlation integral counts of the 64 x 64 cross pairs under 16 radii
    R_0 1.2^-m (R_0 = the largest distance).  Timed twice on the same inputs:
    the batched path (FP32 persistent fused stepper, split-bf16x3 Gram with
    canonical re-check) and the plain FP64 GPU path (one kernel per stage and
    step, direct FP64 distances).  `value` is the batched path's stationary
    patterns/s."""
    import numpy as np
    import torch

    import cil_synth as cs
    import paper_2203_14742_amd as cil

    w = cs.WORKLOADS["fhn32_fixed5000"]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    base = cil.cil_homogeneous_state(w["model"], w["params"])
    ics_host = np.concatenate([cs.initial_conditions(base, w["n"], w["count"], seed=s, law=w["ic_law"])
                               for s in w["seeds"]])
    B, half, M = ics_host.shape[0], w["count"], w["M"]
    probs = cil.make_problems(w["n"], w["L"], w["nu"], w["params"], count=B)

    def run(dtype, path):
        ics = torch.tensor(ics_host, dtype=dtype, device=dev)
        st = torch.empty_like(ics)

        def one_step():
            st.copy_(ics)
            rep = cil.cil_simulate_patterns(w["model"], st, probs, w["dt"], w["max_steps"],
                                            check_every=w["check_every"], path=path)
            P = st.reshape(B, -1)
            _, hi = cil.cil_distance_range(P[:half], P[half:])
            radii = [math.sqrt(hi) * w["radii_base"] ** -(m + 1) for m in range(M)]
            counts, _ = cil.cil_features(P[:half], P[half:], radii)
            return rep, counts

        for _ in range(args.warmup):
            one_step()
        torch.cuda.synchronize()
        cil.cil_profile(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            rep, counts = one_step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = {k: cil.cil_profile_read(k) for k in cil.cil_profile_names()}
        cil.cil_profile(False)
        return el / args.steps, rep, counts, prof

    t_fast, rep, counts, prof = run(torch.float32, cil.CIL_PATH_FUSED)
    t_plain, rep64, counts64, prof64 = run(torch.float64, cil.CIL_PATH_PLAIN)
    # the fused stepper in FP64: the same answers as the plain FP64 path (both
    # within the FP64 trajectory bar of the oracle), so its speedup compares
    # like with like
    t_f64, rep_f64, counts_f64, _ = run(torch.float64, cil.CIL_PATH_FUSED)
    kname = "k_fused_q_f32_n32"
    cnt, tot_ms = prof[kname]
    flops = B * w["max_steps"] * fused_step_flops(w["n"], REACTION_FLOPS[w["model"]])
    ach = flops / (tot_ms / cnt * 1e-3) / 1e12
    roof = {"kernel": kname, "bound": "alu", "achieved": round(ach, 3), "peak": VALU_FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(ach / VALU_FP32_PEAK_TFLOPS, 4), "traffic": None, "launches": cnt,
            "avg_launch_ms": round(tot_ms / cnt, 4),
            "flops_per_solve_step": fused_step_flops(w["n"], REACTION_FLOPS[w["model"]])}
    pairs = half * half
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build()
        threads = cpu_threads()
        k = B                                            # the whole batch: a few seconds
        t1 = time.perf_counter()
        oracle.imex_run(w["model"], w["params"], w["nu"], w["n"], w["L"], w["dt"], w["max_steps"], 0.0,
                        w["check_every"], state=ics_host[:k].copy(), nthreads=threads)
        tp = time.perf_counter() - t1
        cpu = {"value": round(k / tp, 2), "unit": "patterns/s", "cores": threads, "host_cpus": os.cpu_count(),
               "kind": "oracle",
               "sample": "%d solves x 5000 FP64 steps on the host (%.1f s)" % (k, tp)}
    line = {
        "metric": "stationary patterns/s + CIL distance pairs/s, batched FP32 vs plain FP64",
        "value": round(B / t_fast, 2), "unit": "patterns/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * t_fast, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "fhn32_fixed5000", "solves": B, "n": w["n"], "dt": w["dt"],
                   "steps_per_solve": w["max_steps"], "pairs": pairs, "radii": M,
                   "stepping": "fp32 fused persistent; statistic split-bf16x3 Gram + canonical re-check",
                   "parallelism": "none (1 GPU)"},
        "pairs_per_s": round(pairs / t_fast, 1),
        "plain_fp64": {"patterns_per_s": round(B / t_plain, 2), "ms_per_step": round(1e3 * t_plain, 3),
                       "speedup_patterns": round(t_plain / t_fast, 2),
                       "what": "FP64, five kernels per time step (reaction, row and column transforms with the "
                               "divide), direct FP64 distances"},
        "fp64_fused": {"patterns_per_s": round(B / t_f64, 2), "ms_per_step": round(1e3 * t_f64, 3),
                       "speedup_patterns_vs_plain": round(t_plain / t_f64, 2),
                       "counts": [int(c) for c in counts_f64],
                       "what": "the fused stepper in FP64 (the plain path's answers), FP64 statistic"},
        "counts_fp32_path": [int(c) for c in counts], "counts_fp64_path": [int(c) for c in counts64],
        "all_ok": bool(np.all(rep["status"] == 0) and np.all(rep64["status"] == 0) and
                       np.all(rep_f64["status"] == 0)),
        "roofline": roof,
        "kernels": {k: {"launches": v[0], "total_ms": round(v[1], 3)} for k, v in sorted(prof.items())},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def sbdf2_main(args):
    """The second-order IMEX stepper (semi-implicit BDF2) on the plain FP64
    method's configuration: 128 FitzHugh-Nagumo solves on 32x32, 5000 fixed
    steps of dt = 0.01, then the correlation integral counts of the 64 x 64
    cross pairs under 16 radii R_0 1.2^-m, all in FP64.  `value` is the
    fused second-order kernel's patterns/s (one workgroup per solve, history
    in LDS); beside it the same step on the plain back-end and IMEX Euler's
    fused FP64 step.  Roofline: the fused kernel's algorithmic flops (the
    transform count of the Euler step plus the second-order pointwise terms)
    against the FP64 vector peak."""
    import numpy as np
    import torch

    import cil_synth as cs
    import paper_2203_14742_amd as cil

    w = cs.WORKLOADS["fhn32_fixed5000"]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    base = cil.cil_homogeneous_state(w["model"], w["params"])
    ics_host = np.concatenate([cs.initial_conditions(base, w["n"], w["count"], seed=s, law=w["ic_law"])
                               for s in w["seeds"]])
    B, half, M, n = ics_host.shape[0], w["count"], w["M"], w["n"]
    probs = cil.make_problems(n, w["L"], w["nu"], w["params"], count=B)

    def run(scheme, path):
        ics = torch.tensor(ics_host, dtype=torch.float64, device=dev)
        st = torch.empty_like(ics)

        def one_step():
            st.copy_(ics)
            rep = cil.cil_simulate_patterns(w["model"], st, probs, w["dt"], w["max_steps"],
                                            check_every=w["check_every"], path=path, scheme=scheme)
            P = st.reshape(B, -1)
            _, hi = cil.cil_distance_range(P[:half], P[half:])
            radii = [math.sqrt(hi) * w["radii_base"] ** -(m + 1) for m in range(M)]
            counts, _ = cil.cil_features(P[:half], P[half:], radii)
            return rep, counts

        for _ in range(args.warmup):
            one_step()
        torch.cuda.synchronize()
        cil.cil_profile(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            rep, counts = one_step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = {k: cil.cil_profile_read(k) for k in cil.cil_profile_names()}
        cil.cil_profile(False)
        return el / args.steps, rep, counts, prof

    t2, rep2, counts2, prof2 = run("sbdf2", cil.CIL_PATH_AUTO)
    tp, repp, countsp, _ = run("sbdf2", cil.CIL_PATH_PLAIN)
    t1, rep1, counts1, _ = run("euler", cil.CIL_PATH_AUTO)
    kname = "k_fused_sbdf2_f64_n32"
    cnt, tot_ms = prof2[kname]
    step_flops = fused_step_flops(n, REACTION_FLOPS[w["model"]]) + 2 * n * n * 6
    flops = B * w["max_steps"] * step_flops                  # one launch = the whole 5000-step run
    ach = flops / (tot_ms / cnt * 1e-3) / 1e12
    roof = {"kernel": kname, "bound": "alu", "achieved": round(ach, 4), "peak": VALU_FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(ach / VALU_FP64_PEAK_TFLOPS, 5), "traffic": None, "launches": cnt,
            "avg_launch_ms": round(tot_ms / cnt, 3), "flops_per_solve_step": step_flops}
    line = {
        "metric": "stationary patterns/s + CIL distance pairs/s, batched FP32 vs plain FP64",
        "value": round(B / t2, 2), "unit": "patterns/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * t2, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "fhn32_sbdf2", "solves": B, "n": n, "dt": w["dt"], "steps_per_solve": w["max_steps"],
                   "pairs": half * half, "radii": M,
                   "stepping": "second-order IMEX (semi-implicit BDF2), fused FP64 line kernel",
                   "parallelism": "none (1 GPU)"},
        "sbdf2_plain_fp64": {"patterns_per_s": round(B / tp, 2), "ms_per_step": round(1e3 * tp, 3)},
        "imex_euler_fused_fp64": {"patterns_per_s": round(B / t1, 2), "ms_per_step": round(1e3 * t1, 3)},
        "counts_sbdf2": [int(c) for c in counts2], "counts_sbdf2_plain": [int(c) for c in countsp],
        "counts_euler": [int(c) for c in counts1],
        "all_ok": bool(np.all(rep2["status"] == 0) and np.all(repp["status"] == 0) and np.all(rep1["status"] == 0)),
        "roofline": roof,
        "kernels": {k: {"launches": v[0], "total_ms": round(v[1], 3)} for k, v in sorted(prof2.items())},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def mcil_main(args):
    """Multi-feature CIL statistic (Sec. 3.1) on 500 stand-in patterns of side
    64 (halves of 250): derivative augmentation, then per norm the adaptive
    radii, bins and 200 bootstrap vectors -- L2 and W^{1,2} through the
    split-bf16x3 Gram path (patterns / augmented vectors), L-inf, W^{1,inf} and
    its sum variant from the per-segment max-abs distances of the augmented
    vectors, the sum-of-L2 W^{1,2} variant from per-part canonical squared
    distances of all pairs -- and the likelihood of the concatenated 60-entry
    vector.  With --scaled the patterns are min-max scaled first (Sec. 5).
    `value` is distance pairs/s (pairs of patterns, all six norms)."""
    import numpy as np
    import torch

    import cil_synth as cs
    import paper_2203_14742_amd as cil

    w = cs.WORKLOADS["mcil_stripes64"]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    count, n, M, n_boot, L = w["count"], w["n"], w["M"], w["n_boot"], w["L"]
    half = count // 2
    raw = torch.from_numpy(cs.stripe_patterns(count, n, seed=w["seed"]).astype(np.float32)).to(dev)
    ia, ib = cs.resample_halves(half, half, half, half, n_boot, seed=w["boot_seed"])
    idxA = torch.from_numpy(ia).to(dev)
    idxB = torch.from_numpy(ib).to(dev)
    nn2, ne2 = 2 * n * n, 2 * n * (n - 1)
    ends = [nn2, nn2 + ne2, nn2 + 2 * ne2]
    pairs = half * half
    ii = torch.arange(half, device=dev).repeat_interleave(half)
    jj = torch.arange(half, device=dev).repeat(half)

    def one_step():
        P = cil.cil_minmax_scale(raw, n) if args.scaled else raw
        Aug = cil.cil_augment_patterns(P, n, L)
        Ys = []
        for X in (P.reshape(count, -1), Aug):
            _, _, _, bins, _ = cil.cil_pair_bins_adaptive(X[:half], X[half:], M)
            Ys.append(cil.cil_bootstrap_features(bins, idxA, idxB, M, want_counts=False)[1])
        D = cil.cil_pair_maxabs(Aug[:half], Aug[half:], ends)
        parts = []
        for a, b in zip([0] + ends[:-1], ends):
            Xs = Aug[:, a:b].contiguous()
            parts.append(cil.cil_canonical_d2(Xs[:half], Xs[half:], ii, jj).reshape(half, half))
        Wsum = cil.cil_combine_segments(torch.stack(parts, dim=-1).contiguous(), 2)
        for V in (D[..., 0].contiguous(), cil.cil_combine_segments(D, 0), cil.cil_combine_segments(D, 1), Wsum):
            lo, hi = cil.cil_value_range(V)
            bins, _ = cil.cil_bin_values(V, cil.cil_radii(lo * lo, hi * hi, M))
            Ys.append(cil.cil_bootstrap_features(bins, idxA, idxB, M, want_counts=False)[1])
        Y = torch.cat(Ys, dim=1).contiguous()
        return cil.cil_gaussian_loglik(Y, Y[0].contiguous()), Y

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    cil.cil_profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out, Y = one_step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = {k: cil.cil_profile_read(k) for k in cil.cil_profile_names()}
    cil.cil_profile(False)
    K = args.steps
    daug = ends[-1]
    roof = None
    if "k_pair_maxabs" in prof:
        cnt, tot_ms = prof["k_pair_maxabs"]
        ops = 2.0 * daug * pairs               # one FP64 subtract and one max per element pair
        ach = ops * cnt / (tot_ms * 1e-3) / 1e12
        roof = {"kernel": "k_pair_maxabs", "bound": "alu", "achieved": round(ach, 3),
                "peak": VALU_FP64_PEAK_TFLOPS / 2, "unit": "TOP/s (FP64 VALU instructions x lanes)",
                "frac": round(ach / (VALU_FP64_PEAK_TFLOPS / 2), 4), "traffic": None, "launches": cnt,
                "avg_launch_ms": round(tot_ms / cnt, 4), "ops_per_pair": 2 * daug}
    line = {
        "metric": "stationary patterns/s + CIL distance pairs/s, batched FP32 vs plain FP64",
        "value": round(pairs * K / el, 1), "unit": "pairs/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": round(1e3 * el / K, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "mcil_stripes64", "patterns": count, "n": n, "dim": nn2, "augmented_dim": daug,
                   "pairs_per_step": pairs, "norms": ["L2", "W12", "Linf", "W1inf", "W1inf_sum", "W12_sum"],
                   "radii": M,
                   "bootstrap": n_boot, "scaled": bool(args.scaled), "parallelism": "none (1 GPU)"},
        "features": int(Y.shape[1]), "m_eff": int(out[2].cpu()[0]), "loglik_status": int(out[3].cpu()[0]),
        "roofline": roof,
        "kernels": {k: {"launches": v[0], "total_ms": round(v[1], 3)} for k, v in sorted(prof.items())},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def mcmc_main(args):
    """Synthetic-likelihood evaluations (Alg. 3bst) on a window of proposals:
    the window's synthetic patterns in one simulate call (FP32, per-solve
    (mu, eps)), then per proposal the adaptive radii and bins of the
    synthetic self-pairs, 200 resample vectors and the observed vector
    against the data set, and one batched likelihood call.  `value` is
    synthetic patterns/s; likelihood evaluations/s are reported too."""
    import numpy as np
    import torch

    import cil_synth as cs
    import paper_2203_14742_amd as cil

    w = cs.WORKLOADS["fhn128_mcmc"]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    P, nsyn, nset, nboot, M, n = w["window"], w["n_syn"], w["n_set"], w["n_boot"], w["M"], w["n"]
    d = 2 * n * n
    thetas = cs.relative_draws(w["theta0"], P, w["rel"], seed=w["proposal_seed"])
    params = [(t[0], t[1], w["alpha"]) for t in thetas for _ in range(nsyn)]
    p0 = (w["theta0"][0], w["theta0"][1], w["alpha"])
    base = cil.cil_homogeneous_state(w["model"], p0)
    ics = torch.tensor(np.concatenate([cs.initial_conditions(base, n, nsyn, seed=w["ic_seed"] + p)
                                       for p in range(P)]), dtype=torch.float32, device=dev)
    probs = cil.make_problems(n, w["L"], w["nu"], params)
    data = torch.tensor(cs.initial_conditions(base, n, nset, seed=w["data_seed"]), dtype=torch.float32, device=dev)
    cil.cil_simulate_patterns(w["model"], data, cil.make_problems(n, w["L"], w["nu"], p0, count=nset), w["dt"],
                              w["max_steps"], check_every=w["max_steps"])
    data = data.reshape(nset, d)
    idx = [cs.resample_synthetic(nsyn, nset, nboot, seed=w["boot_seed"] + p) for p in range(P)]
    idx = [(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev), torch.from_numpy(c)[None, :].to(dev))
           for a, b, c in idx]
    ident = torch.arange(nset, dtype=torch.int32, device=dev)[None, :]
    st = torch.empty_like(ics)
    copy_calibration(args, dev)
    Y = torch.empty((P, nboot, M), dtype=torch.float64, device=dev)
    yobs = torch.empty((P, M), dtype=torch.float64, device=dev)
    t_sim = [0.0]

    def one_step():
        t0 = time.perf_counter()
        st.copy_(ics)
        cil.cil_simulate_patterns(w["model"], st, probs, w["dt"], w["max_steps"], check_every=w["max_steps"])
        torch.cuda.synchronize()
        t_sim[0] += time.perf_counter() - t0
        S = st.reshape(P * nsyn, d)
        for p in range(P):
            Sp = S[p * nsyn:(p + 1) * nsyn]
            _, _, radii, bins, _ = cil.cil_pair_bins_adaptive(Sp, Sp, M, exclude_diagonal=True)
            _, Y[p] = cil.cil_bootstrap_features(bins, idx[p][0], idx[p][1], M, want_counts=False)
            dbins, _ = cil.cil_pair_bins(data, Sp, radii, want_counts=False)
            _, yobs[p] = cil.cil_bootstrap_features(dbins, ident, idx[p][2], M, want_counts=False)
        return cil.cil_gaussian_loglik(Y, yobs)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    t_sim[0] = 0.0
    cil.cil_profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = one_step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = {k: cil.cil_profile_read(k) for k in cil.cil_profile_names()}
    cil.cil_profile(False)
    K = args.steps
    kname = "k_fused_q_f32_n128"
    roof = None
    if kname in prof:
        cnt, tot_ms = prof[kname]
        flops = P * nsyn * w["max_steps"] * fused_step_flops(n, REACTION_FLOPS[w["model"]]) * cnt / K
        ach = flops / (tot_ms / cnt * 1e-3) / 1e12
        roof = {"kernel": kname, "bound": "alu", "achieved": round(ach, 3), "peak": VALU_FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / VALU_FP32_PEAK_TFLOPS, 4), "traffic": measured_traffic(kname),
                "launches": cnt, "avg_launch_ms": round(tot_ms / cnt, 3),
                "flops_per_solve_step": fused_step_flops(n, REACTION_FLOPS[w["model"]])}
    stt = out[3].cpu().numpy()
    line = {
        "metric": "stationary patterns/s + CIL distance pairs/s, batched FP32 vs plain FP64",
        "value": round(P * nsyn * K / el, 2), "unit": "patterns/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": round(1e3 * el / K, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "fhn128_mcmc", "proposals_timed": P, "of_proposals": w["proposals"],
                   "synthetic_per_proposal": nsyn, "data_patterns": nset, "grid": n, "steps_per_solve": w["max_steps"],
                   "bootstrap": nboot, "radii": M, "parallelism": "none (1 GPU)"},
        "likelihood_evaluations_per_s": round(P * K / el, 3),
        "stepping_share": round(t_sim[0] / el, 3),
        "loglik_ok": int((stt == 0).sum()), "loglik_not_spd": int((stt != 0).sum()),
        "roofline": roof,
        "kernels": {k: {"launches": v[0], "total_ms": round(v[1], 3)} for k, v in sorted(prof.items())},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def de_main(args):
    """Differential evolution on the synthetic likelihood (Sec. 5's
    pre-optimisation): 20 candidates per generation, each generation one
    batched cost evaluation of 20 proposals x 64 synthetic FitzHugh-Nagumo
    patterns (128 x 128, 2000 FP32 steps) through `inference.SyntheticCIL`.
    The timed region is one DE run of `--steps` generations (plus its initial
    population); `value` is synthetic patterns/s."""
    import numpy as np
    import torch

    import cil_synth as cs
    import paper_2203_14742_amd as cil
    from paper_2203_14742_amd.inference import SyntheticCIL, differential_evolution

    w = cs.WORKLOADS["fhn128_mcmc"]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    pop, nsyn, nset, nboot, M, n = w["window"], w["n_syn"], w["n_set"], w["n_boot"], w["M"], w["n"]
    p0 = (w["theta0"][0], w["theta0"][1], w["alpha"])
    base = cil.cil_homogeneous_state(w["model"], p0)
    data = torch.tensor(cs.initial_conditions(base, n, nset, seed=w["data_seed"]), dtype=torch.float32, device=dev)
    cil.cil_simulate_patterns(w["model"], data, cil.make_problems(n, w["L"], w["nu"], p0, count=nset), w["dt"],
                              w["max_steps"], check_every=w["max_steps"])
    scil = SyntheticCIL(w["model"], n, w["L"], w["nu"], lambda t: (t[0], t[1], w["alpha"]), data.reshape(nset, -1),
                        nsyn, nboot, M, w["dt"], w["max_steps"],
                        cs.initial_conditions(base, n, nsyn, seed=w["ic_seed"]),
                        cs.resample_synthetic(nsyn, nset, nboot, seed=w["boot_seed"]))
    t0v = np.asarray(w["theta0"], dtype=np.float64)
    bounds = [(0.8 * t0v[0], 1.2 * t0v[0]), (0.8 * t0v[1], 1.2 * t0v[1])]
    cost = lambda X: scil.costs(X)[0]
    if args.warmup > 0:
        differential_evolution(cost, bounds, pop=pop, generations=args.warmup - 1, seed=99)
    torch.cuda.synchronize()
    K = args.steps
    t0 = time.perf_counter()
    r = differential_evolution(cost, bounds, pop=pop, generations=K, seed=w["proposal_seed"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    evals = K + 1
    line = {
        "metric": "stationary patterns/s + CIL distance pairs/s, batched FP32 vs plain FP64",
        "value": round(pop * nsyn * evals / el, 2), "unit": "patterns/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": round(1e3 * el / evals, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "fhn128_de", "candidates": pop, "generations_timed": K,
                   "batched_evaluations_timed": evals, "synthetic_per_proposal": nsyn, "data_patterns": nset,
                   "grid": n, "steps_per_solve": w["max_steps"], "bootstrap": nboot, "radii": M,
                   "parallelism": "none (1 GPU)"},
        "generations_per_s": round(evals / el, 4),
        "best_cost_history": [round(h, 6) for h in r["history"]],
        "best_theta": [round(float(v), 6) for v in r["x"]],
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def lone_main(args):
    """One Gierer-Meinhardt (source form) 64x64 solve alone on the GPU, 2000
    fixed steps in FP32 and in FP64 on the fused stepper: the per-step latency
    that bounds the stationarity batch's tail (its slowest solve ends up alone
    on its CU); then the batch's slowest solve alone to the tolerance, with
    each polish.  `value` is the FP32 steps per second of the lone solve."""
    import numpy as np
    import torch

    import cil_synth as cs
    import paper_2203_14742_amd as cil

    w = cs.WORKLOADS[WORKLOAD]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    n, steps = w["n"], 2000
    base = cil.cil_homogeneous_state(w["model"], w["params"])
    ics_host = cs.initial_conditions(base, n, 1, seed=w["seeds"][0], law=w["ic_law"])
    probs = cil.make_problems(n, w["L"], w["nu"], w["params"], count=1)
    out = {}
    for name, dtype in (("fp32", torch.float32), ("fp64", torch.float64)):
        ics = torch.tensor(ics_host, dtype=dtype, device=dev)
        st = torch.empty_like(ics)
        best = None
        for _ in range(max(1, args.warmup) + max(1, args.steps)):
            st.copy_(ics)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cil.cil_simulate_patterns(w["model"], st, probs, w["dt"], steps, check_every=w["check_every"], polish=0)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            best = el if best is None else min(best, el)
        out[name] = {"us_per_step": round(1e6 * best / steps, 3)}

    # the stationarity batch's slowest solve alone, to the tolerance: FP32 to
    # its floor (polish 0), then with each polish; the difference over the
    # polish steps is the polish step's latency
    ics_all = cs.initial_conditions(base, n, w["count"], seed=w["seeds"][0], law=w["ic_law"])
    probs_all = cil.make_problems(n, w["L"], w["nu"], w["params"], count=w["count"])
    st_all = torch.tensor(ics_all, dtype=torch.float32, device=dev)
    rep = cil.cil_simulate_patterns(w["model"], st_all, probs_all, w["dt"], w["max_steps"], tol=w["tol"],
                                    check_every=w["check_every"], polish=2)
    k = int(np.argmax(rep["steps_taken"]))
    ics_k = torch.tensor(ics_all[k:k + 1], dtype=torch.float32, device=dev)
    st = torch.empty_like(ics_k)
    slow = {"solve": k, "batch_steps_max": int(rep["steps_taken"][k])}
    # (separate: the polish as a launch of its own after the FP32 kernel, so
    # that the FP32 phase runs in the FP32 kernel in every case)
    for polish, sep in ((0, 0), (1, 0), (2, 0), (1, 1), (2, 1)):
        best, r = None, None
        cil.cil_set_option(cil.CIL_OPT_POLISH_SEPARATE, sep)
        for _ in range(max(1, args.warmup) + max(1, args.steps)):
            st.copy_(ics_k)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = cil.cil_simulate_patterns(w["model"], st, probs, w["dt"], w["max_steps"], tol=w["tol"],
                                          check_every=w["check_every"], polish=polish)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            best = el if best is None else min(best, el)
        cil.cil_set_option(cil.CIL_OPT_POLISH_SEPARATE, 0)
        slow["polish%d%s" % (polish, "_separate" if sep else "")] = {
            "ms": round(1e3 * best, 3), "steps": int(r["steps_taken"][0]), "polish_steps": int(r["steps_fp64"][0]),
            "status": int(r["status"][0])}
    t0 = slow["polish0"]["ms"]
    for key, e in slow.items():
        if isinstance(e, dict) and e["polish_steps"] > 0:
            e["us_per_polish_step"] = round(1e3 * (e["ms"] - t0) / e["polish_steps"], 3)
    line = {
        "metric": "stationary patterns/s + CIL distance pairs/s, batched FP32 vs plain FP64",
        "value": round(1e6 / out["fp32"]["us_per_step"], 1), "unit": "solve-steps/s (one solve alone)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "gm_source64_lone", "solves": 1, "grid": n, "fixed_steps": steps,
                   "parallelism": "none (1 GPU)"},
        "lone_step": out, "slowest_solve_alone": slow, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def cpu_threads() -> int:
    """Threads the oracle runs on: the host's CPUs, capped by OMP_NUM_THREADS
    (when set) and at 16."""
    return min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS") or 16), 16)


def cpu_baseline(w, ics_host, base, n_solves, half, d, n_single):
    """The FP64 oracle on host cores, on the same step: `n_solves` solves to
    stationarity (the whole batch by default) on all the threads it may use,
    the first `n_single` of them again on one thread, and the canonical
    distances of a block of pairs of the resulting patterns; scaled to
    patterns/s of the full step (solve time per pattern + pairs-per-pattern x
    time per pair)."""
    import numpy as np

    import oracle

    oracle.build()
    threads = cpu_threads()
    ics = ics_host[:n_solves].copy()
    t0 = time.perf_counter()
    out, steps, res, status = oracle.imex_run(w["model"], w["params"], w["nu"], w["n"], w["L"], w["dt"],
                                              w["max_steps"], w["tol"], w["check_every"], state=ics,
                                              nthreads=threads)
    t_sim = time.perf_counter() - t0
    k = min(n_solves // 2, 192)
    A = out[:k].reshape(k, -1).astype(np.float32)
    Bm = out[k:2 * k].reshape(k, -1).astype(np.float32)
    t1 = time.perf_counter()
    D = oracle.pair_d2(A, Bm, nthreads=threads)
    t_pairs = time.perf_counter() - t1
    sec_per_pattern = t_sim / n_solves + (half * half / (2 * half)) * (t_pairs / D.size)
    single = None
    if n_single > 0:
        t2 = time.perf_counter()
        _, s1, _, _ = oracle.imex_run(w["model"], w["params"], w["nu"], w["n"], w["L"], w["dt"], w["max_steps"],
                                      w["tol"], w["check_every"], state=ics_host[:n_single].copy(), nthreads=1)
        t_one = time.perf_counter() - t2
        t3 = time.perf_counter()
        D1 = oracle.pair_d2(A[:48], Bm[:48], nthreads=1)
        t_p1 = time.perf_counter() - t3
        # per pattern: this subsample's time per solve-step x the batch's mean
        # steps (the subsample's solves need not have the batch's mean length)
        per_solve = t_one / float(s1.sum()) * float(steps.mean())
        sp1 = per_solve + (half * half / (2 * half)) * (t_p1 / D1.size)
        single = {"value": round(1.0 / sp1, 4), "unit": "patterns/s", "cores": 1,
                  "sample": "%d solves on one thread (%.1f s, %d solve-steps, scaled to the batch's mean of %.0f "
                            "steps per solve) + %d canonical pair distances (%.2f s)"
                            % (n_single, t_one, int(s1.sum()), float(steps.mean()), D1.size, t_p1)}
    return {"value": round(1.0 / sec_per_pattern, 4), "unit": "patterns/s", "cores": threads,
            "host_cpus": os.cpu_count(), "kind": "oracle",
            "sample": "%d solves to residual < %g on %d threads (%.1f s) + %d canonical pair distances (%.1f s), "
                      "scaled to the full step" % (n_solves, w["tol"], threads, t_sim, D.size, t_pairs),
            "pairs_per_s": round(D.size / t_pairs, 1), "mean_steps": float(steps.mean()),
            "single_thread": single}


if __name__ == "__main__":
    main()
