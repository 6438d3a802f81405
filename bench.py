"""Benchmark: population annealing, L = 64, R = 100000, multinomial resampling,
beta 0 -> 0.4407 in 200 steps, theta = 10 checkerboard Metropolis sweeps.

A step is one whole temperature step of the method on the device: histogram,
ln Q, copy counts, offsets, copy/compaction, theta sweeps, measurement and
record.  The timed region runs K consecutive steps of a fresh run with its
population resident in HBM; value = spin-flip attempts (sum R_i N theta) per
nanosecond of wall time.  Both layouts are timed; the multispin one is the
headline.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 200] [--warmup 20] [--no-cpu-baseline]
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

L, R, THETA, BETA_F, N_STEPS = 64, 100_000, 10, 0.4407, 200
SEED = 12345
HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: full-rate 32-bit VALU lane-operations per second
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic VALU work (full-rate lane-operations) of the minimal gfx950 instruction
# sequence for the work actually needed:
SLOTS_PER_PHILOX = 40      # 10 rounds x (2 v_mad_u64_u32 + 2 three-input XORs)
SLOTS_PER_PLANE_PAIR = 16  # two 64-bit planes x two halves x (threshold bit, accept, tie, or)
SLOTS_PER_WORD = 24        # neighbour XORs and the bit-sliced A >= 2 / A = 1 / A = 0 classes


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(kernel: str):
    """FETCH/WRITE bytes per launch from profiles/traffic.json, if taken on this source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    from paper_2102_06611_amd.counters import source_hash
    e = d.get(kernel)
    if not e or e.get("source_hash") != source_hash():
        return None
    return e.get("hbm_bytes_per_launch")


def time_layout(pa, torch, betas, layout, K, W, L=L, R=R, resample="multinomial", seed=SEED,
                update="metropolis"):
    from paper_2102_06611_amd import autotune
    stream = torch.cuda.Stream()
    # warmup: W steps of a separate run (brings clocks and caches up)
    if W > 0:
        w = pa.Run(L, R, betas, THETA, seed + 1, resample, layout, stream=stream, update=update)
        autotune.apply(w, L, R, layout)
        for _ in range(min(W, len(betas) - 1)):
            w.anneal_step()
        w.sync()
        w.close()
    run = pa.Run(L, R, betas, THETA, seed, resample, layout, stream=stream, update=update)
    geometry = autotune.apply(run, L, R, layout) or run.sweep_launch(L)
    run.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        run.anneal_step()
    run.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    recs = [run.observables(i) for i in range(K + 1)]
    attempts = sum(r["R_i"] for r in recs[1:]) * L * L * THETA
    # the rest of the schedule, untimed: the free-energy error at its end
    n_total = len(betas) - 1
    if K < n_total:
        run.run(n_total - K)
        run.sync()
    final = run.observables(n_total)
    # the same K steps again with phase timing, then once more counting the
    # Philox calls (counting slows the sweeps; the runs are deterministic:
    # same populations, same calls)
    prof = None
    for count in (False, True):
        prun = pa.Run(L, R, betas, THETA, seed, resample, layout, stream=stream, update=update)
        autotune.apply(prun, L, R, layout)
        prun.profile(True, count_calls=count)
        for _ in range(K):
            prun.anneal_step()
        prun.sync()
        p = prun.profile_read()
        last = prun.observables(K)
        if (last["R_i"], last["minus_beta_F"]) != (recs[K]["R_i"], recs[K]["minus_beta_F"]):
            raise RuntimeError("the profiled run differs from the timed run")
        prun.close()
        if prof is None:
            prof = p
        else:
            prof["philox_calls"], prof["sweep_words"] = p["philox_calls"], p["sweep_words"]
    prof["geometry"] = list(geometry)
    prof["final"] = final
    return run, wall, prof, recs, attempts


def time_batch(pa, torch, K):
    """64 independent runs, L in {16,32,64,128} x R in {1e3,5e3,2e4,5e4}, graph-replayed."""
    from paper_2102_06611_amd import autotune
    from workloads import batched_design
    design = batched_design(64, beta_final=0.4407, n_steps=200, theta=THETA)
    specs = [dict(L=d.L, R=d.R, theta=d.theta, seed=d.seed, resample=d.resample, layout=d.layout,
                  betas=d.betas()) for d in design]
    stream = torch.cuda.Stream()
    b = pa.Batch(specs, stream=stream)
    for Lc in sorted(set(d.L for d in design)):
        autotune.apply(b, Lc, 20000, "msc64")
    b.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(K)
    b.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    attempts = 0
    for k, d in enumerate(design):
        attempts += sum(b.observables(k, i)["R_i"] for i in range(1, K + 1)) * d.L * d.L * THETA
    b.close()
    return {"attempts_per_ns": attempts / wall / 1e9, "ms_per_step": wall * 1e3 / K, "steps": K,
            "runs": len(design), "spins": sum(d.L * d.L * d.R for d in design),
            "workload": "64 runs, L in {16,32,64,128} x R in {1000,5000,20000,50000} (each pair 4x), "
                        "nearest, multispin, beta 0->0.4407 in 200 steps, theta=10, one HIP graph per step"}


def time_weighted(pa, torch, M=64, L=32, R=2000, n=200):
    """Weighted averages over M runs sharing one schedule (pa_batch_weighted),
    all n + 1 steps in one call, timed by wall clock (the call also checks
    every run's state on the host)."""
    import ctypes
    from workloads import linear_schedule
    betas = linear_schedule(0.4407, n)
    specs = [dict(L=L, R=R, theta=THETA, seed=2000 + m, resample="nearest", layout="msc64",
                  betas=betas) for m in range(M)]
    b = pa.Batch(specs)
    b.run(n)
    b.sync()
    out = torch.empty((n + 1) * ctypes.sizeof(pa.pa_weighted), dtype=torch.uint8, device="cuda")
    call = lambda: pa._check(pa.lib().pa_batch_weighted(b.h, 0, n + 1, ctypes.c_void_p(out.data_ptr())),
                             b.h, batch=True)
    for _ in range(3):  # warm
        call()
    b.sync()
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        call()
    b.sync()
    wall = (time.perf_counter() - t0) / reps
    last = b.weighted(n)[0]
    b.close()
    return {"runs": M, "L": L, "R": R, "steps": n + 1,
            "us_per_call_all_steps": wall * 1e6,
            "at_last_step": {k: last[k] for k in ("e", "e_plain", "c_v", "c_v_plain", "n_eff_runs",
                                                  "var_beta_F", "rho_f", "cov_e")}}


def compare_schedules(pa, torch, n_seeds=16):
    """Plain linear vs self-adaptive vs learned temperature steps at L = 128,
    R = 100000, beta 0 -> 1.0, theta = 10, nearest-integer resampling, on the
    same seeds: steps taken and |(-beta F) - ln Z_exact| / L^2 at beta = 1.0.
    The network is trained on the device from adaptive runs at L = 32 and 64,
    R = 20000 (error-budget targets, paper_2102_06611_amd/schedules.py)."""
    import numpy as np
    from paper_2102_06611_amd import schedules
    from workloads import linear_schedule
    exact = json.load(open(os.path.join(ROOT, "tests", "golden", "exact_lnz.json")))
    ln_z = exact["points"]["L128_1"]
    t0 = time.perf_counter()
    info = []
    X, t = schedules.collect((32, 64), 20000, range(500, 508), THETA, 0.85, 1.0, info=info)
    params, losses = schedules.train(X, t, iters=4000, lr=2e-3)
    t_train = time.perf_counter() - t0
    seeds = [900 + k for k in range(n_seeds)]
    res = schedules.compare(params, 128, 100_000, THETA, seeds, ln_z)
    plain = []
    betas = linear_schedule(1.0, 400)
    for sd in seeds:
        r = pa.Run(128, 100_000, betas, THETA, sd, "nearest", "msc64")
        r.run(400)
        plain.append(abs(r.observables(400)["minus_beta_F"] - ln_z) / (128 * 128))
        r.close()

    def stats(x):
        x = np.asarray(x, dtype=np.float64)
        return {"mean": float(x.mean()), "se": float(x.std(ddof=1) / math.sqrt(len(x)))}
    sa = [r["steps_adaptive"] for r in res]
    sl = [r["steps_learned"] for r in res]
    return {
        "workload": "L=128, R=100000, beta 0->1.0, theta=10, nearest, msc64, %d seeds; "
                    "network trained on adaptive runs at L=32,64, R=20000" % n_seeds,
        "plain": {"steps": 400, "error_per_spin": stats(plain)},
        "adaptive": {"alpha": 0.85, "steps": stats(sa),
                     "error_per_spin": stats([r["error_adaptive"] for r in res])},
        "learned": {"alpha_min": 0.80, "steps": stats(sl),
                    "error_per_spin": stats([r["error_learned"] for r in res]),
                    "accepted": float(np.mean([r["accepted"] for r in res])),
                    "alpha_mean": float(np.mean([r["alpha_mean_learned"] for r in res]))},
        "steps_ratio_learned_to_adaptive": float(np.mean(sl) / np.mean(sa)),
        "training": {"rows": int(X.shape[0]), "loss_first": losses[0], "loss_last": losses[-1],
                     "seconds": t_train,
                     "mean_step_factor": float(np.mean([i["mean_step_factor"] for i in info]))},
        "seconds": time.perf_counter() - t0}


def cpu_baseline(betas, energies):
    """The oracle, single-threaded, on a bounded sample of the same workload.

    Sweeps of one 64-replica group (about 10 s) and one multinomial resampling
    of the full population at step 101 are timed; the value is the whole-step
    rate they imply for R = 100000 (theta sweeps of every group plus one
    resampling per step)."""
    import numpy as np
    from oracle import pa_oracle as po
    beta = betas[-1]
    t4, t8 = po.metropolis_threshold(beta, 4), po.metropolis_threshold(beta, 8)
    spins = po.init_spins(SEED, L, 64)
    t0 = time.perf_counter()
    sweeps = 0
    while True:  # sweeps of one 64-replica group until >= 10 s of CPU work
        po.sweeps(SEED, L, spins, N_STEPS, 1, t4, t8)
        sweeps += 1
        if time.perf_counter() - t0 > 10.0 or sweeps >= 5000:
            break
    t_sweep = time.perf_counter() - t0
    o = po.OracleRun(L, 4, THETA, SEED, "multinomial", betas)
    o.R = R
    o.E = np.asarray(energies, dtype=np.int32)
    t1 = time.perf_counter()
    o.copy_counts(betas[100], betas[101], 101)
    t_res = time.perf_counter() - t1
    groups = math.ceil(R / 64)
    step_s = t_sweep / sweeps * THETA * groups + t_res
    return {"value": R * L * L * THETA / step_s / 1e9, "unit": "attempts/ns", "cores": 1,
            "kind": "oracle",
            "sample": "%d sweeps of 64 replicas (L=64) at beta=%.4f (%.1f s) and one multinomial "
                      "resampling of %d parents (%.2f s), scaled to a step of R=%d, theta=%d"
                      % (sweeps, beta, t_sweep, len(energies), t_res, R, THETA),
            "step_seconds": step_s, "resample_s_per_step": t_res, "sweep_seconds": t_sweep,
            "host": host_cpu()}


def cpu_config3_sample(energies128):
    """The oracle on a bounded sample of the L=128 workload (R = 100000,
    nearest-integer resampling, beta 0 -> 1 in 400 steps): sweeps of one
    64-replica group at beta = 1 (about 5 s) and one nearest-integer
    resampling of the device run's final population, scaled to a step."""
    import numpy as np
    from oracle import pa_oracle as po
    from workloads import linear_schedule
    L3, R3, n3 = 128, 100_000, 400
    betas3 = linear_schedule(1.0, n3)
    beta = betas3[-1]
    t4, t8 = po.metropolis_threshold(beta, 4), po.metropolis_threshold(beta, 8)
    spins = po.init_spins(SEED, L3, 64)
    t0 = time.perf_counter()
    sweeps = 0
    while True:
        po.sweeps(SEED, L3, spins, n3, 1, t4, t8)
        sweeps += 1
        if time.perf_counter() - t0 > 5.0 or sweeps >= 2000:
            break
    t_sweep = time.perf_counter() - t0
    o = po.OracleRun(L3, 4, THETA, SEED, "nearest", betas3)
    o.R = len(energies128)
    o.E = np.asarray(energies128, dtype=np.int32)
    t1 = time.perf_counter()
    o.copy_counts(betas3[n3 - 1], betas3[n3], n3)
    t_res = time.perf_counter() - t1
    step_s = t_sweep / sweeps * THETA * math.ceil(R3 / 64) + t_res
    return {"workload": "L=128, R=100000, nearest, beta 0->1.0 in 400 steps, theta=10",
            "value": R3 * L3 * L3 * THETA / step_s / 1e9, "unit": "attempts/ns", "cores": 1,
            "sample": "%d sweeps of 64 replicas (L=128) at beta=%.1f (%.1f s) and one nearest-integer "
                      "resampling of %d parents (%.2f s), scaled to a step of R=%d, theta=%d"
                      % (sweeps, beta, t_sweep, len(energies128), t_res, R3, THETA),
            "step_seconds": step_s, "resample_s_per_step": t_res}


def cpu_config1(pa):
    """The small workload in full on both sides: L=8, R=1000, beta 0 -> 0.44 in
    101 steps, theta=10, nearest-integer resampling.  The oracle's whole run
    (its copy counts timed apart) beside the device run of the same seed: the
    integer sums of every record must agree exactly, -beta F to rounding."""
    import numpy as np
    import torch
    from oracle import pa_oracle as po
    from workloads import linear_schedule
    L1, R1, n1, seed1 = 8, 1000, 101, SEED
    betas = linear_schedule(0.44, n1)
    o = po.OracleRun(L1, R1, THETA, seed1, "nearest", np.asarray(betas, dtype=np.float64))
    t_counts = [0.0]
    counts = o.copy_counts

    def timed_counts(*a, **k):
        t = time.perf_counter()
        r = counts(*a, **k)
        t_counts[0] += time.perf_counter() - t
        return r
    o.copy_counts = timed_counts
    t0 = time.perf_counter()
    for _ in range(n1):
        o.anneal_step()
    t_oracle = time.perf_counter() - t0
    attempts = sum(rec.R_i for rec in o.records[1:]) * L1 * L1 * THETA
    run = pa.Run(L1, R1, betas, THETA, seed1, "nearest", "msc64")
    run.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    run.run(n1)
    run.sync()
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t1
    keys = ("R_i", "sum_E", "sum_E2", "sum_absM", "sum_M2", "n_families", "sum_cnt2")
    same = all(run.observables(i)[k] == getattr(o.records[i], k) for i in range(n1 + 1) for k in keys)
    f_gpu, f_orc = run.observables(n1)["minus_beta_F"], o.records[n1].minus_beta_F
    run.close()
    return {"workload": "L=8, R=1000, beta 0->0.44 in 101 steps, theta=10, nearest, seed %d" % seed1,
            "oracle_seconds": t_oracle, "oracle_attempts_per_ns": attempts / t_oracle / 1e9,
            "oracle_copy_counts_us_per_step": t_counts[0] / n1 * 1e6,
            "gpu_seconds": t_gpu, "gpu_attempts_per_ns": attempts / t_gpu / 1e9,
            "same_integer_sums_every_step": bool(same),
            "minus_beta_F_rel_diff": abs(f_gpu - f_orc) / abs(f_orc)}


def host_cpu() -> dict:
    """The host's CPU model and the cores this process may use; the oracle
    stays single-threaded, and value x cores is the host's ideal aggregate
    (context only)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def copy_calibration():
    """A plain device-to-device copy of 1 GiB, three times: the reference that
    scales rocprofv3's FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    x = torch.empty(2 ** 28, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    log("copied 3 x 1 GiB")


def head_candidate(layouts: str) -> str:
    names = layouts.split(",")
    return "msc64" if "msc64" in names else names[0]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=N_STEPS)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--layouts", default="msc64,int8")
    ap.add_argument("--headline-only", action="store_true")
    ap.add_argument("--no-schedules", action="store_true",
                    help="skip the plain / adaptive / learned schedule comparison")
    ap.add_argument("--update", choices=("metropolis", "heatbath"), default="metropolis",
                    help="spin update of the layout runs (profiling the heatbath sweep)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB on the device three times (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs each population on one device and "
              "uses no collectives; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    K = max(1, min(args.steps, N_STEPS))
    import numpy as np
    import torch
    import paper_2102_06611_amd as pa
    from workloads import linear_schedule
    if not torch.cuda.is_available():
        print("no GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    betas = linear_schedule(BETA_F, N_STEPS)
    exact = json.load(open(os.path.join(ROOT, "tests", "golden", "exact_lnz.json")))
    lnz = exact["schedules"]["L64_0.4407_200"]["ln_z"]

    results = {}
    energies_mid = None
    energies128 = None
    for layout in args.layouts.split(","):
        log("timing layout %s: %d steps" % (layout, K))
        run, wall, prof, recs, attempts = time_layout(pa, torch, betas, layout, K, args.warmup,
                                                      update=args.update)
        n = prof["steps"]
        sweep_ms = prof["ms_sweep"] / n
        res_ms = prof["ms_resample"] / n
        copy_ms = prof["ms_copy"] / n
        meas_ms = prof["ms_measure"] / n
        words = prof["sweep_words"] / n
        calls = prof["philox_calls"] / n
        alg_slots = calls * (SLOTS_PER_PHILOX + SLOTS_PER_PLANE_PAIR) + words * SLOTS_PER_WORD
        achieved_tops = alg_slots / (sweep_ms * 1e-3) / 1e12
        group_bytes = (L * L * 8) if layout == "msc64" else (L * L * 64)
        copy_bytes = 2 * math.ceil(R / 64) * group_bytes  # a5: read parents, write children
        err = [abs(recs[i]["minus_beta_F"] - lnz[i]) / (L * L) for i in range(K + 1)]
        results[layout] = {
            "attempts_per_ns": attempts / wall / 1e9,
            "sweep_attempts_per_ns": attempts / (prof["ms_sweep"] * 1e-3) / 1e9,
            "ms_per_step": wall * 1e3 / K,
            "sweep_ms_per_step": sweep_ms,
            "resample_us_per_step": res_ms * 1e3,
            "measure_us_per_step": meas_ms * 1e3,
            "philox_calls_per_word": calls / words if words else 0.0,
            "sweep_alu_tops": achieved_tops,
            "resample_copy_bytes": copy_bytes,
            "copy_us_per_step": copy_ms * 1e3,
            "copy_hbm_gbs": copy_bytes / (copy_ms * 1e-3) / 1e9,
            "beta_f_error_per_spin": {
                "beta": prof["final"]["beta"],
                "value": abs(prof["final"]["minus_beta_F"] - lnz[N_STEPS]) / (L * L),
                "jackknife_sigma": math.sqrt(prof["final"]["jk_var_beta_F"]) / (L * L),
                "timed_steps_max": max(err)},
            "beta_last": recs[-1]["beta"],
            "blocking_last": {k: recs[-1][k] for k in ("r_eff_E", "r_eff_absM", "err_e")},
            "sweep_geometry": prof["geometry"],
        }
        # overlap correlation C_q(d), d <= 1024, of the final population (events on
        # the run's stream; the call first reads the run state on the host)
        import torch as _t
        s_ = run.stream
        run.overlap_correlation(1024)
        e0, e1 = _t.cuda.Event(enable_timing=True), _t.cuda.Event(enable_timing=True)
        e0.record(s_)
        cq = run.overlap_correlation(1024)
        e1.record(s_)
        e1.synchronize()
        results[layout]["overlap_correlation"] = {
            "d_max": 1024, "us": e0.elapsed_time(e1) * 1e3,
            "pair_words_per_us": (L * L) * (R / 64) * 1024 / (e0.elapsed_time(e1) * 1e3),
            "C_q": {str(d): float(cq[d]) for d in (1, 2, 4, 16, 64, 256, 1024)}}
        if layout == head_candidate(args.layouts) and not args.no_cpu_baseline:
            # energies entering step 101, for the CPU-baseline resampling sample
            e_run = pa.Run(L, R, betas, THETA, SEED, "multinomial", layout)
            for _ in range(100):
                e_run.anneal_step()
            _, _, energies_mid, _ = e_run.population(spins=False)
            e_run.close()
        run.close()
        torch.cuda.empty_cache()

    extra = {}
    if not args.headline_only:
        log("timing L=128, R=100000, nearest, multispin: 400 steps")
        betas128 = linear_schedule(1.0, 400)
        lnz128 = exact["schedules"]["L128_1_400"]["ln_z"]
        run, wall, prof, recs, attempts = time_layout(pa, torch, betas128, "msc64", 400, 0, L=128,
                                                      R=100_000, resample="nearest")
        n = prof["steps"]
        extra["l128_nearest_msc64"] = {
            "attempts_per_ns": attempts / wall / 1e9, "ms_per_step": wall * 1e3 / 400,
            "sweep_attempts_per_ns": attempts / (prof["ms_sweep"] * 1e-3) / 1e9,
            "resample_us_per_step": prof["ms_resample"] / n * 1e3, "geometry": prof["geometry"],
            "beta_f_error_per_spin": abs(recs[-1]["minus_beta_F"] - lnz128[-1]) / (128 * 128),
            "final_families": recs[-1]["n_families"], "final_rho_t": recs[-1]["rho_t"]}
        if not args.no_cpu_baseline:
            _, _, energies128, _ = run.population(spins=False)
        run.close()
        torch.cuda.empty_cache()
        # the other copy-count rules on the headline workload (same sweeps)
        for rule in ("nearest", "poisson"):
            log("timing L=64, R=100000, %s, multispin: %d steps" % (rule, K))
            run, wall, prof, recs, attempts = time_layout(pa, torch, betas, "msc64", K, 0,
                                                          resample=rule)
            n = prof["steps"]
            sizes = np.array([r["R_i"] for r in recs[1:]], dtype=np.float64)
            err = abs(prof["final"]["minus_beta_F"] - lnz[N_STEPS]) / (L * L)
            extra["l64_%s_msc64" % rule] = {
                "attempts_per_ns": attempts / wall / 1e9, "ms_per_step": wall * 1e3 / K,
                "resample_us_per_step": prof["ms_resample"] / n * 1e3,
                "copy_us_per_step": prof["ms_copy"] / n * 1e3,
                "R_i_mean": float(sizes.mean()), "R_i_std": float(sizes.std()),
                "beta_f_error_per_spin_at_beta_c": err}
            run.close()
            torch.cuda.empty_cache()
        log("timing L=64, R=100000, multinomial, heatbath, multispin: %d steps" % K)
        run, wall, prof, recs, attempts = time_layout(pa, torch, betas, "msc64", K, 0,
                                                      update="heatbath")
        n = prof["steps"]
        words, calls = prof["sweep_words"] / n, prof["philox_calls"] / n
        sweep_ms = prof["ms_sweep"] / n
        alg = calls * (SLOTS_PER_PHILOX + SLOTS_PER_PLANE_PAIR) + words * SLOTS_PER_WORD
        extra["l64_heatbath_msc64"] = {
            "attempts_per_ns": attempts / wall / 1e9, "ms_per_step": wall * 1e3 / K,
            "sweep_attempts_per_ns": attempts / (prof["ms_sweep"] * 1e-3) / 1e9,
            "sweep_ms_per_step": sweep_ms, "philox_calls_per_word": calls / words if words else 0.0,
            "sweep_alu_tops": alg / (sweep_ms * 1e-3) / 1e12,
            "sweep_alu_frac": alg / (sweep_ms * 1e-3) / 1e12 / VALU_PEAK_TOPS,
            "beta_f_error_per_spin_at_beta_c": abs(prof["final"]["minus_beta_F"] - lnz[N_STEPS]) / (L * L)}
        run.close()
        torch.cuda.empty_cache()
        log("timing the 64-run batch: 200 steps")
        extra["batched_64_runs"] = time_batch(pa, torch, 200)
        torch.cuda.empty_cache()
        log("timing the combination of 64 independent runs (L=32, R=2000, nearest): 200 steps")
        extra["runs_combined"] = time_weighted(pa, torch)
        torch.cuda.empty_cache()
        if not args.no_schedules:
            log("plain, adaptive and learned schedules at L=128, R=100000, 16 seeds")
            extra["schedules_compared"] = compare_schedules(pa, torch)
            torch.cuda.empty_cache()

    head_layout = "msc64" if "msc64" in results else list(results)[0]
    head = results[head_layout]
    traffic = measured_traffic("k_sweep_msc64")
    roof = {"bound": "alu", "kernel": "k_sweep<msc64>", "achieved": head["sweep_alu_tops"],
            "peak": VALU_PEAK_TOPS, "unit": "Tops/s (32-bit VALU lane-ops)",
            "frac": head["sweep_alu_tops"] / VALU_PEAK_TOPS, "traffic": traffic}
    # the HBM-bound kernel of the step: copy / compaction of the population
    copy_roof = {"bound": "hbm", "kernel": "k_gather_%s" % head_layout,
                 "achieved": head["copy_hbm_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": head["copy_hbm_gbs"] / HBM_PEAK_GBS, "traffic": measured_traffic("k_gather_%s" % head_layout)}
    out = {
        "metric": "spin-flip attempts/ns + resample/step (L=64,R=1e5); βF error vs exact",
        "value": head["attempts_per_ns"], "unit": "attempts/ns", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64 bit-sliced (int32 counts, f64 ln Q)",
        "data": "synthetic",
        "config": {"workload": "2D Ising L=64 periodic, R=100000, multinomial resampling, beta 0->0.4407 "
                               "in 200 steps, theta=10, %s layout, %s update" % (head_layout, args.update),
                   "L": L, "R": R, "theta": THETA, "n_steps": N_STEPS, "seed": SEED,
                   "steps_timed": "1..%d" % K},
        "resample_us_per_step": head["resample_us_per_step"],
        "beta_f_error_per_spin": head["beta_f_error_per_spin"],
        "roofline": roof,
        "copy_roofline": copy_roof,
        "layouts": results,
        "workloads": extra,
    }
    if not args.no_cpu_baseline and energies_mid is not None:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(betas, energies_mid)
        out["cpu_baseline"]["host"]["ideal_aggregate_attempts_per_ns"] = (
            out["cpu_baseline"]["value"] * out["cpu_baseline"]["host"]["usable_cpus"])
        log("timing the small workload in full on the oracle and the device")
        out["cpu_baseline"]["small_workload_in_full"] = cpu_config1(pa)
        if energies128 is not None:
            log("timing the CPU oracle sample of the L=128 workload")
            out["cpu_baseline"]["l128_sample"] = cpu_config3_sample(energies128)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
