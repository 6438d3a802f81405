"""Autotuner for the sweep kernel's launch geometry.

The sweep kernel keeps whole 64-replica lattices in LDS; its free parameters
are the threads per block, the number of 64-replica groups per block (small
lattices leave threads idle unless several groups share a block) and the
words each thread updates at once (the ABI's variant: one, or two with their
Philox chains interleaved, which trades occupancy for instruction-level
parallelism).  The
random numbers are keyed by replica and site, so every geometry must produce
the same population: the tuner checks that bit for bit while it times each
candidate from one snapshot, and stores the fastest per (arch, L, R bucket,
layout) in a JSON cache.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, List, Optional, Tuple

from . import Run

CACHE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
MAX_LDS = 152 * 1024


def arch_name() -> str:
    import torch
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def r_bucket(R: int) -> int:
    """Population size rounded down to a power of 4 (tuning classes)."""
    return 4 ** int(math.log(max(R, 1), 4))


def key(L: int, R: int, layout: str) -> str:
    return "%s/L%d/R%d/%s" % (arch_name(), L, r_bucket(R), layout)


def candidates(L: int) -> List[Tuple[int, int, int]]:
    """(threads, groups per block, words per thread) triples worth timing."""
    N = L * L
    lds = (L + 2) * (L + 2) * 8  # one lattice with its halo
    out = []
    for gpb in (1, 2, 4, 8):
        if gpb * lds > MAX_LDS:
            continue
        if gpb > 1 and (gpb // 2) * N // 2 >= 1024:
            continue  # one group already fills a 1024-thread block
        for threads in (128, 256, 512, 1024):
            for words in (1, 2):
                out.append((threads, gpb, words))
    return out


def load_cache(path: str = CACHE_PATH) -> Dict[str, dict]:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: Dict[str, dict], path: str = CACHE_PATH) -> None:
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_run(run: Run, L: int, steps: int = 2, cands: Optional[List[Tuple[int, int, int]]] = None):
    """Time every geometry on `steps` steps from the run's current state.

    Returns (best (ms, threads, gpb, variant), all results).  Raises if two geometries
    disagree on the resulting state.  The run is left at its original state
    with the best geometry set.
    """
    blob = run.get_state()
    ref = None
    results = []
    for threads, gpb, variant in (cands or candidates(L)):
        run.set_state(blob)
        run.set_sweep_launch(L, threads, gpb, variant)
        run.profile(True)
        for _ in range(steps):
            run.anneal_step()
        prof = run.profile_read()
        run.profile(False)
        state = run.get_state()
        if ref is None:
            ref = state
        elif state != ref:
            raise RuntimeError("sweep geometry (%d threads, %d groups, variant %d) changed the "
                               "results" % (threads, gpb, variant))
        results.append((prof["ms_sweep"] / steps, threads, gpb, variant))
    best = min(results)
    run.set_state(blob)
    run.set_sweep_launch(L, best[1], best[2], best[3])
    return best, results


def tune(L: int, R: int, layout: str, betas, theta: int = 10, warm_steps: int = 20,
         steps: int = 2, resample: str = "multinomial", save: bool = True) -> dict:
    """Tune a representative run (warmed up to a mid-schedule state) and cache it."""
    run = Run(L, R, betas, theta, 4242, resample, layout)
    for _ in range(min(warm_steps, len(betas) - 1 - steps)):
        run.anneal_step()
    best, results = tune_run(run, L, steps)
    run.close()
    entry = {"threads": best[1], "groups_per_block": best[2], "variant": best[3],
             "ms_sweep": best[0], "candidates": [[t, g, v, ms] for ms, t, g, v in results]}
    if save:
        cache = load_cache()
        cache[key(L, R, layout)] = entry
        save_cache(cache)
    return entry


def apply(target, L: int, R: int, layout: str) -> Optional[Tuple[int, int, int]]:
    """Set the cached geometry on a Run or Batch; returns it (None if not cached)."""
    e = load_cache().get(key(L, R, layout))
    if not e:
        return None
    target.set_sweep_launch(L, e["threads"], e["groups_per_block"], e.get("variant", 0))
    return e["threads"], e["groups_per_block"], e.get("variant", 0)


# The workloads the benchmark runs: (L, R, layout, resampling, beta_final, steps)
WORKLOADS = [
    (64, 100000, "msc64", "multinomial", 0.4407, 200),
    (64, 100000, "int8", "multinomial", 0.4407, 200),
    (128, 100000, "msc64", "nearest", 1.0, 400),
    (16, 20000, "msc64", "nearest", 0.4407, 200),
    (32, 20000, "msc64", "nearest", 0.4407, 200),
    (64, 20000, "msc64", "nearest", 0.4407, 200),
    (128, 20000, "msc64", "nearest", 0.4407, 200),
]


def main():
    """Tune every benchmark workload and write the cache.

        python -m paper_2102_06611_amd.autotune
    """
    import torch
    from workloads import linear_schedule
    torch.cuda.set_device(0)
    for L, R, layout, resample, beta_f, n in WORKLOADS:
        e = tune(L, R, layout, linear_schedule(beta_f, n), warm_steps=n // 2, resample=resample)
        best = sorted(e["candidates"], key=lambda c: c[3])[:4]
        print("L=%d R=%d %s: %d threads, %d groups/block, variant %d, %.4f ms/sweep phase; best %s"
              % (L, R, layout, e["threads"], e["groups_per_block"], e["variant"], e["ms_sweep"], best),
              flush=True)


if __name__ == "__main__":
    main()
