"""Seeded synthetic inputs for population-annealing runs.

This module only builds *inputs*: inverse-temperature schedules, seeds and the
(L, R) design of the batched workload.  It holds none of the method's
arithmetic, so both the HIP path and the CPU oracle may use it.

The Ising lattice itself is the workload (Sec. "Model and observables"): the
initial population is drawn from the seed by each side's own random-number
generator, so no spin data lives here.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

BETA_C = 0.5 * np.log1p(np.sqrt(2.0))  # critical point of the square-lattice Ising model
PARITY_SEED = 12345


def run_seed(k: int) -> int:
    """Seed of independent run k (runs are numbered from 0)."""
    return 1000 + int(k)


def linear_schedule(beta_final: float, n_steps: int, beta0: float = 0.0) -> np.ndarray:
    """beta_i = beta0 + (beta_final - beta0) * i / n_steps for i = 0..n_steps.

    n_steps counts the resampling steps, so the schedule has n_steps + 1
    temperatures including beta0 (Sec. "Free-energy estimate" counts N_T + 1
    temperatures).  Each entry is formed as a multiply followed by a divide in
    IEEE binary64 so every consumer sees the same doubles.
    """
    if n_steps < 0:
        raise ValueError("n_steps must be >= 0")
    out = np.empty(n_steps + 1, dtype=np.float64)
    span = float(beta_final) - float(beta0)
    for i in range(n_steps + 1):
        out[i] = float(beta0) + (span * i) / n_steps if n_steps else float(beta0)
    out[0] = float(beta0)
    return out


@dataclasses.dataclass(frozen=True)
class RunSpec:
    """One population-annealing run: lattice L x L, nominal population R."""

    L: int
    R: int
    theta: int
    seed: int
    resample: str  # "nearest" | "multinomial" | "none"
    beta_final: float
    n_steps: int
    layout: str = "msc64"  # "int8" | "msc64"

    def betas(self) -> np.ndarray:
        return linear_schedule(self.beta_final, self.n_steps)


# The named workloads.  Sizes follow the paper's runs (2D Ising, periodic,
# theta = 10 sweeps, beta from 0 up to or beyond beta_c).
def small_nearest(seed: int = PARITY_SEED, layout: str = "int8") -> RunSpec:
    """L=8, R=1000, beta 0 -> 0.44 in 101 steps, nearest-integer resampling."""
    return RunSpec(8, 1000, 10, seed, "nearest", 0.44, 101, layout)


def l64_multinomial(seed: int = PARITY_SEED, layout: str = "msc64") -> RunSpec:
    """L=64, R=100000, beta 0 -> 0.4407 in 200 steps, multinomial resampling."""
    return RunSpec(64, 100_000, 10, seed, "multinomial", 0.4407, 200, layout)


def l128_nearest(seed: int = PARITY_SEED) -> RunSpec:
    """L=128, R=100000, beta 0 -> 1.0 in 400 steps, multispin, nearest-integer."""
    return RunSpec(128, 100_000, 10, seed, "nearest", 1.0, 400, "msc64")


def batched_design(n_runs: int = 64, beta_final: float = 0.4407, n_steps: int = 200,
                   theta: int = 10, resample: str = "nearest",
                   layout: str = "msc64", draw_seed: Optional[int] = None) -> List[RunSpec]:
    """Independent runs of uneven size.

    By default a covering design: run m gets L = [16,32,64,128][m % 4] and
    R = [1000,5000,20000,50000][(m // 4) % 4], so each (L, R) pair appears
    n_runs / 16 times.  With draw_seed set, L and R are drawn uniformly from
    the same two sets with numpy's PCG64 seeded by draw_seed.
    """
    Ls = [16, 32, 64, 128]
    Rs = [1000, 5000, 20000, 50000]
    out = []
    rng = np.random.default_rng(draw_seed) if draw_seed is not None else None
    for m in range(n_runs):
        if rng is None:
            L, R = Ls[m % 4], Rs[(m // 4) % 4]
        else:
            L, R = int(rng.choice(Ls)), int(rng.choice(Rs))
        out.append(RunSpec(L, R, theta, run_seed(m), resample, beta_final, n_steps, layout))
    return out
