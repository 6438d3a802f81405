"""Adaptive and learned temperature schedules over libpa.

Every decision runs on the device (pa_anneal_step_adaptive / _learned choose
beta_i from the population's histogram without a host round trip); this
module only enqueues steps, detects the end of the schedule and moves the
logged training rows between device tensors.

* Adaptive: each step is the largest dbeta keeping the energy-histogram
  overlap alpha(beta_{i-1}, beta_i) >= alpha_target (self-adaptive steps, Sec.
  "Algorithm"; the paper's runs use alpha = 0.9, with 0.7 as a lower guide).
* Learned: a 35 -> 64 -> 64 -> 1 perceptron proposes log(dbeta sigma_E) from
  the histogram features; a proposal is taken only if its overlap is at least
  alpha_min, otherwise the adaptive step is used.
"""
from __future__ import annotations

from typing import List, Optional, Tuple

import numpy as np

from . import PA_ERR_DONE, PA_MLP_IN, PA_MLP_PARAMS, PAError, Run, mlp_train_step


def _step_until_done(run: Run, enqueue, chunk: int = 32) -> int:
    """Enqueue steps in chunks until the device reports the end of the schedule."""
    while True:
        for _ in range(chunk):
            try:
                enqueue()
            except PAError as e:
                if e.status != PA_ERR_DONE:
                    raise
                break
        try:
            run.sync()
        except PAError as e:
            if e.status != PA_ERR_DONE:
                raise
            return run.current()[0]
        step, _ = run.current()
        if step >= run.max_steps:
            return step


def adaptive_run(L: int, R: int, theta: int, seed: int, alpha: float, beta_final: float,
                 max_steps: int = 4000, resample: str = "nearest", layout: str = "msc64",
                 stream=None) -> Run:
    run = Run(L, R, None, theta, seed, resample, layout, n_steps=max_steps, stream=stream)
    _step_until_done(run, lambda: run.anneal_step_adaptive(alpha, beta_final))
    return run


def learned_run(params, L: int, R: int, theta: int, seed: int, alpha_min: float,
                alpha_target: float, beta_final: float, max_steps: int = 4000,
                resample: str = "nearest", layout: str = "msc64", stream=None) -> Run:
    run = Run(L, R, None, theta, seed, resample, layout, n_steps=max_steps, stream=stream)
    _step_until_done(run, lambda: run.anneal_step_learned(params, alpha_min, alpha_target,
                                                          beta_final))
    return run


def training_rows(run: Run, device: str = "cuda:0"):
    """(X [n, 35], t [n]) device tensors from a run's schedule log (NaN rows dropped)."""
    import torch
    n, _, _ = run.schedule_log()
    X = torch.zeros((max(n, 1), PA_MLP_IN), dtype=torch.float32, device=device)
    t = torch.zeros(max(n, 1), dtype=torch.float32, device=device)
    run.schedule_log(X, t)
    keep = torch.isfinite(t[:n])
    return X[:n][keep].contiguous(), t[:n][keep].contiguous()


def init_params(seed: int, device: str = "cuda:0"):
    """Uniform(+-1/sqrt(fan_in)) weights, zero biases (FP32, on the device)."""
    import torch
    g = torch.Generator().manual_seed(seed)
    p = torch.zeros(PA_MLP_PARAMS, dtype=torch.float32)
    o = 0
    p[o:o + 64 * 35] = (torch.rand(64 * 35, generator=g) * 2 - 1) / np.sqrt(35.0)
    o += 64 * 35 + 64
    p[o:o + 64 * 64] = (torch.rand(64 * 64, generator=g) * 2 - 1) / np.sqrt(64.0)
    o += 64 * 64 + 64
    p[o:o + 64] = (torch.rand(64, generator=g) * 2 - 1) / np.sqrt(64.0)
    return p.to(device)


def train(X, t, iters: int = 3000, lr: float = 3e-3, seed: int = 0,
          params=None) -> Tuple["object", List[float]]:
    """Full-batch Adam on the device (pa_mlp_train_step); returns params and losses."""
    import torch
    if params is None:
        params = init_params(seed, X.device)
    adam = torch.zeros(2 * PA_MLP_PARAMS, dtype=torch.float32, device=X.device)
    loss = torch.zeros(1, dtype=torch.float32, device=X.device)
    losses = []
    for k in range(1, iters + 1):
        mlp_train_step(params, adam, X, t, lr, k, loss)
        if k % 100 == 0 or k == 1:
            losses.append(float(loss.item()))
    return params, losses
