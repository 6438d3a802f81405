"""Unbiasedness of the oracle's partition-function estimate (no GPU).

After step i every replica carries the same weight, (1/Z_{beta_i}) times the
product of the normalisation factors Q_1 ... Q_i (Eq. resampling-weights):
resampling in proportion to tau_i(E_j) and the Metropolis sweeps at beta_i keep
the weighted population distributed as the Boltzmann distribution.  With
multinomial resampling the population stays at R replicas, and this makes the
product an unbiased estimate of Z_{beta_i}/Z_0 at any R:

    E[prod_k Q_k]                    = Z_{beta_i} / Z_0,
    E[prod_k Q_k * (1/R) sum_j e_j]  = (Z_{beta_i} / Z_0) <e>_{beta_i},

while its logarithm, the free-energy estimator (Eq. free-emergy-estimator),
lies below ln(Z_{beta_i}/Z_0) on average by about half the product's relative
variance.  At L = 4 the right-hand sides are exact (Kaufman's closed form), and
R = 8 makes that logarithmic bias large enough to be seen: the test requires
both.  One sweep per step keeps the sweeps from erasing a resampling mistake
before it reaches the estimate: selecting parents with 1.5 times the right
temperature step moves the mean of the product by about 6 standard errors here,
and sweeping at the previous temperature by far more.
"""
import concurrent.futures
import math
import multiprocessing

import numpy as np
import pytest

from oracle import exact
from oracle import pa_oracle as po
from workloads import linear_schedule

L, R, THETA, BETA_F, N_STEPS = 4, 8, 1, 0.4, 6
N_RUNS = 2000
SEED0 = 70_000


def _runs(seeds):
    """(sum_k ln Q_k, e of the last population) of one oracle run per seed."""
    betas = linear_schedule(BETA_F, N_STEPS)
    out = []
    for s in seeds:
        o = po.run(L, R, betas, THETA, s, "multinomial")
        assert all(r.R_i == R for r in o.records)
        out.append((sum(r.ln_Q for r in o.records[1:]), o.records[-1].e))
    return out


@pytest.mark.slow
@pytest.mark.timeout(300)
def test_product_of_q_is_unbiased_for_the_partition_function_ratio():
    po.build()
    seeds = list(range(SEED0, SEED0 + N_RUNS))
    chunks = [seeds[i::8] for i in range(8)]
    ctx = multiprocessing.get_context("spawn")
    with concurrent.futures.ProcessPoolExecutor(max_workers=8, mp_context=ctx) as ex:
        res = [x for part in ex.map(_runs, chunks) for x in part]
    ln_prod = np.array([a for a, _ in res])
    e_run = np.array([b for _, b in res])

    beta = linear_schedule(BETA_F, N_STEPS)[-1]
    ln_ratio = float(exact.ln_z_kaufman(L, beta)) - L * L * math.log(2)
    e_exact = float(exact.energy_per_spin(L, beta))
    w = np.exp(ln_prod - ln_ratio)  # prod Q_k / (Z_beta / Z_0)

    def z(x, target):
        return (x.mean() - target) / (x.std(ddof=1) / math.sqrt(len(x)))

    # the product: unbiased
    assert abs(z(w, 1.0)) < 4.0, (w.mean(), w.std(ddof=1))
    # the product times the population's energy: unbiased for (Z_beta/Z_0) e(beta)
    assert abs(z(w * e_run, e_exact)) < 4.0, ((w * e_run).mean(), e_exact)
    # its logarithm: biased low, by about half the relative variance of w
    z_ln = z(ln_prod, ln_ratio)
    assert z_ln < -5.0, (ln_prod.mean() - ln_ratio, z_ln)
    half_var = 0.5 * w.var(ddof=1)
    assert 0.5 * half_var < ln_ratio - ln_prod.mean() < 2.0 * half_var, (
        ln_ratio - ln_prod.mean(), half_var)
    # the weighted average over runs (Eq. weighted-averages with R^m = R)
    assert abs((w * e_run).sum() / w.sum() - e_exact) < 0.02
