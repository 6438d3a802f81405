"""Pins of the oracle's Poisson resampling (Sec. "Algorithm": r_j ~
Poisson(tau_hat_j), Eq. taus): inversion against scipy's Poisson CDF, the
zero-mean case, copy frequencies against the Poisson pmf, and whole runs whose
population size fluctuates about R."""
import math

import mpmath
import numpy as np
import pytest
from scipy import stats

from oracle import pa_oracle as po
from workloads import linear_schedule


def test_inversion_matches_scipy_cdf():
    rng = np.random.default_rng(11)
    checked = 0
    with mpmath.workprec(po.PREC_BITS):
        for _ in range(400):
            lam = float(rng.uniform(0.01, 12.0))
            U = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
            u = U / 2.0**64
            k = po.poisson_inverse(mpmath.mpf(lam), U)
            cdf = stats.poisson.cdf(np.arange(k + 2), lam)
            # scipy works in binary64: skip draws within its rounding of a CDF value
            if np.min(np.abs(cdf - u)) < 1e-12:
                continue
            want = int(np.argmax(cdf > u))
            assert k == want, (lam, U, k, want)
            checked += 1
    assert checked > 350


def test_zero_mean_gives_no_copies():
    with mpmath.workprec(po.PREC_BITS):
        for U in (0, 1, 2**63, 2**64 - 1):
            assert po.poisson_inverse(mpmath.mpf(0), U) == 0


@pytest.mark.parametrize("lam", [0.3, 1.0, 2.7])
def test_copy_frequencies_follow_the_poisson_pmf(lam):
    rng = np.random.default_rng(int(lam * 100))
    n = 20000
    with mpmath.workprec(po.PREC_BITS):
        ks = [po.poisson_inverse(mpmath.mpf(lam), int(rng.integers(0, 2**63)) * 2 + 1)
              for _ in range(n)]
    kmax = max(ks)
    obs = np.bincount(ks, minlength=kmax + 1).astype(float)
    exp = stats.poisson.pmf(np.arange(kmax + 1), lam) * n
    exp[-1] += stats.poisson.sf(kmax, lam) * n
    # pool the sparse tail
    keep = exp >= 5
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    if e[-1] < 5:
        o[-2] += o[-1]
        e[-2] += e[-1]
        o, e = o[:-1], e[:-1]
    chi2 = float(((o - e) ** 2 / e).sum())
    assert stats.chi2.sf(chi2, len(o) - 1) > 1e-4


def test_population_size_fluctuates_about_R():
    # sum_j tau_hat_j = R exactly, so E[R_i] = R and Var(R_i) = R
    R = 2000
    o = po.run(8, R, linear_schedule(0.45, 12), 1, 41, "poisson")
    sizes = np.array([r.R_i for r in o.records[1:]])
    assert np.all(np.abs(sizes - R) < 6 * math.sqrt(R))
    assert 0 < sizes.std() < 3 * math.sqrt(R)
    # the copy counts of each step add up to that step's population
    assert int(o.last_counts.sum()) == o.records[-1].R_i


def test_extinction_exactly_when_every_draw_falls_below_exp_minus_tau():
    # a parent makes no copy iff U_j < 2^64 e^{-tau_hat_j} (F(0) = e^{-lam});
    # with R = 2 this happens to both parents at the first step for some
    # seeds, and the run then stops with PopulationExtinct
    L, R, b1 = 4, 2, 0.3
    extinct = survived = 0
    for seed in range(40):
        o = po.OracleRun(L, R, 1, seed, "poisson", betas=[0.0, b1])
        E = o.E.astype(int)
        with mpmath.workprec(po.PREC_BITS):
            w = [mpmath.exp(-mpmath.mpf(b1) * int(e)) for e in E]
            tau_hat = [R * x / mpmath.fsum(w) for x in w]
            zero = [po.poisson_uniform(seed, 1, j) < mpmath.ldexp(mpmath.exp(-t), 64)
                    for j, t in enumerate(tau_hat)]
        if all(zero):
            with pytest.raises(po.PopulationExtinct):
                o.anneal_step()
            extinct += 1
        else:
            rec = o.anneal_step()
            assert rec.R_i > 0
            assert [c == 0 for c in o.last_counts] == zero
            survived += 1
    assert extinct > 0 and survived > 0
