"""Pins for the oracle's reweighting and resampling step (no GPU).

Checked against special cases with closed forms (dbeta = 0, a single energy
level), against the defining expectations of the copy-count rules (mean copies
= tau_hat; variance of R_i; multinomial frequencies) and against an
independent binary64 evaluation of Eq. (Q).
"""
import math

import numpy as np
import pytest

from oracle import pa_oracle as po


def _population(L=6, R=300, seed=5, theta=0):
    o = po.OracleRun(L, R, theta, seed, "nearest")
    return o


def test_zero_step_is_the_identity():
    o = _population()
    counts, ln_q = o.copy_counts(0.0, 0.0, 1)
    assert ln_q == 0
    assert np.array_equal(counts, np.ones(len(o.E), dtype=np.int32))


def test_single_level_population_has_q_equal_boltzmann_factor():
    L, R = 6, 70
    o = po.OracleRun(L, R, 0, 1, "nearest")
    o.set_population(0, np.ones((R, L * L), dtype=np.int8), np.arange(R), 0.0)
    for db in (0.01, 0.3):
        counts, ln_q = o.copy_counts(0.0, db, 1)
        assert abs(float(ln_q) - db * 2 * L * L) < 1e-12  # ln Q = -dbeta E, E = -2N
        assert np.all(counts == 1)


def test_log_q_matches_binary64_logsumexp():
    o = _population(R=500)
    E = o.E.astype(np.float64)
    for db in (0.001, 0.02, 0.2):
        _, ln_q = o.copy_counts(0.1, 0.1 + db, 2)
        dbe = (0.1 + db) - 0.1
        a = -dbe * E
        ref = a.max() + math.log(np.exp(a - a.max()).sum()) - math.log(len(E))
        assert abs(float(ln_q) - ref) <= 1e-12 * max(1.0, abs(ref))


def _tau_hat(o, db):
    E = o.E.astype(np.float64)
    w = np.exp(-db * (E - E.min()))
    return o.R * w / w.sum()


def test_nearest_counts_are_floor_or_ceil_with_mean_tau_hat():
    o = _population(R=400)
    db = 0.05
    tau = _tau_hat(o, db)
    K = 300
    acc = np.zeros(len(tau))
    totals = []
    for step in range(1, K + 1):
        c, _ = o.copy_counts(0.2, 0.2 + db, step)
        assert np.all((c == np.floor(tau)) | (c == np.floor(tau) + 1))
        acc += c
        totals.append(c.sum())
    frac = tau - np.floor(tau)
    sigma = np.sqrt(np.maximum(frac * (1 - frac), 1e-12) / K)
    z = (acc / K - tau) / sigma
    assert np.max(np.abs(z)) < 5.5
    # R_i = sum of independent Bernoulli-shifted counts: Var(R_i) = sum frac (1 - frac)
    var_expected = (frac * (1 - frac)).sum()
    var = np.var(totals, ddof=1)
    assert abs(np.mean(totals) - tau.sum()) < 5 * math.sqrt(var_expected / K)
    assert 0.7 * var_expected < var < 1.4 * var_expected


def test_multinomial_keeps_size_and_frequencies():
    o = po.OracleRun(6, 300, 0, 8, "multinomial")
    db = 0.05
    p = _tau_hat(o, db) / o.R
    K = 150
    acc = np.zeros(len(p))
    for step in range(1, K + 1):
        c, _ = o.copy_counts(0.3, 0.3 + db, step)
        assert c.sum() == o.R
        acc += c
    expected = K * o.R * p
    # group parents by energy level to get well-populated cells for a chi^2
    chi2, dof = 0.0, 0
    for e in np.unique(o.E):
        sel = o.E == e
        n_exp = expected[sel].sum()
        if n_exp < 30:
            continue
        chi2 += (acc[sel].sum() - n_exp) ** 2 / n_exp
        dof += 1
    assert chi2 < dof + 5 * math.sqrt(2 * dof) + 10, (chi2, dof)


def test_counts_depend_only_on_energy_level_and_uniform():
    # two parents with equal energy and equal uniforms get equal counts: the
    # rule is a function of (tau_hat(E_j), u_j)
    o = _population(R=256)
    c, _ = o.copy_counts(0.1, 0.15, 3)
    tau = _tau_hat(o, 0.05)
    for j in range(len(c)):
        u = po.resample_uniform(o.seed, 3, j) / 2 ** 32
        fl = math.floor(tau[j])
        if abs((tau[j] - fl) - u) > 1e-9:
            assert c[j] == fl + (1 if u < tau[j] - fl else 0)


@pytest.mark.parametrize("beta_prev,beta_next", [(0.0, 0.37), (0.2, 0.2), (0.31, 0.9)])
def test_one_parent_nearest_count_matches_the_whole_population_rule(beta_prev, beta_next):
    # nearest_count (one parent, from the level counts) against copy_counts
    # (every parent, replica by replica) on the same population and uniforms;
    # the second case is a zero step, whose counts are all one
    o = _population(L=6, R=300, seed=11, theta=2)
    counts, _ = o.copy_counts(beta_prev, beta_next, 3)
    values, mult = np.unique(o.E, return_counts=True)
    levels = {int(e): int(n) for e, n in zip(values, mult)}
    got = [po.nearest_count(o.seed, 3, o.R, levels, beta_prev, beta_next, int(o.E[j]), j)
           for j in range(len(o.E))]
    assert np.array_equal(np.array(got, dtype=np.int32), counts)
    # a population on a single level: tau_hat = R / R_{i-1} whatever dbeta is
    one = {-72: 40}
    assert all(po.nearest_count(7, 2, 40, one, 0.1, 0.5, -72, j) == 1 for j in range(40))
