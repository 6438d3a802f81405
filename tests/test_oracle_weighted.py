"""Pins of the oracle's weighted averages over independent runs (Sec.
"Weighted averages", Eqs. weighted-averages, modified-weights2) and of the
bias estimate (Sec. "Bias with resampling", Eqs. bias_covariance, rho_f):
closed-form weights, invariances, the fixed-size special case, hand-computed
covariances, and a statistical check on whole oracle runs."""
import math
from fractions import Fraction
from types import SimpleNamespace

import numpy as np
import pytest

from oracle import pa_oracle as po
from oracle import weighted as wt


def rec(R_i, sum_E, sum_E2, sum_absM, sum_M2, mbf, beta=0.3, step=1):
    return SimpleNamespace(step=step, beta=beta, R_i=R_i, sum_E=sum_E, sum_E2=sum_E2,
                           sum_absM=sum_absM, sum_M2=sum_M2, minus_beta_F=mbf)


def hist(*recs):
    """A run whose records at steps 0..len-1 are recs (only R_i of earlier steps matter)."""
    return list(recs)


L = 4
N = 16


def test_equal_free_energies_and_sizes_give_the_plain_average():
    r1 = rec(10, -100, 1200, 40, 200, 20.5)
    r2 = rec(10, -60, 500, 20, 60, 20.5)
    out = wt.weighted_averages(L, [hist(r1, r1), hist(r2, r2)], [10, 10], 1)
    for k in ("e", "m", "c_v", "chi"):
        assert out[k] == pytest.approx(out[k + "_plain"], rel=1e-15)
    assert out["omega_max"] == 0.5 and out["n_eff_runs"] == pytest.approx(2.0, rel=1e-15)
    # the plain average combines the moments: <E> = (-10 - 6)/2, <E^2> = (120 + 50)/2
    E1, E2 = Fraction(-8), Fraction(85)
    assert out["e_plain"] == float(E1 / N)
    assert out["c_v_plain"] == float(Fraction(0.3) ** 2 * (E2 - E1 * E1) / N)


def test_weights_follow_exp_minus_beta_F_times_R():
    # -beta F differs by ln 3: weights 3/4 and 1/4; a run twice the size with
    # equal -beta F gets twice the weight (each replica counts the same)
    r1 = rec(10, -100, 1200, 40, 200, 20.0 + math.log(3))
    r2 = rec(10, -60, 500, 20, 60, 20.0)
    out = wt.weighted_averages(L, [hist(r1, r1), hist(r2, r2)], [10, 10], 1)
    assert out["e"] == pytest.approx((0.75 * -10 + 0.25 * -6) / N, rel=1e-14)
    assert out["omega_max"] == pytest.approx(0.75, rel=1e-14)
    r3 = rec(20, -200, 2400, 80, 400, 20.0)
    out = wt.weighted_averages(L, [hist(r2, r2), hist(r3, r3)], [10, 20], 1)
    assert out["omega_max"] == pytest.approx(2 / 3, rel=1e-14)
    assert out["e"] == pytest.approx((-6 / 3 + 2 * -10 / 3) / N, rel=1e-14)


def test_shift_of_every_free_energy_changes_nothing():
    a = [hist(rec(12, -50, 900, 30, 150, 7.0), rec(12, -50, 900, 30, 150, 7.0)),
         hist(rec(9, -40, 300, 27, 90, 6.2), rec(9, -40, 300, 27, 90, 6.2)),
         hist(rec(11, -70, 600, 11, 41, 7.9), rec(11, -70, 600, 11, 41, 7.9))]
    b = [[rec(r.R_i, r.sum_E, r.sum_E2, r.sum_absM, r.sum_M2, r.minus_beta_F + 300.0) for r in run]
         for run in a]
    oa = wt.weighted_averages(L, a, [12, 9, 11], 1)
    ob = wt.weighted_averages(L, b, [12, 9, 11], 1)
    for k in ("e", "m", "c_v", "chi", "e_mod", "omega_max"):
        assert oa[k] == pytest.approx(ob[k], rel=1e-13)
    # variances and covariances of beta F do not move with a constant either
    for k in ("var_beta_F", "cov_e", "cov_chi"):
        assert oa[k] == pytest.approx(ob[k], rel=1e-12)


def test_fixed_population_size_makes_the_modified_weights_equal():
    # R_{k-1} = R for every k: the extra factor of Eq. (modified-weights2) is 1
    runs = []
    for m, (R, x) in enumerate(((50, 30.1), (80, 29.7), (50, 30.4))):
        r = rec(R, -40 * R // 10, 100 * R, 3 * R, 12 * R, x, step=3)
        runs.append([rec(R, 0, 0, 0, 0, 0.0, step=k) for k in range(3)] + [r])
    out = wt.weighted_averages(L, runs, [50, 80, 50], 3)
    for k in ("e", "m", "c_v", "chi"):
        assert out[k + "_mod"] == pytest.approx(out[k], rel=1e-15)


def test_modified_weights_by_hand():
    # run 1: nominal 100, sizes R_0 = 100, R_1 = 110 before step 2, R_2 = 90:
    # factor (100/100)(110/100) = 1.1 -> weight 90 * 1.1 e^x; run 2 fixed at 100
    x = 12.0
    run1 = [rec(100, 0, 0, 0, 0, 0.0, step=0), rec(110, 0, 0, 0, 0, 0.0, step=1),
            rec(90, -900, 9900, 450, 2700, x, step=2)]
    run2 = [rec(100, 0, 0, 0, 0, 0.0, step=0), rec(100, 0, 0, 0, 0, 0.0, step=1),
            rec(100, -500, 3000, 100, 300, x, step=2)]
    out = wt.weighted_averages(L, [run1, run2], [100, 100], 2)
    w1 = 90 * 1.1 / (90 * 1.1 + 100)
    assert out["e_mod"] == pytest.approx((w1 * -10 + (1 - w1) * -5) / N, rel=1e-14)
    w1s = 90 / 190
    assert out["e"] == pytest.approx((w1s * -10 + (1 - w1s) * -5) / N, rel=1e-14)


def test_covariance_and_rho_f_by_hand():
    # three runs with e = -1/16, -2/16, -3/16 (sum_E / (R N)) and beta F =
    # -x = 1, 2, 4: cov = sum (e - ebar)(F - Fbar) / 2 with ebar = -2/16,
    # Fbar = 7/3: ((1/16)(-4/3) + 0 + (-1/16)(5/3)) / 2 = -9/96
    runs, Rs = [], [10, 10, 10]
    for E, F in ((-1, 1.0), (-2, 2.0), (-3, 4.0)):
        r = rec(10, 10 * E, 10 * E * E, 0, 0, -F)
        runs.append([r, r])
    out = wt.weighted_averages(L, runs, Rs, 1)
    assert out["cov_e"] == pytest.approx(-9 / 96, rel=1e-14)
    var = ((1 - 7 / 3) ** 2 + (2 - 7 / 3) ** 2 + (4 - 7 / 3) ** 2) / 2
    assert out["var_beta_F"] == pytest.approx(var, rel=1e-14)
    assert out["rho_f"] == pytest.approx(10 * var, rel=1e-14)
    # every run with E fixed: no specific heat in any run, so no covariance
    assert out["cov_c_v"] == 0.0


def test_one_run_and_identical_runs():
    r = rec(10, -100, 1200, 40, 200, 20.5)
    one = wt.weighted_averages(L, [[r, r]], [10], 1)
    assert one["e"] == one["e_plain"] == -10 / N
    assert math.isnan(one["var_beta_F"]) and math.isnan(one["cov_e"])
    many = wt.weighted_averages(L, [[r, r]] * 5, [10] * 5, 1)
    assert many["e"] == pytest.approx(-10 / N, rel=1e-15)
    assert many["var_beta_F"] == 0.0 and many["cov_m"] == 0.0
    assert many["n_eff_runs"] == pytest.approx(5.0, rel=1e-14)


def test_whole_runs_weighted_energy_near_exact():
    # 12 independent Metropolis runs at L=4, R=40: the weighted and plain
    # energies at beta = 0.5 both lie within a few standard errors of the
    # exact value; omega sums to one by construction, n_eff_runs <= 12
    from oracle import exact
    from workloads import linear_schedule
    betas = linear_schedule(0.5, 10)
    runs = [po.run(4, 40, betas, 2, 300 + k, "nearest") for k in range(12)]
    out = wt.weighted_averages(4, [r.records for r in runs], [40] * 12, 10)
    ex = float(exact.energy_per_spin(4, 0.5))
    es = np.array([r.records[10].e for r in runs])
    se = es.std(ddof=1) / math.sqrt(len(es))
    assert abs(out["e_plain"] - ex) < 5 * se + 0.02
    assert abs(out["e"] - ex) < 5 * se + 0.02
    assert 1.0 <= out["n_eff_runs"] <= 12.0
