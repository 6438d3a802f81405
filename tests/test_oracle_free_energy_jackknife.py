"""Pins of the oracle's single-run jackknife of the free-energy estimator
(Sec. "Conclusions", last guideline; Eq. free-emergy-estimator with Eqs.
jackknife-blocks, jackknife-variance and bias_covariance): a hand-worked case,
the thermodynamic-integration limit (Eq. var-delta-F: for a small step the
jackknife variance of ln Q is dbeta^2 times the jackknife variance of the
mean energy, which equals the blocked variance of Eq. blocked_variance when n
divides R), the sign of the covariance with the energy, degenerate steps and,
statistically, the spread of -beta F over independent runs."""
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from oracle import blocking as bk
from oracle import pa_oracle as po
from workloads import linear_schedule


def _boltz(E, dbeta):
    with mpmath.workprec(bk.PREC_BITS):
        return {int(e): mpmath.exp(-mpmath.mpf(dbeta) * int(e)) for e in set(int(x) for x in E)}


def _jk_after_one_step(E, dbeta, n, ln_z0=0):
    with mpmath.workprec(bk.PREC_BITS):
        return [mpmath.mpf(ln_z0) + q for q in bk.leave_one_block_out_ln_q(E, _boltz(E, dbeta), n)]


def test_hand_example():
    # parents E = 0, 0 | 4, 4 in two blocks, dbeta = ln 2 / 4: weights 1, 1, 1/2, 1/2;
    # without block 0, Q = 1/2; without block 1, Q = 1; so beta F^J = (ln 2, 0) - ln Z_0,
    # deviations +-ln 2 / 2 and sigma^2 = (1/2) (2 (ln 2)^2 / 4) = (ln 2)^2 / 4
    E = [0, 0, 4, 4]
    with mpmath.workprec(bk.PREC_BITS):
        db = mpmath.log(2) / 4
        lnq = bk.leave_one_block_out_ln_q(E, {0: mpmath.mpf(1), 4: mpmath.exp(-4 * db)}, 2)
        assert abs(lnq[0] - mpmath.log(mpmath.mpf(1) / 2)) < mpmath.mpf(2) ** -200
        assert abs(lnq[1]) < mpmath.mpf(2) ** -200
        jk = [mpmath.mpf(7) + q for q in lnq]
    # the record's population, two replicas in two blocks (L = 2 stands for N = 4
    # here): E = 0 | 4, so e^J = (4/N, 0) and
    # cov(e, beta F) = (1/2) [(2/N)(ln 2/2) + (-2/N)(-ln 2/2)] = ln 2 / N
    var, cov_e, cov_m, _, _ = bk.free_energy_errors(2, 0.3, [0, 4], [4, 0], jk, 2)
    assert var == pytest.approx(math.log(2) ** 2 / 4, rel=1e-15)
    assert cov_e == pytest.approx(math.log(2) / 4, rel=1e-15)
    # |M| = 4 | 0: m^J = (0, 4/N), cov(m, beta F) = -ln 2 / N
    assert cov_m == pytest.approx(-math.log(2) / 4, rel=1e-15)
    # a record population with another number of blocks has no covariances
    assert all(math.isnan(x) for x in bk.free_energy_errors(2, 0.3, E, E, jk, 2)[1:])


@pytest.mark.parametrize("R,n", [(1000, 100), (600, 50)])
def test_small_step_limit_is_the_variance_of_the_mean_energy(R, n):
    rng = np.random.default_rng(R)
    E = (4 * rng.integers(-40, 41, size=R) + 4 * np.repeat(rng.integers(-10, 11, size=n), R // n)).tolist()
    dbeta = 1e-7
    jk = _jk_after_one_step(E, dbeta, n)
    var = bk.free_energy_errors(4, 0.1, E, E, jk, n)[0]
    want = float(bk.blocked_variance_of_mean(E, n)) * dbeta ** 2
    assert var == pytest.approx(want, rel=1e-4)


def test_covariance_with_the_energy_has_the_sign_of_the_step():
    # a small step and the same population measured: beta F^J_k = -ln Z_0 + dbeta
    # mean_k^J(E) + O(dbeta^2), so cov(e, beta F) = dbeta N sigma_J^2(e)
    rng = np.random.default_rng(3)
    R, n, L = 1000, 100, 4
    N = L * L
    E = (4 * rng.integers(-8, 9, size=R)).tolist()
    M = (2 * rng.integers(-8, 9, size=R)).tolist()
    for dbeta in (1e-6, -1e-6):
        jk = _jk_after_one_step(E, dbeta, n, ln_z0=N * math.log(2))
        _, cov_e, _, _, _ = bk.free_energy_errors(L, 0.2, E, M, jk, n)
        var_e = float(bk.blocked_variance_of_mean(E, n)) / N ** 2
        assert cov_e == pytest.approx(dbeta * N * var_e, rel=1e-4)


def test_degenerate_steps_have_no_spread():
    E = [0, 4, -4, 8] * 50
    assert bk.free_energy_errors(4, 0.1, E, E, _jk_after_one_step(E, 0.0, 100), 100)[0] == 0.0
    Ec = [12] * 200
    assert bk.free_energy_errors(4, 0.1, Ec, Ec, _jk_after_one_step(Ec, 0.3, 100), 100)[0] == 0.0


def test_empty_and_whole_blocks():
    with mpmath.workprec(bk.PREC_BITS):
        q = bk.leave_one_block_out_ln_q([0, 4, 8], _boltz([0, 4, 8], 0.1), 5)
        full = mpmath.log(mpmath.fsum(mpmath.exp(-mpmath.mpf(0.1) * e) for e in (0, 4, 8)) / 3)
        # three parents in five blocks: blocks 0 and 2 are empty (slots [0, 0), [1, 1))
        assert [k for k in range(5) if abs(q[k] - full) < mpmath.mpf(2) ** -200] == [0, 2]
        assert mpmath.isnan(bk.leave_one_block_out_ln_q([0], _boltz([0], 0.1), 2)[1])
    assert all(math.isnan(x) for x in bk.free_energy_errors(4, 0.1, [0], [0], [mpmath.nan, 1], 2))
    assert all(math.isnan(x) for x in bk.free_energy_errors(4, 0.1, [0], [0], [1], 1))


def test_whole_run_jackknife_matches_the_spread_over_runs():
    # independent runs of L = 4, R = 1000, beta 0 -> 0.35 in 7 steps, theta = 5:
    # the mean single-run jackknife variance of beta F agrees with the sample
    # variance of beta F over the runs (relative standard error sqrt(2 / 39) of
    # the latter, 0.23)
    L, R, steps = 4, 1000, 7
    betas = linear_schedule(0.35, steps)
    fs, jvar = [], []
    for seed in range(40):
        o = po.run(L, R, betas, 5, 100 + seed)
        fs.append(-o.records[-1].minus_beta_F)
        jvar.append(o.records[-1].jk_var_beta_F)
    ratio = np.mean(jvar) / np.var(fs, ddof=1)
    assert 0.5 < ratio < 2.0, ratio
