"""Pins of the oracle's blocking / jackknife analysis (Sec. "Effective
population size", Eqs. blocks, blocked_variance, neff, jackknife-blocks,
jackknife-variance; Sec. "Statistical errors") against hand-computed values,
algebraic identities, closed forms and brute force."""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

from oracle import blocking as bk


def test_hand_example():
    # values 1 2 | 3 5 | 4 9 in n = 3 blocks: block means 3/2, 4, 13/2 with
    # mean 4, squared deviations 25/4 + 0 + 25/4 = 25/2, so the blocked
    # variance of the mean is (25/2) / (3 * 2) = 25/12; the unblocked values
    # have mean 4 and sum of squared deviations 9 + 4 + 1 + 1 + 0 + 25 = 40,
    # variance 40 / 5 = 8; R_eff = 8 / (25/12) = 96/25
    v = [1, 2, 3, 5, 4, 9]
    assert bk.blocked_variance_of_mean(v, 3) == Fraction(25, 12)
    assert bk.variance(v) == 8
    assert bk.r_eff(v, 3) == float(Fraction(96, 25))


@pytest.mark.parametrize("R,n", [(12, 4), (300, 100), (1000, 10), (7, 7)])
def test_jackknife_of_the_mean_equals_the_blocked_variance(R, n):
    # for equal blocks, mean_k^J - mean^J = -(m_k - mbar) / (n - 1), so the two
    # estimators of the variance of the mean coincide exactly
    rng = random.Random(R * 31 + n)
    v = [rng.randint(-50, 50) for _ in range(R)]
    jack = bk.jackknife_variance([v], lambda m: m, n)
    assert jack == bk.blocked_variance_of_mean(v, n)


@pytest.mark.parametrize("n,B", [(10, 5), (100, 3), (4, 25)])
def test_values_constant_within_blocks(n, B):
    # n independent values each repeated B times: sigma^2(O) = B S / (R - 1),
    # sigma^2(mean) = S / (n (n - 1)) with S the scatter of the block values,
    # so R_eff = B n (n - 1) / (R - 1) = R (n - 1) / (R - 1) ~ n
    rng = random.Random(n * 1000 + B)
    vals = [rng.randint(-1000, 1000) for _ in range(n)]
    v = [x for x in vals for _ in range(B)]
    R = n * B
    assert bk.r_eff(v, n) == float(Fraction(R * (n - 1), R - 1))


def _cv_direct(E, beta, N):
    E = np.asarray(E, dtype=np.int64)
    m1 = Fraction(int(E.sum()), len(E))
    m2 = Fraction(int((E * E).sum()), len(E))
    return Fraction(beta) ** 2 * (m2 - m1 * m1) / N


@pytest.mark.parametrize("R", [50, 103, 400])
def test_jackknife_specific_heat_by_brute_force(R):
    # leave each block out, recompute C_V from the remaining raw values, and
    # apply the jackknife variance formula
    rng = np.random.default_rng(R)
    L, beta = 4, 0.37
    N = L * L
    E = rng.integers(-2 * N, 2 * N + 1, R)
    M = rng.integers(-N, N + 1, R)
    n = bk.n_blocks(R)
    fk = []
    for lo, hi in bk.block_bounds(R, n):
        keep = np.concatenate([E[:lo], E[hi:]])
        fk.append(_cv_direct(keep, beta, N))
    fbar = sum(fk) / n
    want = math.sqrt(float(Fraction(n - 1, n) * sum((f - fbar) ** 2 for f in fk)))
    got = bk.population_errors(L, beta, E, M)[4]
    assert got == want
    # chi the same way from |M|
    A = np.abs(M)
    fk = []
    for lo, hi in bk.block_bounds(R, n):
        keep = np.concatenate([A[:lo], A[hi:]])
        m1 = Fraction(int(keep.sum()), len(keep))
        m2 = Fraction(int((keep * keep).sum()), len(keep))
        fk.append(Fraction(beta) * (m2 - m1 * m1) / N)
    fbar = sum(fk) / n
    want = math.sqrt(float(Fraction(n - 1, n) * sum((f - fbar) ** 2 for f in fk)))
    assert bk.population_errors(L, beta, E, M)[5] == want


@pytest.mark.parametrize("R", [1, 2, 99, 100, 101, 1000, 100003])
def test_blocks_partition_the_population(R):
    n = bk.n_blocks(R)
    b = bk.block_bounds(R, n)
    assert b[0][0] == 0 and b[-1][1] == R
    assert all(b[k][1] == b[k + 1][0] for k in range(n - 1))
    sizes = [hi - lo for lo, hi in b]
    assert max(sizes) - min(sizes) <= 1 and min(sizes) >= 1


def test_degenerate_populations():
    assert all(math.isnan(x) for x in bk.population_errors(4, 0.3, [5], [2]))
    # equal block means with varying values: zero blocked variance
    assert bk.r_eff([1, 2, 2, 1], 2) == math.inf
    assert math.isnan(bk.r_eff([3, 3, 3, 3], 2))
    # beta = 0: no specific heat or susceptibility, so no error on them
    r = bk.population_errors(4, 0.0, [1, 5, -3, 8, 2], [4, -2, 0, 6, 2])
    assert r[4] == 0.0 and r[5] == 0.0


def test_uncorrelated_values_have_r_eff_near_r():
    # i.i.d. values: the blocked variance estimates sigma^2 / R from n - 1 = 99
    # degrees of freedom (relative spread about 0.14)
    rng = np.random.default_rng(7)
    R = 20000
    v = rng.integers(-100, 101, R).tolist()
    ratio = bk.r_eff(v, 100) / R
    assert 0.55 < ratio < 1.6
    # and a population of B adjacent copies of independent values has about R / B
    B = 20
    w = [x for x in rng.integers(-100, 101, R // B).tolist() for _ in range(B)]
    assert 0.55 < bk.r_eff(w, 100) / (R / B) < 1.6
