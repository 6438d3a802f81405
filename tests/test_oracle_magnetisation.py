"""Pins of the magnetisation observables (Sec. "Model and observables": m =
<|M|>/N, chi = beta N (<m^2> - <|m|>^2) with m = M/N) against the exact joint
density of states g(E, M) of the L = 4 torus.

The exact side is independent of the oracle's observables: g(E, M) comes from
brute-force enumeration and, separately, from a transfer matrix that carries
the magnetisation; both are checked against closed forms (binomial marginal
in M, g(E) of Kaufman-pinned enumeration, the beta = 0 moments).  Whole
population-annealing runs of the oracle at L = 4 must then reproduce m and
chi within their own statistical errors, and the same check must reject the
three plausible misreadings planted below (beta^2 in chi, M for |M|, a wrong
power of N).
"""
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from oracle import exact as ex
from oracle import pa_oracle as po
from workloads import linear_schedule

L = 4
N = L * L


@pytest.fixture(scope="module")
def g2():
    return ex.joint_dos_enumeration(L)


def test_joint_dos_two_routes_agree(g2):
    assert ex.joint_dos_transfer(L) == g2
    assert sum(g2.values()) == 2 ** N


def test_joint_dos_marginals_and_symmetry(g2):
    # marginal in E is the Kaufman-pinned g(E); marginal in M is binomial
    gE, gM = {}, {}
    for (e, m), c in g2.items():
        gE[e] = gE.get(e, 0) + c
        gM[m] = gM.get(m, 0) + c
        assert g2.get((e, -m)) == c  # spin-flip symmetry
    assert gE == ex.dos_enumeration(L)
    assert gM == {2 * k - N: math.comb(N, k) for k in range(N + 1)}


def test_moments_at_infinite_temperature(g2):
    # independent +-1 spins: <M^2> = N and <|M|> = sum_k C(N, k) |N - 2k| / 2^N
    abs_m, m2 = ex.magnetisation_moments(g2, 0)
    assert abs(m2 - N) < mpmath.mpf(10) ** -60
    want = Fraction(sum(math.comb(N, k) * abs(N - 2 * k) for k in range(N + 1)), 2 ** N)
    assert abs(abs_m - mpmath.mpf(want.numerator) / want.denominator) < mpmath.mpf(10) ** -60
    assert ex.susceptibility(L, g2, 0) == 0


def test_ordered_limit(g2):
    # deep in the ordered phase only the two ground states remain
    assert abs(ex.magnetisation_per_spin(L, g2, 20) - 1) < 1e-30
    assert abs(ex.susceptibility(L, g2, 20)) < 1e-30


# --------------------------------------------------------------- whole runs

def _observables(variant, beta, E, M):
    """m and chi of one population: the oracle's, or a planted misreading."""
    if variant == "oracle":
        _, (_, _, m, chi) = po.observables(L, beta, E, M)
        return m, chi
    E = E.astype(np.int64)
    M = M.astype(np.int64)
    R = len(M)
    A = np.abs(M)
    if variant == "beta_squared":
        m = A.sum() / (N * R)
        return m, beta * beta * ((M * M).sum() / R - (A.sum() / R) ** 2) / N
    if variant == "signed_M":
        return M.sum() / (N * R), beta * ((M * M).sum() / R - (M.sum() / R) ** 2) / N
    if variant == "n_squared":
        return A.sum() / (N * N * R), beta * ((M * M).sum() / R - (A.sum() / R) ** 2) / (N * N)
    raise ValueError(variant)


@pytest.fixture(scope="module")
def runs():
    """Two L = 4 runs, R = 4000, theta = 10, beta 0 -> 0.5 in 10 steps, with the
    population (E, M) and the single-run error bars of every record."""
    out = []
    for seed in (11, 12):
        o = po.OracleRun(L, 4000, 10, seed, "nearest", linear_schedule(0.5, 10))
        steps = []
        for _ in range(10):
            rec = o.anneal_step()
            steps.append((rec.beta, o.E.copy(), o.M.copy(), rec.err_m, rec.err_chi))
        out.append(steps)
    return out


def _max_z(runs, g2, variant):
    z = 0.0
    for steps in runs:
        for beta, E, M, err_m, err_chi in steps:
            m, chi = _observables(variant, beta, E, M)
            z = max(z, abs(m - float(ex.magnetisation_per_spin(L, g2, beta))) / err_m,
                    abs(chi - float(ex.susceptibility(L, g2, beta))) / err_chi)
    return z


def test_runs_reproduce_exact_m_and_chi(runs, g2):
    assert _max_z(runs, g2, "oracle") < 5.0


@pytest.mark.parametrize("variant", ["beta_squared", "signed_M", "n_squared"])
def test_planted_misreadings_are_rejected(runs, g2, variant):
    assert _max_z(runs, g2, variant) > 10.0
