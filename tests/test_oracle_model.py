"""Pins for the oracle's model and Metropolis update (no GPU).

The local update rule is checked against brute-force energy differences, the
thresholds against closed forms, and a chain of sweeps against the exact
Boltzmann distribution of the L = 4 lattice.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import exact
from oracle import pa_oracle as po


def test_energy_of_special_configurations():
    L, N = 6, 36
    up = np.ones((1, N), dtype=np.int8)
    E, M = po.energy_magnetisation(L, up)
    assert (E[0], M[0]) == (-2 * N, N)
    chk = np.array([[1 if (x + y) % 2 == 0 else -1 for y in range(L) for x in range(L)]], dtype=np.int8)
    E, M = po.energy_magnetisation(L, chk)
    assert (E[0], M[0]) == (2 * N, 0)


def test_delta_energy_matches_brute_force_for_all_local_configurations():
    L = 4
    rng = np.random.default_rng(3)
    x0, y0 = 1, 2
    nbrs = [(x0 + 1, y0), (x0 - 1, y0), (x0, y0 + 1), (x0, y0 - 1)]
    for s0, *ns in itertools.product((-1, 1), repeat=5):
        lat = rng.choice([-1, 1], size=(L, L)).astype(np.int8)
        lat[y0, x0] = s0
        for (x, y), v in zip(nbrs, ns):
            lat[y % L, x % L] = v
        flipped = lat.copy()
        flipped[y0, x0] = -s0
        E, _ = po.energy_magnetisation(L, np.stack([lat.ravel(), flipped.ravel()]))
        assert E[1] - E[0] == po.lib().oracle_delta_energy(int(s0), int(sum(ns)))


def test_metropolis_threshold_closed_forms():
    assert po.metropolis_threshold(0.0, 4) == 2 ** 32
    assert po.metropolis_threshold(1e-13, 8) == 2 ** 32       # p within 2^-32 of 1
    assert po.metropolis_threshold(300.0, 8) == 1              # p > 0 but below 2^-32
    for beta in (0.1, 0.25, 0.4406867935097715, 1.0):
        for dE in (4, 8):
            x = 2 ** 32 * math.exp(-beta * dE)
            assert abs(x - round(x)) > 1e-3  # far from a boundary: binary64 suffices
            assert po.metropolis_threshold(beta, dE) == math.ceil(x)


def test_zero_beta_sweep_inverts_each_colour():
    # every move is accepted at beta = 0, so a full sweep negates the lattice
    s = po.init_spins(11, 6, 5)
    before = s.copy()
    po.sweeps(11, 6, s, 1, 1, 2 ** 32, 2 ** 32)
    assert np.array_equal(s, -before)


@pytest.mark.parametrize("beta", [0.3, 0.44])
def test_sweep_chain_samples_exact_boltzmann_distribution_L4(beta):
    L, R = 4, 128
    g = exact.dos_enumeration(L)
    p = exact.energy_distribution(g, beta)
    t4, t8 = po.metropolis_threshold(beta, 4), po.metropolis_threshold(beta, 8)
    s = po.init_spins(77, L, R)
    counts = {e: 0 for e in p}
    for step in range(1, 401):
        po.sweeps(77, L, s, step, 3, t4, t8)
        if step <= 20:
            continue
        E, _ = po.energy_magnetisation(L, s)
        for e in E:
            counts[int(e)] += 1
    n = sum(counts.values())
    chi2, dof = 0.0, 0
    for e, pe in p.items():
        if pe * n < 20:
            continue
        chi2 += (counts[e] - pe * n) ** 2 / (pe * n)
        dof += 1
    # samples are mildly autocorrelated; allow twice the 1e-4 quantile of chi2
    assert chi2 < 2 * (dof + 4 * math.sqrt(2 * dof) + 10), (chi2, dof)
