"""Pins for the exact finite-lattice references (no GPU).

Three independent routes to Z of the periodic L x L Ising model must agree:
brute-force enumeration, an integer transfer matrix and Kaufman's closed form.
Closed forms the paper states are checked too.
"""
import json
import math
import os

import mpmath
import pytest

from oracle import exact


@pytest.fixture(scope="module")
def g4():
    return exact.dos_enumeration(4)


def test_enumeration_matches_transfer_matrix_L4(g4):
    assert exact.dos_transfer(4) == g4
    assert sum(g4.values()) == 2 ** 16
    # symmetric under E -> -E on a bipartite lattice, energies on a step-4 grid
    assert all(g4[e] == g4[-e] for e in g4)
    assert all(e % 4 == 0 for e in g4)
    assert g4[-32] == 2  # the two ground states


@pytest.mark.slow
def test_transfer_matrix_L6_counts_all_states():
    g6 = exact.dos_transfer(6)
    assert sum(g6.values()) == 2 ** 36
    assert g6[-72] == 2
    with mpmath.workprec(200):
        for beta in (0.1, 0.3, 0.4406867935097715, 0.7):
            a = exact.ln_z_from_dos(g6, beta)
            k = exact.ln_z_kaufman(6, beta)
            assert abs((a - k) / a) < mpmath.mpf(10) ** -40


@pytest.mark.parametrize("beta", [0.05, 0.2, 0.44, 0.4406867935097715, 1.0, 2.5])
def test_kaufman_matches_enumeration_L4(g4, beta):
    with mpmath.workprec(200):
        a = exact.ln_z_from_dos(g4, beta)
        k = exact.ln_z_kaufman(4, beta)
        assert abs((a - k) / a) < mpmath.mpf(10) ** -40


def test_paper_closed_forms(golden_dir, g4):
    pv = json.load(open(os.path.join(golden_dir, "paper_values.json")))
    assert abs(0.5 * math.log(1 + math.sqrt(2)) - pv["beta_c"]["value"]) < 1e-15
    # ln Z at beta = 0 is L^2 ln 2
    for L in (4, 8, 16):
        assert abs(float(exact.ln_z_kaufman(L, 0.0)) / (L * L) - pv["ln_z0_per_spin"]["value"]) < 1e-15
    assert abs(float(exact.ln_z_kaufman(4, 1e-30)) - 16 * math.log(2)) < 1e-12
    # Var(E) at beta = 0 is z L^d / 2 = 2N
    n = sum(g4.values())
    mean = sum(e * c for e, c in g4.items()) / n
    var = sum(e * e * c for e, c in g4.items()) / n - mean ** 2
    assert mean == 0 and var == pv["energy_variance_beta0_per_spin"]["value"] * 16


def test_energy_and_specific_heat_by_differentiation(g4):
    # derivatives of Kaufman's ln Z equal the moments of the enumerated g(E)
    with mpmath.workprec(120):
        for beta in (0.3, 0.44):
            p = exact.energy_distribution(g4, beta)
            m1 = sum(e * w for e, w in p.items())
            m2 = sum(e * e * w for e, w in p.items())
            assert abs(float(exact.energy_per_spin(4, beta)) - m1 / 16) < 1e-12
            assert abs(float(exact.specific_heat(4, beta)) - beta ** 2 * (m2 - m1 ** 2) / 16) < 1e-10


def test_large_lattice_magnitudes():
    # ln Z / N tends to the Onsager value; at L = 64, beta_c it is 0.92987...
    v = float(exact.ln_z_kaufman(64, 0.4407)) / 4096
    assert abs(v - 0.929870) < 1e-5
    assert abs(float(exact.ln_z_kaufman(128, 1.0)) / 16384 - 2.000390) < 1e-5
