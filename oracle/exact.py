"""Exact finite-lattice results for the periodic L x L Ising model (J = 1).

TEST INFRASTRUCTURE ONLY.  The paper compares its simulations with exact
finite-size results (Sec. "Model and observables", citing Kaufman 1949 and
Ferdinand & Fisher 1969).  Three independent routes are written here so that
each pins the others:

* ``dos_enumeration(L)``: brute force over all 2^(L^2) states (L = 4).
* ``dos_transfer(L)``: the row-to-row transfer matrix with exact integer
  polynomial entries, giving the integer density of states g(E).
* ``joint_dos_enumeration(L)`` / ``joint_dos_transfer(L)``: the joint density
  of states g(E, M) by brute force (L = 4) and by a transfer matrix that also
  carries the magnetisation, giving the exact <|M|> and <M^2> behind the
  magnetisation m and the susceptibility chi of Sec. "Model and observables".
* ``ln_z_kaufman(L, beta)``: Kaufman's closed form for the torus,
  Z = 1/2 (2 sinh 2K)^(N/2) [P1 + P2 + P3 + P4], with
  P1 = prod_r 2 cosh(L g_{2r+1}/2), P2 = prod_r 2 sinh(L g_{2r+1}/2),
  P3 = prod_r 2 cosh(L g_{2r}/2),   P4 = prod_r 2 sinh(L g_{2r}/2),
  r = 0..L-1, cosh g_l = cosh 2K coth 2K - cos(pi l / L) for l >= 1 and
  g_0 = 2K + ln tanh K (which is negative below the critical coupling).

E here is H = -sum_<ij> s_i s_j, so E ranges over [-2N, 2N] in steps of 4.
"""
from __future__ import annotations

from typing import Dict, Tuple

import mpmath
import numpy as np


def dos_enumeration(L: int) -> Dict[int, int]:
    """g(E) by visiting every configuration (feasible for L <= 4)."""
    N = L * L
    assert N <= 20
    states = np.arange(2 ** N, dtype=np.int64)
    bits = ((states[:, None] >> np.arange(N, dtype=np.int64)[None, :]) & 1).astype(np.int8)
    s = (2 * bits - 1).reshape(-1, L, L)
    E = -(s * np.roll(s, -1, axis=2)).sum(axis=(1, 2)) - (s * np.roll(s, -1, axis=1)).sum(axis=(1, 2))
    vals, counts = np.unique(E.astype(np.int64), return_counts=True)
    return {int(v): int(c) for v, c in zip(vals, counts)}


def dos_transfer(L: int) -> Dict[int, int]:
    """g(E) from a row-to-row transfer matrix with integer polynomial entries.

    A row is an L-bit state; its in-row bond energy and the bond energy to the
    next row are tabulated, and the number of ways to reach (row state, energy)
    is propagated over L rows; the torus closes by returning to the first row.
    """
    nstate = 2 ** L
    rows = ((np.arange(nstate)[:, None] >> np.arange(L)[None, :]) & 1) * 2 - 1
    e_in = -(rows * np.roll(rows, -1, axis=1)).sum(axis=1)          # [nstate]
    e_vert = -(rows[:, None, :] * rows[None, :, :]).sum(axis=2)        # [a, b]
    N = L * L
    span = 4 * N + 1                       # energies -2N..2N, index E + 2N
    total = np.zeros(span, dtype=object)
    for a0 in range(nstate):
        # dist[b, E + 2N] = ways to reach row state b having accumulated energy E
        dist = np.zeros((nstate, span), dtype=object)
        dist[a0, e_in[a0] + 2 * N] = 1
        for _ in range(L - 1):
            new = np.zeros((nstate, span), dtype=object)
            for a in range(nstate):
                row = dist[a]
                nz = np.nonzero(row)[0]
                if len(nz) == 0:
                    continue
                for b in range(nstate):
                    shift = int(e_vert[a, b] + e_in[b])
                    new[b, nz + shift] += row[nz]
            dist = new
        for a in range(nstate):
            shift = int(e_vert[a, a0])
            nz = np.nonzero(dist[a])[0]
            total[nz + shift] += dist[a][nz]
    return {int(i - 2 * N): int(c) for i, c in enumerate(total) if c}


def ln_z_from_dos(g: Dict[int, int], beta) -> mpmath.mpf:
    beta = mpmath.mpf(beta)
    return mpmath.log(mpmath.fsum(c * mpmath.exp(-beta * e) for e, c in g.items()))


def ln_z_kaufman(L: int, beta) -> mpmath.mpf:
    """ln Z of the periodic L x L Ising model at inverse temperature beta."""
    K = mpmath.mpf(beta)
    if K == 0:
        return L * L * mpmath.log(2)
    c2, s2 = mpmath.cosh(2 * K), mpmath.sinh(2 * K)
    base = c2 * c2 / s2  # cosh 2K coth 2K

    def gamma(l):
        if l == 0:
            return 2 * K + mpmath.log(mpmath.tanh(K))
        return mpmath.acosh(base - mpmath.cos(mpmath.pi * l / L))

    p1 = p2 = p3 = p4 = mpmath.mpf(1)
    for r in range(L):
        go, ge = gamma(2 * r + 1), gamma(2 * r)
        p1 *= 2 * mpmath.cosh(L * go / 2)
        p2 *= 2 * mpmath.sinh(L * go / 2)
        p3 *= 2 * mpmath.cosh(L * ge / 2)
        p4 *= 2 * mpmath.sinh(L * ge / 2)
    N = L * L
    return (N / mpmath.mpf(2)) * mpmath.log(2 * s2) + mpmath.log((p1 + p2 + p3 + p4) / 2)


def energy_per_spin(L: int, beta) -> mpmath.mpf:
    """e = <E>/N = -(1/N) d ln Z / d beta."""
    return -mpmath.diff(lambda b: ln_z_kaufman(L, b), mpmath.mpf(beta)) / (L * L)


def specific_heat(L: int, beta) -> mpmath.mpf:
    """C_V = beta^2 Var(E) / N = (beta^2 / N) d^2 ln Z / d beta^2."""
    b = mpmath.mpf(beta)
    return b * b * mpmath.diff(lambda x: ln_z_kaufman(L, x), b, 2) / (L * L)


def energy_distribution(g: Dict[int, int], beta) -> Dict[int, float]:
    """P_beta(E) = g(E) exp(-beta E) / Z."""
    beta = mpmath.mpf(beta)
    w = {e: c * mpmath.exp(-beta * e) for e, c in g.items()}
    z = mpmath.fsum(w.values())
    return {e: float(v / z) for e, v in w.items()}


# ---------------------------------------------------------------- magnetisation

def joint_dos_enumeration(L: int) -> Dict[Tuple[int, int], int]:
    """g(E, M), M = sum of the spins, by visiting every configuration (L <= 4)."""
    N = L * L
    assert N <= 20
    states = np.arange(2 ** N, dtype=np.int64)
    bits = ((states[:, None] >> np.arange(N, dtype=np.int64)[None, :]) & 1).astype(np.int8)
    s = (2 * bits - 1).reshape(-1, L, L)
    E = -(s * np.roll(s, -1, axis=2)).sum(axis=(1, 2)) - (s * np.roll(s, -1, axis=1)).sum(axis=(1, 2))
    M = s.sum(axis=(1, 2))
    key = (E.astype(np.int64) + 2 * N) * (2 * N + 1) + (M.astype(np.int64) + N)
    vals, counts = np.unique(key, return_counts=True)
    return {(int(v // (2 * N + 1)) - 2 * N, int(v % (2 * N + 1)) - N): int(c)
            for v, c in zip(vals, counts)}


def joint_dos_transfer(L: int) -> Dict[Tuple[int, int], int]:
    """g(E, M) from a row-to-row transfer matrix whose entries count states by
    (energy, magnetisation): the row magnetisation is added with each row, the
    bond energies as in dos_transfer."""
    nstate = 2 ** L
    rows = ((np.arange(nstate)[:, None] >> np.arange(L)[None, :]) & 1) * 2 - 1
    e_in = -(rows * np.roll(rows, -1, axis=1)).sum(axis=1)
    e_vert = -(rows[:, None, :] * rows[None, :, :]).sum(axis=2)
    m_row = rows.sum(axis=1)
    total: Dict[Tuple[int, int], int] = {}
    for a0 in range(nstate):
        # dist[b] = {(E, M): ways} over the rows placed so far, last row state b
        dist = [dict() for _ in range(nstate)]
        dist[a0][(int(e_in[a0]), int(m_row[a0]))] = 1
        for _ in range(L - 1):
            new = [dict() for _ in range(nstate)]
            for a in range(nstate):
                if not dist[a]:
                    continue
                for b in range(nstate):
                    de, dm = int(e_vert[a, b] + e_in[b]), int(m_row[b])
                    tgt = new[b]
                    for (e, m), c in dist[a].items():
                        k = (e + de, m + dm)
                        tgt[k] = tgt.get(k, 0) + c
            dist = new
        for a in range(nstate):
            de = int(e_vert[a, a0])
            for (e, m), c in dist[a].items():
                k = (e + de, m)
                total[k] = total.get(k, 0) + c
    return total


def magnetisation_moments(g2: Dict[Tuple[int, int], int], beta):
    """(<|M|>, <M^2>) at inverse temperature beta from the joint density of states."""
    b = mpmath.mpf(beta)
    w = {k: c * mpmath.exp(-b * k[0]) for k, c in g2.items()}
    z = mpmath.fsum(w.values())
    abs_m = mpmath.fsum(abs(k[1]) * v for k, v in w.items()) / z
    m2 = mpmath.fsum(k[1] * k[1] * v for k, v in w.items()) / z
    return abs_m, m2


def magnetisation_per_spin(L: int, g2, beta) -> mpmath.mpf:
    """m = <|M|> / N (the finite-lattice order parameter of Sec. "Model and observables")."""
    return magnetisation_moments(g2, beta)[0] / (L * L)


def susceptibility(L: int, g2, beta) -> mpmath.mpf:
    """chi = beta N (<m^2> - <|m|>^2) = beta (<M^2> - <|M|>^2) / N, m = M / N."""
    abs_m, m2 = magnetisation_moments(g2, beta)
    return mpmath.mpf(beta) * (m2 - abs_m * abs_m) / (L * L)
