"""Pins of the oracle's heatbath update (Sec. "Spin updates": heatbath, the
same as Glauber dynamics for Ising spins): threshold identities and closed
forms, the stream map of its uniforms, the defining property that the new
spin depends only on the neighbours' field, and the exact Boltzmann
distribution of a chain at L = 4."""
import math

import numpy as np
import pytest

from oracle import exact
from oracle import pa_oracle as po

DES = (-8, -4, 0, 4, 8)


def test_threshold_closed_forms_and_symmetry():
    # p(dE) + p(-dE) = 1 and 2^32 p is never an integer for beta > 0, so the
    # two ceilings add up to 2^32 + 1; dE = 0 and beta = 0 give exactly 1/2
    for beta in (1e-9, 0.1, 0.3, 0.4406867935097715, 1.0, 3.0):
        for dE in (4, 8):
            assert po.heatbath_threshold(beta, dE) + po.heatbath_threshold(beta, -dE) == 2 ** 32 + 1
        assert po.heatbath_threshold(beta, 0) == 2 ** 31
    for dE in DES:
        assert po.heatbath_threshold(0.0, dE) == 2 ** 31
    # against binary64 evaluations away from rounding boundaries
    for beta in (0.1, 0.25, 0.4406867935097715, 1.0):
        for dE in DES:
            x = 2 ** 32 / (1 + math.exp(beta * dE))
            if dE:
                assert abs(x - round(x)) > 1e-3
                assert po.heatbath_threshold(beta, dE) == math.ceil(x)
    # far below 2^-32: one uniform value in 2^32 still flips
    assert po.heatbath_threshold(10.0, 8) == 1
    assert po.heatbath_threshold(10.0, -8) == 2 ** 32


def test_heatbath_ties_only_undecided_lanes():
    # a lane ties when its top six bits equal the threshold's AND the
    # threshold's low 26 bits are not zero; tied lanes take the TIE stream's
    # words in ascending lane order exactly like the Metropolis uniforms
    seed, w, g, h = 5, 9, 2, 33
    top = [po.sweep_top6(seed, w, g, h, l) for l in range(64)]
    thr = []
    for l in range(64):
        if l % 3 == 0:
            thr.append((top[l] << 26) | 0x0ABCDEF)  # tied
        elif l % 3 == 1:
            thr.append(top[l] << 26)  # equal top bits, zero low part: decided (u >= thr)
        else:
            thr.append(((top[l] ^ 1) << 26) | 5)  # decided by the top bits
    u = po.word_uniforms_heatbath(seed, w, g, h, thr, [True] * 64)
    tied = [l for l in range(64) if l % 3 == 0]
    for k, l in enumerate(tied):
        x = po.philox4x32_10(seed, [w, g, h, 0x10000100 | (k >> 2)])
        assert int(u[l]) == (top[l] << 26) | (int(x[k & 3]) >> 6)
    for l in range(64):
        if l % 3:
            assert int(u[l]) == top[l] << 26
    # the Metropolis map ties the zero-low-part lanes too (and so shifts the
    # later ties' words): the two maps differ exactly there
    um = po.word_uniforms(seed, w, g, h, thr, [True] * 64)
    assert any(int(a) != int(b) for a, b in zip(u, um))


@pytest.mark.parametrize("T", [1, 0x04000000, 0x7FFFFFFF, 0x80000000, 0xC0000000, 0xFFFFFFFF])
def test_heatbath_comparison_is_exact_bernoulli(T):
    n = 400
    acc = 0
    for w in range(n):
        u = po.word_uniforms_heatbath(3, w, 1, 2, [T] * 64, [True] * 64).astype(np.uint64)
        acc += int((u < np.uint64(T)).sum())
    p = T / 2.0 ** 32
    assert abs(acc / (64 * n) - p) <= 5 * math.sqrt(p * (1 - p) / (64 * n)) + 1e-12


@pytest.mark.parametrize("beta", [0.2, 0.6])
def test_new_spin_depends_only_on_the_field(beta):
    # one sweep: colour-0 sites are updated before any of their neighbours
    # (all colour 1), so the new spin of a colour-0 site is +1 with probability
    # 1 / (1 + exp(-2 beta h)), h the initial field, whatever the old spin was
    L, R = 8, 1024
    thr5 = [po.heatbath_threshold(beta, dE) for dE in DES]
    s = po.init_spins(202, L, R)
    before = s.copy()
    po.sweeps_heatbath(202, L, s, 1, 1, thr5)
    g = before.reshape(R, L, L)
    field = (np.roll(g, 1, 1) + np.roll(g, -1, 1) + np.roll(g, 1, 2) + np.roll(g, -1, 2)).reshape(R, -1)
    colour0 = np.array([((k % L) + (k // L)) % 2 == 0 for k in range(L * L)])
    for old in (-1, 1):
        for hf in (-4, -2, 0, 2, 4):
            sel = (before == old) & (field == hf) & colour0[None, :]
            n = int(sel.sum())
            if n < 200:
                continue
            p = 1 / (1 + math.exp(-2 * beta * hf))
            f = float((s[sel] == 1).mean())
            assert abs(f - p) <= 5 * math.sqrt(p * (1 - p) / n) + 1e-12, (old, hf, f, p, n)


def test_zero_beta_heatbath_gives_fresh_coins():
    # at beta = 0 every spin becomes a fair coin, independent of its past:
    # after one sweep about half of the spins changed
    L, R = 6, 512
    s = po.init_spins(4, L, R)
    before = s.copy()
    po.sweeps_heatbath(4, L, s, 1, 1, [2 ** 31] * 5)
    n = s.size
    changed = int((s != before).sum())
    assert abs(changed / n - 0.5) <= 5 * math.sqrt(0.25 / n)


@pytest.mark.parametrize("beta", [0.3, 0.44])
def test_heatbath_chain_samples_exact_boltzmann_distribution_L4(beta):
    L, R = 4, 128
    g = exact.dos_enumeration(L)
    p = exact.energy_distribution(g, beta)
    thr5 = [po.heatbath_threshold(beta, dE) for dE in DES]
    s = po.init_spins(78, L, R)
    counts = {e: 0 for e in p}
    for step in range(1, 401):
        po.sweeps_heatbath(78, L, s, step, 3, thr5)
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
    assert chi2 < 2 * (dof + 4 * math.sqrt(2 * dof) + 10), (chi2, dof)


def test_heatbath_run_free_energy_at_L4():
    # a whole heatbath run: -beta F at the end within a few standard errors of
    # Kaufman's ln Z (the resampling does not depend on the update)
    from workloads import linear_schedule
    L, R = 4, 2000
    betas = linear_schedule(0.5, 20)
    o = po.run(L, R, betas, 2, 9, "nearest", "heatbath")
    lnz = float(exact.ln_z_kaufman(L, betas[-1]))
    assert abs(o.minus_beta_F - lnz) < 0.08  # about 5 standard deviations over seeds
