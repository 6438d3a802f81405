"""Blocking and jackknife analysis of one tree-ordered population.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle; shares no code with the
HIP library).  Sec. "Effective population size" and Sec. "Statistical
errors": copies of one parent sit at adjacent indices, so correlations between
replicas are local in index space, and the variance of a population mean is
estimated from n consecutive blocks.

* Eq. (blocks): block averages O_k^B over n blocks of the R_i values in slot
  order.  The paper takes n dividing R; for any R this oracle uses the slots
  [floor(k R / n), floor((k + 1) R / n)) for block k = 0 .. n-1 (sizes differ
  by at most one) and n = min(100, R) (the paper's n = 100).
* Eq. (blocked_variance): sigma^2(mean O) = sum_k (O_k^B - mean_k O^B)^2 / (n (n - 1)).
* Eq. (neff): R_eff(O) = sigma^2(O) / sigma^2(mean O), with sigma^2(O) the
  standard unbiased variance of the unblocked values.
* Eqs. (jackknife-blocks, jackknife-variance): the k-th jackknife sample holds
  every value outside block k; for a function f of population means,
  sigma^2(f) = (n - 1) / n sum_k (f_k^J - mean_k f^J)^2.  Used for the specific
  heat and the susceptibility (non-linear), as Sec. "Statistical errors" asks.

* Free-energy jackknife (Sec. "Conclusions", last guideline: the variance and
  covariances involving the free-energy estimator from a jackknife block
  analysis of the tree-ordered population; Eq. free-emergy-estimator).  The
  reading taken: jackknife sample k of -beta_i F_i leaves block k out of every
  normalisation Q_l, l <= i, of Eq. (Q), block k of the parent population of
  step l being its slots [floor(k R_{l-1} / n_F), floor((k + 1) R_{l-1} / n_F))
  with one n_F = min(100, R) (R the nominal size) for the whole run, so that
  the same index range of the tree-ordered populations -- which holds the
  same lineages -- is left out at every step:
      ln Q_l^(k) = ln[ sum_{j not in block k} exp(-dbeta_l E_j) / (R_{l-1} - B_k) ],
      -beta_i F_i^(k) = ln Z_0 + sum_{l <= i} ln Q_l^(k).
  An empty block leaves Q_l unchanged; a block holding every parent makes the
  jackknife undefined (NaN).  sigma^2(beta F) follows Eq. (jackknife-variance);
  cov(O, beta F) = (n - 1)/n sum_k (O_k^J - mean O^J)(beta F_k^J - mean beta F^J)
  (the bias estimate of Eq. bias_covariance) pairs it with the jackknife
  samples of O of the current population, which need the same number of
  blocks there (n = n_F; otherwise NaN).

Everything is exact rational arithmetic (fractions.Fraction) up to the final
conversion to float (and one square root); the free-energy jackknife is
carried in mpmath at 256 bits (its samples are transcendental).  With fewer
than two blocks every quantity is NaN; a zero blocked variance gives R_eff = inf (or NaN when the
values do not vary at all), as IEEE division would.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import Callable, List, Sequence, Tuple

import mpmath

N_BLOCKS = 100  # the paper's n


def n_blocks(R: int) -> int:
    return min(N_BLOCKS, R)


def block_bounds(R: int, n: int) -> List[Tuple[int, int]]:
    """Slot ranges [lo, hi) of the n blocks (Eq. blocks, any R)."""
    return [(k * R // n, (k + 1) * R // n) for k in range(n)]


def _ratio(num: Fraction, den: Fraction) -> float:
    """num / den as IEEE division would give it."""
    if den == 0:
        return math.nan if num == 0 else math.copysign(math.inf, num)
    return float(num / den)


def variance(values: Sequence[int]) -> Fraction:
    """Unbiased variance of the unblocked values: (R sum x^2 - (sum x)^2) / (R (R - 1))."""
    R = len(values)
    s1 = sum(values)
    s2 = sum(x * x for x in values)
    return Fraction(R * s2 - s1 * s1, R * (R - 1))


def blocked_variance_of_mean(values: Sequence[int], n: int) -> Fraction:
    """Eq. (blocked_variance) over the blocks of Eq. (blocks)."""
    means = [Fraction(sum(values[lo:hi]), hi - lo) for lo, hi in block_bounds(len(values), n)]
    mbar = sum(means) / n
    return sum((m - mbar) ** 2 for m in means) / (n * (n - 1))


def jackknife_samples(columns: Sequence[Sequence[int]], f: Callable[..., Fraction],
                      n: int) -> List[Fraction]:
    """Eq. (jackknife-blocks): sample k leaves out block k, f_k = f(mean of each
    column over the other blocks' values)."""
    R = len(columns[0])
    totals = [sum(c) for c in columns]
    fk = []
    for lo, hi in block_bounds(R, n):
        cnt = R - (hi - lo)
        fk.append(f(*[Fraction(t - sum(c[lo:hi]), cnt) for t, c in zip(totals, columns)]))
    return fk


def jackknife_variance(columns: Sequence[Sequence[int]], f: Callable[..., Fraction],
                       n: int) -> Fraction:
    """Eqs. (jackknife-blocks, jackknife-variance) for f of the columns' means."""
    fk = jackknife_samples(columns, f, n)
    fbar = sum(fk) / n
    return Fraction(n - 1, n) * sum((x - fbar) ** 2 for x in fk)


def r_eff(values: Sequence[int], n: int) -> float:
    """Eq. (neff): sigma^2(O) / sigma^2(mean O)."""
    return _ratio(variance(values), blocked_variance_of_mean(values, n))


def population_errors(L: int, beta: float, E: Sequence[int], M: Sequence[int]):
    """(r_eff_E, r_eff_absM, err_e, err_m, err_c_v, err_chi) of one population.

    err_e, err_m: blocked standard errors of e = <E>/N and m = <|M|>/N;
    err_c_v, err_chi: jackknife errors of c_v = beta^2 (<E^2> - <E>^2) / N and
    chi = beta (<M^2> - <|M|>^2) / N (the estimators of the records).
    """
    R = len(E)
    n = n_blocks(R)
    if n < 2:
        return (math.nan,) * 6
    N = L * L
    b = Fraction(beta)
    E = [int(x) for x in E]
    A = [abs(int(x)) for x in M]
    E2 = [x * x for x in E]
    A2 = [x * x for x in A]
    vE = blocked_variance_of_mean(E, n)
    vA = blocked_variance_of_mean(A, n)
    cv = jackknife_variance([E, E2], lambda m1, m2: b * b * (m2 - m1 * m1) / N, n)
    chi = jackknife_variance([A, A2], lambda m1, m2: b * (m2 - m1 * m1) / N, n)
    return (_ratio(variance(E), vE), _ratio(variance(A), vA),
            math.sqrt(float(vE)) / N, math.sqrt(float(vA)) / N,
            math.sqrt(float(cv)), math.sqrt(float(chi)))


# ---------------------------------------------------------------- free energy

PREC_BITS = 256


def n_blocks_free_energy(R_nominal: int) -> int:
    """n_F: the blocks of the free-energy jackknife, fixed for a run."""
    return min(N_BLOCKS, R_nominal)


def leave_one_block_out_ln_q(E: Sequence[int], boltz, n: int):
    """ln Q^(k), k < n, of one step: the normalisation of Eq. (Q) over the
    parents E (slot order) without block k; boltz maps an energy to its
    Boltzmann factor exp(-dbeta E) (mpmath, caller's precision)."""
    R = len(E)
    with mpmath.workprec(PREC_BITS):
        w = [boltz[int(e)] for e in E]
        total = mpmath.fsum(w)
        out = []
        for lo, hi in block_bounds(R, n):
            if hi - lo == R:
                out.append(mpmath.nan)
            elif hi == lo:
                out.append(mpmath.log(total / R))
            else:
                out.append(mpmath.log((total - mpmath.fsum(w[lo:hi])) / (R - (hi - lo))))
        return out


def free_energy_errors(L: int, beta: float, E: Sequence[int], M: Sequence[int],
                       jk_minus_beta_F, n_F: int):
    """(var(beta F), cov(e, beta F), cov(m, beta F), cov(c_v, beta F),
    cov(chi, beta F)) of one record from the jackknife samples of -beta_i F_i
    (one per block of the free-energy jackknife) and the current population."""
    if n_F < 2 or any(mpmath.isnan(x) for x in jk_minus_beta_F):
        return (math.nan,) * 5
    with mpmath.workprec(PREC_BITS):
        bf = [-x for x in jk_minus_beta_F]
        bbar = mpmath.fsum(bf) / n_F
        db = [x - bbar for x in bf]
        jf = mpmath.mpf(n_F - 1) / n_F
        var = float(jf * mpmath.fsum(x * x for x in db))
        R = len(E)
        if n_blocks(R) != n_F:
            return (var,) + (math.nan,) * 4
        N = L * L
        b = Fraction(beta)
        Ei = [int(x) for x in E]
        A = [abs(int(x)) for x in M]
        E2 = [x * x for x in Ei]
        A2 = [x * x for x in A]
        samples = [
            jackknife_samples([Ei], lambda m1: m1 / N, n_F),
            jackknife_samples([A], lambda m1: m1 / N, n_F),
            jackknife_samples([Ei, E2], lambda m1, m2: b * b * (m2 - m1 * m1) / N, n_F),
            jackknife_samples([A, A2], lambda m1, m2: b * (m2 - m1 * m1) / N, n_F),
        ]
        covs = []
        for fk in samples:
            fbar = sum(fk) / n_F
            dev = [mpmath.mpf((x - fbar).numerator) / (x - fbar).denominator for x in fk]
            covs.append(float(jf * mpmath.fsum(u * v for u, v in zip(dev, db))))
        return (var,) + tuple(covs)
