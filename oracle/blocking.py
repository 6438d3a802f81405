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

Everything is exact rational arithmetic (fractions.Fraction) up to the final
conversion to float (and one square root).  With fewer than two blocks every
quantity is NaN; a zero blocked variance gives R_eff = inf (or NaN when the
values do not vary at all), as IEEE division would.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import Callable, List, Sequence, Tuple

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


def jackknife_variance(columns: Sequence[Sequence[int]], f: Callable[..., Fraction],
                       n: int) -> Fraction:
    """Eqs. (jackknife-blocks, jackknife-variance) for f of the columns' means.

    Sample k leaves out block k: f_k = f(mean of each column over the other
    blocks' values).
    """
    R = len(columns[0])
    totals = [sum(c) for c in columns]
    fk = []
    for lo, hi in block_bounds(R, n):
        cnt = R - (hi - lo)
        fk.append(f(*[Fraction(t - sum(c[lo:hi]), cnt) for t, c in zip(totals, columns)]))
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
