"""Weighted averages over independent runs, and the bias estimate.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle; shares no code with the
HIP library).  Sec. "Weighted averages": the replicas of run m at beta_i carry
a weight proportional to exp(-beta_i F_i^m) (the product of that run's Q_k),
so observables of M independent runs are combined as

    O(beta_i) = sum_m omega_i^m O_m(beta_i),
    omega_i^m = R_i^m exp(-beta_i F_i^m) / sum_m' (same)              Eq. (weighted-averages)

and, for resampling with a fluctuating population size (nearest-integer,
Poisson), with the extra factor prod_{k=1}^{i} (R_{k-1}^m / R^m), R^m the
run's nominal size                                                    Eq. (modified-weights2).

Sec. "Bias with resampling": the bias of an estimator is cov(O, beta F)
(Eq. bias_covariance), estimated here by the sample covariance over the runs,
and rho_f = R sigma^2(beta F) (Eq. rho_f), with sigma^2 the sample variance
over the runs and R the mean nominal size.

The combined observables are the per-run thermal averages <E>, <E^2>, <|M|>,
<M^2> (each from the run's exact population sums); e = <E>/N, m = <|M|>/N,
c_v = beta^2 (<E^2> - <E>^2)/N and chi = beta (<M^2> - <|M|>^2)/N are then
formed from the combined moments.  The plain average uses omega = 1/M in the
same formulas.  The covariances pair each run's own estimates (e, m, c_v, chi
of that run) with its beta_i F_i = -(-beta_i F_i).

Inputs are each run's records (steps 0 .. i) as the oracle produces them; the
weights are evaluated in mpmath at 256 bits, the moments in exact rationals.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import Dict, List, Sequence

import mpmath

PREC_BITS = 256

FIELDS = ("e", "m", "c_v", "chi", "e_mod", "m_mod", "c_v_mod", "chi_mod", "e_plain", "m_plain",
          "c_v_plain", "chi_plain", "omega_max", "n_eff_runs", "var_beta_F", "rho_f", "cov_e",
          "cov_m", "cov_c_v", "cov_chi")


def _moments(rec) -> List[Fraction]:
    """<E>, <E^2>, <|M|>, <M^2> of one run's population at one step."""
    R = rec.R_i
    return [Fraction(rec.sum_E, R), Fraction(rec.sum_E2, R), Fraction(rec.sum_absM, R),
            Fraction(rec.sum_M2, R)]


def _observables(mom, beta, N) -> List:
    """e, m, c_v, chi from combined moments (mpmath or Fraction)."""
    E1, E2, A1, A2 = mom
    return [E1 / N, A1 / N, beta * beta * (E2 - E1 * E1) / N, beta * (A2 - A1 * A1) / N]


def _combine(weights, moms, beta, N):
    comb = [sum(w * m[k] for w, m in zip(weights, moms)) for k in range(4)]
    return _observables(comb, beta, N)


def weighted_averages(L: int, runs: Sequence[Sequence], R_nominal: Sequence[int], step: int) -> Dict:
    """Combine M runs at step i.  runs[m][k] is run m's record of step k
    (k = 0 .. i at least); R_nominal[m] its nominal population size R^m."""
    M = len(runs)
    N = L * L
    recs = [r[step] for r in runs]
    beta_f = recs[0].beta
    assert all(r.beta == beta_f for r in recs), "the runs must share the temperature"
    out: Dict = {"step": step, "n_runs": M, "beta": beta_f}
    with mpmath.workprec(PREC_BITS):
        beta = mpmath.mpf(beta_f)
        x = [mpmath.mpf(r.minus_beta_F) for r in recs]  # -beta_i F_i^m
        # Eq. (weighted-averages): R_i^m exp(-beta F)
        a = [r.R_i * mpmath.exp(xm) for r, xm in zip(recs, x)]
        # Eq. (modified-weights2): times prod_{k=1}^{i} R_{k-1}^m / R^m
        b = []
        for m in range(M):
            f = Fraction(1)
            for k in range(1, step + 1):
                f *= Fraction(runs[m][k - 1].R_i, R_nominal[m])
            b.append(a[m] * mpmath.mpf(f.numerator) / f.denominator)
        w = [am / mpmath.fsum(a) for am in a]
        wb = [bm / mpmath.fsum(b) for bm in b]
        moms = [[mpmath.mpf(v.numerator) / v.denominator for v in _moments(r)] for r in recs]
        for key, vals in (("", _combine(w, moms, beta, N)), ("_mod", _combine(wb, moms, beta, N))):
            for name, v in zip(("e", "m", "c_v", "chi"), vals):
                out[name + key] = float(v)
        # plain average: equal weights, exact
        fmoms = [_moments(r) for r in recs]
        plain = _combine([Fraction(1, M)] * M, fmoms, Fraction(beta_f), N)
        for name, v in zip(("e", "m", "c_v", "chi"), plain):
            out[name + "_plain"] = float(v)
        out["omega_max"] = float(max(w))
        out["n_eff_runs"] = float(1 / mpmath.fsum(wm * wm for wm in w))
        if M < 2:
            for k in ("var_beta_F", "rho_f", "cov_e", "cov_m", "cov_c_v", "cov_chi"):
                out[k] = math.nan
            return out
        F = [-xm for xm in x]  # beta_i F_i^m
        Fbar = mpmath.fsum(F) / M
        var = mpmath.fsum((f - Fbar) ** 2 for f in F) / (M - 1)
        out["var_beta_F"] = float(var)
        out["rho_f"] = float(mpmath.mpf(sum(R_nominal)) / M * var)
        # each run's own estimates, exact from its sums
        own = [_observables(fm, Fraction(beta_f), N) for fm in fmoms]
        for k, name in enumerate(("cov_e", "cov_m", "cov_c_v", "cov_chi")):
            vals = [mpmath.mpf(o[k].numerator) / o[k].denominator for o in own]
            vbar = mpmath.fsum(vals) / M
            out[name] = float(mpmath.fsum((v - vbar) * (f - Fbar) for v, f in zip(vals, F)) / (M - 1))
    return out
