"""Population-annealing CPU oracle.

TEST INFRASTRUCTURE ONLY.  A plain, slow, obviously correct implementation of
population annealing for the 2D Ising ferromagnet, written from the paper
(Weigel, Barash, Shchur & Janke, "Understanding population annealing Monte
Carlo simulations", arXiv:2102.06611).  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; it shares no code
with the HIP library.

The integer core (Philox streams, initial spins, checkerboard Metropolis,
energy/magnetisation) is plain C in pa_oracle.c, reached through ctypes.  This
file takes the per-step decisions, following Sec. "Algorithm" steps 1-5:

* Eq. (Q): Q_i = (1/R_{i-1}) sum_j exp[-(beta_i - beta_{i-1}) E_j], evaluated
  per replica in mpmath at 256-bit precision.
* Eq. (taus) and Eq. (resampling-factors): tau_hat_j = (R / R_{i-1}) tau_i(E_j)
  with tau_i(E_j) = exp[-(beta_i - beta_{i-1}) E_j] / Q_i; the copy count is
  floor(tau_hat) + 1 when u < tau_hat - floor(tau_hat) and floor(tau_hat)
  otherwise, u = u32 / 2^32 the parent's resampling uniform (strict "<": the
  reading taken where the paper's "r > frac" leaves r = frac to the "+1" side).
* Poisson resampling (Sec. "Algorithm", fluctuating population size): parent
  j makes r_j ~ Poisson(tau_hat_j) copies, drawn by inversion of a 64-bit
  uniform U (the smallest k with U < 2^64 F(k), F the Poisson CDF).
* Multinomial resampling (Sec. "Algorithm", fixed population size): R draws
  with probability proportional to tau_i(E_j); each weight relative to the
  largest one, exp[-dbeta (E_j - E_min)], is quantised to floor(2^40 x) and a
  draw with 64-bit uniform U picks the first parent whose cumulative quantised
  weight exceeds floor(U * W / 2^64), W the total.
* Copies of one parent sit at adjacent slots, parents in ascending order
  (Sec. "Overlap correlation": place the r copies at adjacent indices).
* Metropolis thresholds ceil(2^32 exp(-beta dE)) for dE = 4, 8; heatbath
  (Sec. "Spin updates") thresholds ceil(2^32 / (1 + exp(beta dE))) for
  dE = -8, -4, 0, 4, 8 (every move compares).
* Eq. (free-emergy-estimator): -beta_i F_i = ln Z_0 + sum_k ln Q_k with
  ln Z_0 = L^2 ln 2.
* Sec. "Model and observables": e, C_V, m, chi from population sums (N -> R_i).
* Sec. "Families": f, rho_t = R_i sum n_k^2 (Eq. rhot), S_f and
  rho_s = R_i / exp(S_f) (Eq. rhos); the one-step rho_t(beta_{i-1}, beta_i)
  = R_i sum_k (r_k / R_i)^2 of Eq. (one-step-Reff).
* Sec. "Effective population size" and Sec. "Statistical errors": blocking
  R_eff(E), R_eff(|M|) and single-run error bars of e, m, C_V, chi over the
  tree-ordered population (oracle/blocking.py).
* Sec. "Conclusions" (last guideline) with Eqs. (free-emergy-estimator,
  jackknife-variance, bias_covariance): the single-run jackknife of -beta F,
  each sample leaving one block of every parent population out of every Q
  (oracle/blocking.py gives the reading), and the covariances of e, m, C_V,
  chi with beta F.

Every integer decision is taken on a 256-bit value and is checked to be at
least 2^-100 away from its rounding boundary unless the value is exact.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from fractions import Fraction
from typing import Dict, List, Optional

import mpmath
import numpy as np

from oracle import blocking

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pa_oracle.c")
_LIB = os.path.join(_HERE, "libpa_oracle.so")
PREC_BITS = 256
_lib = None


class OracleAmbiguity(RuntimeError):
    """A decision value sits too close to its rounding boundary to be trusted."""


class PopulationExtinct(RuntimeError):
    """Resampling gave every parent zero copies (possible with Poisson resampling)."""


def build(force: bool = False) -> str:
    """Compile pa_oracle.c with gcc (no FP contraction; the core is integer-only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC",
                               "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        p_u32 = ctypes.POINTER(ctypes.c_uint32)
        p_i8 = ctypes.POINTER(ctypes.c_int8)
        p_i32 = ctypes.POINTER(ctypes.c_int32)
        L.oracle_philox4x32_10.argtypes = [u32, u32, p_u32, p_u32]
        L.oracle_philox4x32_10.restype = None
        L.oracle_philox4x32_10_n.argtypes = [u32, u32, ctypes.c_int64, p_u32, p_u32]
        L.oracle_philox4x32_10_n.restype = None
        L.oracle_sweep_top6.argtypes = [u64, u32, u32, u32, u32]
        L.oracle_sweep_top6.restype = u32
        L.oracle_word_uniforms.argtypes = [u64, u32, u32, u32, ctypes.POINTER(ctypes.c_uint64),
                                           ctypes.POINTER(ctypes.c_int), p_u32]
        L.oracle_word_uniforms.restype = None
        L.oracle_resample_uniform.argtypes = [u64, u32, u32]
        L.oracle_resample_uniform.restype = u32
        L.oracle_multinomial_uniform.argtypes = [u64, u32, u32]
        L.oracle_multinomial_uniform.restype = u64
        L.oracle_poisson_uniform.argtypes = [u64, u32, u32]
        L.oracle_poisson_uniform.restype = u64
        L.oracle_init_spins.argtypes = [u64, i32, i32, p_i8]
        L.oracle_init_spins.restype = None
        L.oracle_energy_magnetisation.argtypes = [i32, i32, p_i8, p_i32, p_i32]
        L.oracle_energy_magnetisation.restype = None
        L.oracle_delta_energy.argtypes = [i32, i32]
        L.oracle_delta_energy.restype = i32
        L.oracle_sweeps.argtypes = [u64, i32, i32, p_i8, i32, i32, u64, u64, i32]
        L.oracle_sweeps.restype = None
        L.oracle_word_uniforms_heatbath.argtypes = L.oracle_word_uniforms.argtypes
        L.oracle_word_uniforms_heatbath.restype = None
        L.oracle_sweeps_heatbath.argtypes = [u64, i32, i32, p_i8, i32, i32,
                                             ctypes.POINTER(ctypes.c_uint64), i32]
        L.oracle_sweeps_heatbath.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


# ---------------------------------------------------------------- RNG streams

def philox4x32_10(key: int, ctr) -> np.ndarray:
    """Philox4x32-10 of a 128-bit counter (4 words) under a 64-bit key."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(key & 0xFFFFFFFF, key >> 32, _ptr(c, ctypes.c_uint32),
                               _ptr(out, ctypes.c_uint32))
    return out


def philox4x32_10_many(key: int, ctrs) -> np.ndarray:
    """Philox4x32-10 of every row of an [n, 4] array of counters under one key."""
    c = np.ascontiguousarray(np.asarray(ctrs, dtype=np.uint32).reshape(-1, 4))
    out = np.zeros_like(c)
    lib().oracle_philox4x32_10_n(key & 0xFFFFFFFF, key >> 32, len(c), _ptr(c, ctypes.c_uint32),
                                 _ptr(out, ctypes.c_uint32))
    return out


def sweep_top6(seed: int, w: int, g: int, h: int, lane: int) -> int:
    """Top six bits of lane `lane`'s Metropolis uniform in word (w, g, h)."""
    return int(lib().oracle_sweep_top6(seed, w, g, h, lane))


def word_uniforms(seed: int, w: int, g: int, h: int, thr, needs) -> np.ndarray:
    """The 64 Metropolis uniforms of word (w, g, h) for per-lane thresholds thr
    and the lanes that compare at all (needs); 0 where needs is false."""
    t = np.ascontiguousarray(np.asarray(thr, dtype=np.uint64))
    n = np.ascontiguousarray(np.asarray(needs, dtype=np.intc))
    assert t.shape == (64,) and n.shape == (64,)
    u = np.zeros(64, dtype=np.uint32)
    lib().oracle_word_uniforms(seed, w, g, h, _ptr(t, ctypes.c_uint64), _ptr(n, ctypes.c_int),
                               _ptr(u, ctypes.c_uint32))
    return u


def word_uniforms_heatbath(seed: int, w: int, g: int, h: int, thr, needs) -> np.ndarray:
    """The 64 heatbath uniforms of word (w, g, h): as word_uniforms, but a lane
    is tied only when its top six bits leave u < thr undecided."""
    t = np.ascontiguousarray(np.asarray(thr, dtype=np.uint64))
    n = np.ascontiguousarray(np.asarray(needs, dtype=np.intc))
    assert t.shape == (64,) and n.shape == (64,)
    u = np.zeros(64, dtype=np.uint32)
    lib().oracle_word_uniforms_heatbath(seed, w, g, h, _ptr(t, ctypes.c_uint64),
                                        _ptr(n, ctypes.c_int), _ptr(u, ctypes.c_uint32))
    return u


def resample_uniform(seed: int, step: int, j: int) -> int:
    return int(lib().oracle_resample_uniform(seed, step, j))


def multinomial_uniform(seed: int, step: int, d: int) -> int:
    return int(lib().oracle_multinomial_uniform(seed, step, d))


def poisson_uniform(seed: int, step: int, j: int) -> int:
    return int(lib().oracle_poisson_uniform(seed, step, j))


def nearest_count(seed: int, step: int, R: int, levels: Dict[int, int], beta_prev: float,
                  beta_next: float, e_j: int, j: int) -> int:
    """Copy count of one parent under the nearest-integer rule, for
    populations too large to resample whole here.

    Parent j (energy e_j) of a population with levels[e] replicas of energy e
    (R_{i-1} = their sum) at the move beta_prev -> beta_next, dbeta their
    difference: Q_i = (1/R_{i-1}) sum_e levels[e] exp(-dbeta e) (Eq. Q, the replicas
    grouped by energy), tau_hat_j = (R / R_{i-1}) exp(-dbeta e_j) / Q_i (Eq.
    taus), and r_j = floor(tau_hat_j) + [u_j < frac(tau_hat_j)] with u_j the
    parent's resampling uniform (Eq. resampling-factors).  The rule of
    OracleRun.copy_counts, one parent at a time.
    """
    Rp = sum(levels.values())
    with mpmath.workprec(PREC_BITS):
        db = mpmath.mpf(beta_next) - mpmath.mpf(beta_prev)
        if len(levels) == 1:
            tau = mpmath.mpf(1)  # one level: every weight equals Q
        else:
            Q = mpmath.fsum(n * mpmath.exp(-db * e) for e, n in levels.items()) / Rp
            tau = mpmath.exp(-db * e_j) / Q
        tau_hat = mpmath.mpf(R) / Rp * tau
        _check_margin(mpmath.ldexp(tau_hat, 32), "2^32 tau_hat")
        fl = mpmath.floor(tau_hat)
        u = mpmath.ldexp(resample_uniform(seed, step, j), -32)
        return int(fl) + (1 if u < tau_hat - fl else 0)


def poisson_inverse(lam, U: int) -> int:
    """Copies for Poisson resampling by inversion: the smallest k >= 0 with
    U < 2^64 F(k), F(k) = e^-lam sum_{m<=k} lam^m / m! (the Poisson CDF of mean
    lam, Sec. "Algorithm"); lam is a high-precision real, U a 64-bit integer."""
    term = mpmath.exp(-lam)
    F = term
    k = 0
    while True:
        x = mpmath.ldexp(F, 64)
        gap = abs(x - U)
        if gap < mpmath.ldexp(mpmath.mpf(1), 64 - 100):
            raise OracleAmbiguity("2^64 F(%d) = %s is within 2^-100 (relative) of U" % (k, mpmath.nstr(x, 40)))
        if U < x:
            return k
        k += 1
        term = term * lam / k
        F = F + term


# ---------------------------------------------------------------- model

def init_spins(seed: int, L: int, R: int) -> np.ndarray:
    """Simple sampling at beta_0 = 0 (Sec. "Algorithm", step 1): [R, L*L] int8 of +-1."""
    s = np.zeros((R, L * L), dtype=np.int8)
    lib().oracle_init_spins(seed, L, R, _ptr(s, ctypes.c_int8))
    return s


def energy_magnetisation(L: int, spins: np.ndarray):
    spins = np.ascontiguousarray(spins, dtype=np.int8)
    R = spins.shape[0]
    E = np.zeros(R, dtype=np.int32)
    M = np.zeros(R, dtype=np.int32)
    if R:
        lib().oracle_energy_magnetisation(L, R, _ptr(spins, ctypes.c_int8),
                                          _ptr(E, ctypes.c_int32), _ptr(M, ctypes.c_int32))
    return E, M


def sweeps(seed: int, L: int, spins: np.ndarray, step: int, theta: int, t4: int, t8: int,
           slot0: int = 0) -> None:
    """theta checkerboard Metropolis sweeps, in place, for step >= 1.

    spins[k] is the replica in population slot slot0 + k; a group's 64
    uniforms are drawn together, so slot0 is a multiple of 64 and spins holds
    whole groups (the last may be short only where the population ends).
    """
    assert spins.dtype == np.int8 and spins.flags.c_contiguous
    assert slot0 % 64 == 0, "sweeps take whole 64-replica groups"
    R = spins.shape[0]
    if R and theta:
        lib().oracle_sweeps(seed, L, R, _ptr(spins, ctypes.c_int8), step, theta, t4, t8, slot0)


def sweeps_heatbath(seed: int, L: int, spins: np.ndarray, step: int, theta: int, thr5,
                    slot0: int = 0) -> None:
    """theta checkerboard heatbath sweeps, in place, for step >= 1; thr5[c] is
    heatbath_threshold(beta, 4c - 8).  Groups as in sweeps()."""
    assert spins.dtype == np.int8 and spins.flags.c_contiguous
    assert slot0 % 64 == 0, "sweeps take whole 64-replica groups"
    t = np.ascontiguousarray(np.asarray(thr5, dtype=np.uint64))
    assert t.shape == (5,)
    R = spins.shape[0]
    if R and theta:
        lib().oracle_sweeps_heatbath(seed, L, R, _ptr(spins, ctypes.c_int8), step, theta,
                                     _ptr(t, ctypes.c_uint64), slot0)


# ---------------------------------------------------------------- decisions

def _check_margin(x, what: str):
    """x is a high-precision real about to be rounded to an integer."""
    if x == mpmath.floor(x):
        return  # exact integer: no rounding ambiguity
    gap = min(x - mpmath.floor(x), mpmath.ceil(x) - x)
    if gap < abs(x) * mpmath.mpf(2) ** -100:
        raise OracleAmbiguity("%s = %s is within 2^-100 (relative) of an integer"
                              % (what, mpmath.nstr(x, 40)))


def metropolis_threshold(beta: float, dE: int) -> int:
    """ceil(2^32 exp(-beta dE)): accept a dE > 0 move iff u32 < this value."""
    with mpmath.workprec(PREC_BITS):
        x = mpmath.ldexp(mpmath.exp(-mpmath.mpf(beta) * dE), 32)
        _check_margin(x, "2^32 exp(-beta dE)")
        return int(mpmath.ceil(x))


def heatbath_threshold(beta: float, dE: int) -> int:
    """ceil(2^32 / (1 + exp(beta dE))): the heatbath flip (Sec. "Spin updates")
    of a move with energy change dE happens iff u32 < this value.  beta = 0 or
    dE = 0 give probability 1/2, i.e. 2^31 exactly."""
    if beta == 0.0 or dE == 0:
        return 1 << 31
    # for dE < 0, 2^32 p lies about 2^32 exp(-beta |dE|) below 2^32: carry
    # enough extra bits that the rounding error stays far below that distance
    prec = PREC_BITS + int(abs(beta * dE) * 1.5) + 64
    with mpmath.workprec(prec):
        x = mpmath.ldexp(1 / (1 + mpmath.exp(mpmath.mpf(beta) * dE)), 32)
        gap = min(x - mpmath.floor(x), mpmath.ceil(x) - x)
        if gap < mpmath.mpf(2) ** (32 + 100 - prec):
            raise OracleAmbiguity("2^32 / (1 + exp(beta dE)) = %s is too close to an integer"
                                  % mpmath.nstr(x, 40))
        return int(mpmath.ceil(x))


def overlap(E: np.ndarray, dbeta: float) -> float:
    """Histogram overlap alpha(beta, beta + dbeta) = sum_E min(P(E), P'(E)).

    P is the population's energy histogram, P' the same histogram reweighted
    by exp(-dbeta E) and renormalised; this equals (1/R) sum_j min(1, tau_j).
    """
    with mpmath.workprec(PREC_BITS):
        db = mpmath.mpf(dbeta)
        cache: Dict[int, mpmath.mpf] = {}
        for e in np.unique(E):
            cache[int(e)] = mpmath.exp(-db * int(e))
        Q = mpmath.fsum(cache[int(e)] for e in E) / len(E)
        a = mpmath.fsum(min(mpmath.mpf(1), cache[int(e)] / Q) for e in E) / len(E)
        return float(a)


@dataclasses.dataclass
class Record:
    step: int
    beta: float
    R_i: int
    sum_E: int
    sum_E2: int
    sum_absM: int
    sum_M2: int
    e: float
    c_v: float
    m: float
    chi: float
    ln_Q: float
    minus_beta_F: float
    n_families: int
    sum_fam2: int
    sum_cnt2: int
    rho_t: float
    rho_s: float
    rho_t_step: float
    r_eff_E: float
    r_eff_absM: float
    err_e: float
    err_m: float
    err_c_v: float
    err_chi: float
    jk_var_beta_F: float
    jk_cov_e: float
    jk_cov_m: float
    jk_cov_c_v: float
    jk_cov_chi: float


def observables(L: int, beta: float, E: np.ndarray, M: np.ndarray):
    """e, C_V, m, chi (Sec. "Model and observables") from exact integer sums."""
    N = L * L
    R = len(E)
    E64 = E.astype(np.int64)
    M64 = M.astype(np.int64)
    sE, sE2 = int(E64.sum()), int((E64 * E64).sum())
    sM, sM2 = int(np.abs(M64).sum()), int((M64 * M64).sum())
    b = Fraction(beta)
    e = Fraction(sE, N * R)
    c_v = b * b * N * (Fraction(sE2, N * N * R) - e * e)
    m = Fraction(sM, N * R)
    chi = b * N * (Fraction(sM2, N * N * R) - m * m)
    return (sE, sE2, sM, sM2), (float(e), float(c_v), float(m), float(chi))


def family_stats(fam: np.ndarray):
    """f, sum_k c_k^2, rho_t = R_i sum n_k^2, rho_s = R_i / exp(S_f) (Eqs. rhot, rhos)."""
    R = len(fam)
    _, counts = np.unique(fam, return_counts=True)
    f = len(counts)
    sum_c2 = int((counts.astype(np.int64) ** 2).sum())
    with mpmath.workprec(PREC_BITS):
        S_f = -mpmath.fsum(mpmath.mpf(int(c)) / R * mpmath.log(mpmath.mpf(int(c)) / R)
                           for c in counts)
        rho_s = float(R / mpmath.exp(S_f))
    rho_t = float(Fraction(sum_c2, R))
    return f, sum_c2, rho_t, rho_s


class OracleRun:
    """One population-annealing run, executed step by step on the CPU.

    State: spins [R_i, N] int8 (+-1), fam [R_i] (index of the initial replica
    each one descends from), E and M [R_i], the running sum of ln Q.
    """

    def __init__(self, L: int, R: int, theta: int, seed: int, resample: str = "nearest",
                 betas: Optional[np.ndarray] = None, update: str = "metropolis"):
        assert L >= 4 and L % 2 == 0
        assert resample in ("nearest", "multinomial", "poisson", "none")
        assert update in ("metropolis", "heatbath")
        self.L, self.N, self.R, self.theta, self.seed = L, L * L, R, theta, seed
        self.resample = resample
        self.update = update
        self.betas: List[float] = [0.0] if betas is None else [float(b) for b in betas]
        assert self.betas[0] == 0.0
        self.step = 0
        self.spins = init_spins(seed, L, R)
        self.fam = np.arange(R, dtype=np.int32)
        self.E, self.M = energy_magnetisation(L, self.spins)
        with mpmath.workprec(PREC_BITS):
            self._acc = self.N * mpmath.log(2)  # ln Z_{beta_0} = L^2 ln 2
            # jackknife samples of -beta F, one per block of the free-energy jackknife
            self.n_F = blocking.n_blocks_free_energy(R)
            self._jk = [self._acc] * self.n_F
        self._jk_lnq = None
        self.last_counts = np.zeros(0, dtype=np.int32)
        self.records: List[Record] = [self._record(0.0, 0, 0.0)]

    # -- the population at the current step ------------------------------------
    def _record(self, ln_q, sum_cnt2, beta=None) -> Record:
        beta = self.betas[self.step] if beta is None else beta
        sums, obs = observables(self.L, beta, self.E, self.M)
        f, sum_c2, rho_t, rho_s = family_stats(self.fam)
        R_i = len(self.E)
        rho_step = float(Fraction(sum_cnt2, R_i)) if self.step > 0 else 0.0
        errs = blocking.population_errors(self.L, beta, self.E, self.M)
        jk = blocking.free_energy_errors(self.L, beta, self.E, self.M, self._jk, self.n_F)
        return Record(self.step, beta, R_i, *sums, *obs, float(ln_q), float(self._acc),
                      f, sum_c2, int(sum_cnt2), rho_t, rho_s, rho_step, *errs, *jk)

    # -- step 2 of the algorithm ------------------------------------------------
    def copy_counts(self, beta_prev: float, beta_next: float, step: int):
        """Return (copy counts per parent, ln Q) for the move beta_prev -> beta_next."""
        E = self.E
        Rp = len(E)
        with mpmath.workprec(PREC_BITS):
            db = mpmath.mpf(beta_next) - mpmath.mpf(beta_prev)
            boltz: Dict[int, mpmath.mpf] = {}
            for e in np.unique(E):
                boltz[int(e)] = mpmath.exp(-db * int(e))
            Q = mpmath.fsum(boltz[int(e)] for e in E) / Rp  # Eq. (Q)
            ln_q = mpmath.log(Q)
            self._jk_lnq = blocking.leave_one_block_out_ln_q(E, boltz, self.n_F)
            if self.resample == "none":
                return np.ones(Rp, dtype=np.int32), ln_q
            if self.resample == "poisson":
                # r_j ~ Poisson(tau_hat_j) by inversion of its 64-bit uniform (Sec.
                # "Algorithm", following Machta: a sum of Poisson distributions)
                counts = np.zeros(Rp, dtype=np.int32)
                single_level = len(boltz) == 1
                for j in range(Rp):
                    tau = mpmath.mpf(1) if single_level else boltz[int(E[j])] / Q
                    tau_hat = mpmath.mpf(self.R) / Rp * tau  # Eq. (taus)
                    counts[j] = poisson_inverse(tau_hat, poisson_uniform(self.seed, step, j))
                return counts, ln_q
            if self.resample == "nearest":
                counts = np.zeros(Rp, dtype=np.int32)
                single_level = len(boltz) == 1
                for j in range(Rp):
                    # tau_i(E_j); with one energy level every replica's weight equals Q,
                    # so tau = 1 exactly (a floating evaluation would only be close to it)
                    tau = mpmath.mpf(1) if single_level else boltz[int(E[j])] / Q
                    tau_hat = mpmath.mpf(self.R) / Rp * tau  # Eq. (taus)
                    _check_margin(mpmath.ldexp(tau_hat, 32), "2^32 tau_hat")
                    fl = mpmath.floor(tau_hat)
                    u = mpmath.ldexp(resample_uniform(self.seed, step, j), -32)
                    counts[j] = int(fl) + (1 if u < tau_hat - fl else 0)  # Eq. (resampling-factors)
                return counts, ln_q
            # multinomial: R draws, probability of parent j proportional to tau_i(E_j)
            e_min = int(E.min())
            q = []
            for j in range(Rp):
                rel = mpmath.exp(-db * (int(E[j]) - e_min))
                x = mpmath.ldexp(rel, 40)
                _check_margin(x, "2^40 w")
                q.append(int(mpmath.floor(x)))
        cum = np.cumsum(np.array(q, dtype=np.uint64), dtype=np.uint64)
        W = int(cum[-1])
        counts = np.zeros(Rp, dtype=np.int32)
        for d in range(self.R):
            U = multinomial_uniform(self.seed, step, d)
            x = (U * W) >> 64
            parent = int(np.searchsorted(cum, np.uint64(x), side="right"))
            counts[parent] += 1
        return counts, ln_q

    def anneal_step(self, beta_next: Optional[float] = None) -> Record:
        """One temperature step: reweight/resample, theta sweeps, measure."""
        i = self.step + 1
        if beta_next is not None:
            if len(self.betas) > i:
                self.betas[i] = float(beta_next)
            else:
                self.betas.append(float(beta_next))
        beta_prev, beta = self.betas[i - 1], self.betas[i]
        counts, ln_q = self.copy_counts(beta_prev, beta, i)
        if int(counts.sum()) == 0:
            raise PopulationExtinct("no copies at step %d" % i)
        # tree order: the copies of parent j sit at adjacent slots, parents ascending
        self.spins = np.ascontiguousarray(np.repeat(self.spins, counts, axis=0))
        self.fam = np.repeat(self.fam, counts)
        self.last_counts = counts
        with mpmath.workprec(PREC_BITS):
            self._acc = self._acc + ln_q
            self._jk = [a + b for a, b in zip(self._jk, self._jk_lnq)]
        self.step = i
        if self.update == "heatbath":
            thr5 = [heatbath_threshold(beta, dE) for dE in (-8, -4, 0, 4, 8)]
            sweeps_heatbath(self.seed, self.L, self.spins, i, self.theta, thr5)
        else:
            t4 = metropolis_threshold(beta, 4)
            t8 = metropolis_threshold(beta, 8)
            sweeps(self.seed, self.L, self.spins, i, self.theta, t4, t8)
        self.E, self.M = energy_magnetisation(self.L, self.spins)
        rec = self._record(ln_q, int((counts.astype(np.int64) ** 2).sum()))
        self.records.append(rec)
        return rec

    @property
    def minus_beta_F(self) -> float:
        return float(self._acc)

    def set_population(self, step: int, spins: np.ndarray, fam: np.ndarray, acc: float,
                       betas: Optional[List[float]] = None) -> None:
        """Adopt a population (e.g. a snapshot) at the given step; E, M recomputed."""
        self.step = step
        self.spins = np.ascontiguousarray(spins, dtype=np.int8).copy()
        self.fam = np.asarray(fam, dtype=np.int32).copy()
        self.E, self.M = energy_magnetisation(self.L, self.spins)
        with mpmath.workprec(PREC_BITS):
            self._acc = mpmath.mpf(acc)
            # the jackknife starts again from the adopted population
            self._jk = [self._acc] * self.n_F
        if betas is not None:
            self.betas = [float(b) for b in betas]


def run(L: int, R: int, betas, theta: int, seed: int, resample: str = "nearest",
        update: str = "metropolis") -> OracleRun:
    """A whole run over the schedule betas[0] = 0 < betas[1] < ... ."""
    o = OracleRun(L, R, theta, seed, resample, np.asarray(betas, dtype=np.float64), update)
    for _ in range(len(betas) - 1):
        o.anneal_step()
    return o
