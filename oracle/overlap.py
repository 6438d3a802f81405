"""Overlap correlation along the population index.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle; shares no code with the
HIP library).  Sec. "Effective population size" (overlap correlation):
copies of one parent sit at adjacent indices, so the overlap of two replicas,

    q(i, j) = (1/N) sum_k s_k^(i) s_k^(j)                    Eq. (overlap_correlation)

decays with their distance |i - j| in index space.  Taking the overlap as
translation invariant in the index, C_q(d) is its mean over all R - d pairs
(i, i + d) of the population; C_q(0) = 1.  The sum over pairs and sites is an
integer, so the value is exact up to the final division.
"""
from __future__ import annotations

from fractions import Fraction
from typing import List

import numpy as np


def overlap_correlation(spins: np.ndarray, d_max: int) -> List[float]:
    """C_q(d) for d = 0 .. d_max of a population spins [R, N] of +-1."""
    s = np.asarray(spins, dtype=np.int64)
    R, N = s.shape
    assert 0 <= d_max < R
    out = []
    for d in range(d_max + 1):
        total = int((s[: R - d] * s[d:]).sum())  # sum over pairs (i, i + d) and sites
        out.append(float(Fraction(total, N * (R - d))))
    return out
