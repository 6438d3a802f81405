"""Pins of the oracle's overlap correlation C_q(d) along the population index
(Eq. overlap_correlation): closed forms for populations built from blocks of
mutually orthogonal (Walsh) patterns, alternating signs, brute force over
explicit pairs, and the decay in a real tree-ordered population."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import overlap as ov
from oracle import pa_oracle as po


def walsh(n_bits: int) -> np.ndarray:
    """2^n_bits mutually orthogonal +-1 rows of length 2^n_bits (Sylvester)."""
    H = np.array([[1]], dtype=np.int64)
    for _ in range(n_bits):
        H = np.block([[H, H], [H, -H]])
    return H


@pytest.mark.parametrize("B,n_blocks", [(1, 40), (5, 12), (64, 3), (7, 9)])
def test_blocks_of_orthogonal_patterns(B, n_blocks):
    # replicas i in block b are all the b-th Walsh row; rows are orthogonal,
    # so q(i, i + d) = 1 inside a block and 0 across blocks: C_q(d) = the
    # fraction of the R - d pairs that stay inside one block
    H = walsh(6)  # N = 64, an 8 x 8 lattice
    spins = np.repeat(H[:n_blocks], B, axis=0)
    R = B * n_blocks
    got = ov.overlap_correlation(spins, R - 1)
    for d in range(R):
        inside = n_blocks * max(B - d, 0)
        assert got[d] == float(Fraction(inside, R - d)), d


def test_alternating_signs():
    # replica i = (-1)^i times one pattern: C_q(d) = (-1)^d exactly
    rng = np.random.default_rng(3)
    p = rng.choice([-1, 1], size=36)
    spins = np.array([p * (1 if i % 2 == 0 else -1) for i in range(21)])
    assert ov.overlap_correlation(spins, 20) == [(-1.0) ** d for d in range(21)]


def test_brute_force_pairs():
    rng = np.random.default_rng(4)
    spins = rng.choice([-1, 1], size=(17, 16))
    got = ov.overlap_correlation(spins, 16)
    for d in range(17):
        pairs = [sum(int(spins[i, k]) * int(spins[i + d, k]) for k in range(16)) for i in range(17 - d)]
        assert got[d] == float(Fraction(sum(pairs), 16 * (17 - d)))


def test_tree_ordered_population_decays():
    # near the critical point with theta = 1 neighbouring replicas often share
    # a recent parent: C_q is clearly positive at small d and decays with d
    from workloads import linear_schedule
    o = po.run(8, 2000, linear_schedule(0.44, 30), 1, 17, "nearest")
    c = ov.overlap_correlation(o.spins, 200)
    assert c[0] == 1.0
    assert c[1] > c[2] > c[5] > 0.05
    assert max(abs(x) for x in c[50:]) < c[1] / 4
