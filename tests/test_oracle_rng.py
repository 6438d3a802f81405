"""Pins for the oracle's Philox4x32-10 and its random streams (no GPU).

The oracle's Philox is checked against rocRAND's Philox4x32-10 (a separate
implementation, compiled here from its header and run on the host), and the
streams built on it are checked for the properties the method relies on.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import pa_oracle as po

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND header / hipcc not available")
    exe = str(tmp_path_factory.mktemp("rocrand") / "philox_ref")
    subprocess.check_call([hipcc, "-O1", "-o", exe, os.path.join(HERE, "rocrand_philox_ref.cpp")])
    return exe


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(7)
    queries = []
    for _ in range(2000):
        seed = int(rng.integers(0, 2 ** 63)) * 2 + int(rng.integers(0, 2))
        ctr = [int(x) for x in rng.integers(0, 2 ** 32, size=4, dtype=np.uint64)]
        ctr[1] &= 2 ** 30 - 1  # rocRAND's offset counts 32-bit outputs in 64 bits
        queries.append((seed, ctr))
    # edge counters and keys
    for seed in (0, 1, 2 ** 64 - 1, 12345):
        for ctr in ([0, 0, 0, 0], [2 ** 32 - 1, 2 ** 30 - 1, 2 ** 32 - 1, 2 ** 32 - 1],
                    [1, 0, 0, 0], [0, 0, 0, 0x10000000]):
            queries.append((seed, ctr))
    text = "".join("%d %d %d %d %d\n" % (s, *c) for s, c in queries)
    out = subprocess.run([rocrand_ref], input=text, capture_output=True, text=True, check=True).stdout
    ref = [list(map(int, line.split())) for line in out.strip().splitlines()]
    assert len(ref) == len(queries)
    for (seed, ctr), r in zip(queries, ref):
        assert list(po.philox4x32_10(seed, ctr)) == r, (seed, ctr)
    # the batched form, one key over many counters
    for seed in (0, 12345, 2 ** 64 - 1):
        idx = [i for i, (s, _) in enumerate(queries) if s == seed]
        ctrs = np.array([queries[i][1] for i in idx], dtype=np.uint32)
        got = po.philox4x32_10_many(seed, ctrs)
        assert got.shape == (len(idx), 4)
        assert [list(map(int, g)) for g in got] == [ref[i] for i in idx]
    assert po.philox4x32_10_many(7, np.zeros((0, 4), dtype=np.uint32)).shape == (0, 4)


def test_sweep_uniform_top_bits_and_ties_follow_the_stream_map():
    # lane l's top six bits: bit (5 - b) is bit l of plane b; planes 2p, 2p+1
    # come from call (w, g, h, 0x10000000 | p).  A lane whose top six bits equal
    # its threshold's takes its low 26 bits from word k & 3 of call (w, g, h,
    # 0x10000100 | k >> 2), k = its rank among the tied lanes.
    seed, w, g, h = 99, 5, 3, 17
    planes = []
    for p in range(3):
        x = po.philox4x32_10(seed, [w, g, h, 0x10000000 | p]).astype(np.uint64)
        planes += [int(x[0] | (x[1] << np.uint64(32))), int(x[2] | (x[3] << np.uint64(32)))]
    top = [sum(((planes[b] >> lane) & 1) << (5 - b) for b in range(6)) for lane in range(64)]
    for lane in (0, 1, 31, 32, 63):
        assert po.sweep_top6(seed, w, g, h, lane) == top[lane]
    # thresholds that tie every other lane, skip lane 7 entirely
    thr = [((top[l] if l % 2 == 0 else top[l] ^ 1) << 26) | 0x1234567 for l in range(64)]
    needs = [l != 7 for l in range(64)]
    u = po.word_uniforms(seed, w, g, h, thr, needs)
    tied = [l for l in range(64) if needs[l] and l % 2 == 0]
    for k, l in enumerate(tied):
        x = po.philox4x32_10(seed, [w, g, h, 0x10000100 | (k >> 2)])
        assert int(u[l]) == (top[l] << 26) | (int(x[k & 3]) >> 6)
    for l in range(64):
        if not needs[l]:
            assert u[l] == 0
        elif l % 2:
            assert int(u[l]) == top[l] << 26


def _acceptance(seed, thr_of_lane, n_words):
    """Fraction of u < thr over n_words words (all lanes comparing)."""
    acc = np.zeros(64)
    for w in range(n_words):
        thr = [thr_of_lane(l) for l in range(64)]
        u = po.word_uniforms(seed, w, 1, 2, thr, [True] * 64).astype(np.uint64)
        acc += u < np.asarray(thr, dtype=np.uint64)
    return acc / n_words


@pytest.mark.parametrize("T", [1, 0x02000000, 0x03FFFFFF, 0x7C000001, 0x8000_0000, 0xB504F334,
                               0xFFFFFFFF])
def test_comparison_with_tied_top_bits_is_exact_bernoulli(T):
    # u < T must hold with probability T / 2^32 whether it is decided by the
    # top six bits or by a tie's 26 fresh bits (thresholds with small, zero and
    # full low parts; one per lane class)
    n = 400
    p = T / 2.0 ** 32
    frac = _acceptance(31, lambda l: T, n).mean()
    sigma = np.sqrt(p * (1 - p) / (64 * n))
    assert abs(frac - p) <= 5 * sigma + 1e-12


def test_comparison_with_mixed_thresholds_per_lane():
    # lanes of one word comparing with two thresholds (the dE = 4 and dE = 8
    # classes) keep their own acceptance probabilities while sharing tie draws
    t4, t8 = 0x9A3C2B11, 0x07A5D003
    n = 600
    frac = _acceptance(7, lambda l: t4 if l % 3 else t8, n)
    for lanes, t in (([l for l in range(64) if l % 3], t4), ([l for l in range(64) if l % 3 == 0], t8)):
        p = t / 2.0 ** 32
        f = frac[lanes].mean()
        assert abs(f - p) <= 5 * np.sqrt(p * (1 - p) / (len(lanes) * n))


def test_stream_uniformity():
    # top six bits of the sweep uniforms, resampling and multinomial uniforms
    # are flat
    ts = np.array([po.sweep_top6(5, w, 0, 1, lane) for w in range(64) for lane in range(64)],
                  dtype=np.float64) / 64
    rs = np.array([po.resample_uniform(5, 3, j) for j in range(4096)], dtype=np.float64) / 2 ** 32
    ms = np.array([po.multinomial_uniform(5, 3, d) for d in range(4096)], dtype=np.float64) / 2 ** 64
    for x in (ts, rs, ms):
        hist, _ = np.histogram(x, bins=16, range=(0, 1))
        expected = len(x) / 16
        chi2 = ((hist - expected) ** 2 / expected).sum()
        assert chi2 < 50  # 15 dof: p ~ 1e-5
        assert abs(x.mean() + (1 / 128 if x is ts else 0) - 0.5) < 5 * np.sqrt(1 / 12 / len(x))


def test_init_spins_are_fair_and_seeded():
    s = po.init_spins(1, 8, 640)
    assert set(np.unique(s)) == {-1, 1}
    assert abs(s.astype(np.float64).mean()) < 5 / np.sqrt(s.size)
    assert np.array_equal(s, po.init_spins(1, 8, 640))
    assert not np.array_equal(s, po.init_spins(2, 8, 640))
    # replicas r and r + 64 use different groups of the INIT stream
    assert not np.array_equal(s[0], s[64])
