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


def test_sweep_uniform_is_built_from_bit_planes():
    # lane l's uniform: bit (31 - b) is bit l of plane b; planes 2p, 2p+1 come
    # from Philox call p with counter (w, g, h, 0x10000000 | p)
    seed, w, g, h = 99, 5, 3, 17
    planes = []
    for p in range(16):
        x = po.philox4x32_10(seed, [w, g, h, 0x10000000 | p]).astype(np.uint64)
        planes += [int(x[0] | (x[1] << np.uint64(32))), int(x[2] | (x[3] << np.uint64(32)))]
    for lane in (0, 1, 31, 32, 63):
        u = sum(((planes[b] >> lane) & 1) << (31 - b) for b in range(32))
        assert po.sweep_uniform(seed, w, g, h, lane) == u


def test_stream_uniformity():
    # 64-lane sweep uniforms and resampling uniforms are flat on [0, 2^32)
    us = np.array([po.sweep_uniform(5, w, 0, 1, lane) for w in range(64) for lane in range(64)],
                  dtype=np.float64) / 2 ** 32
    rs = np.array([po.resample_uniform(5, 3, j) for j in range(4096)], dtype=np.float64) / 2 ** 32
    ms = np.array([po.multinomial_uniform(5, 3, d) for d in range(4096)], dtype=np.float64) / 2 ** 64
    for x in (us, rs, ms):
        hist, _ = np.histogram(x, bins=16, range=(0, 1))
        expected = len(x) / 16
        chi2 = ((hist - expected) ** 2 / expected).sum()
        assert chi2 < 50  # 15 dof: p ~ 1e-5
        assert abs(x.mean() - 0.5) < 5 * np.sqrt(1 / 12 / len(x))


def test_init_spins_are_fair_and_seeded():
    s = po.init_spins(1, 8, 640)
    assert set(np.unique(s)) == {-1, 1}
    assert abs(s.astype(np.float64).mean()) < 5 / np.sqrt(s.size)
    assert np.array_equal(s, po.init_spins(1, 8, 640))
    assert not np.array_equal(s, po.init_spins(2, 8, 640))
    # replicas r and r + 64 use different groups of the INIT stream
    assert not np.array_equal(s[0], s[64])
