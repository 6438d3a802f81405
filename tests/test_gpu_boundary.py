"""GPU tests of boundary calls and input validation: the energy histogram and
caller-chosen temperatures against the oracle, snapshots that must be
rejected, and the single-run jackknife of the free energy against the spread
of independent runs."""
import math
import struct
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_2102_06611_amd as pa
from oracle import pa_oracle as po
from workloads import linear_schedule, run_seed

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pa.lib()


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("L,R,resample", [(8, 300, "nearest"), (16, 2000, "multinomial"),
                                          (6, 5000, "poisson")])
def test_energy_histogram_matches_oracle(L, R, resample):
    log("histogram", L, R, resample)
    betas = linear_schedule(0.5, 6)
    run = pa.Run(L, R, betas, 2, 77, resample, "msc64")
    ref = po.OracleRun(L, R, 2, 77, resample, betas)
    N = L * L
    for i in range(7):
        if i:
            run.anneal_step()
            ref.anneal_step()
        kmin, counts = run.energy_histogram()
        levels = (ref.E.astype(np.int64) + 2 * N) // 4
        want = np.bincount(levels - levels.min())
        assert kmin == int(levels.min()), i
        assert np.array_equal(counts, want), i
        assert counts.sum() == len(ref.E) and counts[0] > 0 and counts[-1] > 0
    # a cap below the number of bins is refused, nothing written
    kmin = pa.ctypes.c_int32()
    nb = pa.ctypes.c_int32()
    small = np.zeros(1, dtype=np.int32)
    st = pa.lib().pa_energy_histogram(run.h, small.ctypes.data_as(pa.ctypes.POINTER(pa.ctypes.c_int32)),
                                      0, pa.ctypes.byref(kmin), pa.ctypes.byref(nb))
    assert st == pa.PA_ERR_ARG and small[0] == 0
    run.close()


@pytest.mark.parametrize("resample", ["nearest", "multinomial"])
def test_anneal_step_to_matches_oracle(resample):
    # caller-chosen, uneven temperatures (a zero step and a large one included)
    L, R, theta = 8, 400, 3
    betas = [0.0, 0.05, 0.05, 0.2, 0.21, 0.5, 0.9]
    run = pa.Run(L, R, None, theta, 91, resample, "msc64", n_steps=len(betas) - 1)
    ref = po.OracleRun(L, R, theta, 91, resample, np.array([0.0]))
    from test_gpu_parity import check_population, check_record
    for i, b in enumerate(betas[1:], 1):
        run.anneal_step_to(b)
        ref.anneal_step(b)
        check_record(run.observables(i), ref.records[i], "step %d" % i)
        check_population(run, ref, "step %d" % i)
    # no room for another temperature
    with pytest.raises(pa.PAError) as ei:
        run.anneal_step_to(1.0)
    assert ei.value.status == pa.PA_ERR_DONE
    run.close()


def _snapshot_parts(run, blob):
    """Offsets of the snapshot's family, energy and magnetisation arrays: they
    are followed only by the schedule (max_steps + 1 doubles) and the records
    0 .. step."""
    step, R_i = run.current()
    tail = 8 * (run.max_steps + 1) + pa.ctypes.sizeof(pa.pa_obs) * (step + 1)
    fam = len(blob) - tail - 12 * R_i
    return fam, fam + 4 * R_i, fam + 8 * R_i, R_i


def test_corrupted_snapshots_are_rejected():
    betas = linear_schedule(0.4, 8)
    a = pa.Run(8, 300, betas, 2, 5, "nearest", "msc64")
    a.run(4)
    blob = bytearray(a.get_state())
    fam_at, E_at, M_at, R_i = _snapshot_parts(a, blob)
    b = pa.Run(8, 300, betas, 2, 5, "nearest", "msc64")

    def rejected(bad):
        with pytest.raises(pa.PAError) as ei:
            b.set_state(bytes(bad))
        return ei.value.status == pa.PA_ERR_STATE

    # an energy outside [-2N, 2N] (it would index past the histogram)
    bad = bytearray(blob)
    bad[E_at:E_at + 4] = struct.pack("<i", 1 << 20)
    assert rejected(bad)
    # an energy in range that does not belong to the spins
    bad = bytearray(blob)
    e0 = struct.unpack("<i", bytes(bad[E_at:E_at + 4]))[0]
    bad[E_at:E_at + 4] = struct.pack("<i", e0 + 4 if e0 < 128 else e0 - 4)
    assert rejected(bad)
    # a magnetisation of the wrong parity, a family label out of order
    bad = bytearray(blob)
    bad[M_at:M_at + 4] = struct.pack("<i", 1)
    assert rejected(bad)
    bad = bytearray(blob)
    bad[fam_at:fam_at + 4] = struct.pack("<i", 299)
    assert rejected(bad)
    # the good snapshot still restores the run exactly
    b.set_state(bytes(blob))
    a.run(4)
    b.run(4)
    assert a.get_state() == b.get_state()
    a.close()
    b.close()


@pytest.mark.parametrize("L,R,beta_f,n_steps", [(16, 4000, 0.4, 40), (32, 4000, 0.35, 40)])
def test_single_run_free_energy_jackknife_matches_spread_over_runs(L, R, beta_f, n_steps):
    """sigma^2(beta F) from one run's jackknife (averaged over 64 runs) against the
    sample variance of beta F over the same 64 independent runs (pa_batch_weighted,
    relative standard error sqrt(2/63) = 0.18)."""
    log("jackknife vs runs", L, R)
    betas = linear_schedule(beta_f, n_steps)
    specs = [dict(L=L, R=R, theta=10, seed=run_seed(k), resample="nearest", layout="msc64",
                  betas=betas) for k in range(64)]
    b = pa.Batch(specs, stream=torch.cuda.Stream())
    b.run(n_steps)
    b.sync()
    w = b.weighted(0, n_steps + 1)
    for i in (n_steps // 2, n_steps):
        jk = np.array([b.observables(k, i)["jk_var_beta_F"] for k in range(64)])
        assert np.all(jk > 0)
        ratio = jk.mean() / w[i]["var_beta_F"]
        log("step", i, "jackknife", jk.mean(), "runs", w[i]["var_beta_F"], "ratio", ratio)
        assert 0.55 < ratio < 1.7, (i, ratio)
        # the bias estimate cov(e, beta F): one run's jackknife against the runs' covariance,
        # compared on the scale of its standard error over the runs
        cj = np.array([b.observables(k, i)["jk_cov_e"] for k in range(64)])
        sd = math.sqrt(w[i]["var_beta_F"]) * np.std([b.observables(k, i)["e"] for k in range(64)])
        assert abs(cj.mean() - w[i]["cov_e"]) < 3 * sd / math.sqrt(63) + 3 * cj.std() / 8
    b.close()


@pytest.mark.parametrize("resample", ["nearest", "multinomial"])
def test_lower_temperature_stops_the_run_on_the_device(resample):
    # A caller-chosen step to a lower beta is refused by the step's
    # normalisation on the device (sticky PA_ERR_ARG).  The population, its
    # records and the copy counts stay those of the last good step, whichever
    # kernels normalise (multinomial runs at L <= 64 fold it into the weights).
    run = pa.Run(8, 300, None, 2, 17, resample, "msc64", n_steps=6)
    for b in (0.1, 0.2):
        run.anneal_step_to(b)
    run.sync()
    step, R_i = run.current()
    spins, fam, E, M = run.population()
    counts = run.copy_counts()
    rec = run.observables(step)
    run.anneal_step_to(0.15)
    with pytest.raises(pa.PAError) as ei:
        run.sync()
    assert ei.value.status == pa.PA_ERR_ARG
    assert run.current() == (step, R_i)
    s2, f2, E2, M2 = run.population()
    assert np.array_equal(s2, spins) and np.array_equal(f2, fam)
    assert np.array_equal(E2, E) and np.array_equal(M2, M)
    assert np.array_equal(run.copy_counts(), counts)
    assert run.observables(step) == rec
    with pytest.raises(pa.PAError) as ei:
        run.observables(step + 1)
    assert ei.value.status == pa.PA_ERR_ARG
    run.close()
