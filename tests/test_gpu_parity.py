"""GPU parity: the HIP library (through its C-ABI) against the CPU oracle.

Integer results (spins, copy counts, energies, family labels, population
sums) must match bit for bit; ln Q and -beta F within 1e-12 relative; the
other floating-point observables within 1e-12 relative as well (they are
formed from exact integer sums on both sides), and the blocking / jackknife
fields within 1e-9 (see BLOCK_FIELDS).
"""
import ctypes
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_2102_06611_amd as pa
from recordcmp import same_record
from oracle import pa_oracle as po
from workloads import PARITY_SEED, linear_schedule

pytestmark = pytest.mark.gpu

INT_FIELDS = ("step", "R_i", "sum_E", "sum_E2", "sum_absM", "sum_M2", "n_families", "sum_fam2",
              "sum_cnt2")
FP_FIELDS = ("beta", "e", "c_v", "m", "chi", "ln_Q", "minus_beta_F", "rho_t", "rho_s",
             "rho_t_step")
# blocking / jackknife fields: the device forms block means and jackknife
# variances in binary64 from exact integer sums (the oracle in exact rationals);
# a block mean is rounded to ~1e-16 relative and enters differences about 1e-3
# of its size, so the results agree to ~1e-12; 1e-9 leaves a margin
BLOCK_FIELDS = ("r_eff_E", "r_eff_absM", "err_e", "err_m", "err_c_v", "err_chi")
# free-energy jackknife: the device sums each step's ln Q^(k) - ln Q =
# ln(1 - W_k / S) - ln(1 - B_k / R_{i-1}) in binary64 (W_k a binary64 sum of
# level weights, S double-double), about 1e-13 relative per step against the
# oracle's 256-bit samples; a covariance can cancel to far below its terms
# (sum_k (O_k^J - O) d_k with |O_k^J - O| up to about sigma_O + |O|), so it is
# compared on the scale sigma_F (sigma_O + |O|) of those terms
JK_COV = (("jk_cov_e", "err_e", "e"), ("jk_cov_m", "err_m", "m"),
          ("jk_cov_c_v", "err_c_v", "c_v"), ("jk_cov_chi", "err_chi", "chi"))


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pa.lib()


def close(a, b, rel=1e-12):
    if math.isnan(a) or math.isnan(b):
        return math.isnan(a) and math.isnan(b)
    return a == b or abs(a - b) <= rel * max(abs(a), abs(b))


def check_record(got: dict, want, ctx=""):
    for k in INT_FIELDS:
        assert got[k] == getattr(want, k), (ctx, k, got[k], getattr(want, k))
    for k in FP_FIELDS:
        assert close(got[k], getattr(want, k)), (ctx, k, got[k], getattr(want, k))
    for k in BLOCK_FIELDS:
        assert close(got[k], getattr(want, k), 1e-9), (ctx, k, got[k], getattr(want, k))
    check_jackknife(got, want, ctx)


def check_jackknife(got: dict, want, ctx=""):
    vF = want.jk_var_beta_F
    assert close(got["jk_var_beta_F"], vF, 1e-9), (ctx, got["jk_var_beta_F"], vF)
    for k, err, obs in JK_COV:
        a, b = got[k], getattr(want, k)
        if math.isnan(b) or math.isnan(a):
            assert math.isnan(a) and math.isnan(b), (ctx, k, a, b)
            continue
        sd = getattr(want, err)
        scale = math.sqrt(vF) * ((0.0 if math.isnan(sd) else sd) + abs(getattr(want, obs))) \
            if vF > 0 else 0.0
        assert abs(a - b) <= 1e-9 * (abs(b) + scale), (ctx, k, a, b, scale)


def check_population(run: "pa.Run", ref: po.OracleRun, ctx=""):
    spins, fam, E, M = run.population()
    assert spins.shape == ref.spins.shape, ctx
    assert np.array_equal(spins, ref.spins), ctx
    assert np.array_equal(fam, ref.fam), ctx
    assert np.array_equal(E, ref.E), ctx
    assert np.array_equal(M, ref.M), ctx


def test_philox_device_matches_oracle():
    """Every output word of 10^6 counters under three keys, bit for bit."""
    rng = np.random.default_rng(0)
    n = 1_000_000
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:16] = 0
    ctr[16:32] = 0xFFFFFFFF
    ctr[32:96] = np.arange(64, dtype=np.uint32)[:, None]  # neighbouring counters
    dev_ctr = torch.from_numpy(ctr.view(np.int32)).cuda()
    dev_out = torch.zeros_like(dev_ctr)
    for key in (0, 12345, 2 ** 64 - 1):
        log("philox", key, n)
        pa.philox4x32_10(key, dev_ctr, dev_out)
        torch.cuda.synchronize()
        out = dev_out.cpu().numpy().view(np.uint32)
        ref = po.philox4x32_10_many(key, ctr)
        bad = np.flatnonzero((out != ref).any(axis=1))
        assert bad.size == 0, (key, bad[:8])
    # odd lengths: the grid's last block is partial and nothing past n is written
    for m in (1, 255, 257):
        dev_out.fill_(-1)
        pa.philox4x32_10(99, dev_ctr[:m], dev_out[:m])
        torch.cuda.synchronize()
        out = dev_out.cpu().numpy().view(np.uint32)
        assert np.array_equal(out[:m], po.philox4x32_10_many(99, ctr[:m]))
        assert (out[m:m + 300] == 0xFFFFFFFF).all()


@pytest.mark.parametrize("layout", ["msc64", "int8"])
@pytest.mark.parametrize("L,R", [(8, 200), (6, 64), (4, 1), (12, 130)])
def test_initial_population_matches_oracle(layout, L, R):
    log("init", layout, L, R)
    betas = linear_schedule(0.3, 2)
    run = pa.Run(L, R, betas, 1, PARITY_SEED, "nearest", layout)
    ref = po.OracleRun(L, R, 1, PARITY_SEED, "nearest", betas)
    check_record(run.observables(0), ref.records[0], "record 0")
    check_population(run, ref, "init")
    run.close()


CASES = [
    # L, R, theta, n_steps, beta_f, resample, layout
    (8, 200, 3, 8, 0.44, "nearest", "msc64"),
    (8, 200, 3, 8, 0.44, "nearest", "int8"),
    (6, 130, 2, 6, 0.6, "multinomial", "msc64"),
    (6, 130, 2, 6, 0.6, "multinomial", "int8"),
    (4, 64, 5, 10, 1.2, "nearest", "msc64"),
    (10, 1, 2, 5, 0.5, "nearest", "msc64"),
    (8, 300, 0, 5, 0.8, "nearest", "msc64"),
    (16, 150, 2, 4, 0.44, "multinomial", "msc64"),
    (12, 100, 2, 4, 2.0, "none", "int8"),
    # several 1024-slot blocks and strong selection: families span block
    # boundaries (the first grows one family over five blocks)
    (6, 5000, 0, 6, 2.0, "nearest", "msc64"),
    (4, 5000, 1, 6, 3.0, "multinomial", "int8"),
    (6, 5000, 0, 6, 2.0, "multinomial", "msc64"),
    # one jump to beta = 5: a few parents fill whole 64-replica child groups
    # (the multispin copy's spread network at its deepest shifts)
    (4, 3000, 0, 2, 5.0, "nearest", "msc64"),
    (4, 3000, 0, 2, 5.0, "multinomial", "msc64"),
    # a thousand sweeps per step: half-sweep counters h = 2 (theta (i - 1) + s)
    # + colour up to 6000, in both layouts
    (4, 130, 1000, 3, 0.44, "nearest", "msc64"),
    (4, 130, 1000, 3, 0.44, "multinomial", "int8"),
    # more than 4096 stretches of 64 parents: the multinomial draws search the
    # parent blocks' bases and the dense stretch ends instead of the LDS index
    # of every stretch
    (4, 300000, 1, 2, 0.6, "multinomial", "msc64"),
    # L = 128 multinomial: the normalisation runs in its own launch (the
    # weights kernel folds it in only up to L = 64), with a partial second group
    (128, 130, 1, 3, 0.5, "multinomial", "msc64"),
    # strong selection at other sizes and with the other copy rules: one or a
    # few parents take nearly all the weight in the first steps
    (128, 130, 1, 3, 0.5, "nearest", "int8"),
    (128, 100, 1, 3, 0.5, "poisson", "msc64"),
    (64, 70, 2, 3, 1.0, "multinomial", "msc64"),
    (32, 200, 1, 2, 1.5, "nearest", "msc64"),
    # Poisson resampling: fluctuating R_i, several blocks, strong selection
    (8, 200, 3, 8, 0.44, "poisson", "msc64"),
    (6, 130, 2, 6, 0.6, "poisson", "int8"),
    (4, 64, 5, 10, 1.2, "poisson", "msc64"),
    (6, 5000, 0, 6, 2.0, "poisson", "msc64"),
]


@pytest.mark.parametrize("L,R,theta,n,bf,resample,layout", CASES)
def test_run_parity_step_by_step(L, R, theta, n, bf, resample, layout):
    log("run parity", L, R, theta, n, bf, resample, layout)
    betas = linear_schedule(bf, n)
    run = pa.Run(L, R, betas, theta, PARITY_SEED, resample, layout)
    ref = po.OracleRun(L, R, theta, PARITY_SEED, resample, betas)
    for i in range(1, n + 1):
        run.anneal_step()
        ref.anneal_step()
        check_record(run.observables(i), ref.records[i], "step %d" % i)
        assert np.array_equal(run.copy_counts(), ref.last_counts), i
        check_population(run, ref, "step %d" % i)
    run.close()


@pytest.mark.slow
def test_small_nearest_workload_full_run():
    """L=8, R=1000, beta 0 -> 0.44 in 101 steps, theta=10, nearest, int8."""
    L, R, theta, n = 8, 1000, 10, 101
    betas = linear_schedule(0.44, n)
    run = pa.Run(L, R, betas, theta, PARITY_SEED, "nearest", "int8")
    run.run(n)
    run.sync()
    ref = po.run(L, R, betas, theta, PARITY_SEED, "nearest")
    for i in range(n + 1):
        check_record(run.observables(i), ref.records[i], "step %d" % i)
    check_population(run, ref, "final")
    run.close()


def test_layouts_give_identical_trajectories():
    L, R, n = 32, 5000, 10
    betas = linear_schedule(0.44, n)
    a = pa.Run(L, R, betas, 4, 7, "nearest", "msc64")
    b = pa.Run(L, R, betas, 4, 7, "nearest", "int8")
    a.run(n)
    b.run(n)
    for i in range(n + 1):
        assert same_record(a.observables(i), b.observables(i)), i
    sa, fa, Ea, Ma = a.population()
    sb, fb, Eb, Mb = b.population()
    assert np.array_equal(sa, sb) and np.array_equal(fa, fb) and np.array_equal(Ea, Eb)


def test_graph_replay_matches_stepping():
    L, R, n = 16, 3000, 12
    betas = linear_schedule(0.5, n)
    s = torch.cuda.Stream()
    a = pa.Run(L, R, betas, 3, 11, "nearest", "msc64", stream=s)
    b = pa.Run(L, R, betas, 3, 11, "nearest", "msc64")
    a.run(n)
    for _ in range(n):
        b.anneal_step()
    a.sync()
    b.sync()
    for i in range(n + 1):
        assert same_record(a.observables(i), b.observables(i)), i
    assert a.get_state() == b.get_state()


def test_same_seed_is_bit_identical_and_seed_matters():
    betas = linear_schedule(0.44, 6)
    blobs = []
    for seed in (5, 5, 6):
        r = pa.Run(16, 700, betas, 3, seed, "multinomial", "msc64")
        r.run(6)
        blobs.append(r.get_state())
        r.close()
    assert blobs[0] == blobs[1]
    assert blobs[0] != blobs[2]


@pytest.mark.parametrize("L,R,resample,layout,update", [(12, 500, "nearest", "int8", "metropolis"),
                                                       (128, 700, "multinomial", "msc64", "metropolis"),
                                                       (64, 300, "poisson", "int8", "heatbath")])
def test_checkpoint_resume_is_bit_identical(L, R, resample, layout, update):
    betas = linear_schedule(0.6, 10)
    a = pa.Run(L, R, betas, 2, 3, resample, layout, update=update)
    a.run(4)
    blob = a.get_state()
    a.run(6)
    b = pa.Run(L, R, betas, 2, 3, resample, layout, update=update)
    b.set_state(blob)
    b.run(6)
    assert a.get_state() == b.get_state()
    for i in range(11):
        assert same_record(a.observables(i), b.observables(i))


def test_set_population_resumes_like_the_oracle():
    L, R, theta = 8, 150, 2
    betas = linear_schedule(0.5, 6)
    ref = po.OracleRun(L, R, theta, 9, "nearest", betas)
    for _ in range(3):
        ref.anneal_step()
    run = pa.Run(L, R, betas, theta, 9, "nearest", "msc64")
    run.set_population(3, ref.spins, ref.fam, ref.minus_beta_F)
    # both sides adopt: the free-energy jackknife starts again at step 3
    ref.set_population(3, ref.spins, ref.fam, ref.minus_beta_F)
    check_population(run, ref, "adopted")
    for i in range(4, 7):
        run.anneal_step()
        ref.anneal_step()
        check_record(run.observables(i), ref.records[i], "step %d" % i)
        check_population(run, ref, "step %d" % i)


def test_zero_temperature_step_is_the_identity_before_sweeps():
    betas = np.array([0.0, 0.0, 0.0])
    run = pa.Run(8, 256, betas, 0, 4, "nearest", "msc64")
    s0, f0, _, _ = run.population()
    run.anneal_step()
    o = run.observables(1)
    assert o["ln_Q"] == 0.0 and o["R_i"] == 256
    assert np.all(run.copy_counts() == 1)
    s1, f1, _, _ = run.population()
    assert np.array_equal(s0, s1) and np.array_equal(f0, f1)


def test_capacity_overflow_is_reported_and_state_kept():
    L, R = 8, 128
    betas = linear_schedule(0.6, 40)
    run = pa.Run(L, R, betas, 1, 2, "nearest", "msc64", capacity=128)
    ref = po.OracleRun(L, R, 1, 2, "nearest", betas)
    for _ in range(40):
        run.anneal_step()
    with pytest.raises(pa.PAError) as ei:
        run.sync()
    assert ei.value.status == pa.PA_ERR_CAPACITY
    step, R_i = run.current()
    # the oracle (no capacity limit) reaches the same population at that step
    for _ in range(step):
        ref.anneal_step()
    assert len(ref.E) == R_i <= 128
    check_population(run, ref, "kept step %d" % step)
    ref.anneal_step()
    assert len(ref.E) > 128  # the step that overflowed


HEATBATH_CASES = [
    # L, R, theta, betas, resample, layout
    (8, 200, 3, linear_schedule(0.44, 8), "nearest", "msc64"),
    (8, 200, 3, linear_schedule(0.44, 8), "nearest", "int8"),
    (6, 130, 2, linear_schedule(0.6, 6), "multinomial", "int8"),
    (4, 64, 5, linear_schedule(1.2, 10), "poisson", "msc64"),
    (12, 100, 2, linear_schedule(3.0, 4), "none", "msc64"),  # large beta: small T'
    (10, 1, 2, linear_schedule(0.5, 5), "nearest", "msc64"),
    (16, 150, 2, [0.0, 0.0, 0.0, 0.2, 0.4], "nearest", "msc64"),  # beta = 0: fair coins
    # L = 128 and strong selection (normalisation in its own launch)
    (128, 130, 1, linear_schedule(0.5, 3), "multinomial", "msc64"),
    (64, 100, 2, linear_schedule(0.8, 3), "nearest", "int8"),
]


@pytest.mark.parametrize("L,R,theta,betas,resample,layout", HEATBATH_CASES)
def test_heatbath_run_parity_step_by_step(L, R, theta, betas, resample, layout):
    log("heatbath parity", L, R, theta, betas[-1], resample, layout)
    n = len(betas) - 1
    run = pa.Run(L, R, betas, theta, PARITY_SEED, resample, layout, update="heatbath")
    ref = po.OracleRun(L, R, theta, PARITY_SEED, resample, betas, update="heatbath")
    for i in range(1, n + 1):
        run.anneal_step()
        ref.anneal_step()
        check_record(run.observables(i), ref.records[i], "step %d" % i)
        assert np.array_equal(run.copy_counts(), ref.last_counts), i
        check_population(run, ref, "step %d" % i)
    run.close()


def test_update_rules_differ_and_snapshots_keep_the_rule():
    betas = linear_schedule(0.44, 3)
    a = pa.Run(8, 128, betas, 2, 3, "nearest", "msc64")
    b = pa.Run(8, 128, betas, 2, 3, "nearest", "msc64", update="heatbath")
    a.run(3)
    b.run(3)
    assert not np.array_equal(a.population()[0], b.population()[0])
    with pytest.raises(pa.PAError) as ei:
        b.set_state(a.get_state())
    assert ei.value.status == pa.PA_ERR_STATE
    a.close()
    b.close()


@pytest.mark.slow
def test_poisson_mean_limit():
    """beta 0 -> 50 in one step at L=6, R=100000 with theta = 0: nearly all the
    weight sits on the lowest occupied level.  Seed 4 has one replica there,
    so tau_hat ~ 1e5 exceeds the supported 65536 and the step stops with
    PA_ERR_NUMERIC; seed 1 has four (tau_hat ~ 25000) and its copy counts match
    the oracle's."""
    L, R, betas = 6, 100_000, [0.0, 50.0]
    run = pa.Run(L, R, betas, 0, 4, "poisson", "msc64")
    run.anneal_step()
    with pytest.raises(pa.PAError) as ei:
        run.sync()
    assert ei.value.status == pa.PA_ERR_NUMERIC
    assert run.current() == (0, R)
    run.close()
    run = pa.Run(L, R, betas, 0, 1, "poisson", "msc64")
    run.anneal_step()
    run.sync()
    ref = po.OracleRun(L, R, 0, 1, "poisson", betas)
    ref.anneal_step()
    counts = run.copy_counts()
    assert np.array_equal(counts, ref.last_counts)
    assert counts.max() > 10000
    check_record(run.observables(1), ref.records[1], "seed 1")
    run.close()


def test_extinct_population_is_reported():
    # R = 2, Poisson: for some seeds both parents draw zero copies at step 1
    # (seeds 27 and 35 among 20..39); the device reports PA_ERR_EXTINCT
    # exactly where the oracle stops
    L, R, betas = 4, 2, [0.0, 0.3, 0.6]
    extinct = 0
    for seed in range(20, 40):
        ref = po.OracleRun(L, R, 1, seed, "poisson", betas)
        run = pa.Run(L, R, betas, 1, seed, "poisson", "msc64")
        try:
            ref.anneal_step()
            ok = True
        except po.PopulationExtinct:
            ok = False
        run.anneal_step()
        if ok:
            run.sync()
            check_record(run.observables(1), ref.records[1], "seed %d" % seed)
        else:
            with pytest.raises(pa.PAError) as ei:
                run.sync()
            assert ei.value.status == pa.PA_ERR_EXTINCT, seed
            assert run.current() == (0, R)  # the population before the step is kept
            extinct += 1
        run.close()
    assert extinct > 0


def test_schedule_end_is_reported():
    run = pa.Run(8, 64, linear_schedule(0.3, 2), 1, 1, "nearest", "msc64")
    run.anneal_step()
    run.anneal_step()
    with pytest.raises(pa.PAError) as ei:
        run.anneal_step()
    assert ei.value.status == pa.PA_ERR_DONE
    run.sync()


def _sampled_step_parity(L, R, resample, layout, n_steps, beta_f, k, theta, seed, n_groups=6,
                         update="metropolis"):
    """GPU step k -> k+1 at full size; the oracle recomputes the copy counts of
    all parents and the sweeps of a sample of replica groups."""
    betas = linear_schedule(beta_f, n_steps)
    s = torch.cuda.Stream()
    run = pa.Run(L, R, betas, theta, seed, resample, layout, stream=s, update=update)
    run.run(k)
    run.sync()
    snap_spins, snap_fam, snap_E, _ = run.population()
    acc = run.observables(k)["minus_beta_F"]
    run.anneal_step()
    got = run.observables(k + 1)
    counts = run.copy_counts()
    ref = po.OracleRun(L, 4, theta, seed, resample, betas)  # population replaced below
    ref.R = R
    ref.E = snap_E.copy()
    ref_counts, ln_q = ref.copy_counts(betas[k], betas[k + 1], k + 1)
    assert np.array_equal(counts, ref_counts)
    assert got["R_i"] == int(ref_counts.sum())
    assert close(got["ln_Q"], float(ln_q))
    assert close(got["minus_beta_F"], acc + float(ln_q), 1e-12)
    off = np.concatenate([[0], np.cumsum(ref_counts)])
    R_new = int(off[-1])
    G = (R_new + 63) // 64
    rng = np.random.default_rng(seed)
    groups = sorted(set([0, G - 1] + list(rng.integers(0, G, n_groups))))
    t4, t8 = po.metropolis_threshold(betas[k + 1], 4), po.metropolis_threshold(betas[k + 1], 8)
    thr5 = [po.heatbath_threshold(betas[k + 1], dE) for dE in (-8, -4, 0, 4, 8)]
    for g in groups:
        lo, hi = 64 * g, min(64 * g + 64, R_new)
        parents = np.searchsorted(off, np.arange(lo, hi), side="right") - 1
        kids = np.ascontiguousarray(snap_spins[parents])
        if update == "heatbath":
            po.sweeps_heatbath(seed, L, kids, k + 1, theta, thr5, slot0=lo)
        else:
            po.sweeps(seed, L, kids, k + 1, theta, t4, t8, slot0=lo)
        E, M = po.energy_magnetisation(L, kids)
        gs, gf, gE, gM = run.population(lo, hi - lo)
        assert np.array_equal(gs, kids), g
        assert np.array_equal(gf, snap_fam[parents]), g
        assert np.array_equal(gE, E) and np.array_equal(gM, M), g
    run.close()


@pytest.mark.slow
@pytest.mark.parametrize("layout,k", [("msc64", 120), ("int8", 120), ("msc64", 199)])
def test_l64_multinomial_sampled_step_parity(layout, k):
    """L=64, R=100000, multinomial, beta 0 -> 0.4407 in 200 steps: step k -> k + 1
    (k = 199: the last step, into beta_c, where few families are left)."""
    log("L64 sampled", layout, k)
    _sampled_step_parity(64, 100_000, "multinomial", layout, 200, 0.4407, k, 10, PARITY_SEED)


@pytest.mark.slow
@pytest.mark.parametrize("L,k,layout,resample", [(64, 120, "msc64", "nearest"),
                                                (64, 150, "msc64", "multinomial"),
                                                (128, 180, "msc64", "nearest"),
                                                (128, 180, "int8", "nearest")])
def test_heatbath_sampled_step_parity(L, k, layout, resample):
    """Heatbath at full size: L=64 (one group per block, one word per thread;
    nearest and multinomial copies) and L=128 (two words per thread, both
    layouts), R=100000."""
    log("heatbath sampled", L, layout, resample)
    n, bf = (200, 0.4407) if L == 64 else (400, 1.0)
    _sampled_step_parity(L, 100_000, resample, layout, n, bf, k, 10, PARITY_SEED, 3,
                         update="heatbath")


@pytest.mark.slow
@pytest.mark.parametrize("layout", ["msc64", "int8"])
def test_l64_poisson_sampled_step_parity(layout):
    """L=64, R=100000, Poisson, beta 0 -> 0.4407 in 200 steps: step 120 -> 121."""
    log("L64 sampled poisson", layout)
    _sampled_step_parity(64, 100_000, "poisson", layout, 200, 0.4407, 120, 10, PARITY_SEED)


@pytest.mark.slow
@pytest.mark.parametrize("layout", ["msc64", "int8"])
def test_l128_nearest_sampled_step_parity(layout):
    """L=128, R=100000, nearest, beta 0 -> 1.0 in 400 steps: step 180 -> 181 (the
    lattice fills most of a CU's LDS, so the sweep takes two words per thread)."""
    log("L128 sampled", layout)
    _sampled_step_parity(128, 100_000, "nearest", layout, 400, 1.0, 180, 10, PARITY_SEED, 3)


def _check_full_population(run, rec, L, rng, n_samples=8):
    """Record sums against every replica's E and M, tree order of the family
    labels and their count, and E, M of sampled stretches of 64 replicas
    against the oracle's evaluation of their spins."""
    _, fam, E, M = run.population(spins=False)
    E64, M64 = E.astype(np.int64), M.astype(np.int64)
    assert rec["sum_E"] == int(E64.sum()) and rec["sum_E2"] == int((E64 * E64).sum())
    assert rec["sum_absM"] == int(np.abs(M64).sum()) and rec["sum_M2"] == int((M64 * M64).sum())
    assert np.all(np.diff(fam) >= 0)  # copies of one parent adjacent, parents ascending
    assert rec["n_families"] == len(np.unique(fam))
    for first in rng.choice(rec["R_i"] - 64, n_samples, replace=False):
        spins, _, Es, Ms = run.population(int(first), 64)
        Eo, Mo = po.energy_magnetisation(L, spins)
        assert np.array_equal(Es, Eo) and np.array_equal(Ms, Mo), first
    return E


def test_largest_population_nearest():
    # R = 2^24, the largest population the boundary accepts, at L = 4: two
    # steps of nearest-integer resampling with one sweep each.  The copy counts
    # of 2000 random parents are compared with the oracle's one-parent rule;
    # the rest holds at any size (count totals, record sums, tree order).
    L, R, theta = 4, 1 << 24, 1
    log("largest population, nearest", L, R)
    betas = linear_schedule(0.5, 2)
    run = pa.Run(L, R, betas, theta, PARITY_SEED, "nearest", "msc64")
    rng = np.random.default_rng(5)
    _, _, E_prev, _ = run.population(spins=False)
    for i in (1, 2):
        values, mult = np.unique(E_prev, return_counts=True)
        levels = {int(e): int(n) for e, n in zip(values, mult)}
        run.anneal_step()
        rec = run.observables(i)
        counts = run.copy_counts()
        assert len(counts) == len(E_prev)
        assert int(counts.sum(dtype=np.int64)) == rec["R_i"]
        assert int((counts.astype(np.int64) ** 2).sum()) == rec["sum_cnt2"]
        for j in rng.choice(len(E_prev), 2000, replace=False):
            want = po.nearest_count(PARITY_SEED, i, R, levels, betas[i - 1], betas[i],
                                    int(E_prev[j]), int(j))
            assert counts[j] == want, (i, int(j))
        E_prev = _check_full_population(run, rec, L, rng)
    run.close()


def test_largest_multinomial_population():
    # R = 2^23 - 1, the largest multinomial population (its quantised weights
    # total below 2^63), at L = 4.  The first step has dbeta = 0: every weight
    # is 2^40, so the draws' total W = R 2^40 is the largest the kernels meet,
    # and the copy counts are multinomial with equal probabilities, whose share
    # of childless parents is (1 - 1/R)^R (within six standard deviations).
    L, R = 4, (1 << 23) - 1
    log("largest population, multinomial", L, R)
    betas = [0.0, 0.0, 0.3]
    run = pa.Run(L, R, betas, 1, PARITY_SEED, "multinomial", "msc64")
    rng = np.random.default_rng(6)
    for i in (1, 2):
        run.anneal_step()
        rec = run.observables(i)
        counts = run.copy_counts()
        assert rec["R_i"] == R and int(counts.sum(dtype=np.int64)) == R
        assert int((counts.astype(np.int64) ** 2).sum()) == rec["sum_cnt2"]
        if i == 1:
            p0 = (1.0 - 1.0 / R) ** R
            assert abs(float(np.mean(counts == 0)) - p0) < 6.0 * math.sqrt(p0 * (1 - p0) / R)
            assert rec["ln_Q"] == 0.0
        _check_full_population(run, rec, L, rng)
    run.close()
