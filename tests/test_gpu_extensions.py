"""GPU tests of the batched engine, the adaptive schedule and the learned
(perceptron) schedule, against the CPU oracle and against single runs."""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_2102_06611_amd as pa
from recordcmp import same_record
from paper_2102_06611_amd import schedules
from oracle import mlp
from oracle import pa_oracle as po
from workloads import PARITY_SEED, linear_schedule

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pa.lib()


def log(*a):
    print(*a, flush=True)


def test_batch_of_uneven_runs_matches_single_runs_and_oracle():
    n = 5
    specs = [dict(L=8, R=100, theta=2, seed=21, resample="nearest", layout="msc64"),
             dict(L=16, R=300, theta=3, seed=22, resample="multinomial", layout="int8"),
             dict(L=6, R=70, theta=1, seed=23, resample="nearest", layout="msc64"),
             dict(L=8, R=64, theta=2, seed=24, resample="nearest", layout="int8"),
             dict(L=16, R=129, theta=2, seed=25, resample="nearest", layout="msc64")]
    for k, s in enumerate(specs):
        s["betas"] = linear_schedule(0.3 + 0.1 * k, n)
    stream = torch.cuda.Stream()
    b = pa.Batch(specs, stream=stream)
    b.run(n)
    b.sync()
    for k, s in enumerate(specs):
        single = pa.Run(s["L"], s["R"], s["betas"], s["theta"], s["seed"], s["resample"],
                        s["layout"])
        single.run(n)
        for i in range(n + 1):
            assert same_record(b.observables(k, i), single.observables(i)), (k, i)
        single.close()
    ref = po.run(8, 100, specs[0]["betas"], 2, 21, "nearest")
    for i in range(n + 1):
        got = b.observables(0, i)
        assert got["sum_E"] == ref.records[i].sum_E and got["R_i"] == ref.records[i].R_i
    b.close()


def test_batch_mixing_every_copy_rule_and_size_matches_single_runs():
    """One batch holding L = 128 and 64 multinomial runs beside nearest, Poisson
    and heatbath ones: the batch normalises every run in k_norm (a multinomial
    run alone at L <= 64 folds it into its weights' launch instead), and every
    record must equal that of the same run made alone."""
    n = 4
    specs = [dict(L=128, R=130, theta=1, seed=31, resample="multinomial", layout="msc64"),
             dict(L=64, R=700, theta=2, seed=32, resample="multinomial", layout="int8"),
             dict(L=64, R=300, theta=1, seed=33, resample="poisson", layout="msc64"),
             dict(L=32, R=1000, theta=2, seed=34, resample="nearest", layout="msc64",
                  update="heatbath"),
             dict(L=8, R=65, theta=3, seed=35, resample="none", layout="int8")]
    for k, s in enumerate(specs):
        s["betas"] = linear_schedule(0.4 + 0.2 * k, n)
    b = pa.Batch(specs)
    b.run(n)
    b.sync()
    for k, s in enumerate(specs):
        single = pa.Run(s["L"], s["R"], s["betas"], s["theta"], s["seed"], s["resample"],
                        s["layout"], update=s.get("update", "metropolis"))
        single.run(n)
        for i in range(n + 1):
            assert same_record(b.observables(k, i), single.observables(i)), (k, i)
        single.close()
    b.close()


def _close_weighted(got, want, ctx):
    from oracle import weighted as wt
    assert got["step"] == want["step"] and got["n_runs"] == want["n_runs"], ctx
    # the device combines the runs in binary64 from its own records, whose
    # -beta F agree with the oracle's to ~1e-15 relative; covariances are
    # compared on the scale sqrt(var(O) var(beta F)) of their Cauchy-Schwarz bound
    for k in wt.FIELDS:
        a, b = got[k], want[k]
        if math.isnan(b):
            assert math.isnan(a), (ctx, k, a, b)
            continue
        tol = 1e-8 * max(abs(a), abs(b))
        if k.startswith("cov_"):
            tol = max(tol, 1e-8 * math.sqrt(want["var_beta_F"]) * want["_sd_" + k[4:]])
        assert abs(a - b) <= tol + 1e-300, (ctx, k, a, b)


@pytest.mark.parametrize("resample", ["nearest", "poisson", "multinomial"])
def test_weighted_averages_over_runs_match_oracle(resample):
    from oracle import weighted as wt
    L, n, M = 8, 6, 7
    betas = linear_schedule(0.6, n)
    Rs = [100, 160, 100, 220, 130, 100, 190]
    specs = [dict(L=L, R=Rs[m], theta=2, seed=500 + m, resample=resample,
                  layout="msc64" if m % 2 else "int8", betas=betas) for m in range(M)]
    b = pa.Batch(specs)
    b.run(n)
    got = b.weighted(0, n + 1)
    refs = [po.run(L, Rs[m], betas, 2, 500 + m, resample) for m in range(M)]
    for i in range(n + 1):
        want = wt.weighted_averages(L, [r.records for r in refs], Rs, i)
        for k in ("e", "m", "c_v", "chi"):
            want["_sd_" + k] = float(np.std([getattr(r.records[i], k) for r in refs], ddof=1))
        _close_weighted(got[i], want, "%s step %d" % (resample, i))
    # one step alone gives the same record
    assert b.weighted(3)[0] == got[3]
    b.close()


def test_weighted_averages_reject_mixed_runs():
    specs = [dict(L=8, R=64, theta=1, seed=1, betas=linear_schedule(0.3, 3)),
             dict(L=8, R=64, theta=1, seed=2, betas=linear_schedule(0.4, 3))]
    b = pa.Batch(specs)
    b.run(3)
    w = b.weighted(0, 4)
    assert w[0]["n_runs"] == 2  # beta_0 = 0 is shared
    assert all(x["n_runs"] == 0 and math.isnan(x["e"]) for x in w[1:])
    with pytest.raises(pa.PAError):
        b.weighted(3, 2)  # step 4 not queued
    b.close()
    # a run that stops (capacity) leaves the later steps uncombined
    betas = linear_schedule(0.6, 40)
    b = pa.Batch([dict(L=8, R=128, theta=1, seed=2, betas=betas, capacity=128),
                  dict(L=8, R=128, theta=1, seed=3, betas=betas)])
    b.run(40)
    w = b.weighted(0, 41)
    stop = next(i for i, x in enumerate(w) if x["n_runs"] == 0)
    assert stop > 1 and all(x["n_runs"] == 2 for x in w[:stop])
    assert all(x["n_runs"] == 0 and math.isnan(x["e"]) for x in w[stop:])
    b.close()
    b = pa.Batch([dict(L=8, R=64, theta=1, seed=1, betas=linear_schedule(0.3, 2)),
                  dict(L=6, R=64, theta=1, seed=2, betas=linear_schedule(0.3, 2))])
    b.run(2)
    with pytest.raises(pa.PAError) as ei:
        b.weighted(1)
    assert ei.value.status == pa.PA_ERR_ARG
    b.close()


def _cq_integer(c, N, R):
    """The exact integer sum over pairs and sites behind each C_q(d)."""
    return [int(round(c[d] * N * (R - d))) for d in range(len(c))]


@pytest.mark.parametrize("L,R,n,layout", [(8, 300, 10, "msc64"), (8, 300, 10, "int8"),
                                          (6, 1000, 6, "msc64"), (4, 64, 3, "int8")])
def test_overlap_correlation_matches_oracle(L, R, n, layout):
    from oracle import overlap as ov
    betas = linear_schedule(0.44, n)
    run = pa.Run(L, R, betas, 1, PARITY_SEED, "nearest", layout)
    run.run(n)
    ref = po.run(L, R, betas, 1, PARITY_SEED, "nearest")
    R_i = len(ref.E)
    assert run.current() == (n, R_i)
    d_max = R_i - 1
    got = run.overlap_correlation(d_max)
    want = ov.overlap_correlation(ref.spins, d_max)
    assert _cq_integer(got, L * L, R_i) == _cq_integer(want, L * L, R_i)
    assert np.allclose(got, want, rtol=0, atol=1e-14)
    # a shorter range gives the same values
    assert np.array_equal(run.overlap_correlation(5), got[:6])
    for bad in (0, R_i):
        with pytest.raises(pa.PAError):
            run.overlap_correlation(bad)
    run.close()


@pytest.mark.slow
def test_overlap_correlation_full_size_sampled():
    """L=64, R=100000 after 120 of 200 steps to 0.4407: C_q at sampled
    distances (within a group, across one and several group boundaries, past
    the first 256-distance chunk) against the plain sum over the downloaded
    population."""
    L, R = 64, 100_000
    run = pa.Run(L, R, linear_schedule(0.4407, 200), 10, PARITY_SEED, "multinomial", "msc64")
    run.run(120)
    got = run.overlap_correlation(1100)
    spins, _, _, _ = run.population()
    R_i = spins.shape[0]
    N = L * L
    for d in (1, 2, 63, 64, 65, 127, 255, 256, 257, 700, 1100):
        total = N * (R_i - d) - 2 * int(np.count_nonzero(spins[: R_i - d] != spins[d:]))
        assert _cq_integer(got, N, R_i)[d] == total, d
    # beta = 0.26 with theta = 10: the population is nearly uncorrelated
    assert got[0] == 1.0 and np.abs(got[1:]).max() < 0.05
    run.close()


def test_batch_covering_design_runs_and_replays():
    from workloads import batched_design
    specs = []
    for rs in batched_design(8, beta_final=0.4407, n_steps=6, theta=2):
        specs.append(dict(L=rs.L // 2, R=rs.R // 10, theta=rs.theta, seed=rs.seed,
                          resample=rs.resample, layout=rs.layout, betas=rs.betas()))
    stream = torch.cuda.Stream()
    b = pa.Batch(specs, stream=stream)
    b.run(3)
    b.run(3)  # the captured graph is replayed
    b.sync()
    for k in (0, 5):
        s = specs[k]
        single = pa.Run(s["L"], s["R"], s["betas"], s["theta"], s["seed"], s["resample"],
                        s["layout"])
        single.run(6)
        assert same_record(b.observables(k, 6), single.observables(6))
        single.close()
    b.close()


def _population_after(L, R, steps, bf=0.44, theta=3, seed=31):
    betas = linear_schedule(bf, 20)
    run = pa.Run(L, R, betas, theta, seed, "nearest", "msc64")
    for _ in range(steps):
        run.anneal_step()
    _, _, E, _ = run.population(spins=False)
    return run, E, betas[steps]


@pytest.mark.parametrize("dbeta", [0.0, 0.003, 0.02, 0.1])
def test_overlap_matches_oracle(dbeta):
    run, E, _ = _population_after(16, 3000, 8)
    a = run.overlap(dbeta)
    assert abs(a - po.overlap(E, dbeta)) < 1e-9
    if dbeta == 0.0:
        assert a == 1.0
    run.close()


def test_histogram_overlap_at_the_critical_point():
    """Sec. "Bias with resampling": for L = 32 at beta_c the overlap of the
    energy histograms at beta_c and beta_c + dbeta is about 0.3 for dbeta =
    0.02 and below 10 % for dbeta >= 0.05, decaying away from dbeta = 0.  A
    population at beta_c (R = 100000, theta = 10, dbeta = 0.01 steps) is required
    to give 0.3 within 50 % and less than 0.1 at 0.05, decreasing in dbeta."""
    betas = linear_schedule(0.4407, 44)
    run = pa.Run(32, 100000, betas, 10, 77, "nearest", "msc64")
    run.run(44)
    a = {d: run.overlap(d) for d in (0.005, 0.01, 0.02, 0.05, 0.1)}
    run.close()
    log("overlap at beta_c", a)
    assert 0.15 < a[0.02] < 0.45, a
    assert a[0.05] < 0.1, a
    assert a[0.005] > a[0.01] > a[0.02] > a[0.05] > a[0.1], a


def test_adaptive_dbeta_hits_the_target_overlap():
    run, E, _ = _population_after(16, 3000, 10)
    for target in (0.7, 0.85, 0.95):
        d = run.adaptive_dbeta(target, 0.5)
        assert 0 < d < 0.5
        assert abs(po.overlap(E, d) - target) < 1e-6
    # a target already met by the largest step returns that step
    assert run.adaptive_dbeta(1e-6, 0.001) == 0.001
    run.close()


@pytest.mark.parametrize("update,resample", [("metropolis", "nearest"), ("heatbath", "poisson")])
def test_adaptive_schedule_replays_in_the_oracle(update, resample):
    L, R, theta = 8, 400, 2
    run = schedules.adaptive_run(L, R, theta, 41, 0.85, 0.6, max_steps=300, resample=resample,
                                 update=update)
    n, acc, alpha = run.schedule_log()
    assert n > 3 and run.observables(n)["beta"] == 0.6
    assert np.all(alpha >= 0.85 - 1e-9) and not acc.any()
    betas = [run.observables(i)["beta"] for i in range(n + 1)]
    ref = po.OracleRun(L, R, theta, 41, resample, np.array(betas), update=update)
    for i in range(1, n + 1):
        # the step the device chose has the target overlap in the oracle too
        if i < n:
            assert abs(po.overlap(ref.E, betas[i] - betas[i - 1]) - 0.85) < 1e-6
        ref.anneal_step()
        got = run.observables(i)
        assert got["sum_E"] == ref.records[i].sum_E and got["R_i"] == ref.records[i].R_i
        assert abs(got["minus_beta_F"] - ref.records[i].minus_beta_F) < 1e-12 * abs(got["minus_beta_F"])
    run.close()


def _rand_params(seed):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(seed) + rng.normal(0, 0.05, mlp.N_PARAMS)
    return p


def test_mlp_forward_matches_fp64_oracle():
    p = _rand_params(1)
    X = np.random.default_rng(2).normal(0, 1, (301, mlp.N_IN))
    dp = torch.tensor(p, dtype=torch.float32, device="cuda")
    dx = torch.tensor(X, dtype=torch.float32, device="cuda")
    dy = torch.zeros(301, dtype=torch.float32, device="cuda")
    pa.mlp_forward(dp, dx, dy)
    torch.cuda.synchronize()
    y, _, _ = mlp.forward(p, X)
    assert np.max(np.abs(dy.cpu().numpy() - y) / (1 + np.abs(y))) < 1e-4


def test_mlp_backward_matches_fp64_oracle():
    p = _rand_params(3)
    rng = np.random.default_rng(4)
    X = rng.normal(0, 1, (257, mlp.N_IN))
    T = rng.normal(0, 1, 257)
    dp = torch.tensor(p, dtype=torch.float32, device="cuda")
    dx = torch.tensor(X, dtype=torch.float32, device="cuda")
    dt = torch.tensor(T, dtype=torch.float32, device="cuda")
    dg = torch.zeros(mlp.N_PARAMS, dtype=torch.float32, device="cuda")
    dl = torch.zeros(1, dtype=torch.float32, device="cuda")
    pa.mlp_backward(dp, dx, dt, dg, dl)
    torch.cuda.synchronize()
    L0, g = mlp.loss_and_grad(p, X, T)
    gd = dg.cpu().numpy()
    assert abs(dl.item() - L0) < 1e-4 * (1 + L0)
    assert np.max(np.abs(gd - g)) < 1e-4 * (np.max(np.abs(g)) + 1e-3)


def test_mlp_training_follows_fp64_adam():
    rng = np.random.default_rng(5)
    X = rng.normal(0, 1, (200, mlp.N_IN))
    T = np.sin(X[:, 0]) + 0.5 * X[:, 1]
    p0 = _rand_params(6)
    dp = torch.tensor(p0, dtype=torch.float32, device="cuda")
    adam = torch.zeros(2 * mlp.N_PARAMS, dtype=torch.float32, device="cuda")
    dl = torch.zeros(1, dtype=torch.float32, device="cuda")
    dx = torch.tensor(X, dtype=torch.float32, device="cuda")
    dt = torch.tensor(T, dtype=torch.float32, device="cuda")
    p, m, v = p0.copy(), np.zeros(mlp.N_PARAMS), np.zeros(mlp.N_PARAMS)
    for t in range(1, 51):
        pa.mlp_train_step(dp, adam, dx, dt, 1e-3, t, dl)
        _, g = mlp.loss_and_grad(p, X, T)
        p, m, v = mlp.adam_step(p, m, v, g, 1e-3, t)
    torch.cuda.synchronize()
    assert np.max(np.abs(dp.cpu().numpy() - p)) < 2e-4
    assert mlp.loss(p, X, T) < mlp.loss(p0, X, T)


def test_features_match_oracle():
    run, E, beta = _population_after(16, 2000, 7)
    f = torch.zeros(mlp.N_IN, dtype=torch.float32, device="cuda")
    run.features(f)
    torch.cuda.synchronize()
    want = mlp.features(E, beta, 256)
    assert np.allclose(f.cpu().numpy(), want.astype(np.float32), rtol=1e-6, atol=1e-7)
    run.close()


def test_learned_proposal_is_guarded_by_the_overlap():
    run, E, beta = _population_after(16, 3000, 9)
    for seed in range(4):
        p = _rand_params(10 + seed)
        p[-1] = -1.0 + 0.6 * seed  # spread the proposals
        dp = torch.tensor(p, dtype=torch.float32, device="cuda")
        d, accepted = run.learned_dbeta(dp, 0.8, 0.85, 0.3)
        if accepted:
            assert po.overlap(E, d) >= 0.8 - 1e-9
            y, _, _ = mlp.forward(p, mlp.features(E, beta, 256)[None, :])
            sd = math.sqrt(mlp.features(E, beta, 256)[34] * 256)
            assert abs(d - min(math.exp(y[0]) / sd, 0.3)) < 1e-4 * d
        else:
            assert d == run.adaptive_dbeta(0.85, 0.3)
    run.close()


def test_learned_schedule_runs_and_logs():
    L, R = 16, 2000
    p = _rand_params(20)
    p[-1] = -1.0
    dp = torch.tensor(p, dtype=torch.float32, device="cuda")
    run = schedules.learned_run(dp, L, R, 2, 51, 0.8, 0.85, 0.5, max_steps=500)
    n, acc, alpha = run.schedule_log()
    assert run.observables(n)["beta"] == 0.5
    assert np.all(alpha >= 0.8 - 1e-9)
    X, t = schedules.training_rows(run)
    assert X.shape[0] == t.shape[0] <= n and torch.isfinite(t).all()
    run.close()


GEOMETRIES = {
    16: ((256, 4), (64, 1), (1024, 2), (128, 8), (512, 1), (192, 3)),
    # the thread stride is not a multiple of a row: the word walk carries
    # across rows and groups
    6: ((256, 4), (64, 1), (1024, 2), (128, 8), (512, 1), (192, 3)),
    # three or four groups fill more than half the LDS: two words per thread;
    # one group per block: a thread keeps its column
    64: ((512, 1), (256, 3), (1024, 4), (320, 3), (192, 1)),
    # one group fills more than half the LDS; with 64, 192 or 320 threads a
    # thread's rows are 1, 3 or 5 apart, so its word alternates between the
    # two columns of its pair
    128: ((1024, 1), (192, 1), (64, 1), (320, 1)),
}


@pytest.mark.parametrize("update", ["metropolis", "heatbath"])
@pytest.mark.parametrize("L", sorted(GEOMETRIES))
def test_sweep_geometry_does_not_change_results(L, update):
    betas = linear_schedule(0.5, 4)
    states = []
    for k, (threads, gpb) in enumerate(GEOMETRIES[L]):
        for words in (0, 1 + k % 2):  # the default, and one or two words per thread
            r = pa.Run(L, 1000, betas, 3, 61, "nearest", "msc64", update=update)
            r.set_sweep_launch(L, threads, gpb, words)
            assert r.sweep_launch(L) == (threads, gpb, words)
            r.run(4)
            states.append(r.get_state())
            r.close()
    assert all(s == states[0] for s in states)
    r = pa.Run(L, 64, betas, 3, 61, "nearest", "msc64")
    for words in (-1, 3):
        with pytest.raises(pa.PAError):
            r.set_sweep_launch(L, 256, 1, words)
    r.close()


def test_profiling_modes():
    """Timing alone counts nothing; counting gives the Philox calls the words
    need (three plane calls at most, plus tie calls) and every word update;
    neither changes the results; other enable bits are rejected."""
    L, R, theta, n = 16, 3000, 3, 4
    betas = linear_schedule(0.44, n)
    ref = pa.Run(L, R, betas, theta, 63, "nearest", "msc64")
    ref.run(n)
    want = ref.observables(n)
    ref.close()
    for count in (False, True):
        r = pa.Run(L, R, betas, theta, 63, "nearest", "msc64")
        r.profile(True, count_calls=count)
        r.run(n)
        p = r.profile_read()
        assert same_record(r.observables(n), want)
        assert p["steps"] == n and p["ms_sweep"] > 0.0
        if not count:
            assert p["philox_calls"] == 0 and p["sweep_words"] == 0
        else:
            # step i sweeps its new population of R_i replicas: one word per site and group
            groups = sum(math.ceil(r.observables(i)["R_i"] / 64) for i in range(1, n + 1))
            assert p["sweep_words"] == groups * theta * L * L
            assert 2.0 < p["philox_calls"] / p["sweep_words"] < 4.0, p
        with pytest.raises(pa.PAError):
            pa._check(pa.lib().pa_profile(r.h, 4), r.h)
        r.close()


def test_effective_population_size_is_bounded_below_by_the_families():
    """Sec. "Effective population size": R / rho_t from the family statistics is
    a lower bound of the blocking estimate R_eff(E) (far from tight).  The
    blocked variance is itself an estimate (99 degrees of freedom), hence the
    factor 1/2; at beta = 0 the population is uncorrelated and R_eff is about R."""
    L, R, theta, n = 16, 20000, 5, 30
    r = pa.Run(L, R, linear_schedule(0.44, n), theta, 64, "nearest", "msc64")
    r.run(n)
    recs = [r.observables(i) for i in range(n + 1)]
    r.close()
    assert 0.6 * R < recs[0]["r_eff_E"] < 1.6 * R
    for o in recs[1:]:
        assert o["r_eff_E"] > 0.5 * o["R_i"] / o["rho_t"], o
        assert o["err_e"] > 0.0 and o["err_c_v"] > 0.0


def test_blocked_error_bar_of_e_matches_the_spread_of_independent_runs():
    """Sec. "Statistical errors" (the comparison of its error-bar figure): at
    L = 32, R = 50000, theta = 10, dbeta = 0.01 the single-run error bar of e
    from the blocking analysis agrees with the standard deviation of e over
    independent runs (64 runs here; the standard deviation of 64 values has a
    relative standard error of 9 %)."""
    betas = linear_schedule(0.44, 44)
    specs = [dict(L=32, R=50000, theta=10, seed=1000 + s, betas=betas, resample="nearest")
             for s in range(64)]
    b = pa.Batch(specs)
    b.run(44)
    for i in (10, 25, 35, 44):
        e = np.array([b.observables(k, i)["e"] for k in range(64)])
        err = np.array([b.observables(k, i)["err_e"] for k in range(64)])
        ratio = err.mean() / e.std(ddof=1)
        log("step", i, "mean err_e / std e", ratio)
        assert 0.7 < ratio < 1.4, (i, ratio)
    b.close()


def test_effective_population_size_near_criticality():
    """Sec. "Statistical errors": with one sweep per step the population near
    criticality is strongly correlated; the paper finds R_eff of about 600 for
    R = 50000 (L = 32).  Here dbeta = 0.01 up to beta = 0.44 with
    checkerboard instead of sequential updates: the mean R_eff(E) over three
    seeds at beta = 0.44 is required within a factor 2.5 of 600, and ten sweeps
    per step keep it at least twenty times larger."""
    betas = linear_schedule(0.44, 44)
    reff = {}
    for theta in (1, 10):
        vals = []
        for seed in (11, 12, 13):
            r = pa.Run(32, 50000, betas, theta, seed, "nearest", "msc64")
            r.run(44)
            vals.append(r.observables(44)["r_eff_E"])
            r.close()
        reff[theta] = float(np.mean(vals))
        log("theta", theta, "R_eff(E) at beta 0.44", vals)
    assert 600 / 2.5 < reff[1] < 600 * 2.5, reff
    assert reff[10] > 20 * reff[1], reff


def _tau_eff(bf, n, thetas, R=128000, seeds=(5, 6)):
    """Fit of Eq. Reff, R_eff / R = 1 - c exp(-theta / tau_eff), to R_eff(E) / R
    averaged over the last five steps of runs at L = 64 with dbeta = 0.005
    (points with R_eff / R >= 0.97 carry no information on the decay)."""
    ys = []
    for th in thetas:
        vals = []
        for seed in seeds:
            r = pa.Run(64, R, linear_schedule(bf, n), th, seed, "nearest", "msc64")
            r.run(n)
            vals += [r.observables(i)["r_eff_E"] / r.observables(i)["R_i"] for i in range(n - 4, n + 1)]
            r.close()
        ys.append(float(np.mean(vals)))
    th, y = np.array(thetas, dtype=float), np.array(ys)
    ok = y < 0.97
    slope = np.polyfit(th[ok], np.log(1.0 - y[ok]), 1)[0]
    log("beta_f", bf, "R_eff/R", dict(zip(thetas, ys)), "tau_eff", -1.0 / slope)
    return -1.0 / slope


@pytest.mark.slow
def test_theta_dependence_of_the_effective_population_size():
    """Sec. "Statistical errors", Eq. Reff: at L = 64, dbeta = 0.005 and R =
    128000 the paper fits tau_eff = 2.2 at T = 2.5 and 51.2 at T = 2.325.  These
    checkerboard runs (nearest-integer copies, 100 blocks) are required to give
    tau_eff within a factor 2 of 2.2 at T = 2.5 and within a factor 2.5 of 51.2
    at T = 2.325, the latter at least five times the former."""
    t_hot = _tau_eff(0.4, 80, (1, 2, 3, 4, 6, 8))
    t_crit = _tau_eff(1.0 / 2.325, 86, (5, 10, 20, 40, 80))
    assert 2.2 / 2 < t_hot < 2.2 * 2, t_hot
    assert 51.2 / 2.5 < t_crit < 51.2 * 2.5, t_crit
    assert t_crit > 5 * t_hot, (t_hot, t_crit)


@pytest.mark.slow
def test_energy_relaxation_time_without_resampling():
    """Sec. "Bias", behaviour without resampling: at L = 32, R = 10000, with
    resampling off and steps of dbeta = 0.1 to beta_c, the relative deviation of
    the energy from Kaufman's, averaged over 200 runs, follows
    eps = a exp(-theta / tau_rel) (1 + b / theta) with tau_rel = 45.4(6).  Here
    256 runs per theta, the steps 0, 0.1, 0.2, 0.3, 0.4, beta_c; the fitted
    tau_rel is required within 25 % of 45.4 and |eps| to fall with theta."""
    from scipy.optimize import curve_fit
    from oracle import exact
    bc = 0.5 * math.log(1.0 + math.sqrt(2.0))
    betas = np.array([0.0, 0.1, 0.2, 0.3, 0.4, bc])
    e_ex = float(exact.energy_per_spin(32, bc))
    thetas = [1, 2, 5, 10, 20, 40, 60, 80, 120, 160, 200]
    eps, se = [], []
    for th in thetas:
        es = []
        for chunk in range(4):
            specs = [dict(L=32, R=10000, theta=th, seed=5000 + 64 * chunk + k, betas=betas,
                          resample="none") for k in range(64)]
            b = pa.Batch(specs)
            b.run(5)
            es += [b.observables(k, 5)["e"] for k in range(64)]
            b.close()
        es = np.array(es)
        eps.append((es.mean() - e_ex) / e_ex)
        se.append(es.std(ddof=1) / math.sqrt(len(es)) / abs(e_ex))
    th, y = np.array(thetas, dtype=float), np.array(eps)
    fit = lambda t, a, tau, b: a * np.exp(-t / tau) * (1.0 + b / t)
    p, _ = curve_fit(fit, th, y, p0=(y[3], 40.0, 1.0), sigma=np.array(se), maxfev=20000)
    log("eps", dict(zip(thetas, eps)), "tau_rel", p[1])
    assert np.all(np.diff(np.abs(y)) < 0), y
    assert 45.4 * 0.75 < p[1] < 45.4 * 1.25, p


def test_error_bars_fall_as_one_over_sqrt_population():
    """Sec. "Statistical errors": with theta = 10 the population stays close to
    equilibrium and the statistical error of the energy falls as 1 / sqrt(R).
    L = 32, dbeta = 0.01 to beta = 0.44, R = 12500, 50000 and 200000 (the
    blocked error bar err_e of each run, averaged over four seeds and over the
    steps to beta = 0.3, 0.4 and 0.44): err_e sqrt(R) is required to agree
    within 25 % across the three sizes."""
    betas = linear_schedule(0.44, 44)
    steps = (30, 40, 44)
    scaled = {}
    for R in (12500, 50000, 200000):
        specs = [dict(L=32, R=R, theta=10, seed=300 + s, betas=betas, resample="nearest")
                 for s in range(4)]
        b = pa.Batch(specs)
        b.run(44)
        scaled[R] = np.array([[b.observables(k, i)["err_e"] for k in range(4)] for i in steps]
                             ).mean(axis=1) * math.sqrt(R)
        b.close()
    log("err_e sqrt(R) at steps", steps, scaled)
    ref = scaled[50000]
    for R in (12500, 200000):
        assert np.all(np.abs(scaled[R] / ref - 1.0) < 0.25), scaled


@pytest.mark.slow
def test_effective_population_size_falls_linearly_with_the_step():
    """Sec. "Statistical errors", Eq. Reff-deltabeta: close to criticality
    (L = 64, beta = 0.43, R = 10000, averaged over independent runs) the
    paper fits 1 - R_eff / R = A dbeta.  64 runs with theta = 40 per step
    size dbeta = 0.0025, 0.005 and 0.01 (the last three steps of each run): the
    slope (1 - R_eff / R) / dbeta is required to agree within 30 % across the
    three step sizes."""
    slopes = []
    for db in (0.0025, 0.005, 0.01):
        n = int(round(0.43 / db))
        betas = np.linspace(0.0, 0.43, n + 1)
        specs = [dict(L=64, R=10000, theta=40, seed=700 + s, betas=betas, resample="nearest")
                 for s in range(64)]
        b = pa.Batch(specs)
        b.run(n)
        y = np.mean([1.0 - b.observables(k, i)["r_eff_E"] / b.observables(k, i)["R_i"]
                     for k in range(64) for i in range(n - 2, n + 1)])
        b.close()
        slopes.append(y / db)
    log("(1 - R_eff/R) / dbeta", slopes)
    assert max(slopes) < 1.3 * min(slopes), slopes


def test_autotuner_times_candidates_and_keeps_results():
    from paper_2102_06611_amd import autotune
    betas = linear_schedule(0.44, 10)
    run = pa.Run(32, 3000, betas, 4, 62, "multinomial", "int8")
    for _ in range(3):
        run.anneal_step()
    best, results = autotune.tune_run(run, 32, steps=1)
    assert len(results) == len(autotune.candidates(32)) and best == min(results)
    assert run.sweep_launch(32) == (best[1], best[2], best[3])
    run.close()


def test_learned_schedule_against_plain_adaptive():
    """Trained on error-budget targets from adaptive runs at L = 16 and 32
    (R = 5000), the learned schedule reaches beta_f = 0.8 at L = 32, R = 20000
    in at most 0.9 times the adaptive schedule's steps, its proposals passing
    the overlap guard, at a free-energy error (against Kaufman's ln Z, 16
    seeds) no worse than the adaptive schedule's within two standard errors
    and below 1e-4 per spin."""
    from oracle import exact
    info = []
    X, t = schedules.collect((16, 32), 5000, range(500, 508), 5, 0.85, 0.8, info=info)
    log(info)
    assert X.shape[0] > 100 and torch.isfinite(t).all()
    params, losses = schedules.train(X, t, iters=2000, lr=3e-3)
    assert losses[-1] < 0.1 * losses[0]
    lnz = float(exact.ln_z_kaufman(32, 0.8))
    res = schedules.compare(params, 32, 20000, 5, list(range(900, 916)), lnz, beta_final=0.8)
    sa = np.array([r["steps_adaptive"] for r in res], dtype=float)
    sl = np.array([r["steps_learned"] for r in res], dtype=float)
    ea = np.array([r["error_adaptive"] for r in res])
    el = np.array([r["error_learned"] for r in res])
    log("steps", sa.mean(), sl.mean(), "errors", ea.mean(), el.mean(),
        "accepted", np.mean([r["accepted"] for r in res]))
    assert sl.mean() <= 0.9 * sa.mean()
    assert np.mean([r["accepted"] for r in res]) > 0.9
    assert np.all([r["alpha_mean_learned"] >= 0.80 for r in res])
    se = math.sqrt(ea.var(ddof=1) / len(ea) + el.var(ddof=1) / len(el))
    assert el.mean() <= ea.mean() + 2 * se
    assert ea.mean() < 1e-4 and el.mean() < 1e-4


def _tail_decay_length(cq):
    """tau_R of the exponential tail C_q(d) ~ exp(-d / tau_R) (Eq. exponential_R):
    a least-squares line through ln C_q(d) from the first d where C_q has fallen
    to 0.3 C_q(1) (past the faster initial decay) to the last d before it drops
    below 0.03 (far above the noise of the average, about 0.002)."""
    d_b = 1
    while d_b + 1 < len(cq) and cq[d_b + 1] >= 0.03:
        d_b += 1
    d_a = next(d for d in range(1, len(cq)) if cq[d] <= 0.3 * cq[1] or d >= d_b - 1)
    d_a = min(d_a, d_b - 1)
    d = np.arange(d_a, d_b + 1)
    slope = np.polyfit(d, np.log(cq[d_a:d_b + 1]), 1)[0]
    return -1.0 / slope


def test_overlap_correlation_tail_matches_the_paper():
    """Sec. "Effective population size" (Fig. correlation_function, Eq.
    exponential_R): L = 16, R = 50000 near beta_c = 0.44, theta = 1, 5, 10 give
    tau_R = 32.3, 3.0, 1.8.  The step size is not stated there; Delta beta = 0.01
    (44 steps), the paper's usual step at these sizes, is taken.  The paper's
    runs use sequential Metropolis updates and these checkerboard ones (a
    reading of the update order), so each tau_R is required within 50 %, and
    the order theta = 1 > 5 > 10."""
    betas = linear_schedule(0.44, 44)
    taus = {}
    for theta in (1, 5, 10):
        cqs = []
        for seed in range(4):
            r = pa.Run(16, 50000, betas, theta, 300 + seed, "nearest", "msc64")
            r.run(44)
            cqs.append(r.overlap_correlation(256))
            r.close()
        taus[theta] = _tail_decay_length(np.mean(cqs, axis=0))
    log("tau_R", taus)
    assert taus[1] > taus[5] > taus[10]
    for theta, want in ((1, 32.3), (5, 3.0), (10, 1.8)):
        assert 0.5 * want <= taus[theta] <= 1.5 * want, (theta, taus[theta], want)


def test_full_size_covering_design_members_match_single_runs():
    """The 64-run covering design at full size (L in {16, 32, 64, 128} x R in
    {1000, 5000, 20000, 50000}, beta 0 -> 0.4407 in 200 steps, theta = 10), run
    60 steps in one batch: the members L = 128 / R = 50000 and L = 16 / R = 1000
    (and one with L = 32 and one with L = 64) equal single runs record by
    record, and on sampled replica groups spin by spin."""
    from workloads import batched_design
    design = batched_design(64)
    specs = [dict(L=d.L, R=d.R, theta=d.theta, seed=d.seed, resample=d.resample,
                  layout=d.layout, betas=d.betas()) for d in design]
    b = pa.Batch(specs, stream=torch.cuda.Stream())
    k = 60
    b.run(k)
    b.sync()
    members = [m for m, d in enumerate(design) if (d.L, d.R) in ((128, 50000), (16, 1000))][:2]
    members += [m for m, d in enumerate(design) if (d.L, d.R) in ((32, 20000), (64, 5000))][:2]
    rng = np.random.default_rng(5)
    for m in members:
        d = design[m]
        log("member", m, d.L, d.R)
        single = pa.Run(d.L, d.R, d.betas(), d.theta, d.seed, d.resample, d.layout)
        single.run(k)
        for i in range(k + 1):
            assert same_record(b.observables(m, i), single.observables(i)), (m, i)
        _, R_i = single.current()
        G = (R_i + 63) // 64
        for g in sorted(set([0, G - 1] + list(rng.integers(0, G, 3)))):
            lo, hi = 64 * g, min(64 * g + 64, R_i)
            got = b.population(m, lo, hi - lo)
            want = single.population(lo, hi - lo)
            for x, y in zip(got, want):
                assert np.array_equal(x, y), (m, g)
        single.close()
    b.close()
