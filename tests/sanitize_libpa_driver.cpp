// Host sanitizer driver for libpa's host code (the C-ABI of include/pa.h).
//
// Linked with libpa's objects built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host side only (the device code is not
// instrumented).  Every host buffer handed to the library is a heap block of
// exactly the size the header documents, so a write past it is reported.
//
//   sanitize_libpa_driver host    configuration checks, workspace layouts,
//                                 argument and handle errors: no device needed
//   sanitize_libpa_driver device  the above, then every entry point on small
//                                 runs and batches on device 0
//
// Exit status 0 when every check holds; 3 on a failed check (the message names
// it); the sanitizers' own exit codes are set by the caller.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <vector>

#include "pa.h"

#define CHECK(cond)                                                                      \
    do {                                                                                 \
        if (!(cond)) {                                                                   \
            std::fprintf(stderr, "check failed at line %d: %s (last error: %s)\n", __LINE__, \
                         #cond, pa_last_error(nullptr));                                 \
            std::exit(3);                                                                \
        }                                                                                \
    } while (0)
#define HIP_OK(call) CHECK((call) == hipSuccess)

namespace {

// A heap block of exactly n elements (never a rounded-up container capacity).
template <typename T>
struct Exact {
    std::unique_ptr<T[]> p;
    size_t n;
    explicit Exact(size_t n_) : p(new T[n_ ? n_ : 1]()), n(n_) {}
    T *get() { return n ? p.get() : nullptr; }
    T &operator[](size_t i) { return p[i]; }
};

pa_config config(int L, int R, const double *betas, int n_steps, int theta, int resample,
                 int layout, int update = PA_UPDATE_METROPOLIS) {
    pa_config c{};
    c.L = L;
    c.R = R;
    c.betas = betas;
    c.n_steps = n_steps;
    c.theta = theta;
    c.seed = 0x5EEDu + (uint64_t)L * 131u + (uint64_t)R;
    c.resample = resample;
    c.layout = layout;
    c.capacity = 0;
    c.update = update;
    return c;
}

std::vector<double> linear_betas(double beta_f, int n) {
    std::vector<double> b(n + 1);
    for (int i = 0; i <= n; ++i) b[i] = beta_f * i / n;
    return b;
}

// ---------------------------------------------------------------- host part

void workspace_layouts() {
    const int Ls[] = {4, 6, 8, 16, 64, 128};
    const int Rs[] = {1, 63, 64, 65, 1000, 100000, (1 << 23) - 1, 1 << 24};
    std::vector<double> betas = linear_betas(0.4407, 200);
    for (int L : Ls)
        for (int layout = 0; layout <= 1; ++layout)
            for (int rule = 0; rule <= 3; ++rule)
                for (int with_betas = 0; with_betas <= 1; ++with_betas) {
                    size_t prev = 0;
                    for (int R : Rs) {
                        if (rule == PA_RESAMPLE_MULTINOMIAL && R >= (1 << 23)) continue;
                        pa_config c = config(L, R, with_betas ? betas.data() : nullptr, 200, 10,
                                             rule, layout);
                        size_t bytes = 0;
                        CHECK(pa_workspace_size(&c, &bytes) == PA_OK);
                        // two population buffers at least, and growing with R
                        size_t groups = ((size_t)R + 63) / 64;
                        size_t pop = groups * L * L * (layout == PA_LAYOUT_MSC64 ? 8 : 64);
                        CHECK(bytes >= 2 * pop);
                        CHECK(bytes >= prev);
                        prev = bytes;
                    }
                }
}

void invalid_configurations() {
    std::vector<double> good = linear_betas(0.44, 4);
    std::vector<double> bad0 = good, decreasing = good, nan = good;
    bad0[0] = 0.1;
    decreasing[3] = 0.05;
    nan[2] = std::nan("");
    pa_config base = config(8, 100, good.data(), 4, 2, PA_RESAMPLE_NEAREST, PA_LAYOUT_MSC64);
    std::vector<pa_config> bad;
    auto with = [&](auto edit) {
        pa_config c = base;
        edit(c);
        bad.push_back(c);
    };
    with([](pa_config &c) { c.L = 2; });
    with([](pa_config &c) { c.L = 7; });
    with([](pa_config &c) { c.L = 130; });
    with([](pa_config &c) { c.R = 0; });
    with([](pa_config &c) { c.R = (1 << 24) + 1; });
    with([](pa_config &c) { c.n_steps = -1; });
    with([](pa_config &c) { c.theta = -1; });
    with([](pa_config &c) { c.resample = 4; });
    with([](pa_config &c) { c.resample = -1; });
    with([](pa_config &c) {
        c.resample = PA_RESAMPLE_MULTINOMIAL;
        c.R = 1 << 23;
    });
    with([](pa_config &c) {
        c.betas = nullptr;
        c.theta = 1000000;
        c.n_steps = 10000;
    });
    with([](pa_config &c) { c.layout = 2; });
    with([](pa_config &c) { c.capacity = -1; });
    with([](pa_config &c) { c.capacity = 64; });
    with([](pa_config &c) { c.update = 2; });
    with([&](pa_config &c) { c.betas = bad0.data(); });
    with([&](pa_config &c) { c.betas = decreasing.data(); });
    with([&](pa_config &c) { c.betas = nan.data(); });
    for (const pa_config &c : bad) {
        size_t bytes = 12345;
        CHECK(pa_workspace_size(&c, &bytes) == PA_ERR_ARG);
        CHECK(std::strlen(pa_last_error(nullptr)) > 0);
        pa_ctx *ctx = reinterpret_cast<pa_ctx *>(0x1);
        Exact<uint8_t> ws(4096);
        CHECK(pa_create(&c, ws.get(), ws.n, nullptr, &ctx) == PA_ERR_ARG);
        CHECK(ctx == nullptr);
    }
    size_t bytes = 0;
    CHECK(pa_workspace_size(nullptr, &bytes) == PA_ERR_ARG);
    CHECK(pa_workspace_size(&base, nullptr) == PA_ERR_ARG);
    // batches: sizes, counts, one bad member
    std::vector<pa_config> mixed;
    std::vector<double> b64 = linear_betas(0.44, 64);
    for (int r = 0; r < 64; ++r)
        mixed.push_back(config(4 << (r % 6) > 128 ? 128 : 4 << (r % 6), 100 + 37 * r, b64.data(),
                               64, 1 + r % 3, r % 4, r % 2));
    size_t one = 0, all = 0;
    CHECK(pa_batch_workspace_size(mixed.data(), 64, &all) == PA_OK);
    for (const pa_config &c : mixed) {
        CHECK(pa_workspace_size(&c, &one) == PA_OK);
        CHECK(all >= one);
    }
    CHECK(pa_batch_workspace_size(mixed.data(), 0, &all) == PA_ERR_ARG);
    CHECK(pa_batch_workspace_size(mixed.data(), 4097, &all) == PA_ERR_ARG);
    CHECK(pa_batch_workspace_size(nullptr, 3, &all) == PA_ERR_ARG);
    mixed[17].L = 9;
    CHECK(pa_batch_workspace_size(mixed.data(), 64, &all) == PA_ERR_ARG);
}

// Creation failures that the library detects before touching a device.
void create_failures() {
    std::vector<double> betas = linear_betas(0.44, 4);
    pa_config c = config(8, 100, betas.data(), 4, 2, PA_RESAMPLE_NEAREST, PA_LAYOUT_MSC64);
    size_t bytes = 0;
    CHECK(pa_workspace_size(&c, &bytes) == PA_OK);
    pa_ctx *ctx = nullptr;
    Exact<uint8_t> ws(bytes + 256);
    uint8_t *aligned = reinterpret_cast<uint8_t *>(
        (reinterpret_cast<uintptr_t>(ws.get()) + 255) / 256 * 256);
    CHECK(pa_create(nullptr, aligned, bytes, nullptr, &ctx) == PA_ERR_ARG);
    CHECK(pa_create(&c, aligned, bytes, nullptr, nullptr) == PA_ERR_ARG);
    CHECK(pa_create(&c, nullptr, bytes, nullptr, &ctx) == PA_ERR_ARG);
    CHECK(pa_create(&c, aligned + 8, bytes, nullptr, &ctx) == PA_ERR_ARG);
    CHECK(pa_create(&c, aligned, bytes - 1, nullptr, &ctx) == PA_ERR_NOMEM);
    CHECK(ctx == nullptr);
    pa_batch *b = nullptr;
    pa_config two[2] = {c, c};
    CHECK(pa_batch_create(two, 0, aligned, bytes, nullptr, &b) == PA_ERR_ARG);
    CHECK(pa_batch_create(nullptr, 2, aligned, bytes, nullptr, &b) == PA_ERR_ARG);
    CHECK(pa_batch_create(two, 2, aligned, 0, nullptr, &b) == PA_ERR_NOMEM);
    CHECK(b == nullptr);
}

// Every call that takes a handle rejects a NULL one.
void null_handles() {
    int32_t i32 = 0, i32b = 0, i32c = 0;
    int64_t i64 = 0;
    size_t sz = 0;
    double d = 0;
    uint64_t u64 = 0, u64b = 0;
    pa_obs obs;
    CHECK(pa_anneal_step(nullptr) == PA_ERR_ARG);
    CHECK(pa_anneal_step_to(nullptr, 0.1) == PA_ERR_ARG);
    CHECK(pa_run(nullptr, 1) == PA_ERR_ARG);
    CHECK(pa_sync(nullptr) == PA_ERR_ARG);
    CHECK(pa_observables(nullptr, 0, &obs) == PA_ERR_ARG);
    CHECK(pa_current(nullptr, &i32, &i32b) == PA_ERR_ARG);
    CHECK(pa_energy_histogram(nullptr, nullptr, 0, &i32, &i32b) == PA_ERR_ARG);
    CHECK(pa_copy_counts(nullptr, nullptr, 0, &i64) == PA_ERR_ARG);
    CHECK(pa_get_population(nullptr, 0, 1, nullptr, &i32, &i32b, &i32c) == PA_ERR_ARG);
    CHECK(pa_get_state(nullptr, nullptr, 0, &sz) == PA_ERR_ARG);
    CHECK(pa_set_state(nullptr, &d, sizeof d) == PA_ERR_ARG);
    CHECK(pa_set_population(nullptr, 0, 1, nullptr, nullptr, 0.0) == PA_ERR_ARG);
    CHECK(pa_overlap(nullptr, 0.1, &d) == PA_ERR_ARG);
    CHECK(pa_adaptive_dbeta(nullptr, 0.85, 0.1, &d) == PA_ERR_ARG);
    CHECK(pa_profile(nullptr, 1) == PA_ERR_ARG);
    CHECK(pa_profile_read(nullptr, &i32, &d, &d, &d, &u64, &u64b, &d) == PA_ERR_ARG);
    CHECK(pa_set_sweep_launch(nullptr, 8, 256, 1, 0) == PA_ERR_ARG);
    CHECK(pa_get_sweep_launch(nullptr, 8, &i32, &i32b, &i32c) == PA_ERR_ARG);
    CHECK(pa_overlap_correlation(nullptr, 1, nullptr) == PA_ERR_ARG);
    CHECK(pa_features(nullptr, nullptr) == PA_ERR_ARG);
    CHECK(pa_anneal_step_adaptive(nullptr, 0.85, 1.0) == PA_ERR_ARG);
    CHECK(pa_anneal_step_learned(nullptr, nullptr, 0.5, 0.85, 1.0) == PA_ERR_ARG);
    CHECK(pa_schedule_log(nullptr, nullptr, nullptr, nullptr, nullptr, 0, &i32) == PA_ERR_ARG);
    CHECK(pa_learned_dbeta(nullptr, nullptr, 0.5, 0.85, 0.1, nullptr, &d, &i32) == PA_ERR_ARG);
    CHECK(pa_batch_run(nullptr, 1) == PA_ERR_ARG);
    CHECK(pa_batch_observables(nullptr, 0, 0, &obs) == PA_ERR_ARG);
    CHECK(pa_batch_get_population(nullptr, 0, 0, 1, nullptr, &i32, &i32b, &i32c) == PA_ERR_ARG);
    CHECK(pa_batch_sync(nullptr) == PA_ERR_ARG);
    CHECK(pa_batch_set_sweep_launch(nullptr, 8, 256, 1, 0) == PA_ERR_ARG);
    CHECK(pa_batch_get_sweep_launch(nullptr, 8, &i32, &i32b, &i32c) == PA_ERR_ARG);
    CHECK(pa_batch_weighted(nullptr, 0, 1, nullptr) == PA_ERR_ARG);
    // free functions: argument errors come before any device work
    uint32_t word = 0;
    float f = 0;
    double two[2];
    int32_t e = 0;
    CHECK(pa_philox4x32_10(0u, 0u, nullptr, 1, &word, nullptr) == PA_ERR_ARG);
    CHECK(pa_philox4x32_10(0u, 0u, &word, -1, &word, nullptr) == PA_ERR_ARG);
    CHECK(pa_philox4x32_10(0u, 0u, nullptr, 0, nullptr, nullptr) == PA_OK);
    CHECK(pa_mlp_forward(&f, &f, -1, &f, nullptr) == PA_ERR_ARG);
    CHECK(pa_mlp_forward(nullptr, nullptr, 0, nullptr, nullptr) == PA_OK);
    CHECK(pa_mlp_backward(&f, &f, &f, 0, &f, &f, nullptr) == PA_ERR_ARG);
    CHECK(pa_mlp_train_step(&f, &f, &f, &f, 1, 1e-3f, 0, &f, nullptr) == PA_ERR_ARG);
    CHECK(pa_mlp_train_step(&f, &f, &f, &f, 1, 0.0f, 1, &f, nullptr) == PA_ERR_ARG);
    CHECK(pa_adaptive_dbeta_noalloc(&e, 1, 7, 0.85, 0.1, two, nullptr) == PA_ERR_ARG);
    CHECK(pa_adaptive_dbeta_noalloc(&e, 1, 8, 1.0, 0.1, two, nullptr) == PA_ERR_ARG);
    CHECK(pa_adaptive_dbeta_noalloc(&e, 1, 8, 0.85, 0.0, two, nullptr) == PA_ERR_ARG);
    CHECK(pa_adaptive_dbeta_noalloc(&e, 0, 8, 0.85, 0.1, two, nullptr) == PA_ERR_ARG);
    pa_destroy(nullptr);
    pa_batch_destroy(nullptr);
    CHECK(pa_last_error(nullptr) != nullptr);
    CHECK(pa_batch_last_error(nullptr) != nullptr);
}

// ---------------------------------------------------------------- device part

template <typename T>
struct Dev {
    T *p = nullptr;
    size_t n = 0;
    explicit Dev(size_t n_) : n(n_) {
        HIP_OK(hipMalloc((void **)&p, (n ? n : 1) * sizeof(T)));
        HIP_OK(hipMemset(p, 0, (n ? n : 1) * sizeof(T)));
    }
    ~Dev() { (void)hipFree(p); }
    Dev(const Dev &) = delete;
    Dev &operator=(const Dev &) = delete;
};

// Reads everything a run exposes, with exact host buffers, and the calls'
// own capacity checks one element short.
void read_back(pa_ctx *ctx, int N, int steps_done) {
    pa_obs obs;
    for (int i = 0; i <= steps_done; ++i) {
        CHECK(pa_observables(ctx, i, &obs) == PA_OK);
        CHECK(obs.step == i);
    }
    CHECK(pa_observables(ctx, steps_done + 1, &obs) == PA_ERR_ARG);
    CHECK(pa_observables(ctx, -1, &obs) == PA_ERR_ARG);
    int32_t step = -1, R_i = -1;
    CHECK(pa_current(ctx, &step, &R_i) == PA_OK);
    CHECK(step == steps_done && R_i >= 1);

    int32_t k_min = 0, n_bins = 0;
    CHECK(pa_energy_histogram(ctx, nullptr, 0, &k_min, &n_bins) == PA_OK);
    Exact<int32_t> hist(n_bins);
    if (n_bins > 1) CHECK(pa_energy_histogram(ctx, hist.get(), n_bins - 1, &k_min, &n_bins) == PA_ERR_ARG);
    CHECK(pa_energy_histogram(ctx, hist.get(), n_bins, &k_min, &n_bins) == PA_OK);
    int64_t total = 0;
    for (int32_t k = 0; k < n_bins; ++k) total += hist[k];
    CHECK(total == R_i);

    int64_t n_cnt = 0;
    CHECK(pa_copy_counts(ctx, nullptr, 0, &n_cnt) == PA_OK);
    Exact<int32_t> cnt(n_cnt);
    if (n_cnt > 1) CHECK(pa_copy_counts(ctx, cnt.get(), n_cnt - 1, &n_cnt) == PA_ERR_ARG);
    CHECK(pa_copy_counts(ctx, cnt.get(), n_cnt, &n_cnt) == PA_OK);

    Exact<int8_t> spins((size_t)R_i * N);
    Exact<int32_t> fam(R_i), E(R_i), M(R_i);
    CHECK(pa_get_population(ctx, 0, R_i, spins.get(), fam.get(), E.get(), M.get()) == PA_OK);
    CHECK(pa_get_population(ctx, 1, R_i, spins.get(), fam.get(), E.get(), M.get()) == PA_ERR_ARG);
    for (int32_t r = 0; r < R_i; ++r) {
        int32_t m = 0;
        for (int s = 0; s < N; ++s) m += spins[(size_t)r * N + s];
        CHECK(m == M[r]);
    }

    size_t used = 0;
    CHECK(pa_get_state(ctx, nullptr, 0, &used) == PA_OK);
    Exact<uint8_t> blob(used);
    CHECK(pa_get_state(ctx, blob.get(), used - 1, &used) == PA_ERR_ARG);
    CHECK(pa_get_state(ctx, blob.get(), used, &used) == PA_OK);
    CHECK(pa_set_state(ctx, blob.get(), used - 1) == PA_ERR_STATE);
    CHECK(pa_set_state(ctx, blob.get(), used) == PA_OK);
    CHECK(pa_sync(ctx) == PA_OK);
    CHECK(pa_set_population(ctx, step, R_i, spins.get(), fam.get(), obs.minus_beta_F) == PA_OK);
    CHECK(pa_sync(ctx) == PA_OK);
    CHECK(pa_set_state(ctx, blob.get(), used) == PA_OK);

    double alpha = -1, dbeta = -1;
    CHECK(pa_overlap(ctx, 0.01, &alpha) == PA_OK);
    CHECK(alpha >= 0.0 && alpha <= 1.0);
    CHECK(pa_adaptive_dbeta(ctx, 0.85, 0.1, &dbeta) == PA_OK);
    CHECK(dbeta > 0.0 && dbeta <= 0.1);
    if (R_i >= 2) {
        Dev<double> cq(2);
        CHECK(pa_overlap_correlation(ctx, 1, cq.p) == PA_OK);
        CHECK(pa_overlap_correlation(ctx, R_i, cq.p) == PA_ERR_ARG);
        CHECK(pa_sync(ctx) == PA_OK);
    }
    Dev<float> feat(PA_MLP_IN);
    CHECK(pa_features(ctx, feat.p) == PA_OK);
    CHECK(pa_sync(ctx) == PA_OK);
}

void fixed_schedule_runs() {
    const int L = 8, R = 130, n = 5;
    std::vector<double> betas = linear_betas(0.4, n);
    for (int layout = 0; layout <= 1; ++layout)
        for (int rule = 0; rule <= 3; ++rule)
            for (int update = 0; update <= 1; ++update) {
                pa_config c = config(L, R, betas.data(), n, 2, rule, layout, update);
                size_t bytes = 0;
                CHECK(pa_workspace_size(&c, &bytes) == PA_OK);
                Dev<uint8_t> ws(bytes);
                pa_ctx *ctx = nullptr;
                CHECK(pa_create(&c, ws.p, bytes, nullptr, &ctx) == PA_OK);
                CHECK(pa_run(ctx, 2) == PA_OK);
                CHECK(pa_profile(ctx, 1 | 2) == PA_OK);
                CHECK(pa_anneal_step(ctx) == PA_OK);
                int32_t ns = 0;
                double t[4];
                uint64_t calls = 0, words = 0;
                CHECK(pa_profile_read(ctx, &ns, &t[0], &t[1], &t[2], &calls, &words, &t[3]) == PA_OK);
                CHECK(ns == 1);
                CHECK(pa_profile(ctx, 0) == PA_OK);
                int32_t th = 0, gpb = 0, var = 0;
                CHECK(pa_set_sweep_launch(ctx, L, 128, 1, 0) == PA_OK);
                CHECK(pa_get_sweep_launch(ctx, L, &th, &gpb, &var) == PA_OK);
                CHECK(th == 128 && gpb == 1);
                CHECK(pa_set_sweep_launch(ctx, L, 100, 1, 0) == PA_ERR_ARG);
                CHECK(pa_sync(ctx) == PA_OK);
                read_back(ctx, L * L, 3);
                CHECK(pa_run(ctx, 2) == PA_OK);
                CHECK(pa_sync(ctx) == PA_OK);
                read_back(ctx, L * L, 5);
                CHECK(pa_anneal_step(ctx) == PA_ERR_DONE);  // past the schedule
                CHECK(pa_run(ctx, 1) == PA_ERR_DONE);
                CHECK(std::strlen(pa_last_error(ctx)) > 0);
                CHECK(pa_sync(ctx) == PA_OK);
                pa_destroy(ctx);
            }
}

void caller_driven_run() {
    const int L = 8, R = 200;
    pa_config c = config(L, R, nullptr, 8, 2, PA_RESAMPLE_NEAREST, PA_LAYOUT_MSC64);
    size_t bytes = 0;
    CHECK(pa_workspace_size(&c, &bytes) == PA_OK);
    Dev<uint8_t> ws(bytes);
    pa_ctx *ctx = nullptr;
    CHECK(pa_create(&c, ws.p, bytes, nullptr, &ctx) == PA_OK);
    CHECK(pa_anneal_step_to(ctx, 0.05) == PA_OK);
    CHECK(pa_anneal_step_adaptive(ctx, 0.85, 0.3) == PA_OK);
    std::vector<float> host_params(PA_MLP_PARAMS);
    for (int k = 0; k < PA_MLP_PARAMS; ++k) host_params[k] = 0.01f * (float)((k * 37) % 19 - 9);
    Dev<float> params(PA_MLP_PARAMS);
    HIP_OK(hipMemcpy(params.p, host_params.data(), PA_MLP_PARAMS * sizeof(float), hipMemcpyHostToDevice));
    CHECK(pa_anneal_step_learned(ctx, params.p, 0.5, 0.85, 0.3) == PA_OK);
    CHECK(pa_sync(ctx) == PA_OK);
    double dbeta = 0;
    int32_t accepted = -1;
    Dev<float> feat(PA_MLP_IN);
    CHECK(pa_learned_dbeta(ctx, params.p, 0.5, 0.85, 0.1, feat.p, &dbeta, &accepted) == PA_OK);
    CHECK(dbeta > 0.0 && dbeta <= 0.1 && (accepted == 0 || accepted == 1));
    int32_t n = 0;
    CHECK(pa_schedule_log(ctx, nullptr, nullptr, nullptr, nullptr, 0, &n) == PA_OK);
    CHECK(n == 3);
    Dev<float> f(n * PA_MLP_IN), tg(n);
    Exact<int32_t> acc(n);
    Exact<double> alpha(n);
    CHECK(pa_schedule_log(ctx, f.p, tg.p, acc.get(), alpha.get(), n, &n) == PA_OK);
    CHECK(pa_schedule_log(ctx, f.p, tg.p, acc.get(), alpha.get(), n - 1, &n) == PA_OK);  // cap bounds the rows
    read_back(ctx, L * L, 3);
    pa_destroy(ctx);
}

void batches() {
    const int n = 4;
    std::vector<double> betas = linear_betas(0.44, n);
    pa_config mixed[3] = {config(8, 100, betas.data(), n, 2, PA_RESAMPLE_NEAREST, PA_LAYOUT_MSC64),
                          config(16, 200, betas.data(), n, 2, PA_RESAMPLE_MULTINOMIAL, PA_LAYOUT_INT8),
                          config(8, 64, betas.data(), n, 3, PA_RESAMPLE_POISSON, PA_LAYOUT_MSC64)};
    pa_config same[3] = {mixed[0], mixed[0], mixed[0]};
    same[1].seed += 1;
    same[2].seed += 2;
    same[2].resample = PA_RESAMPLE_MULTINOMIAL;
    for (int which = 0; which < 2; ++which) {
        pa_config *cfgs = which ? same : mixed;
        size_t bytes = 0;
        CHECK(pa_batch_workspace_size(cfgs, 3, &bytes) == PA_OK);
        Dev<uint8_t> ws(bytes);
        pa_batch *b = nullptr;
        CHECK(pa_batch_create(cfgs, 3, ws.p, bytes, nullptr, &b) == PA_OK);
        CHECK(pa_batch_set_sweep_launch(b, 8, 256, 2, 0) == PA_OK);
        int32_t th = 0, gpb = 0, var = 0;
        CHECK(pa_batch_get_sweep_launch(b, 8, &th, &gpb, &var) == PA_OK);
        CHECK(th == 256 && gpb == 2);
        CHECK(pa_batch_get_sweep_launch(b, 32, &th, &gpb, &var) == PA_ERR_ARG);
        CHECK(pa_batch_run(b, n) == PA_OK);
        CHECK(pa_batch_sync(b) == PA_OK);
        pa_obs obs;
        for (int r = 0; r < 3; ++r) {
            for (int i = 0; i <= n; ++i) CHECK(pa_batch_observables(b, r, i, &obs) == PA_OK);
            CHECK(pa_batch_observables(b, r, n + 1, &obs) == PA_ERR_ARG);
            int N = cfgs[r].L * cfgs[r].L, R_i = obs.R_i;
            Exact<int8_t> spins((size_t)R_i * N);
            Exact<int32_t> fam(R_i), E(R_i), M(R_i);
            CHECK(pa_batch_get_population(b, r, 0, R_i, spins.get(), fam.get(), E.get(), M.get()) == PA_OK);
            CHECK(pa_batch_get_population(b, r, 0, R_i + 1, spins.get(), fam.get(), E.get(), M.get()) == PA_ERR_ARG);
        }
        CHECK(pa_batch_observables(b, 3, 0, &obs) == PA_ERR_ARG);
        Dev<pa_weighted> w(n + 1);
        if (which) {
            CHECK(pa_batch_weighted(b, 0, n + 1, w.p) == PA_OK);
            CHECK(pa_batch_weighted(b, 0, n + 2, w.p) == PA_ERR_ARG);
            CHECK(pa_batch_sync(b) == PA_OK);
        } else {
            CHECK(pa_batch_weighted(b, 0, 1, w.p) == PA_ERR_ARG);  // lattice sizes differ
        }
        pa_batch_destroy(b);
    }
}

void free_functions() {
    const int n = 5;
    Dev<uint32_t> ctr(4 * n), out(4 * n);
    CHECK(pa_philox4x32_10(1u, 2u, ctr.p, n, out.p, nullptr) == PA_OK);
    Dev<float> params(PA_MLP_PARAMS), adam(2 * PA_MLP_PARAMS), x(n * PA_MLP_IN), y(n), t(n),
        grad(PA_MLP_PARAMS), loss(1);
    CHECK(pa_mlp_forward(params.p, x.p, n, y.p, nullptr) == PA_OK);
    CHECK(pa_mlp_backward(params.p, x.p, t.p, n, grad.p, loss.p, nullptr) == PA_OK);
    CHECK(pa_mlp_train_step(params.p, adam.p, x.p, t.p, n, 1e-3f, 1, loss.p, nullptr) == PA_OK);
    const int L = 8, R = 100;
    std::vector<int32_t> hostE(R);
    for (int r = 0; r < R; ++r) hostE[r] = -2 * L * L + 4 * (r % 20);
    Dev<int32_t> E(R);
    Dev<double> res(2);
    HIP_OK(hipMemcpy(E.p, hostE.data(), R * sizeof(int32_t), hipMemcpyHostToDevice));
    CHECK(pa_adaptive_dbeta_noalloc(E.p, R, L, 0.85, 0.1, res.p, nullptr) == PA_OK);
    CHECK(pa_adaptive_dbeta_noalloc(E.p, R, 130, 0.85, 0.1, res.p, nullptr) == PA_ERR_ARG);
    HIP_OK(hipDeviceSynchronize());
}

}  // namespace

int main(int argc, char **argv) {
    bool device = argc > 1 && std::strcmp(argv[1], "device") == 0;
    workspace_layouts();
    invalid_configurations();
    create_failures();
    null_handles();
    std::printf("host checks ok\n");
    std::fflush(stdout);
    if (device) {
        int count = 0;
        HIP_OK(hipGetDeviceCount(&count));
        CHECK(count > 0);
        HIP_OK(hipSetDevice(0));
        fixed_schedule_runs();
        std::printf("fixed-schedule runs ok\n");
        std::fflush(stdout);
        caller_driven_run();
        std::printf("caller-driven run ok\n");
        std::fflush(stdout);
        batches();
        free_functions();
        std::printf("device checks ok\n");
    }
    return 0;
}
