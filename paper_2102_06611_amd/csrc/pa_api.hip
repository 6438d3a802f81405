// libpa host side: configuration checks, workspace carving, kernel sequencing
// and the extern "C" entry points declared in pa.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pa.h"
#include "pa_device.hpp"
#include "pa_internal.hpp"

using namespace pa;

namespace {

thread_local std::string g_last_error;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int default_capacity(const pa_config &c) {
    int64_t cap;
    if (c.capacity > 0)
        cap = c.capacity;
    else if (c.resample == PA_RESAMPLE_NEAREST || c.resample == PA_RESAMPLE_POISSON)
        cap = (int64_t)c.R + (int64_t)std::ceil(10.0 * std::sqrt((double)c.R));
    else
        cap = c.R;
    return (int)((cap + 63) / 64 * 64);
}

bool validate(const pa_config &c, std::string *why) {
    auto fail = [&](const char *m) {
        *why = m;
        return false;
    };
    if (c.L < 4 || c.L > kMaxL || (c.L & 1)) return fail("L must be even and in [4, 128]");
    if (c.R < 1 || c.R > (1 << 24)) return fail("R must be in [1, 2^24]");
    if (c.n_steps < 0 || c.n_steps > 10000000) return fail("n_steps must be in [0, 1e7]");
    if (c.theta < 0 || c.theta > 1000000) return fail("theta must be in [0, 1e6]");
    if (c.resample < 0 || c.resample > 3) return fail("unknown resampling rule");
    // multinomial: the quantised weights are at most 2^40 each, so their total
    // over R parents stays below 2^63 (signed 64-bit block sums) for R < 2^23
    if (c.resample == PA_RESAMPLE_MULTINOMIAL && c.R >= (1 << 23))
        return fail("multinomial resampling needs R < 2^23 (64-bit total of the 2^40-quantised weights)");
    // the global half-sweep index 2 (theta (i - 1) + s) + colour is a 32-bit Philox
    // counter word: it must not wrap over the run's steps
    if (2 * (int64_t)c.theta * (int64_t)c.n_steps > (int64_t)1 << 32)
        return fail("2 theta n_steps must not exceed 2^32 (half-sweep counter of the random stream)");
    if (c.layout < 0 || c.layout > 1) return fail("unknown layout");
    if (c.capacity < 0) return fail("capacity must be >= 0");
    if (c.capacity > 0 && c.capacity < c.R) return fail("capacity must be >= R");
    if (c.update != PA_UPDATE_METROPOLIS && c.update != PA_UPDATE_HEATBATH)
        return fail("unknown spin update");
    if (c.betas) {
        if (c.betas[0] != 0.0) return fail("betas[0] must be 0 (simple sampling start)");
        for (int i = 1; i <= c.n_steps; ++i) {
            if (!(c.betas[i] >= c.betas[i - 1]) || !std::isfinite(c.betas[i]))
                return fail("betas must be finite and non-decreasing");
        }
    }
    return true;
}

struct RunPlan {
    int L, N, R, C, G, K, nblk, max_steps;
    size_t off_ms[2], off_s8[2], off_E, off_M, off_fam[2], off_hist, off_zlev, off_wlev,
        off_plev, off_cnt, off_off, off_par, off_cum, off_send, off_e8, off_part, off_partd, off_blk, off_betas, off_records, off_st,
        off_stage, off_feat, off_flog, off_tlog, off_alog, off_alpha, off_jkw;
    size_t bytes;
};

RunPlan plan_run(const pa_config &c) {
    RunPlan p{};
    p.L = c.L;
    p.N = c.L * c.L;
    p.R = c.R;
    p.C = default_capacity(c);
    p.G = p.C / 64;
    p.K = p.N + 1;
    p.nblk = (p.C + kSlotBlock - 1) / kSlotBlock;
    p.max_steps = c.n_steps;
    size_t o = 0;
    auto take = [&](size_t n) {
        size_t at = o;
        o = align_up(o + n, 256);
        return at;
    };
    size_t pop = (c.layout == PA_LAYOUT_MSC64) ? (size_t)p.G * p.N * 8 : (size_t)p.G * p.N * 64;
    for (int b = 0; b < 2; ++b) {
        if (c.layout == PA_LAYOUT_MSC64) {
            p.off_ms[b] = take(pop);
            p.off_s8[b] = SIZE_MAX;
        } else {
            p.off_s8[b] = take(pop);
            p.off_ms[b] = SIZE_MAX;
        }
    }
    p.off_E = take((size_t)p.C * 4);
    p.off_M = take((size_t)p.C * 4);
    p.off_fam[0] = take((size_t)p.C * 4);
    p.off_fam[1] = take((size_t)p.C * 4);
    p.off_hist = take((size_t)p.K * 4);
    p.off_zlev = take((size_t)p.K * 8);
    p.off_wlev = take((size_t)p.K * 16);
    p.off_plev = take((size_t)p.K * 48);
    p.off_cnt = take((size_t)p.C * 4);
    p.off_off = take((size_t)(p.C + 1) * 4);
    p.off_par = take((size_t)p.C * 4);
    p.off_cum = take((size_t)p.C * 8);
    p.off_send = take((size_t)p.G * 8);
    p.off_e8 = take((size_t)p.C);  // C / 8 entries of 8 bytes
    p.off_part = take((size_t)p.nblk * 8 * 8);
    p.off_partd = take((size_t)p.nblk * 2 * 8);
    p.off_blk = take((size_t)kBlocks * 4 * 8);
    p.off_betas = take((size_t)(p.max_steps + 1) * 8);
    p.off_records = take((size_t)(p.max_steps + 1) * sizeof(pa_obs));
    p.off_st = take(sizeof(RunState));
    p.off_stage = take((size_t)64 * p.N);
    p.off_feat = take(64 * sizeof(float));
    p.off_flog = take((size_t)(p.max_steps + 1) * PA_MLP_IN * sizeof(float));
    p.off_tlog = take((size_t)(p.max_steps + 1) * sizeof(float));
    p.off_alog = take((size_t)(p.max_steps + 1) * sizeof(int32_t));
    p.off_alpha = take((size_t)(p.max_steps + 1) * sizeof(double));
    p.off_jkw = take((size_t)kBlocks * sizeof(double));
    p.bytes = o;
    return p;
}

// Map arrays (blk_off and run_id) of every launch, laid out in one int32 buffer.
struct MapBuild {
    std::vector<int32_t> ints;
    size_t add(const std::vector<int> &runs, const std::vector<int> &blocks, int *total) {
        size_t at = ints.size();
        int acc = 0;
        for (size_t k = 0; k < runs.size(); ++k) {
            ints.push_back(acc);
            acc += blocks[k];
        }
        ints.push_back(acc);
        for (int r : runs) ints.push_back(r);
        *total = acc;
        return at;
    }
};

struct EngineLayout {
    std::vector<RunPlan> plans;
    std::vector<size_t> run_base;
    size_t off_descs, off_maps, bytes;
    MapBuild maps;
    // map positions (int offsets into maps.ints)
    size_t m_slots, m_groups;
    int t_slots, t_groups;
    struct Cls {
        int L;
        size_t at;
        int total;
        int n;
        bool msc, i8;
        std::vector<int> runs;  // runs with this L
    };
    std::vector<Cls> classes;
};

EngineLayout layout_engine(const pa_config *cfgs, int n) {
    EngineLayout E;
    size_t o = 0;
    for (int r = 0; r < n; ++r) {
        E.plans.push_back(plan_run(cfgs[r]));
        E.run_base.push_back(o);
        o = align_up(o + E.plans.back().bytes, 256);
    }
    std::vector<int> all, nblk, groups;
    for (int r = 0; r < n; ++r) {
        all.push_back(r);
        nblk.push_back(E.plans[r].nblk);
        groups.push_back(E.plans[r].G);
    }
    E.m_slots = E.maps.add(all, nblk, &E.t_slots);
    E.m_groups = E.maps.add(all, groups, &E.t_groups);
    // sweep classes by L, larger lattices first
    std::vector<int> Ls;
    for (int r = 0; r < n; ++r)
        if (std::find(Ls.begin(), Ls.end(), cfgs[r].L) == Ls.end()) Ls.push_back(cfgs[r].L);
    std::sort(Ls.begin(), Ls.end(), [](int a, int b) { return a > b; });
    for (int L : Ls) {
        std::vector<int> rs, gs;
        bool msc = false, i8 = false;
        for (int r = 0; r < n; ++r) {
            if (cfgs[r].L != L) continue;
            rs.push_back(r);
            gs.push_back(E.plans[r].G);
            (cfgs[r].layout == PA_LAYOUT_MSC64 ? msc : i8) = true;
        }
        EngineLayout::Cls c;
        c.L = L;
        c.n = (int)rs.size();
        c.at = E.maps.add(rs, gs, &c.total);
        c.msc = msc;
        c.i8 = i8;
        c.runs = rs;
        E.classes.push_back(c);
    }
    E.off_descs = o;
    o = align_up(o + sizeof(RunDesc) * n, 256);
    E.off_maps = o;
    o = align_up(o + E.maps.ints.size() * 4, 256);
    E.bytes = o;
    return E;
}

void dd_n_ln2(int N, double *hi, double *lo) {
    const double l_hi = 6.93147180559945286227e-01, l_lo = 2.31904681384629955842e-17;
    double p = N * l_hi;
    double e = std::fma((double)N, l_hi, -p) + N * l_lo;
    double s = p + e;
    *hi = s;
    *lo = e - (s - p);
}

// Default sweep geometry (what the autotuner finds on gfx950 for the usual
// population sizes): one 64-replica group per block, 128 threads for L <= 16,
// 512 up to L = 64 and 1024 above, where a lattice fills most of a CU's LDS.
void default_sweep_launch(int L, int *threads, int *gpb) {
    *gpb = 1;
    *threads = L <= 16 ? 128 : (L <= 64 ? 512 : 1024);
}

std::once_flag g_config_once;
hipError_t g_config_err = hipSuccess;

}  // namespace

// ----------------------------------------------------------------------------
constexpr int kProfEvents = 5;  // before counts, copy, sweeps, measurement, and after

struct pa_batch {
    std::vector<pa_config> cfg;
    std::vector<std::vector<double>> betas;
    int n = 0;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    EngineLayout lay;
    std::vector<RunDesc> desc;
    RunDesc *d_runs = nullptr;
    LaunchCtx lc;
    std::vector<int> host_step;  // steps enqueued per run
    std::string err;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool dead = false;
    std::vector<std::vector<int32_t>> class_maps;  // host copies of uploaded sweep maps
    // phase timing (pa_profile)
    bool profiling = false;
    std::vector<hipEvent_t> events;  // kProfEvents per profiled step
    int profiled_steps = 0;
};

struct pa_ctx {
    pa_batch b;
};

namespace {

pa_status fail(pa_batch *b, pa_status s, const std::string &msg) {
    if (b) b->err = msg;
    g_last_error = msg;
    return s;
}

pa_status hip_fail(pa_batch *b, hipError_t e, const char *what) {
    if (b) b->dead = true;
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    return fail(b, PA_ERR_DEVICE, buf);
}

#define PA_HIP(b, call)                                   \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(b, e_, #call); \
    } while (0)

pa_status workspace_size(const pa_config *cfgs, int n, size_t *bytes) {
    if (!cfgs || !bytes || n < 1 || n > 4096) return fail(nullptr, PA_ERR_ARG, "bad arguments");
    std::string why;
    for (int r = 0; r < n; ++r)
        if (!validate(cfgs[r], &why)) return fail(nullptr, PA_ERR_ARG, why);
    *bytes = layout_engine(cfgs, n).bytes;
    return PA_OK;
}

// (Re)write the block offsets of sweep class k for its groups-per-block.
pa_status upload_class_map(pa_batch *B, int k) {
    const auto &c = B->lay.classes[k];
    SweepClass &sc = B->lc.sweep_classes[k];
    std::vector<int32_t> off(c.runs.size() + 1);
    int acc = 0;
    for (size_t q = 0; q < c.runs.size(); ++q) {
        off[q] = acc;
        acc += (B->lay.plans[c.runs[q]].G + sc.gpb - 1) / sc.gpb;
    }
    off[c.runs.size()] = acc;
    sc.total = acc;
    B->class_maps.push_back(off);  // keep the host copy alive for the async copy
    PA_HIP(B, hipMemcpyAsync((void *)sc.map.blk_off, B->class_maps.back().data(), off.size() * 4,
                             hipMemcpyHostToDevice, B->stream));
    return PA_OK;
}

pa_status engine_create(pa_batch *B, const pa_config *cfgs, int n, void *ws, size_t bytes,
                        void *stream) {
    std::string why;
    for (int r = 0; r < n; ++r)
        if (!validate(cfgs[r], &why)) return fail(B, PA_ERR_ARG, why);
    if (!ws) return fail(B, PA_ERR_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(B, PA_ERR_ARG, "workspace must be 256-byte aligned");
    B->n = n;
    B->stream = (hipStream_t)stream;
    B->ws = (char *)ws;
    B->lay = layout_engine(cfgs, n);
    if (bytes < B->lay.bytes) return fail(B, PA_ERR_NOMEM, "workspace smaller than pa_workspace_size()");
    std::call_once(g_config_once, [] { g_config_err = configure_kernels(); });
    if (g_config_err != hipSuccess) return hip_fail(B, g_config_err, "configure_kernels");

    B->cfg.assign(cfgs, cfgs + n);
    B->betas.resize(n);
    B->desc.resize(n);
    std::vector<RunState> states(n);
    for (int r = 0; r < n; ++r) {
        const pa_config &c = cfgs[r];
        const RunPlan &p = B->lay.plans[r];
        char *base = B->ws + B->lay.run_base[r];
        auto &bt = B->betas[r];
        bt.assign((size_t)p.max_steps + 1, 0.0);
        if (c.betas)
            for (int i = 0; i <= p.max_steps; ++i) bt[i] = c.betas[i];
        B->cfg[r].betas = nullptr;  // the caller's array is not retained
        RunDesc &d = B->desc[r];
        std::memset(&d, 0, sizeof d);
        d.L = p.L;
        d.N = p.N;
        d.R = p.R;
        d.C = p.C;
        d.G = p.G;
        d.K = p.K;
        d.theta = c.theta;
        d.resample = c.resample;
        d.update = c.update;
        d.layout = c.layout;
        d.max_steps = p.max_steps;
        d.key0 = (uint32_t)c.seed;
        d.key1 = (uint32_t)(c.seed >> 32);
        d.nblk = p.nblk;
        for (int b = 0; b < 2; ++b) {
            d.ms[b] = p.off_ms[b] == SIZE_MAX ? nullptr : (uint64_t *)(base + p.off_ms[b]);
            d.s8[b] = p.off_s8[b] == SIZE_MAX ? nullptr : (int8_t *)(base + p.off_s8[b]);
            d.fam[b] = (int32_t *)(base + p.off_fam[b]);
        }
        d.E = (int32_t *)(base + p.off_E);
        d.M = (int32_t *)(base + p.off_M);
        d.hist = (int32_t *)(base + p.off_hist);
        d.zlev = (uint64_t *)(base + p.off_zlev);
        d.wlev = (double *)(base + p.off_wlev);
        d.plev = (double *)(base + p.off_plev);
        d.cnt = (int32_t *)(base + p.off_cnt);
        d.off = (int32_t *)(base + p.off_off);
        d.par = (int32_t *)(base + p.off_par);
        d.cum = (uint64_t *)(base + p.off_cum);
        d.send = (uint64_t *)(base + p.off_send);
        d.e8 = (uint64_t *)(base + p.off_e8);
        d.part = (int64_t *)(base + p.off_part);
        d.partd = (double *)(base + p.off_partd);
        d.blk = (int64_t *)(base + p.off_blk);
        d.betas = (double *)(base + p.off_betas);
        d.records = (pa_obs *)(base + p.off_records);
        d.st = (RunState *)(base + p.off_st);
        d.stage = (int8_t *)(base + p.off_stage);
        d.feat = (float *)(base + p.off_feat);
        d.feat_log = (float *)(base + p.off_flog);
        d.tgt_log = (float *)(base + p.off_tlog);
        d.acc_log = (int32_t *)(base + p.off_alog);
        d.alpha_log = (double *)(base + p.off_alpha);
        d.jkw = (double *)(base + p.off_jkw);
        RunState &s = states[r];
        std::memset(&s, 0, sizeof s);
        s.step = -1;
        s.cur = 1;
        s.R_new = p.R;
        s.kmin = INT32_MAX;  // empty histogram; the first reduction fills it
        s.kmax = -1;
        dd_n_ln2(p.N, &s.acc_hi, &s.acc_lo);  // ln Z_0 = L^2 ln 2
    }
    PA_HIP(B, launch_fill_zero(B->ws, B->lay.bytes, B->stream));  // deterministic contents
    B->d_runs = (RunDesc *)(B->ws + B->lay.off_descs);
    int32_t *d_maps = (int32_t *)(B->ws + B->lay.off_maps);
    hipStream_t st = B->stream;
    PA_HIP(B, hipMemcpyAsync(B->d_runs, B->desc.data(), sizeof(RunDesc) * n, hipMemcpyHostToDevice, st));
    PA_HIP(B, hipMemcpyAsync(d_maps, B->lay.maps.ints.data(), B->lay.maps.ints.size() * 4,
                             hipMemcpyHostToDevice, st));
    for (int r = 0; r < n; ++r) {
        PA_HIP(B, hipMemcpyAsync(B->desc[r].st, &states[r], sizeof(RunState), hipMemcpyHostToDevice, st));
        PA_HIP(B, hipMemcpyAsync(B->desc[r].betas, B->betas[r].data(), B->betas[r].size() * 8,
                                 hipMemcpyHostToDevice, st));
    }
    LaunchCtx &lc = B->lc;
    lc.runs = B->d_runs;
    lc.n_runs = n;
    lc.stream = st;
    auto mk = [&](size_t at, int nn) {
        WorkMap m;
        m.n = nn;
        m.blk_off = d_maps + at;
        m.run_id = d_maps + at + nn + 1;
        return m;
    };
    lc.slots.map = mk(B->lay.m_slots, n);
    lc.slots.total = B->lay.t_slots;
    lc.groups.map = mk(B->lay.m_groups, n);
    lc.groups.total = B->lay.t_groups;
    lc.sweep_classes.clear();
    for (auto &c : B->lay.classes) {
        SweepClass sc;
        sc.L = c.L;
        sc.N = c.L * c.L;
        sc.map = mk(c.at, c.n);
        sc.total = c.total;
        sc.has_msc = c.msc;
        sc.has_int8 = c.i8;
        default_sweep_launch(c.L, &sc.threads, &sc.gpb);
        lc.sweep_classes.push_back(sc);
    }
    for (size_t k = 0; k < lc.sweep_classes.size(); ++k) {
        pa_status e = upload_class_map(B, (int)k);
        if (e) return e;
    }
    if (lc.sweep_classes.size() > 1) {  // the classes' sweeps side by side
        for (size_t k = 0; k < lc.sweep_classes.size(); ++k) {
            hipStream_t s = nullptr;
            PA_HIP(B, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            lc.class_streams.push_back(s);
        }
        for (size_t k = 0; k <= lc.sweep_classes.size(); ++k) {
            hipEvent_t ev = nullptr;
            PA_HIP(B, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            lc.class_events.push_back(ev);
        }
    }
    lc.max_nblk = 1;  // multinomial runs (R < 2^23): at most 8192 blocks, 64 KiB of draw LDS
    for (int r = 0; r < n; ++r)
        if (cfgs[r].resample == PA_RESAMPLE_MULTINOMIAL)
            lc.max_nblk = std::max(lc.max_nblk, B->lay.plans[r].nblk);
    lc.any_nearest = lc.any_multi = lc.any_poisson = false;
    lc.any_msc = lc.any_int8 = false;
    lc.any_update[0] = lc.any_update[1] = false;
    lc.max_L = 0;
    for (int r = 0; r < n; ++r) {
        lc.max_L = std::max(lc.max_L, (int)cfgs[r].L);
        if (cfgs[r].resample == PA_RESAMPLE_MULTINOMIAL) lc.any_multi = true;
        else if (cfgs[r].resample == PA_RESAMPLE_POISSON) lc.any_poisson = true;
        else lc.any_nearest = true;
        lc.any_update[cfgs[r].update] = true;
        if (cfgs[r].layout == PA_LAYOUT_MSC64) lc.any_msc = true;
        else lc.any_int8 = true;
    }
    PA_HIP(B, launch_init(lc));
    PA_HIP(B, launch_sweeps(lc, 1));
    PA_HIP(B, launch_reduce(lc));
    PA_HIP(B, hipStreamSynchronize(st));  // the host arrays above are now consumed
    B->class_maps.clear();
    B->host_step.assign(n, 0);
    return PA_OK;
}

pa_status read_state(pa_batch *B, int r, RunState *s) {
    PA_HIP(B, hipStreamSynchronize(B->stream));
    PA_HIP(B, hipMemcpy(s, B->desc[r].st, sizeof(RunState), hipMemcpyDeviceToHost));
    return PA_OK;
}

pa_status engine_sync(pa_batch *B) {
    if (B->dead) return fail(B, PA_ERR_DEVICE, "handle is unusable after a device error");
    pa_status worst = PA_OK;
    for (int r = 0; r < B->n; ++r) {
        RunState s;
        pa_status e = read_state(B, r, &s);
        if (e) return e;
        B->host_step[r] = s.step;
        if (s.err && worst == PA_OK) {
            char buf[160];
            std::snprintf(buf, sizeof buf, "run %d: device status %d raised at step %d", r, s.err,
                          s.err_step);
            worst = fail(B, s.err, buf);
        }
    }
    return worst;
}

pa_status engine_step(pa_batch *B) {
    if (B->dead) return fail(B, PA_ERR_DEVICE, "handle is unusable after a device error");
    if (!B->profiling) {
        PA_HIP(B, launch_step(B->lc));
    } else {
        const size_t base = (size_t)B->profiled_steps * kProfEvents;
        while (B->events.size() < base + kProfEvents) {
            hipEvent_t ev;
            PA_HIP(B, hipEventCreate(&ev));
            B->events.push_back(ev);
        }
        PA_HIP(B, hipEventRecord(B->events[base], B->stream));
        PA_HIP(B, launch_counts(B->lc));
        PA_HIP(B, hipEventRecord(B->events[base + 1], B->stream));
        PA_HIP(B, launch_copy(B->lc));
        PA_HIP(B, hipEventRecord(B->events[base + 2], B->stream));
        PA_HIP(B, launch_sweeps(B->lc, 0));
        PA_HIP(B, hipEventRecord(B->events[base + 3], B->stream));
        PA_HIP(B, launch_reduce(B->lc));
        PA_HIP(B, hipEventRecord(B->events[base + 4], B->stream));
        ++B->profiled_steps;
    }
    for (auto &s : B->host_step) ++s;
    return PA_OK;
}

pa_status engine_run(pa_batch *B, int n_steps) {
    if (B->dead) return fail(B, PA_ERR_DEVICE, "handle is unusable after a device error");
    if (n_steps < 0) return fail(B, PA_ERR_ARG, "n_steps < 0");
    if (n_steps == 0) return PA_OK;
    if (B->stream == nullptr) {  // the null stream cannot be captured
        for (int k = 0; k < n_steps; ++k) {
            pa_status e = engine_step(B);
            if (e) return e;
        }
        return PA_OK;
    }
    if (!B->exec) {
        PA_HIP(B, hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
        hipError_t le = launch_step(B->lc);
        hipGraph_t g = nullptr;
        hipError_t ce = hipStreamEndCapture(B->stream, &g);
        if (le != hipSuccess) return hip_fail(B, le, "launch_step (capture)");
        if (ce != hipSuccess) return hip_fail(B, ce, "hipStreamEndCapture");
        B->graph = g;
        PA_HIP(B, hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0));
    }
    for (int k = 0; k < n_steps; ++k) PA_HIP(B, hipGraphLaunch(B->exec, B->stream));
    for (auto &s : B->host_step) s += n_steps;
    return PA_OK;
}

pa_status engine_observables(pa_batch *B, int r, int step, pa_obs *out) {
    if (!out || r < 0 || r >= B->n) return fail(B, PA_ERR_ARG, "bad arguments");
    if (B->dead) return fail(B, PA_ERR_DEVICE, "handle is unusable after a device error");
    RunState s;
    pa_status e = read_state(B, r, &s);
    if (e) return e;
    if (step < 0 || step > s.step) {
        if (s.err) return fail(B, s.err, "step not reached: the run stopped on a device status");
        return fail(B, PA_ERR_ARG, "step not reached yet");
    }
    PA_HIP(B, hipMemcpy(out, B->desc[r].records + step, sizeof(pa_obs), hipMemcpyDeviceToHost));
    return PA_OK;
}

void engine_destroy(pa_batch *B) {
    for (hipEvent_t ev : B->events) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : B->lc.class_events) (void)hipEventDestroy(ev);
    for (hipStream_t s : B->lc.class_streams) (void)hipStreamDestroy(s);
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
}

}  // namespace

// ============================================================================ C ABI

extern "C" {

pa_status pa_workspace_size(const pa_config *cfg, size_t *bytes) { return workspace_size(cfg, 1, bytes); }

pa_status pa_create(const pa_config *cfg, void *ws, size_t bytes, void *stream, pa_ctx **out) {
    if (!cfg || !out) return fail(nullptr, PA_ERR_ARG, "bad arguments");
    *out = nullptr;
    pa_ctx *c = new pa_ctx();
    pa_status e = engine_create(&c->b, cfg, 1, ws, bytes, stream);
    if (e) {
        g_last_error = c->b.err;
        engine_destroy(&c->b);
        delete c;
        return e;
    }
    *out = c;
    return PA_OK;
}

pa_status pa_anneal_step(pa_ctx *ctx) {
    if (!ctx) return fail(nullptr, PA_ERR_ARG, "NULL handle");
    pa_batch *B = &ctx->b;
    if (B->host_step[0] >= B->desc[0].max_steps) return fail(B, PA_ERR_DONE, "schedule exhausted");
    return engine_step(B);
}

pa_status pa_anneal_step_to(pa_ctx *ctx, double beta_next) {
    if (!ctx) return fail(nullptr, PA_ERR_ARG, "NULL handle");
    pa_batch *B = &ctx->b;
    if (B->dead) return fail(B, PA_ERR_DEVICE, "handle is unusable after a device error");
    int i = B->host_step[0] + 1;
    if (i > B->desc[0].max_steps) return fail(B, PA_ERR_DONE, "no room for another step");
    if (!std::isfinite(beta_next)) return fail(B, PA_ERR_ARG, "beta_next must be finite");
    B->betas[0][i] = beta_next;
    PA_HIP(B, launch_set_beta(B->lc, 0, i, beta_next));
    return engine_step(B);
}

pa_status pa_run(pa_ctx *ctx, int32_t n_steps) {
    if (!ctx) return fail(nullptr, PA_ERR_ARG, "NULL handle");
    pa_batch *B = &ctx->b;
    if (B->host_step[0] + (int64_t)n_steps > B->desc[0].max_steps)
        return fail(B, PA_ERR_DONE, "n_steps runs past the end of the schedule");
    return engine_run(B, n_steps);
}

pa_status pa_sync(pa_ctx *ctx) {
    if (!ctx) return fail(nullptr, PA_ERR_ARG, "NULL handle");
    return engine_sync(&ctx->b);
}

pa_status pa_observables(pa_ctx *ctx, int32_t step, pa_obs *out) {
    if (!ctx) return fail(nullptr, PA_ERR_ARG, "NULL handle");
    return engine_observables(&ctx->b, 0, step, out);
}

pa_status pa_current(pa_ctx *ctx, int32_t *step, int32_t *R_i) {
    if (!ctx) return fail(nullptr, PA_ERR_ARG, "NULL handle");
    pa_batch *B = &ctx->b;
    RunState s;
    pa_status e = read_state(B, 0, &s);
    if (e) return e;
    if (step) *step = s.step;
    if (R_i) *R_i = s.R_cur;
    return PA_OK;
}

pa_status pa_energy_histogram(pa_ctx *ctx, int32_t *counts, int32_t cap, int32_t *k_min,
                              int32_t *n_bins) {
    if (!ctx || !n_bins || !k_min) return fail(nullptr, PA_ERR_ARG, "bad arguments");
    pa_batch *B = &ctx->b;
    RunState s;
    pa_status e = read_state(B, 0, &s);
    if (e) return e;
    if (s.kmax < s.kmin) return fail(B, PA_ERR_STATE, "no histogram has been computed yet");
    int nb = s.kmax - s.kmin + 1;
    *k_min = s.kmin;
    *n_bins = nb;
    if (counts) {
        if (cap < nb) return fail(B, PA_ERR_ARG, "cap smaller than n_bins");
        PA_HIP(B, hipMemcpy(counts, B->desc[0].hist + s.kmin, (size_t)nb * 4, hipMemcpyDeviceToHost));
    }
    return PA_OK;
}

pa_status pa_copy_counts(pa_ctx *ctx, int32_t *cnt, int64_t cap, int64_t *n) {
    if (!ctx || !n) return fail(nullptr, PA_ERR_ARG, "bad arguments");
    pa_batch *B = &ctx->b;
    RunState s;
    pa_status e = read_state(B, 0, &s);
    if (e) return e;
    *n = s.r_parents;
    if (cnt && s.r_parents) {
        if (cap < s.r_parents) return fail(B, PA_ERR_ARG, "cap smaller than R_{i-1}");
        PA_HIP(B, hipMemcpy(cnt, B->desc[0].cnt, (size_t)s.r_parents * 4, hipMemcpyDeviceToHost));
    }
    return PA_OK;
}

static pa_status engine_get_population(pa_batch *B, int r, int32_t first, int32_t count,
                                       int8_t *spins, int32_t *fam, int32_t *E, int32_t *M) {
    if (r < 0 || r >= B->n) return fail(B, PA_ERR_ARG, "run index outside the batch");
    RunState s;
    pa_status e = read_state(B, r, &s);
    if (e) return e;
    const RunDesc &d = B->desc[r];
    if (first < 0 || count < 0 || (int64_t)first + count > s.R_cur)
        return fail(B, PA_ERR_ARG, "replica range outside the population");
    if (count == 0) return PA_OK;
    if (spins) {
        std::vector<int8_t> tmp((size_t)64 * d.N);
        for (int g = first / 64; g <= (first + count - 1) / 64; ++g) {
            PA_HIP(B, launch_unpack_group(B->lc, r, g, d.N));
            PA_HIP(B, hipStreamSynchronize(B->stream));
            PA_HIP(B, hipMemcpy(tmp.data(), d.stage, tmp.size(), hipMemcpyDeviceToHost));
            int lo = std::max(first, g * 64), hi = std::min(first + count, g * 64 + 64);
            for (int rr = lo; rr < hi; ++rr)
                std::memcpy(spins + (size_t)(rr - first) * d.N, tmp.data() + (size_t)(rr - g * 64) * d.N, d.N);
        }
    }
    if (fam) PA_HIP(B, hipMemcpy(fam, d.fam[s.cur] + first, (size_t)count * 4, hipMemcpyDeviceToHost));
    if (E) PA_HIP(B, hipMemcpy(E, d.E + first, (size_t)count * 4, hipMemcpyDeviceToHost));
    if (M) PA_HIP(B, hipMemcpy(M, d.M + first, (size_t)count * 4, hipMemcpyDeviceToHost));
    return PA_OK;
}

pa_status pa_get_population(pa_ctx *ctx, int32_t first, int32_t count, int8_t *spins,
                            int32_t *fam, int32_t *E, int32_t *M) {
    if (!ctx) return fail(nullptr, PA_ERR_ARG, "NULL handle");
    return engine_get_population(&ctx->b, 0, first, count, spins, fam, E, M);
}

pa_status pa_batch_get_population(pa_batch *b, int32_t run, int32_t first, int32_t count,
                                  int8_t *spins, int32_t *fam, int32_t *E, int32_t *M) {
    if (!b) return fail(nullptr, PA_ERR_ARG, "NULL handle");
    return engine_get_population(b, run, first, count, spins, fam, E, M);
}

pa_status pa_set_population(pa_ctx *ctx, int32_t step, int32_t R_i, const int8_t *spins,
                            const int32_t *fam, double minus_beta_F) {
    if (!ctx || !spins || !fam) return fail(nullptr, PA_ERR_ARG, "bad arguments");
    pa_batch *B = &ctx->b;
    if (B->dead) return fail(B, PA_ERR_DEVICE, "handle is unusable after a device error");
    const RunDesc &d = B->desc[0];
    if (R_i < 1 || R_i > d.C) return fail(B, PA_ERR_ARG, "R_i must be in [1, capacity]");
    if (step < 0 || step > d.max_steps) return fail(B, PA_ERR_ARG, "step outside the schedule");
    for (int64_t k = 0; k < (int64_t)R_i * d.N; ++k)
        if (spins[k] != 1 && spins[k] != -1) return fail(B, PA_ERR_STATE, "spins must be +1 or -1");
    PA_HIP(B, hipStreamSynchronize(B->stream));
    PA_HIP(B, launch_adopt_begin(B->lc, 0, R_i));
    std::vector<int8_t> tmp((size_t)64 * d.N, (int8_t)-1);
    for (int g = 0; g * 64 < R_i; ++g) {
        int nv = std::min(64, R_i - g * 64);
        std::memcpy(tmp.data(), spins + (size_t)g * 64 * d.N, (size_t)nv * d.N);
        PA_HIP(B, hipMemcpyAsync(d.stage, tmp.data(), tmp.size(), hipMemcpyHostToDevice, B->stream));
        PA_HIP(B, launch_pack_group(B->lc, 0, g, 0, nv, d.N));
        PA_HIP(B, hipStreamSynchronize(B->stream));
    }
    PA_HIP(B, hipMemcpyAsync(d.fam[0], fam, (size_t)R_i * 4, hipMemcpyHostToDevice, B->stream));
    PA_HIP(B, hipStreamSynchronize(B->stream));
    PA_HIP(B, launch_sweeps(B->lc, 1));  // E, M of the adopted population
    PA_HIP(B, launch_adopt_end(B->lc, 0, step, minus_beta_F));
    PA_HIP(B, launch_hist_current(B->lc));  // the next step reads the histogram
    PA_HIP(B, hipStreamSynchronize(B->stream));
    B->host_step[0] = step;
    return PA_OK;
}

namespace {
// Snapshot layout: header, RunState, the live population groups, then family
// labels, energies and magnetisations of the R_i replicas, the schedule and
// the records 0..step.  Nothing outside the live population is stored, so two
// runs in the same state give identical snapshots.
struct StateHeader {
    char magic[8];
    int32_t L, R, C, layout, resample, max_steps, theta, step, R_i, update;
    uint64_t seed;
};

size_t group_bytes(const RunDesc &d) {
    return d.layout == PA_LAYOUT_MSC64 ? (size_t)d.N * 8 : (size_t)d.N * 64;
}

size_t snapshot_bytes(const RunDesc &d, int step, int R_i) {
    const size_t groups = (size_t)(R_i + 63) / 64;
    return sizeof(StateHeader) + sizeof(RunState) + groups * group_bytes(d) + (size_t)R_i * 12 +
           (size_t)(d.max_steps + 1) * 8 + (size_t)(step + 1) * sizeof(pa_obs);
}
}  // namespace

pa_status pa_get_state(pa_ctx *ctx, void *buf, size_t cap, size_t *used) {
    if (!ctx || !used) return fail(nullptr, PA_ERR_ARG, "bad arguments");
    pa_batch *B = &ctx->b;
    const RunDesc &d = B->desc[0];
    RunState s;
    pa_status e = read_state(B, 0, &s);
    if (e) return e;
    if (s.err) return fail(B, s.err, "the run stopped on a device status");
    const size_t need = snapshot_bytes(d, s.step, s.R_cur);
    *used = need;
    if (!buf) return PA_OK;
    if (cap < need) return fail(B, PA_ERR_ARG, "cap smaller than the state");
    char *p = (char *)buf;
    StateHeader h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, "PASTATE3", 8);
    h.L = d.L; h.R = d.R; h.C = d.C; h.layout = d.layout; h.resample = d.resample;
    h.max_steps = d.max_steps; h.theta = d.theta; h.step = s.step; h.R_i = s.R_cur;
    h.update = d.update;
    h.seed = B->cfg[0].seed;
    std::memcpy(p, &h, sizeof h); p += sizeof h;
    std::memcpy(p, &s, sizeof s); p += sizeof s;
    const size_t pop = (size_t)(s.R_cur + 63) / 64 * group_bytes(d);
    const void *src = d.layout == PA_LAYOUT_MSC64 ? (const void *)d.ms[s.cur] : (const void *)d.s8[s.cur];
    PA_HIP(B, hipMemcpy(p, src, pop, hipMemcpyDeviceToHost)); p += pop;
    const size_t n4 = (size_t)s.R_cur * 4;
    PA_HIP(B, hipMemcpy(p, d.fam[s.cur], n4, hipMemcpyDeviceToHost)); p += n4;
    PA_HIP(B, hipMemcpy(p, d.E, n4, hipMemcpyDeviceToHost)); p += n4;
    PA_HIP(B, hipMemcpy(p, d.M, n4, hipMemcpyDeviceToHost)); p += n4;
    PA_HIP(B, hipMemcpy(p, d.betas, (size_t)(d.max_steps + 1) * 8, hipMemcpyDeviceToHost));
    p += (size_t)(d.max_steps + 1) * 8;
    PA_HIP(B, hipMemcpy(p, d.records, (size_t)(s.step + 1) * sizeof(pa_obs), hipMemcpyDeviceToHost));
    return PA_OK;
}

pa_status pa_set_state(pa_ctx *ctx, const void *buf, size_t len) {
    if (!ctx || !buf) return fail(nullptr, PA_ERR_ARG, "bad arguments");
    pa_batch *B = &ctx->b;
    if (B->dead) return fail(B, PA_ERR_DEVICE, "handle is unusable after a device error");
    const RunDesc &d = B->desc[0];
    const char *p = (const char *)buf;
    if (len < sizeof(StateHeader)) return fail(B, PA_ERR_STATE, "snapshot too short");
    StateHeader h;
    std::memcpy(&h, p, sizeof h); p += sizeof h;
    if (std::memcmp(h.magic, "PASTATE3", 8) || h.L != d.L || h.R != d.R || h.C != d.C ||
        h.layout != d.layout || h.resample != d.resample || h.max_steps != d.max_steps ||
        h.theta != d.theta || h.update != d.update || h.seed != B->cfg[0].seed)
        return fail(B, PA_ERR_STATE, "snapshot belongs to another configuration");
    if (h.step < 0 || h.step > d.max_steps || h.R_i < 1 || h.R_i > d.C)
        return fail(B, PA_ERR_STATE, "snapshot state is inconsistent");
    if (len != snapshot_bytes(d, h.step, h.R_i)) return fail(B, PA_ERR_STATE, "snapshot size mismatch");
    RunState s;
    std::memcpy(&s, p, sizeof s); p += sizeof s;
    if (s.cur < 0 || s.cur > 1 || s.R_cur != h.R_i || s.step != h.step || s.err != 0 ||
        s.r_parents < 0 || s.r_parents > d.C || !std::isfinite(s.acc_hi) || !std::isfinite(s.acc_lo))
        return fail(B, PA_ERR_STATE, "snapshot state is inconsistent");
    for (int k = 0; k < kBlocks; ++k)
        if (!std::isfinite(s.jk_F[k])) return fail(B, PA_ERR_STATE, "snapshot state is inconsistent");
    // the fields below are derived during a step: nothing of the snapshot's is kept
    s.R_new = s.R_cur;
    s.err_step = 0;
    s.kmin = INT32_MAX;
    s.kmax = -1;
    s.lnq_hi = s.lnq_lo = 0.0;
    s.w_total = 0;
    s.sum_cnt2 = 0;
    s.reduce_done = 0;
    // family labels, energies and magnetisations are checked before anything
    // reaches the device (the energies index the histogram there): labels are
    // beta_0 replica indices in tree order (non-decreasing), E in [-2N, 2N] with
    // E = 2N mod 4, M in [-N, N] with M = N mod 2
    const size_t pop = (size_t)(s.R_cur + 63) / 64 * group_bytes(d);
    const size_t n4 = (size_t)s.R_cur * 4;
    std::vector<int32_t> fam(s.R_cur), E(s.R_cur), M(s.R_cur);
    std::memcpy(fam.data(), p + pop, n4);
    std::memcpy(E.data(), p + pop + n4, n4);
    std::memcpy(M.data(), p + pop + 2 * n4, n4);
    for (int j = 0; j < s.R_cur; ++j) {
        if (fam[j] < 0 || fam[j] >= d.R || (j > 0 && fam[j] < fam[j - 1]))
            return fail(B, PA_ERR_STATE, "snapshot family labels are not in tree order");
        if (E[j] < -2 * d.N || E[j] > 2 * d.N || (E[j] + 2 * d.N) % 4 != 0 || M[j] < -d.N ||
            M[j] > d.N || (M[j] + d.N) % 2 != 0)
            return fail(B, PA_ERR_STATE, "snapshot energies or magnetisations out of range");
    }
    PA_HIP(B, hipStreamSynchronize(B->stream));
    void *dst = d.layout == PA_LAYOUT_MSC64 ? (void *)d.ms[s.cur] : (void *)d.s8[s.cur];
    PA_HIP(B, hipMemcpy(d.st, &s, sizeof s, hipMemcpyHostToDevice));
    PA_HIP(B, hipMemcpy(dst, p, pop, hipMemcpyHostToDevice)); p += pop;
    PA_HIP(B, hipMemcpy(d.fam[s.cur], p, n4, hipMemcpyHostToDevice)); p += 3 * n4;
    PA_HIP(B, hipMemcpy(d.betas, p, (size_t)(d.max_steps + 1) * 8, hipMemcpyHostToDevice));
    std::memcpy(B->betas[0].data(), p, (size_t)(d.max_steps + 1) * 8);
    p += (size_t)(d.max_steps + 1) * 8;
    PA_HIP(B, hipMemcpy(d.records, p, (size_t)(s.step + 1) * sizeof(pa_obs), hipMemcpyHostToDevice));
    // E and M are measured again from the restored spins and must equal the
    // snapshot's: a snapshot whose spins do not fit its energies is rejected
    PA_HIP(B, launch_swap_buffers(B->lc, 0));
    PA_HIP(B, launch_sweeps(B->lc, 1));
    PA_HIP(B, launch_swap_buffers(B->lc, 0));
    PA_HIP(B, hipStreamSynchronize(B->stream));
    std::vector<int32_t> E2(s.R_cur), M2(s.R_cur);
    PA_HIP(B, hipMemcpy(E2.data(), d.E, n4, hipMemcpyDeviceToHost));
    PA_HIP(B, hipMemcpy(M2.data(), d.M, n4, hipMemcpyDeviceToHost));
    if (E2 != E || M2 != M) {
        PA_HIP(B, launch_set_error(B->lc, 0, PA_ERR_STATE));  // no valid run is left
        PA_HIP(B, hipStreamSynchronize(B->stream));
        return fail(B, PA_ERR_STATE, "snapshot energies do not match its spins");
    }
    PA_HIP(B, launch_hist_current(B->lc));  // the next step reads the histogram
    PA_HIP(B, hipStreamSynchronize(B->stream));
    B->host_step[0] = s.step;
    return PA_OK;
}

pa_status pa_overlap(pa_ctx *ctx, double dbeta, double *alpha) {
    if (!ctx || !alpha) return fail(nullptr, PA_ERR_ARG, "bad arguments");
    pa_batch *B = &ctx->b;
    if (!(dbeta >= 0) || !std::isfinite(dbeta)) return fail(B, PA_ERR_ARG, "dbeta must be finite and >= 0");
    PA_HIP(B, launch_hist_current(B->lc));
    PA_HIP(B, launch_overlap(B->lc, 0, dbeta));
    RunState s;
    pa_status e = read_state(B, 0, &s);
    if (e) return e;
    *alpha = s.alpha_out;
    return PA_OK;
}

pa_status pa_adaptive_dbeta(pa_ctx *ctx, double alpha_target, double dbeta_max, double *dbeta) {
    if (!ctx || !dbeta) return fail(nullptr, PA_ERR_ARG, "bad arguments");
    pa_batch *B = &ctx->b;
    if (!(alpha_target > 0 && alpha_target < 1)) return fail(B, PA_ERR_ARG, "alpha_target must be in (0, 1)");
    if (!(dbeta_max > 0) || !std::isfinite(dbeta_max)) return fail(B, PA_ERR_ARG, "dbeta_max must be > 0");
    PA_HIP(B, launch_hist_current(B->lc));
    PA_HIP(B, launch_schedule(B->lc, 0, nullptr, 0.0, alpha_target, dbeta_max, 0, nullptr));
    RunState s;
    pa_status e = read_state(B, 0, &s);
    if (e) return e;
    *dbeta = s.dbeta_out;
    return PA_OK;
}

pa_status pa_profile(pa_ctx *ctx, int32_t enable) {
    if (!ctx) return fail(nullptr, PA_ERR_ARG, "NULL handle");
    pa_batch *B = &ctx->b;
    if (B->dead) return fail(B, PA_ERR_DEVICE, "handle is unusable after a device error");
    PA_HIP(B, hipStreamSynchronize(B->stream));
    if (enable & ~3) return fail(B, PA_ERR_ARG, "enable must be a combination of 1 and 2");
    B->profiling = enable != 0;
    if (B->profiling) B->profiled_steps = 0;
    if (B->lc.count_calls != ((enable & 2) != 0)) {
        B->lc.count_calls = (enable & 2) != 0;  // another sweep kernel: drop the captured graph
        if (B->exec) {
            (void)hipGraphExecDestroy(B->exec);
            (void)hipGraphDestroy(B->graph);
            B->exec = nullptr;
            B->graph = nullptr;
        }
    }
    for (int r = 0; r < B->n; ++r) {
        if (!B->profiling) continue;
        unsigned long long zero[2] = {0, 0};
        PA_HIP(B, hipMemcpy(&B->desc[r].st->philox_calls, zero, sizeof zero, hipMemcpyHostToDevice));
    }
    return PA_OK;
}

pa_status pa_profile_read(pa_ctx *ctx, int32_t *n_steps, double *ms_resample, double *ms_sweep,
                          double *ms_measure, uint64_t *philox_calls, uint64_t *sweep_words,
                          double *ms_copy) {
    if (!ctx) return fail(nullptr, PA_ERR_ARG, "NULL handle");
    pa_batch *B = &ctx->b;
    RunState s;
    pa_status e = read_state(B, 0, &s);
    if (e) return e;
    double t[kProfEvents - 1] = {0, 0, 0, 0};  // counts, copy, sweep, measure
    for (int k = 0; k < B->profiled_steps; ++k) {
        for (int ph = 0; ph < kProfEvents - 1; ++ph) {
            float ms = 0;
            PA_HIP(B, hipEventElapsedTime(&ms, B->events[kProfEvents * k + ph],
                                          B->events[kProfEvents * k + ph + 1]));
            t[ph] += ms;
        }
    }
    if (n_steps) *n_steps = B->profiled_steps;
    if (ms_resample) *ms_resample = t[0] + t[1];
    if (ms_copy) *ms_copy = t[1];
    if (ms_sweep) *ms_sweep = t[2];
    if (ms_measure) *ms_measure = t[3];
    if (philox_calls) *philox_calls = s.philox_calls;
    if (sweep_words) *sweep_words = s.sweep_words;
    return PA_OK;
}

static pa_status set_sweep_launch(pa_batch *B, int32_t L, int32_t threads, int32_t gpb,
                                  int32_t variant) {
    if (B->dead) return fail(B, PA_ERR_DEVICE, "handle is unusable after a device error");
    if (threads < 64 || threads > 1024 || threads % 64) return fail(B, PA_ERR_ARG, "threads must be a multiple of 64 in [64, 1024]");
    if (gpb < 1 || gpb > 8) return fail(B, PA_ERR_ARG, "groups_per_block must be in [1, 8]");
    if (variant < 0 || variant > 2) return fail(B, PA_ERR_ARG, "variant must be 0, 1 or 2");
    if (sweep_lds_bytes(L, gpb) > (size_t)kMaxSweepLds)
        return fail(B, PA_ERR_ARG, "groups_per_block * (L + 2)^2 * 8 bytes exceed the LDS budget");
    for (size_t k = 0; k < B->lc.sweep_classes.size(); ++k) {
        SweepClass &sc = B->lc.sweep_classes[k];
        if (sc.L != L) continue;
        PA_HIP(B, hipStreamSynchronize(B->stream));
        sc.threads = threads;
        sc.gpb = gpb;
        sc.words = variant;
        pa_status e = upload_class_map(B, (int)k);
        if (e) return e;
        PA_HIP(B, hipStreamSynchronize(B->stream));
        B->class_maps.clear();
        if (B->exec) {  // the captured graph holds the old geometry
            (void)hipGraphExecDestroy(B->exec);
            (void)hipGraphDestroy(B->graph);
            B->exec = nullptr;
            B->graph = nullptr;
        }
        return PA_OK;
    }
    return fail(B, PA_ERR_ARG, "no run with this L");
}

static pa_status get_sweep_launch(pa_batch *B, int32_t L, int32_t *threads, int32_t *gpb,
                                  int32_t *variant) {
    for (const SweepClass &sc : B->lc.sweep_classes) {
        if (sc.L != L) continue;
        if (threads) *threads = sc.threads;
        if (gpb) *gpb = sc.gpb;
        if (variant) *variant = sc.words;
        return PA_OK;
    }
    return fail(B, PA_ERR_ARG, "no run with this L");
}

pa_status pa_set_sweep_launch(pa_ctx *ctx, int32_t L, int32_t threads, int32_t groups_per_block,
                              int32_t variant) {
    if (!ctx) return fail(nullptr, PA_ERR_ARG, "NULL handle");
    return set_sweep_launch(&ctx->b, L, threads, groups_per_block, variant);
}

pa_status pa_get_sweep_launch(pa_ctx *ctx, int32_t L, int32_t *threads, int32_t *groups_per_block,
                              int32_t *variant) {
    if (!ctx) return fail(nullptr, PA_ERR_ARG, "NULL handle");
    return get_sweep_launch(&ctx->b, L, threads, groups_per_block, variant);
}

pa_status pa_batch_set_sweep_launch(pa_batch *b, int32_t L, int32_t threads,
                                    int32_t groups_per_block, int32_t variant) {
    if (!b) return fail(nullptr, PA_ERR_ARG, "NULL handle");
    return set_sweep_launch(b, L, threads, groups_per_block, variant);
}

pa_status pa_batch_get_sweep_launch(pa_batch *b, int32_t L, int32_t *threads,
                                    int32_t *groups_per_block, int32_t *variant) {
    if (!b) return fail(nullptr, PA_ERR_ARG, "NULL handle");
    return get_sweep_launch(b, L, threads, groups_per_block, variant);
}

void pa_destroy(pa_ctx *ctx) {
    if (!ctx) return;
    engine_destroy(&ctx->b);
    delete ctx;
}

const char *pa_last_error(const pa_ctx *ctx) {
    if (ctx) return ctx->b.err.c_str();
    return g_last_error.c_str();
}

// ---- batch
pa_status pa_batch_workspace_size(const pa_config *cfgs, int32_t n_runs, size_t *bytes) {
    return workspace_size(cfgs, n_runs, bytes);
}

pa_status pa_batch_create(const pa_config *cfgs, int32_t n_runs, void *ws, size_t bytes,
                          void *stream, pa_batch **out) {
    if (!cfgs || !out || n_runs < 1 || n_runs > 4096) return fail(nullptr, PA_ERR_ARG, "bad arguments");
    *out = nullptr;
    pa_batch *b = new pa_batch();
    pa_status e = engine_create(b, cfgs, n_runs, ws, bytes, stream);
    if (e) {
        g_last_error = b->err;
        engine_destroy(b);
        delete b;
        return e;
    }
    *out = b;
    return PA_OK;
}

pa_status pa_batch_run(pa_batch *b, int32_t n_steps) {
    if (!b) return fail(nullptr, PA_ERR_ARG, "NULL handle");
    return engine_run(b, n_steps);
}

pa_status pa_batch_observables(pa_batch *b, int32_t run, int32_t step, pa_obs *out) {
    if (!b) return fail(nullptr, PA_ERR_ARG, "NULL handle");
    return engine_observables(b, run, step, out);
}

pa_status pa_batch_sync(pa_batch *b) {
    if (!b) return fail(nullptr, PA_ERR_ARG, "NULL handle");
    return engine_sync(b);
}

pa_status pa_overlap_correlation(pa_ctx *ctx, int32_t d_max, double *dev_cq) {
    if (!ctx || !dev_cq) return fail(nullptr, PA_ERR_ARG, "bad arguments");
    pa_batch *B = &ctx->b;
    if (B->dead) return fail(B, PA_ERR_DEVICE, "handle is unusable after a device error");
    RunState s;
    pa_status e = read_state(B, 0, &s);
    if (e) return e;
    if (s.err) return fail(B, s.err, "the run stopped on a device status");
    if (d_max < 1 || d_max >= s.R_cur || d_max > kMaxOverlapDistance)
        return fail(B, PA_ERR_ARG, "d_max outside [1, min(R_i - 1, 65536)]");
    PA_HIP(B, launch_overlap_correlation(B->lc, B->desc[0].N, s.R_cur, d_max, dev_cq));
    return PA_OK;
}

pa_status pa_batch_weighted(pa_batch *b, int32_t first, int32_t count, pa_weighted *dev_out) {
    if (!b) return fail(nullptr, PA_ERR_ARG, "NULL handle");
    if (!dev_out || count < 1 || first < 0) return fail(b, PA_ERR_ARG, "bad arguments");
    if (b->dead) return fail(b, PA_ERR_DEVICE, "handle is unusable after a device error");
    const int last = first + count - 1;
    if (last < first) return fail(b, PA_ERR_ARG, "bad arguments");
    for (int r = 0; r < b->n; ++r) {
        if (b->cfg[r].L != b->cfg[0].L) return fail(b, PA_ERR_ARG, "the runs differ in L");
        if (last > b->host_step[r]) return fail(b, PA_ERR_ARG, "step not queued yet");
    }
    PA_HIP(b, launch_weighted(b->lc, first, count, dev_out));
    return PA_OK;
}

void pa_batch_destroy(pa_batch *b) {
    if (!b) return;
    engine_destroy(b);
    delete b;
}

const char *pa_batch_last_error(const pa_batch *b) {
    if (b) return b->err.c_str();
    return g_last_error.c_str();
}

pa_status pa_features(pa_ctx *ctx, float *dev_feat) {
    if (!ctx || !dev_feat) return fail(nullptr, PA_ERR_ARG, "bad arguments");
    pa_batch *B = &ctx->b;
    if (B->dead) return fail(B, PA_ERR_DEVICE, "handle is unusable after a device error");
    PA_HIP(B, launch_hist_current(B->lc));
    PA_HIP(B, launch_features(B->lc, 0, dev_feat));
    return PA_OK;
}

pa_status pa_learned_dbeta(pa_ctx *ctx, const float *dev_params, double alpha_min,
                           double alpha_target, double dbeta_max, float *dev_feat,
                           double *dbeta, int32_t *accepted) {
    if (!ctx || !dev_params || !dbeta) return fail(nullptr, PA_ERR_ARG, "bad arguments");
    pa_batch *B = &ctx->b;
    if (!(alpha_min > 0 && alpha_min < 1) || !(alpha_target > 0 && alpha_target < 1))
        return fail(B, PA_ERR_ARG, "overlap thresholds must be in (0, 1)");
    if (!(dbeta_max > 0) || !std::isfinite(dbeta_max)) return fail(B, PA_ERR_ARG, "dbeta_max must be > 0");
    PA_HIP(B, launch_hist_current(B->lc));
    PA_HIP(B, launch_schedule(B->lc, 0, dev_params, alpha_min, alpha_target, dbeta_max, 0, dev_feat));
    RunState s;
    pa_status e = read_state(B, 0, &s);
    if (e) return e;
    *dbeta = s.dbeta_out;
    if (accepted) *accepted = s.accepted;
    return PA_OK;
}

static pa_status schedule_step(pa_ctx *ctx, const float *params, double alpha_min,
                               double alpha_target, double beta_final) {
    if (!ctx) return fail(nullptr, PA_ERR_ARG, "NULL handle");
    pa_batch *B = &ctx->b;
    if (B->dead) return fail(B, PA_ERR_DEVICE, "handle is unusable after a device error");
    if (!(alpha_target > 0 && alpha_target < 1)) return fail(B, PA_ERR_ARG, "alpha_target must be in (0, 1)");
    if (params && !(alpha_min > 0 && alpha_min < 1)) return fail(B, PA_ERR_ARG, "alpha_min must be in (0, 1)");
    if (!std::isfinite(beta_final)) return fail(B, PA_ERR_ARG, "beta_final must be finite");
    if (B->host_step[0] >= B->desc[0].max_steps) return fail(B, PA_ERR_DONE, "no room for another step");
    PA_HIP(B, launch_hist_current(B->lc));
    PA_HIP(B, launch_schedule(B->lc, 0, params, alpha_min, alpha_target, beta_final, 1, nullptr));
    return engine_step(B);
}

pa_status pa_anneal_step_adaptive(pa_ctx *ctx, double alpha_target, double beta_final) {
    return schedule_step(ctx, nullptr, 0.5, alpha_target, beta_final);
}

pa_status pa_anneal_step_learned(pa_ctx *ctx, const float *dev_params, double alpha_min,
                                 double alpha_target, double beta_final) {
    if (!dev_params) return fail(ctx ? &ctx->b : nullptr, PA_ERR_ARG, "dev_params is NULL");
    return schedule_step(ctx, dev_params, alpha_min, alpha_target, beta_final);
}

pa_status pa_schedule_log(pa_ctx *ctx, float *dev_feat, float *dev_target, int32_t *accepted,
                          double *alpha, int32_t cap, int32_t *n) {
    if (!ctx || !n || cap < 0) return fail(nullptr, PA_ERR_ARG, "bad arguments");
    pa_batch *B = &ctx->b;
    RunState s;
    pa_status e = read_state(B, 0, &s);
    if (e) return e;
    const RunDesc &d = B->desc[0];
    const int rows = std::min(s.step, cap);
    *n = s.step;
    if (rows <= 0) return PA_OK;
    if (dev_feat)
        PA_HIP(B, hipMemcpyAsync(dev_feat, d.feat_log + PA_MLP_IN, (size_t)rows * PA_MLP_IN * 4,
                                 hipMemcpyDeviceToDevice, B->stream));
    if (dev_target)
        PA_HIP(B, hipMemcpyAsync(dev_target, d.tgt_log + 1, (size_t)rows * 4, hipMemcpyDeviceToDevice,
                                 B->stream));
    PA_HIP(B, hipStreamSynchronize(B->stream));
    if (accepted) PA_HIP(B, hipMemcpy(accepted, d.acc_log + 1, (size_t)rows * 4, hipMemcpyDeviceToHost));
    if (alpha) PA_HIP(B, hipMemcpy(alpha, d.alpha_log + 1, (size_t)rows * 8, hipMemcpyDeviceToHost));
    return PA_OK;
}

pa_status pa_mlp_forward(const float *dev_params, const float *dev_x, int32_t n, float *dev_y,
                         void *stream) {
    if (n < 0 || (n > 0 && (!dev_params || !dev_x || !dev_y))) return fail(nullptr, PA_ERR_ARG, "bad arguments");
    if (n == 0) return PA_OK;
    hipError_t e = launch_mlp_forward(dev_params, dev_x, n, dev_y, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(nullptr, e, "launch_mlp_forward");
    return PA_OK;
}

pa_status pa_mlp_backward(const float *dev_params, const float *dev_x, const float *dev_t,
                          int32_t n, float *dev_grad, float *dev_loss, void *stream) {
    if (n < 1 || !dev_params || !dev_x || !dev_t || !dev_grad) return fail(nullptr, PA_ERR_ARG, "bad arguments");
    hipError_t e = launch_mlp_backward(dev_params, dev_x, dev_t, n, dev_grad, dev_loss, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(nullptr, e, "launch_mlp_backward");
    return PA_OK;
}

pa_status pa_mlp_train_step(float *dev_params, float *dev_adam, const float *dev_x,
                            const float *dev_t, int32_t n, float lr, int32_t t, float *dev_loss,
                            void *stream) {
    if (n < 1 || t < 1 || !dev_params || !dev_adam || !dev_x || !dev_t || !(lr > 0))
        return fail(nullptr, PA_ERR_ARG, "bad arguments");
    hipError_t e = launch_adam_step(dev_params, dev_adam, dev_x, dev_t, n, lr, t, dev_loss, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(nullptr, e, "launch_adam_step");
    return PA_OK;
}

pa_status pa_philox4x32_10(uint32_t key0, uint32_t key1, const uint32_t *dev_ctr, int64_t n,
                           uint32_t *dev_out, void *stream) {
    if (n < 0 || (n > 0 && (!dev_ctr || !dev_out))) return fail(nullptr, PA_ERR_ARG, "bad arguments");
    if (n == 0) return PA_OK;
    hipError_t e = launch_philox(key0, key1, dev_ctr, n, dev_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(nullptr, e, "launch_philox");
    return PA_OK;
}

}  // extern "C"

// Message of a failing handle-free call made outside this file (pa_last_error(NULL)).
void pa::set_last_error(const char *msg) { g_last_error = msg; }
