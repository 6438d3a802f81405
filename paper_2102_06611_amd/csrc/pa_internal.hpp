// Host-side launch descriptions shared by the engine and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "pa_device.hpp"

namespace pa {

constexpr int kMaxOverlapDistance = 65536;  // largest d of pa_overlap_correlation

struct MapInfo {
    WorkMap map;  // device arrays
    int total;    // blocks in the launch
};

struct SweepClass {
    int L, N;
    WorkMap map;
    int total;
    bool has_msc, has_int8;
    int threads;  // block size of k_sweep for this lattice size
    int gpb;      // 64-replica groups per block
    int words = 0;  // words each thread updates at once: 0 = default (1), 1 or 2
};

struct LaunchCtx {
    const RunDesc *runs;  // device array [n_runs]
    int n_runs;
    hipStream_t stream;
    MapInfo slots;   // per run: nblk blocks of kSlotBlock slots
    MapInfo groups;  // per run: G blocks, one per 64-replica group
    std::vector<SweepClass> sweep_classes;  // one launch per distinct L
    // with several classes: one stream per class (default priority), forked
    // from and joined back to `stream` by events, so the classes' sweeps run
    // side by side (also inside a captured graph)
    std::vector<hipStream_t> class_streams;
    std::vector<hipEvent_t> class_events;  // [0] fork, [1 + k] class k done
    bool any_nearest, any_multi, any_poisson;
    bool any_msc, any_int8;  // layouts present in the batch
    bool any_update[2];      // spin-update rules present in the batch (PA_UPDATE_*)
    bool count_calls = false;  // sweeps count the Philox calls the words need (pa_profile 3)
    int max_nblk = 1;          // most slot blocks of a multinomial run (LDS of its draws)
    int max_L = 0;             // largest lattice side of the batch
};

void set_last_error(const char *msg);  // for pa_last_error(NULL)
hipError_t configure_kernels();
size_t sweep_lds_bytes(int L, int gpb);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t stream);
hipError_t launch_init(const LaunchCtx &c);
hipError_t launch_sweeps(const LaunchCtx &c, int init);
hipError_t launch_reduce(const LaunchCtx &c);
hipError_t launch_step(const LaunchCtx &c);
hipError_t launch_counts(const LaunchCtx &c);  // reweighting, copy counts, offsets
hipError_t launch_weighted(const LaunchCtx &c, int first, int count, pa_weighted *out);
hipError_t launch_overlap_correlation(const LaunchCtx &c, int N, int R, int d_max, double *cq);
hipError_t launch_copy(const LaunchCtx &c);    // copy / compaction
hipError_t launch_resample(const LaunchCtx &c);
hipError_t launch_hist_current(const LaunchCtx &c);
hipError_t launch_overlap(const LaunchCtx &c, int r, double dbeta);
hipError_t launch_set_beta(const LaunchCtx &c, int r, int idx, double beta);
hipError_t launch_swap_buffers(const LaunchCtx &c, int r);
hipError_t launch_set_error(const LaunchCtx &c, int r, int status);
hipError_t launch_unpack_group(const LaunchCtx &c, int r, int g, int N);
hipError_t launch_pack_group(const LaunchCtx &c, int r, int g, int buf, int n_valid, int N);
hipError_t launch_adopt_begin(const LaunchCtx &c, int r, int R_i);
hipError_t launch_adopt_end(const LaunchCtx &c, int r, int step, double acc);
hipError_t launch_philox(uint32_t k0, uint32_t k1, const uint32_t *ctr, int64_t n, uint32_t *out,
                         hipStream_t stream);
hipError_t launch_features(const LaunchCtx &c, int r, float *feat);
hipError_t launch_schedule(const LaunchCtx &c, int r, const float *params, double alpha_min,
                           double alpha_target, double dmax_or_final, int mode, float *feat_out);
hipError_t launch_mlp_forward(const float *params, const float *x, int n, float *y,
                              hipStream_t stream);
hipError_t launch_mlp_backward(const float *params, const float *x, const float *t, int n,
                               float *grad, float *loss, hipStream_t stream);
hipError_t launch_adam_step(float *params, float *adam, const float *x, const float *t, int n,
                            float lr, int step, float *loss, hipStream_t stream);

}  // namespace pa
