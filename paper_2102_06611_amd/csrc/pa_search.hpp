// Self-adaptive temperature steps (Sec. "Algorithm"): the histogram overlap
// at many trial steps at once and the bracket search for the largest step
// that keeps the overlap at a target, over an energy histogram on the device.
#pragma once

#include "pa_block.hpp"
#include "pa_device.hpp"

namespace pa {

// Overlap alpha(d) = (1/R) sum_l n_l min(1, R w_l(d) / S(d)), w_l(d) =
// exp(-4 d l), S(d) = sum_l n_l w_l(d), at kSearch trial steps d[0..kSearch)
// at once: wave v takes the trials v, v + 4, ...; lane j runs over the levels
// l = j, j + 64, ..., stepping w_l by the factor exp(-256 d) (two exp per
// lane and trial instead of one per level; the schedule search needs no
// last-ulp agreement with pa_overlap).  Needs a 256-thread block; alpha[] is
// shared.
constexpr int kSearch = 16;
constexpr int kPerWave = kSearch / 4;

__device__ inline void overlap_trials(const RunDesc &rd, int kmin, int nlev, int R, const double *d,
                               double *alpha) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double S[kPerWave], A[kPerWave], w0[kPerWave], q[kPerWave], w[kPerWave];
#pragma unroll
    for (int c = 0; c < kPerWave; ++c) {
        const double dc = d[wave + 4 * c];
        w0[c] = exp(-4.0 * dc * lane);
        q[c] = exp(-256.0 * dc);
        S[c] = A[c] = 0.0;
        w[c] = w0[c];
    }
    for (int l = lane; l < nlev; l += 64) {
        const double n = rd.hist[kmin + l];
#pragma unroll
        for (int c = 0; c < kPerWave; ++c) {
            S[c] += n * w[c];
            w[c] *= q[c];
        }
    }
#pragma unroll
    for (int c = 0; c < kPerWave; ++c) {
        S[c] = (double)R / wave_sum_f64(S[c]);
        w[c] = w0[c];
    }
    for (int l = lane; l < nlev; l += 64) {
        const double n = rd.hist[kmin + l];
#pragma unroll
        for (int c = 0; c < kPerWave; ++c) {
            A[c] += n * fmin(1.0, w[c] * S[c]);
            w[c] *= q[c];
        }
    }
#pragma unroll
    for (int c = 0; c < kPerWave; ++c) {
        const double a = wave_sum_f64(A[c]);
        if (lane == 0) alpha[wave + 4 * c] = a / R;
    }
}

// Largest step in (0, dmax] whose overlap is >= alpha_target, by a
// (kSearch + 1)-ary bracket search: lo always has overlap >= target (alpha(0)
// = 1) and hi below it; each round evaluates kSearch equally spaced interior
// points and keeps the last one at or above the target together with its right
// neighbour, so 12 rounds narrow the bracket to dmax / 17^12 (< dmax 2^-49).
// Returns lo; *alo receives its overlap.  Every thread returns the same values.
__device__ inline double search_dbeta(const RunDesc &rd, int kmin, int nlev, int R, double dmax,
                               double alpha_target, double *alo) {
    __shared__ double d[2][kSearch], al[2][kSearch];
    __shared__ double shd[32];
    double lo = 0.0, a_lo = 1.0, hi = dmax;
    const double a_hi = overlap_block(rd, kmin, nlev, R, hi, shd);
    if (a_hi >= alpha_target) {
        *alo = a_hi;
        return hi;
    }
    for (int it = 0; it < 12; ++it) {
        const int b = it & 1;  // alternate buffers: one barrier per round
        const double step = (hi - lo) / (kSearch + 1);
        if (threadIdx.x < kSearch) d[b][threadIdx.x] = lo + step * (threadIdx.x + 1);
        __syncthreads();
        overlap_trials(rd, kmin, nlev, R, d[b], al[b]);
        __syncthreads();
        int k = -1;
        for (int c = 0; c < kSearch; ++c)
            if (al[b][c] >= alpha_target) k = c;
        const double nlo = k >= 0 ? d[b][k] : lo;
        const double nhi = k + 1 < kSearch ? d[b][k + 1] : hi;
        if (k >= 0) a_lo = al[b][k];
        lo = nlo;
        hi = nhi;
    }
    *alo = a_lo;
    return lo;
}

}  // namespace pa
