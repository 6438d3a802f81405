// Block-level reductions and scans shared by the kernels of libpa.
#pragma once

#include "pa_device.hpp"

namespace pa {

// Block-wide exclusive scan of one int64 per thread (blockDim.x <= 1024).
__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t *sh, int64_t *total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int w = 0; w < nw; ++w) {
            int64_t t = sh[w];
            sh[w] = run;
            run += t;
        }
        sh[16] = run;
    }
    __syncthreads();
    int64_t res = x - v + sh[wave];
    *total = sh[16];
    __syncthreads();
    return res;
}

// Block-wide sum of int64 values in a fixed order (deterministic).
__device__ inline int64_t block_sum_i64(int64_t v, int64_t *sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    v = wave_sum_i64(v);
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    int64_t t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < nw; ++w) t += sh[w];
    __syncthreads();
    return t;  // valid in thread 0
}
// K sums at once (one pass of barriers): v[k] <- block sum of v[k], valid in
// thread 0; sh holds K values per wavefront of the block.
template <int K>
__device__ inline void block_sum_i64v(int64_t (&v)[K], int64_t *sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum_i64(v[k]);
    if (lane == 0)
        for (int k = 0; k < K; ++k) sh[wave * K + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < K; ++k) {
            int64_t t = 0;
            for (int w = 0; w < nw; ++w) t += sh[w * K + k];
            v[k] = t;
        }
    }
    __syncthreads();
}
__device__ inline double block_sum_f64(double v, double *sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    v = wave_sum_f64(v);
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < nw; ++w) t += sh[w];
    __syncthreads();
    return t;
}

// alpha(dbeta) = (1/R) sum_l n_l min(1, R w_l / S) over the histogram of the
// current population (binary64; the schedule generator needs no exact ties).
__device__ inline double overlap_block(const RunDesc &rd, int kmin, int nlev, int R, double dbeta,
                                double *shd) {
    double s = 0.0;
    for (int l = threadIdx.x; l < nlev; l += blockDim.x) {
        int n = rd.hist[kmin + l];
        if (n) s += n * exp(-4.0 * dbeta * l);
    }
    __shared__ double S_sh;
    double S = block_sum_f64(s, shd);
    if (threadIdx.x == 0) S_sh = S;
    __syncthreads();
    S = S_sh;
    double a = 0.0;
    for (int l = threadIdx.x; l < nlev; l += blockDim.x) {
        int n = rd.hist[kmin + l];
        if (n) a += n * fmin(1.0, R * exp(-4.0 * dbeta * l) / S);
    }
    double A = block_sum_f64(a, shd);
    __shared__ double A_sh;
    if (threadIdx.x == 0) A_sh = A / R;
    __syncthreads();
    return A_sh;
}

}  // namespace pa
