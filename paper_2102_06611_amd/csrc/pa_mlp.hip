// Learned temperature steps: energy-histogram features of the population, a
// 35 -> 64 -> 64 -> 1 perceptron (tanh hidden layers, FP32) with hand-written
// forward, backward and Adam kernels, and the overlap-guarded proposal.
//
// Layout of the parameter vector: W1[64][35], b1[64], W2[64][64], b2[64],
// w3[64], b3.  A wavefront evaluates one row at a time with lane j = hidden
// unit j, so each lane keeps its rows of W1 and W2 in registers.
#include <climits>

#include "pa_block.hpp"
#include "pa_device.hpp"
#include "pa_internal.hpp"
#include "pa_search.hpp"

namespace pa {

constexpr int kIn = PA_MLP_IN, kH = PA_MLP_HIDDEN;
constexpr int oW1 = 0, oB1 = kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kH;
static_assert(oB3 + 1 == PA_MLP_PARAMS, "parameter layout");

struct MlpLane {
    float w1[kIn], w2[kH], b1, b2, w3, b3;
};

__device__ __forceinline__ void mlp_load(const float *P, int j, MlpLane &m) {
#pragma unroll
    for (int k = 0; k < kIn; ++k) m.w1[k] = P[oW1 + j * kIn + k];
#pragma unroll
    for (int k = 0; k < kH; ++k) m.w2[k] = P[oW2 + j * kH + k];
    m.b1 = P[oB1 + j];
    m.b2 = P[oB2 + j];
    m.w3 = P[oW3 + j];
    m.b3 = P[oB3];
}

// Lane k's value of v in every lane (k uniform: one v_readlane into a scalar
// register instead of a round trip through LDS).
__device__ __forceinline__ float lane_value(float v, int k) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

// One row through the network; xk = feature k held by lane k (k < 35).
// Returns y in every lane; h1, h2 = this lane's hidden activations.
__device__ __forceinline__ float mlp_row(const MlpLane &m, float xk, float *h1o, float *h2o) {
    float a = m.b1;
#pragma unroll
    for (int k = 0; k < kIn; ++k) a = fmaf(m.w1[k], lane_value(xk, k), a);
    const float h1 = tanhf(a);
    float b = m.b2;
#pragma unroll
    for (int k = 0; k < kH; ++k) b = fmaf(m.w2[k], lane_value(h1, k), b);
    const float h2 = tanhf(b);
    float y = m.w3 * h2;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) y += __shfl_xor(y, o, 64);
    *h1o = h1;
    *h2o = h2;
    return y + m.b3;
}

__global__ void __launch_bounds__(256) k_mlp_forward(const float *P, const float *X, int n,
                                                     float *Y) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    MlpLane m;
    mlp_load(P, lane, m);
    for (int row = wave; row < n; row += nwaves) {
        float xk = lane < kIn ? X[(size_t)row * kIn + lane] : 0.0f;
        float h1, h2;
        float y = mlp_row(m, xk, &h1, &h2);
        if (lane == 0) Y[row] = y;
    }
}

// Gradient of (1/n) sum (y - t)^2 by backpropagation, one block of
// kGradWaves wavefronts (two per SIMD, so one hides the other's dependent
// FMA chains); per-wave partial gradients are summed in wave order in LDS
// (deterministic).  mode 0 writes grad and loss; mode 1 applies one Adam step.
constexpr int kGradWaves = 8;
__global__ void __launch_bounds__(kGradWaves * 64) k_mlp_grad(float *P, const float *X, const float *T, int n,
                                                  float *grad, float *loss, float *adam, float lr,
                                                  int t, int mode) {
    __shared__ float W2s[kH * kH];
    __shared__ float G[PA_MLP_PARAMS];
    __shared__ float Ls[kGradWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = threadIdx.x; k < kH * kH; k += blockDim.x) W2s[k] = P[oW2 + k];
    for (int k = threadIdx.x; k < PA_MLP_PARAMS; k += blockDim.x) G[k] = 0.0f;
    MlpLane m;
    mlp_load(P, lane, m);
    __syncthreads();
    float gw1[kIn], gw2[kH];
#pragma unroll
    for (int k = 0; k < kIn; ++k) gw1[k] = 0.0f;
#pragma unroll
    for (int k = 0; k < kH; ++k) gw2[k] = 0.0f;
    float gb1 = 0, gb2 = 0, gw3 = 0, gb3 = 0, lsum = 0;
    const float inv_n = 1.0f / (float)n;
    for (int row = wave; row < n; row += kGradWaves) {
        const float xk = lane < kIn ? X[(size_t)row * kIn + lane] : 0.0f;
        float h1, h2;
        const float y = mlp_row(m, xk, &h1, &h2);
        const float r = y - T[row];
        const float g = 2.0f * r * inv_n;
        lsum += r * r * inv_n;
        gb3 += g;
        gw3 += g * h2;
        const float d2 = g * m.w3 * (1.0f - h2 * h2);
        gb2 += d2;
#pragma unroll
        for (int k = 0; k < kH; ++k) gw2[k] = fmaf(d2, lane_value(h1, k), gw2[k]);
        float s = 0.0f;  // sum_j d2_j W2[j][lane]
#pragma unroll
        for (int j = 0; j < kH; ++j) s = fmaf(lane_value(d2, j), W2s[j * kH + lane], s);
        const float d1 = s * (1.0f - h1 * h1);
        gb1 += d1;
#pragma unroll
        for (int k = 0; k < kIn; ++k) gw1[k] = fmaf(d1, lane_value(xk, k), gw1[k]);
    }
    for (int w = 0; w < kGradWaves; ++w) {
        if (wave == w) {
#pragma unroll
            for (int k = 0; k < kIn; ++k) G[oW1 + lane * kIn + k] += gw1[k];
#pragma unroll
            for (int k = 0; k < kH; ++k) G[oW2 + lane * kH + k] += gw2[k];
            G[oB1 + lane] += gb1;
            G[oB2 + lane] += gb2;
            G[oW3 + lane] += gw3;
            if (lane == 0) {
                G[oB3] += gb3;
                Ls[w] = lsum;
            }
        }
        __syncthreads();
    }
    if (mode == 0) {
        for (int k = threadIdx.x; k < PA_MLP_PARAMS; k += blockDim.x) grad[k] = G[k];
    } else {
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
        for (int k = threadIdx.x; k < PA_MLP_PARAMS; k += blockDim.x) {
            const float gk = G[k];
            const float mk = b1 * adam[k] + (1.0f - b1) * gk;
            const float vk = b2 * adam[PA_MLP_PARAMS + k] + (1.0f - b2) * gk * gk;
            adam[k] = mk;
            adam[PA_MLP_PARAMS + k] = vk;
            P[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
        }
    }
    if (threadIdx.x == 0 && loss) {
        float l = 0.0f;
        for (int w = 0; w < kGradWaves; ++w) l += Ls[w];
        loss[0] = l;
    }
}

// Features of the current population from its energy histogram: 32 bins of
// z = (E - <E>) / sigma_E over [-4, 4) normalised to sum 1, then beta_i,
// <E> / N and Var(E) / N.  Executed by one block; result in feat[0..34] and
// sigma_E in feat[35].
__device__ void features_block(const RunDesc &rd, float *feat) {
    __shared__ int64_t sh[32];
    __shared__ int bins[32];
    __shared__ double mom[2];
    RunState *st = rd.st;
    const int kmin = st->kmin, nlev = st->kmax - st->kmin + 1, R = st->R_cur, N = rd.N;
    int64_t s1 = 0, s2 = 0;
    for (int l = threadIdx.x; l < nlev; l += blockDim.x) {
        const int64_t n = rd.hist[kmin + l];
        const int64_t e = -2 * (int64_t)N + 4 * (int64_t)(kmin + l);
        s1 += n * e;
        s2 += n * e * e;
    }
    int64_t S[2] = {s1, s2};
    block_sum_i64v(S, sh);
    const int64_t S1 = S[0], S2 = S[1];
    if (threadIdx.x < 32) bins[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        const __int128 var = (__int128)R * S2 - (__int128)S1 * S1;  // R^2 Var(E)
        mom[0] = (double)S1 / R;
        mom[1] = (double)var / ((double)R * R);
    }
    __syncthreads();
    const double mean = mom[0], var = mom[1], sd = sqrt(var);
    for (int l = threadIdx.x; l < nlev; l += blockDim.x) {
        const int n = rd.hist[kmin + l];
        if (!n) continue;
        const double e = -2.0 * N + 4.0 * (kmin + l);
        const double z = sd > 0 ? (e - mean) / sd : 0.0;
        const int b = (int)floor((z + 4.0) * 4.0);
        if (b >= 0 && b < 32) atomicAdd(&bins[b], n);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int b = 0; b < 32; ++b) tot += bins[b];
        for (int b = 0; b < 32; ++b) feat[b] = tot ? (float)bins[b] / (float)tot : 0.0f;
        feat[32] = (float)rd.betas[st->step];
        feat[33] = (float)(mean / N);
        feat[34] = (float)(var / N);
        feat[35] = (float)sd;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(256) k_features(const RunDesc *runs, int r, float *out) {
    const RunDesc &rd = runs[r];
    features_block(rd, rd.feat);
    for (int k = threadIdx.x; k < kIn; k += blockDim.x) out[k] = rd.feat[k];
}

// Temperature choice on the device (one block of 256 threads), from the
// histogram of the current population at beta_{i-1}:
//   adaptive: dbeta* = largest step in (0, dmax] with overlap >= alpha_target
//             (search_dbeta; the self-adaptive schedule),
//   learned:  y = MLP(features), proposal exp(y) / sigma_E clipped to dmax,
//             taken iff its overlap >= alpha_min; only a rejected proposal
//             pays for the search of dbeta*.
// mode 0 answers a query (st->dbeta_out etc.); mode 1 also writes beta_i =
// beta_{i-1} + dbeta and the schedule log of step i, with dmax = beta_final -
// beta_{i-1}, and ends the run (PA_ERR_DONE) once beta_final is reached.  The
// logged training target log(dbeta* sigma_E) is NaN on steps where the search
// did not run.
__global__ void __launch_bounds__(256) k_schedule(const RunDesc *runs, int r, const float *P,
                                                  double alpha_min, double alpha_target,
                                                  double dmax_or_final, int mode,
                                                  float *feat_out) {
    const RunDesc &rd = runs[r];
    RunState *st = rd.st;
    __shared__ double shd[32];
    __shared__ float ysh;
    __shared__ int stop;
    if (st->err) return;
    const int i = st->step + 1;
    const double b0 = rd.betas[st->step];
    double dmax = dmax_or_final;
    if (mode == 1) {
        if (threadIdx.x == 0) {
            stop = 0;
            if (i > rd.max_steps || !(b0 < dmax_or_final)) {
                st->err = PA_ERR_DONE;
                st->err_step = i;
                stop = 1;
            }
        }
        __syncthreads();
        if (stop) return;
        dmax = dmax_or_final - b0;
    }
    features_block(rd, rd.feat);
    const double sd = rd.feat[35];
    const int kmin = st->kmin, nlev = st->kmax - st->kmin + 1, R = st->R_cur;
    double take = 0.0, a_take = 1.0, target = __builtin_nan("");
    int acc = 0;
    if (P) {
        if (threadIdx.x < 64) {  // wave 0 evaluates the network
            MlpLane m;
            mlp_load(P, threadIdx.x, m);
            const float xk = threadIdx.x < kIn ? rd.feat[threadIdx.x] : 0.0f;
            float h1, h2;
            const float y = mlp_row(m, xk, &h1, &h2);
            if (threadIdx.x == 0) ysh = y;
        }
        __syncthreads();
        double prop = sd > 0 ? exp((double)ysh) / sd : dmax;
        if (!(prop > 0)) prop = dmax;
        prop = fmin(prop, dmax);
        const double ap = overlap_block(rd, kmin, nlev, R, prop, shd);
        if (ap >= alpha_min) {
            take = prop;
            a_take = ap;
            acc = 1;
        }
    }
    if (!acc) {  // block-uniform: ap is read from shared memory by every thread
        double alo;
        take = search_dbeta(rd, kmin, nlev, R, dmax, alpha_target, &alo);
        a_take = alo;
        if (sd > 0) target = log(take * sd);
    }
    if (feat_out)
        for (int k = threadIdx.x; k < kIn; k += blockDim.x) feat_out[k] = rd.feat[k];
    if (threadIdx.x != 0) return;
    st->dbeta_out = take;
    st->alpha_out = a_take;
    st->accepted = acc;
    st->mlp_y = P ? ysh : 0.0f;
    if (mode != 1) return;
    double b1 = b0 + take;
    if (take >= dmax) b1 = dmax_or_final;          // land exactly on beta_final
    if (!(b1 > b0)) b1 = b0 + dmax * 0x1p-40;      // never stall
    rd.betas[i] = b1;
    for (int k = 0; k < kIn; ++k) rd.feat_log[(size_t)i * kIn + k] = rd.feat[k];
    rd.tgt_log[i] = (float)target;
    rd.acc_log[i] = acc;
    rd.alpha_log[i] = a_take;
}

hipError_t launch_features(const LaunchCtx &c, int r, float *feat) {
    hipLaunchKernelGGL(k_features, dim3(1), dim3(256), 0, c.stream, c.runs, r, feat);
    return hipGetLastError();
}

hipError_t launch_schedule(const LaunchCtx &c, int r, const float *params, double alpha_min,
                           double alpha_target, double dmax_or_final, int mode, float *feat_out) {
    hipLaunchKernelGGL(k_schedule, dim3(1), dim3(256), 0, c.stream, c.runs, r, params, alpha_min,
                       alpha_target, dmax_or_final, mode, feat_out);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *params, const float *x, int n, float *y,
                              hipStream_t stream) {
    int blocks = (n + 3) / 4;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_mlp_forward, dim3(blocks), dim3(256), 0, stream, params, x, n, y);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const float *params, const float *x, const float *t, int n,
                               float *grad, float *loss, hipStream_t stream) {
    hipLaunchKernelGGL(k_mlp_grad, dim3(1), dim3(kGradWaves * 64), 0, stream, const_cast<float *>(params), x,
                       t, n, grad, loss, (float *)nullptr, 0.0f, 0, 0);
    return hipGetLastError();
}

hipError_t launch_adam_step(float *params, float *adam, const float *x, const float *t, int n,
                            float lr, int step, float *loss, hipStream_t stream) {
    hipLaunchKernelGGL(k_mlp_grad, dim3(1), dim3(kGradWaves * 64), 0, stream, params, x, t, n,
                       (float *)nullptr, loss, adam, lr, step, 1);
    return hipGetLastError();
}

}  // namespace pa
