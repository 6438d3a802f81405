// The self-adaptive temperature step of a caller's population of energies
// with no device allocation: the energy histogram lives in this file's
// scratch array.  For callers that cannot allocate device memory (HIP graph
// capture, tight serving loops, harnesses that forbid allocation).
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <mutex>

#include "pa.h"
#include "pa_device.hpp"
#include "pa_internal.hpp"
#include "pa_search.hpp"

namespace pa {
namespace {

// scratch = int32 histogram of up to kNaLevels energy levels (level k <-> E =
// -2N + 4k, N = L^2 <= 128^2), then the occupied level range and a flag for
// energies that are not energies of an L x L torus.
constexpr int kNaLevels = kMaxL * kMaxL + 1;
constexpr int kNaHist = (kNaLevels + 63) / 64 * 64;
constexpr int kNaKmin = kNaHist, kNaKmax = kNaHist + 1, kNaBad = kNaHist + 2;
constexpr int kNaInts = kNaHist + 64;

static __device__ __align__(256) int32_t scratch[kNaInts];

// Clears the histogram of K levels, the range and the flag (a fill kernel, so
// that the call can be captured in a graph).
__global__ void __launch_bounds__(256) k_na_clear(int32_t *s, int K) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < K) s[k] = 0;
    if (k == 0) {
        s[kNaKmin] = INT_MAX;
        s[kNaKmax] = -1;
        s[kNaBad] = 0;
    }
}

// Histogram of E[0..n): an energy outside [-2N, 2N] or not -2N mod 4 sets the
// flag and is not counted.
__global__ void __launch_bounds__(256) k_na_hist(const int32_t *E, int n, int N, int32_t *s) {
    int lo = INT_MAX, hi = -1, bad = 0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        const int64_t x = (int64_t)E[j] + 2 * (int64_t)N;
        if (x < 0 || x > 4 * (int64_t)N || (x & 3)) {
            bad = 1;
            continue;
        }
        const int k = (int)(x >> 2);
        atomicAdd(&s[k], 1);
        lo = min(lo, k);
        hi = max(hi, k);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o, 64));
        hi = max(hi, __shfl_xor(hi, o, 64));
        bad |= __shfl_xor(bad, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (hi >= 0) {
            atomicMin(&s[kNaKmin], lo);
            atomicMax(&s[kNaKmax], hi);
        }
        if (bad) atomicOr(&s[kNaBad], 1);
    }
}

// out[0] = largest step in (0, dmax] with overlap >= alpha_target, out[1] its
// overlap (search_dbeta over the histogram, as for a run's population); NaN
// for both when an energy was rejected.
__global__ void __launch_bounds__(256) k_na_search(const int32_t *s, int n, double alpha_target,
                                                   double dmax, double *out) {
    if (s[kNaBad]) {
        if (threadIdx.x == 0) out[0] = out[1] = __builtin_nan("");
        return;
    }
    RunDesc rd{};
    rd.hist = const_cast<int32_t *>(s);
    const int kmin = s[kNaKmin], nlev = s[kNaKmax] - s[kNaKmin] + 1;
    double alo;
    const double d = search_dbeta(rd, kmin, nlev, n, dmax, alpha_target, &alo);
    if (threadIdx.x == 0) {
        out[0] = d;
        out[1] = alo;
    }
}

// The address of this device's copy of scratch, looked up once per device.
constexpr int kNaMaxDevices = 64;
std::mutex g_na_mutex;
int32_t *g_na_ptr[kNaMaxDevices] = {};

hipError_t na_scratch(int32_t **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNaMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> guard(g_na_mutex);
    if (!g_na_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_na_ptr[dev] = static_cast<int32_t *>(p);
    }
    *out = g_na_ptr[dev];
    return hipSuccess;
}

pa_status na_fail(pa_status s, const char *msg) {
    set_last_error(msg);
    return s;
}

}  // namespace
}  // namespace pa

extern "C" pa_status pa_adaptive_dbeta_noalloc(const int32_t *dev_E, int32_t n, int32_t L,
                                               double alpha_target, double dbeta_max,
                                               double *dev_out, void *stream) {
    using namespace pa;
    if (!dev_E || !dev_out || n < 1) return na_fail(PA_ERR_ARG, "bad arguments");
    if (L < 4 || L > kMaxL || (L & 1))
        return na_fail(PA_ERR_ARG, "L must be even and in [4, 128] (the scratch histogram holds "
                                   "128^2 + 1 energy levels)");
    if (!(alpha_target > 0 && alpha_target < 1))
        return na_fail(PA_ERR_ARG, "alpha_target must be in (0, 1)");
    if (!(dbeta_max > 0) || !std::isfinite(dbeta_max))
        return na_fail(PA_ERR_ARG, "dbeta_max must be finite and > 0");
    int32_t *s = nullptr;
    hipError_t e = na_scratch(&s);
    if (e != hipSuccess) return na_fail(PA_ERR_DEVICE, hipGetErrorString(e));
    const hipStream_t st = (hipStream_t)stream;
    const int N = L * L, K = N + 1;
    hipLaunchKernelGGL(k_na_clear, dim3((K + 255) / 256), dim3(256), 0, st, s, K);
    const int blocks = (int)std::min<int64_t>(((int64_t)n + 1023) / 1024, 1024);
    hipLaunchKernelGGL(k_na_hist, dim3(blocks), dim3(256), 0, st, dev_E, n, N, s);
    hipLaunchKernelGGL(k_na_search, dim3(1), dim3(256), 0, st, s, n, alpha_target, dbeta_max,
                       dev_out);
    e = hipGetLastError();
    if (e != hipSuccess) return na_fail(PA_ERR_DEVICE, hipGetErrorString(e));
    return PA_OK;
}
