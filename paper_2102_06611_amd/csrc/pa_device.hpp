// Device-side building blocks of libpa: run descriptors, Philox4x32-10,
// double-double arithmetic and the exact integer decisions of the method.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pa.h"

namespace pa {

// Device buffers as global-address-space pointers: loads and stores through
// them are global (not flat) accesses, which the compiler knows cannot alias
// LDS, so it can keep several in flight around LDS traffic.
template <class T>
using gptr = T __attribute__((address_space(1))) *;
template <class T>
__device__ __forceinline__ gptr<T> global(T *p) {
    return (gptr<T>)p;
}
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));  // 16-byte copies

constexpr int kLanes = 64;        // replicas per group = bits per multispin word
constexpr int kSlotBlock = 1024;  // replica slots per block of the per-slot kernels
constexpr int kMaxL = 128;
constexpr int kBlocks = 100;      // blocks of the blocking / jackknife analysis
// dynamic LDS available to one sweep block (the static part is 4 KiB)
constexpr int kMaxSweepLds = 152 * 1024;

// Stream tags in the top nibble of the fourth Philox counter word.
constexpr uint32_t kTagSweep = 0x10000000u;
constexpr uint32_t kTagInit = 0x20000000u;
constexpr uint32_t kTagResample = 0x30000000u;
constexpr uint32_t kTagMulti = 0x40000000u;
constexpr uint32_t kTagPoisson = 0x50000000u;

// Dynamic per-run state, written only by kernels once a run exists.
struct RunState {
    int32_t step;      // record index of the current population (-1 before init)
    int32_t cur;       // ping-pong buffer holding the current population
    int32_t R_cur;     // R_i of the current population
    int32_t R_new;     // size of the population being built in buffer cur ^ 1
    int32_t err;       // sticky pa_status
    int32_t err_step;  // step that raised err
    int32_t kmin, kmax;          // occupied energy levels of the current population
    double acc_hi, acc_lo;       // running -beta F (double-double)
    double lnq_hi, lnq_lo;       // ln Q of the step in progress (committed by k_reduce)
    uint64_t t4, t8;             // thresholds at beta_i (2^32: beta_i = 0), by update rule
    uint64_t w_total;            // multinomial: total quantised weight
    int64_t sum_cnt2;            // sum of squared copy counts of the step
    double dbeta_out, alpha_out; // results of the overlap / adaptive kernels
    int32_t r_parents;           // R_{i-1} of the last resampling (parents of cnt[])
    int32_t accepted;            // learned proposal passed the overlap guard
    float mlp_y;                 // last MLP output of the learned step
    int32_t reserved;            // 0
    unsigned long long philox_calls;  // Philox calls counted by the sweeps (profiling)
    unsigned long long sweep_words;   // 64-replica words updated by the sweeps
    double s_hi, s_lo;                // S = sum_l n_l w_l of the step in progress (Eq. Q)
    int32_t kmin_step;                // level origin of wlev / zlev of the step in progress
    int32_t reduce_done;              // k_reduce blocks finished in the step (0 between steps)
    // free-energy jackknife: for block k of the n_F = min(kBlocks, R) blocks,
    // sum over the steps so far of ln Q^(k) - ln Q (Q without block k of the
    // parents, Eq. Q), so that sample k of -beta F is -beta F + jk_F[k]
    double jk_F[kBlocks];
};

// Static description of one run plus pointers into its slice of the workspace.
struct RunDesc {
    int32_t L, N, R, C, G, K;  // side, sites, nominal R, capacity, groups, levels
    int32_t theta, resample, layout, max_steps;
    int32_t update;            // PA_UPDATE_*
    uint32_t key0, key1;
    int32_t nblk;              // ceil(C / kSlotBlock)
    int32_t pad;
    uint64_t *ms[2];           // multispin [G][N]
    int8_t *s8[2];             // int8 [G][N][64]
    int32_t *E, *M;            // [C] energies / magnetisations of the current population
    int32_t *fam[2];           // [C] family labels
    int32_t *hist;             // [K] energy histogram, level k <-> E = -2N + 4k
    uint64_t *zlev;            // [K] per-level decision integers (from kmin)
    double *wlev;              // [2K] per-level Boltzmann factor (double-double, from kmin)
    double *plev;              // [6K] Poisson, per level: tau_hat, m, k with e^-tau_hat = m 2^-k
    int32_t *cnt;              // [C] copy counts of the last resampling
    int32_t *off;              // [C + 1] exclusive offsets of the children
    int32_t *par;              // [C] parent of each child slot of the last resampling
    uint64_t *cum;             // [C] multinomial cumulative quantised weights
    uint64_t *send;            // [C / 64] cum at the last parent of each stretch of 64
    uint64_t *e8;              // [C / 8] cum at the last parent of each eighth of a stretch
    int64_t *part;             // [nblk * 4] per-block partial sums
    int64_t *blk;              // [kBlocks * 4] blocking sums of E, E^2, |M|, M^2 (zero between steps)
    double *partd;             // [nblk * 2] per-block FP partials
    double *betas;             // [max_steps + 1]
    pa_obs *records;           // [max_steps + 1]
    RunState *st;
    int8_t *stage;             // [64 * N] staging for host transfers
    float *feat;               // [64] features of the learned step
    float *feat_log;           // [(max_steps + 1) * 35] features entering each step
    float *tgt_log;            // [max_steps + 1] log(dbeta* sigma_E) of each step
    int32_t *acc_log;          // [max_steps + 1] learned proposal taken
    double *alpha_log;         // [max_steps + 1] overlap of the step taken
    double *jkw;               // [kBlocks] parents' weight sum per free-energy jackknife block
};

// Maps a flat block index of a batched launch to (run, item within the run).
struct WorkMap {
    int32_t n;                 // number of runs covered
    const int32_t *blk_off;    // [n + 1] first block of each covered run
    const int32_t *run_id;     // [n] run index of each entry
};

// Workgroups are handed to the 8 XCDs round-robin (block b runs on XCD b % 8).
// This permutation gives each XCD a contiguous range of blocks, so that
// neighbouring work items (which share input data) meet in the same L2.
constexpr int kXcds = 8;
__device__ inline int xcd_swizzle(int b, int total) {
    const int per = total / kXcds;
    if (b >= per * kXcds) return b;  // the ragged tail keeps its order
    return (b % kXcds) * per + b / kXcds;
}

__device__ inline int map_block(const WorkMap &m, int b, int *item) {
    int lo = 0, hi = m.n - 1;
    while (lo < hi) {  // last entry with blk_off <= b
        int mid = (lo + hi + 1) >> 1;
        if (m.blk_off[mid] <= b) lo = mid; else hi = mid - 1;
    }
    *item = b - m.blk_off[lo];
    return m.run_id[lo];
}

// ---------------------------------------------------------------- Philox4x32-10
// Salmon, Moraes, Dror & Shaw (SC'11): ten rounds; each multiplies counter
// words 0 and 2 by fixed odd constants, swaps the halves and mixes in the
// round key; the key advances by a Weyl sequence between rounds.
struct U4 { uint32_t x, y, z, w; };

// Three-input bitwise functions in one gfx950 instruction (v_bitop3_b32).  The
// 8-bit table is the function applied to the operand patterns 0xF0, 0xCC, 0xAA.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);  // 0xF0 ^ 0xCC ^ 0xAA
}

// In every use the counter word c3 (the stream tag) is the same across a
// wavefront: the first round XORs it with the key first (no three-input XOR
// with two scalar operands, one of which would need a move).
__device__ __forceinline__ U4 philox(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1,
                                     uint32_t c2, uint32_t c3) {
    {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ (c3 ^ k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
#pragma unroll
    for (int r = 1; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// ---------------------------------------------------------------- double-double
// Error-free transformations (Knuth two-sum, FMA two-product) and the usual
// double-double operations; relative error ~2^-104 per operation.  The
// library is built with -ffp-contract=off so these stay exact.
struct dd { double hi, lo; };

__device__ __forceinline__ dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return dd{s, e};
}
__device__ __forceinline__ dd quick_two_sum(double a, double b) {
    double s = a + b;
    return dd{s, b - (s - a)};
}
__device__ __forceinline__ dd two_prod(double a, double b) {
    double p = a * b;
    return dd{p, __builtin_fma(a, b, -p)};
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd dd_neg(dd a) { return dd{-a.hi, -a.lo}; }
__device__ __forceinline__ dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }
__device__ __forceinline__ dd dd_mul(dd a, dd b) {
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return quick_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ dd dd_mul_d(dd a, double b) {
    dd p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return quick_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ dd dd_div(dd a, dd b) {
    double q1 = a.hi / b.hi;
    dd r = dd_sub(a, dd_mul_d(b, q1));
    double q2 = r.hi / b.hi;
    r = dd_sub(r, dd_mul_d(b, q2));
    double q3 = r.hi / b.hi;
    return dd_add(quick_two_sum(q1, q2), dd{q3, 0.0});
}
__device__ __forceinline__ dd dd_div_d(dd a, double b) { return dd_div(a, dd{b, 0.0}); }
__device__ __forceinline__ dd dd_ldexp(dd a, int e) { return dd{ldexp(a.hi, e), ldexp(a.lo, e)}; }

// ln 2 to ~107 bits.
__device__ __forceinline__ dd dd_ln2() { return dd{6.93147180559945286227e-01, 2.31904681384629955842e-17}; }

// 1/n for n = 1..14 as double-double (hi + lo, |lo| <= ulp(hi)/2): the Taylor
// terms multiply by these instead of dividing.
__device__ constexpr dd kRecip[14] = {
    {0x1.0000000000000p+0, 0x0.0p+0},  // 1/1
    {0x1.0000000000000p-1, 0x0.0p+0},  // 1/2
    {0x1.5555555555555p-2, 0x1.5555555555555p-56},  // 1/3
    {0x1.0000000000000p-2, 0x0.0p+0},  // 1/4
    {0x1.999999999999ap-3, -0x1.999999999999ap-57},  // 1/5
    {0x1.5555555555555p-3, 0x1.5555555555555p-57},  // 1/6
    {0x1.2492492492492p-3, 0x1.2492492492492p-57},  // 1/7
    {0x1.0000000000000p-3, 0x0.0p+0},  // 1/8
    {0x1.c71c71c71c71cp-4, 0x1.c71c71c71c71cp-58},  // 1/9
    {0x1.999999999999ap-4, -0x1.999999999999ap-58},  // 1/10
    {0x1.745d1745d1746p-4, -0x1.745d1745d1746p-59},  // 1/11
    {0x1.5555555555555p-4, 0x1.5555555555555p-58},  // 1/12
    {0x1.3b13b13b13b14p-4, -0x1.3b13b13b13b14p-58},  // 1/13
    {0x1.2492492492492p-4, 0x1.2492492492492p-58},  // 1/14
};

// exp(-x) = m 2^-k for x >= 0 given in double-double (m in [0.7, 1.42]).
// Range reduction x = k ln 2 + r, |r| <= ln 2 / 2; then r / 16 and a Taylor
// series of 14 terms, squared four times.  Relative error of m below 2^-98
// plus k 2^-106 from the reduction.
__device__ inline dd dd_exp_neg_split(dd x, int *kexp) {
    double k = rint(x.hi / 6.93147180559945286227e-01);
    dd r = dd_sub(x, dd_mul_d(dd_ln2(), k));  // e^-x = 2^-k e^-r
    dd rs = dd_ldexp(dd_neg(r), -4);          // -r / 16
    dd term = dd{1.0, 0.0};
    dd sum = dd{1.0, 0.0};
#pragma unroll
    for (int n = 1; n <= 14; ++n) {
        term = dd_mul(dd_mul(term, rs), kRecip[n - 1]);  // term_n = term_{n-1} (-r/16) / n
        sum = dd_add(sum, term);
    }
    for (int s = 0; s < 4; ++s) sum = dd_mul(sum, sum);
    *kexp = (int)k;
    return sum;
}
// exp(-x) for x >= 0 given in double-double.  Returns false (and sets *out to
// 0) when exp(-x) < 2^-1000, i.e. far below every decision boundary here.
__device__ inline bool dd_exp_neg(dd x, dd *out) {
    if (x.hi > 690.0) {
        *out = dd{0.0, 0.0};
        return false;
    }
    int k;
    const dd m = dd_exp_neg_split(x, &k);
    *out = dd_ldexp(m, -k);
    return true;
}

// ln(x) for x > 0 in double-double: one Newton step y + x e^-y - 1 from the
// binary64 logarithm.
__device__ inline dd dd_log(dd x) {
    double y0 = log(x.hi);
    dd e;
    if (y0 >= 0) {
        dd_exp_neg(dd{y0, 0.0}, &e);  // e^-y0
    } else {
        dd t;
        dd_exp_neg(dd{-y0, 0.0}, &t);  // e^y0, then e^-y0 = 1 / e^y0
        e = dd_div(dd{1.0, 0.0}, t);
    }
    dd corr = dd_sub(dd_mul(x, e), dd{1.0, 0.0});
    return dd_add(dd{y0, 0.0}, corr);
}

// floor of a non-negative double-double below 2^62, plus the distance of x to
// the nearest integer (0 when x is an integer).
__device__ inline uint64_t dd_floor(dd x, double *gap) {
    double fh = floor(x.hi);
    double f;
    if (fh == x.hi) {
        f = fh + floor(x.lo);  // x.hi integral: floor(hi + lo) = hi + floor(lo)
    } else {
        f = fh;  // |lo| < half an ulp of hi: hi + lo cannot cross an integer
    }
    dd frac = dd_add(dd{x.hi - f, 0.0}, dd{x.lo, 0.0});
    double fr = frac.hi + frac.lo;
    *gap = fmin(fr, 1.0 - fr);
    return (uint64_t)f;
}

// Relative margin below which a decision is reported as undecidable: the
// double-double pipelines here are accurate to better than 2^-90, so a value
// x whose nearest integer lies within x 2^-86 cannot be rounded safely.
__device__ constexpr double kDecisionMargin = 0x1p-86;

// ceil(x) for x = a transcendental non-integer value known to ~2^-90.
__device__ inline uint64_t dd_ceil_decided(dd x, bool *ambiguous) {
    double gap;
    uint64_t f = dd_floor(x, &gap);
    if (gap < x.hi * kDecisionMargin) *ambiguous = true;
    return f + 1;
}
__device__ inline uint64_t dd_floor_decided(dd x, bool *ambiguous) {
    double gap;
    uint64_t f = dd_floor(x, &gap);
    if (gap < x.hi * kDecisionMargin) *ambiguous = true;
    return f;
}

// Metropolis threshold ceil(2^32 exp(-beta dE)) for beta >= 0, dE in {4, 8};
// 2^32 means "always accept".  beta = 0 is the only exact case.
__device__ inline uint64_t metropolis_threshold(double beta, int dE, bool *ambiguous) {
    if (beta == 0.0) return 1ull << 32;
    dd p;
    if (!dd_exp_neg(dd{beta * dE, 0.0}, &p)) return 1;  // 0 < p < 2^-1000
    return dd_ceil_decided(dd_ldexp(p, 32), ambiguous);
}

__device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

// Wavefront reductions (64 lanes).
__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace pa
