// HIP kernels of one population-annealing temperature step, batched over
// independent runs (a single run is a batch of one).
//
// Step i (Sec. "Algorithm", steps 2-4), with the population entering the step
// in buffer `cur` and the new one built in buffer `cur ^ 1`:
//   k_norm         Metropolis thresholds for beta_i; Q_i of Eq. (Q) over the
//                  energy histogram; per-level decision integers for the copy
//                  counts (Eq. taus / resampling-factors)
//   k_counts_* / k_multi_*   copy counts r_j and per-block partial sums
//   k_offsets      exclusive prefix sum of r_j (tree order of the children), R_i
//   k_gather_*     children <- parents: spins and family labels
//   k_sweep        theta checkerboard Metropolis sweeps in LDS + E, M
//   k_reduce       population sums, family statistics, next energy histogram;
//                  its last block writes record i and makes the new population current
#include <algorithm>
#include <climits>
#include <type_traits>

#include "pa_block.hpp"
#include "pa_device.hpp"
#include "pa_internal.hpp"

namespace pa {

// ------------------------------------------------------------------ helpers

// 4 int8 spins (+1 = 0x01, -1 = 0xFF) -> 4 bits, bit = 1 for +1.  Bit 7 of each
// byte is moved to the top nibble by one multiply (no carries cross into it).
__device__ __forceinline__ uint32_t spins_to_nibble(uint32_t d) {
    uint32_t neg = (d >> 7) & 0x01010101u;
    uint32_t dn = (neg * 0x10204080u) >> 28;
    return ~dn & 0xFu;
}
// Inverse of spins_to_nibble.
__device__ __forceinline__ uint32_t nibble_to_spins(uint32_t up4) {
    uint32_t dn = ~up4 & 0xFu;
    uint32_t spread = (dn & 1u) | ((dn & 2u) << 7) | ((dn & 4u) << 14) | ((dn & 8u) << 21);
    return 0x01010101u | (spread * 0xFEu);
}
__device__ __forceinline__ uint32_t pack16(uint4 v) {
    return spins_to_nibble(v.x) | (spins_to_nibble(v.y) << 4) | (spins_to_nibble(v.z) << 8) |
           (spins_to_nibble(v.w) << 12);
}
__device__ __forceinline__ uint4 unpack16(uint32_t b) {
    return uint4{nibble_to_spins(b & 0xF), nibble_to_spins((b >> 4) & 0xF),
                 nibble_to_spins((b >> 8) & 0xF), nibble_to_spins((b >> 12) & 0xF)};
}

__device__ __forceinline__ uint64_t lane_mask(int n_valid) {
    if (n_valid >= 64) return ~0ull;
    if (n_valid <= 0) return 0ull;
    return (1ull << n_valid) - 1ull;
}

// ------------------------------------------------------------------ init

// Simple sampling at beta_0 = 0 (Sec. "Algorithm", step 1): spin lane of group
// g at `site` is bit lane of x0 | x1 << 32 of Philox(site, g, 0, INIT).
__global__ void k_init_population(const RunDesc *runs, WorkMap map) {
    int g;
    const RunDesc &rd = runs[map_block(map, blockIdx.x, &g)];
    if (g >= rd.G) return;
    const uint64_t valid = lane_mask(rd.R - g * kLanes);
    for (int site = threadIdx.x; site < rd.N; site += blockDim.x) {
        U4 x = philox(rd.key0, rd.key1, (uint32_t)site, (uint32_t)g, 0u, kTagInit);
        uint64_t bits = (((uint64_t)x.y << 32) | x.x) & valid;
        size_t w = (size_t)g * rd.N + site;
        if (rd.layout == PA_LAYOUT_MSC64) {
            rd.ms[0][w] = bits;
        } else {
            uint4 *dst = reinterpret_cast<uint4 *>(rd.s8[0] + w * kLanes);
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[q] = unpack16((uint32_t)(bits >> (16 * q)) & 0xFFFFu);
        }
    }
    if (threadIdx.x < kLanes) {
        int c = g * kLanes + threadIdx.x;
        if (c < rd.C) rd.fam[0][c] = c < rd.R ? c : 0;
    }
}

// ------------------------------------------------------------------ histogram

// Histogram of the energies of slots [j0, j1): level k = (E + 2N) / 4 <-> E.
// The block first finds its own level range; when it spans at most kLdsBins
// levels the counts are gathered in LDS and only occupied levels touch global
// memory, otherwise each slot adds to the global histogram directly.
constexpr int kLdsBins = 4096;

// lev[m]: levels of the block's slots held by this thread (-1: none)
template <int M>
__device__ void block_histogram(const RunDesc &rd, RunState *st, const int (&lev)[M]) {
    __shared__ int32_t bins[kLdsBins];
    __shared__ int32_t rng[2];
    int kmin = INT_MAX, kmax = -1;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        if (lev[m] >= 0) {
            kmin = min(kmin, lev[m]);
            kmax = max(kmax, lev[m]);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        kmin = min(kmin, __shfl_xor(kmin, o, 64));
        kmax = max(kmax, __shfl_xor(kmax, o, 64));
    }
    if (threadIdx.x == 0) {
        rng[0] = INT_MAX;
        rng[1] = -1;
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&rng[0], kmin);
        atomicMax(&rng[1], kmax);
    }
    __syncthreads();
    const int lo = rng[0], hi = rng[1];
    if (hi < lo) return;  // empty range (no slots in this block)
    if (threadIdx.x == 0) {
        atomicMin(&st->kmin, lo);
        atomicMax(&st->kmax, hi);
    }
    const int span = hi - lo + 1;
    if (span > kLdsBins) {
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (lev[m] >= 0) atomicAdd(&rd.hist[lev[m]], 1);
        return;
    }
    for (int k = threadIdx.x; k < span; k += blockDim.x) bins[k] = 0;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < M; ++m)
        if (lev[m] >= 0) atomicAdd(&bins[lev[m] - lo], 1);
    __syncthreads();
    for (int k = threadIdx.x; k < span; k += blockDim.x)
        if (bins[k]) atomicAdd(&rd.hist[lo + k], bins[k]);
}

// Clear the histogram and rebuild it from the current population (after a
// population was adopted from the host, and for the overlap / feature queries).
__global__ void k_hist_clear(const RunDesc *runs) {
    const RunDesc &rd = runs[blockIdx.x];
    if (threadIdx.x == 0) {
        rd.st->kmin = INT_MAX;
        rd.st->kmax = -1;
    }
    for (int k = threadIdx.x; k < rd.K; k += blockDim.x) rd.hist[k] = 0;
}

__global__ void __launch_bounds__(256) k_hist(const RunDesc *runs, WorkMap map) {
    int b;
    const RunDesc &rd = runs[map_block(map, blockIdx.x, &b)];
    RunState *st = rd.st;
    const int Rc = st->R_cur, j1 = min((b + 1) * kSlotBlock, Rc);
    int lev[kSlotBlock / 256];
#pragma unroll
    for (int m = 0; m < kSlotBlock / 256; ++m) {
        const int j = b * kSlotBlock + m * 256 + (int)threadIdx.x;
        lev[m] = j < j1 ? (rd.E[j] + 2 * rd.N) >> 2 : -1;
    }
    block_histogram(rd, st, lev);
}

// ------------------------------------------------------------------ normalisation

// One block per run, first kernel of step i.  The population entering the
// step is the current one; its energy histogram n_l (levels kmin + l) was
// built by the previous step's reduction.  With dB = beta_i - beta_{i-1}
// (exact, double-double) and w_l = exp(-4 dB l) the Boltzmann factor of level
// kmin + l relative to the lowest occupied energy E_min:
//   S = sum_l n_l w_l,   ln Q_i = -dB E_min + ln(S / R_{i-1})          (Eq. Q,
//                        the logarithm taken by k_offsets, see log_q)
//   nearest:     Z_l = ceil(2^32 R w_l / S) = ceil(2^32 tau_hat)      (Eq. taus)
//   multinomial: q_l = floor(2^40 w_l)
//   Poisson:     lambda_l = R w_l / S = tau_hat and e^{-lambda_l} = m 2^-e,
//                double-double (plev[6l .. 6l+4]); an occupied level with
//                lambda_l > kPoissonMaxMean fails with PA_ERR_NUMERIC
// Z_l and q_l are the exact integers of the real-valued definitions: they are
// computed in double-double and a value within the error margin of an integer
// boundary aborts the run with PA_ERR_NUMERIC.  dB = 0 or a single occupied
// level make every w_l = 1 and S = R_{i-1} exactly; those use integer math.
// Also: the Metropolis thresholds t4 = ceil(2^32 e^{-4 beta_i}), t8 =
// ceil(2^32 e^{-8 beta_i}) (heatbath: floor(2^32 / (1 + e^{4 beta_i})) and
// floor(2^32 / (1 + e^{8 beta_i}))) and the end-of-schedule check.
constexpr double kPoissonMaxMean = 65536.0;  // largest supported tau_hat
constexpr int kPoissonMax = 1 << 18;          // > kPoissonMaxMean + 40 sqrt(kPoissonMaxMean)
constexpr double kPoissonMargin = 0x1p-8;     // in units of U

__device__ void norm_run(const RunDesc &rd) {
    RunState *st = rd.st;
    __shared__ double sh_hi[4], sh_lo[4];
    __shared__ int amb_any, ok;
    const int i = st->step + 1;
    if (threadIdx.x == 0) {
        ok = st->err == 0;
        amb_any = 0;
        if (ok && i > rd.max_steps) {
            st->err = PA_ERR_DONE;
            st->err_step = i;
            ok = 0;
        }
        if (ok) {
            const double b0 = rd.betas[i - 1], b1 = rd.betas[i];
            if (!(b1 >= b0) || !(b1 <= 1e300)) {
                st->err = PA_ERR_ARG;
                st->err_step = i;
                ok = 0;
            }
        }
        st->sum_cnt2 = 0;
    }
    __syncthreads();
    if (!ok) return;
    const int Rp = st->R_cur, kmin = st->kmin, kmax = st->kmax;
    const int nlev = kmax - kmin + 1;
    const double b1 = rd.betas[i];
    const dd db = two_sum(b1, -rd.betas[i - 1]);
    const bool exact = (db.hi == 0.0) || (nlev == 1);
    // One double-double exponential per thread, all in the same code path:
    // thread 0 (whose level weight is 1) takes e^{-4 beta_i} for the
    // thresholds, thread t > 0 its first level weight w_t = e^{-4 dbeta t}.
    dd e{1.0, 0.0};
    bool e_ok = true;
    if (threadIdx.x == 0 ? b1 != 0.0 : !exact)
        e_ok = dd_exp_neg(threadIdx.x == 0 ? dd{4.0 * b1, 0.0} : dd_mul_d(db, 4.0 * threadIdx.x), &e);
    dd w = threadIdx.x == 0 ? dd{1.0, 0.0} : e;
    if (threadIdx.x == 0) {
        if (b1 == 0.0) {
            st->t4 = st->t8 = 1ull << 32;  // heatbath: every flip has probability 1/2
        } else if (rd.update == PA_UPDATE_HEATBATH) {
            // T'_dE = floor(2^32 q / (1 + q)), q = e^{-beta dE}, dE = 4, 8: the
            // dE > 0 classes flip iff u <= T', the dE < 0 classes iff ~u >= T'
            bool amb = false;
            if (!e_ok) {
                st->t4 = st->t8 = 0;  // q < 2^-1000
            } else {
                const dd q8 = dd_mul(e, e);
                const dd p4 = dd_div(e, dd_add(dd{1.0, 0.0}, e));
                const dd p8 = dd_div(q8, dd_add(dd{1.0, 0.0}, q8));
                st->t4 = dd_floor_decided(dd_ldexp(p4, 32), &amb);
                st->t8 = p8.hi < 0x1p-990 ? 0 : dd_floor_decided(dd_ldexp(p8, 32), &amb);
            }
            if (amb) atomicOr(&amb_any, 1);
        } else {
            bool amb = false;
            if (!e_ok) {
                st->t4 = st->t8 = 1;  // 0 < p < 2^-1000
            } else {
                const dd p8 = dd_mul(e, e);  // e^{-8 beta} = (e^{-4 beta})^2
                st->t4 = dd_ceil_decided(dd_ldexp(e, 32), &amb);
                st->t8 = p8.hi < 0x1p-990 ? 1 : dd_ceil_decided(dd_ldexp(p8, 32), &amb);
            }
            if (amb) atomicOr(&amb_any, 1);
        }
    }
    // Levels beyond the first blockDim: repeated multiplication by
    // e^{-4 dbeta blockDim} = w_1 w_{blockDim-1} (at most nlev / blockDim
    // double-double products; relative error far below the decision margin).
    dd stride{1.0, 0.0};
    if (!exact && nlev > (int)blockDim.x) {
        if (threadIdx.x == 1 || threadIdx.x == blockDim.x - 1) {
            sh_hi[threadIdx.x == 1 ? 0 : 1] = w.hi;
            sh_lo[threadIdx.x == 1 ? 0 : 1] = w.lo;
        }
        __syncthreads();
        stride = dd_mul(dd{sh_hi[0], sh_lo[0]}, dd{sh_hi[1], sh_lo[1]});
        __syncthreads();
    }
    dd part{0.0, 0.0};
    for (int l = threadIdx.x; l < nlev; l += blockDim.x) {
        rd.wlev[2 * l] = w.hi;
        rd.wlev[2 * l + 1] = w.lo;
        int n = rd.hist[kmin + l];
        if (n) part = dd_add(part, dd_mul_d(w, (double)n));
        if (!exact) w = dd_mul(w, stride);
    }
    // S: a butterfly within each wavefront (the double-double sum is
    // commutative, so every lane ends with the same value), then the four
    // wavefronts' sums in a fixed order
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        part = dd_add(part, dd{__shfl_xor(part.hi, o, 64), __shfl_xor(part.lo, o, 64)});
    if ((threadIdx.x & 63) == 0) {
        sh_hi[threadIdx.x >> 6] = part.hi;
        sh_lo[threadIdx.x >> 6] = part.lo;
    }
    __syncthreads();
    const dd S = dd_add(dd_add(dd{sh_hi[0], sh_lo[0]}, dd{sh_hi[1], sh_lo[1]}),
                        dd_add(dd{sh_hi[2], sh_lo[2]}, dd{sh_hi[3], sh_lo[3]}));
    if (threadIdx.x == 0) {  // ln Q_i itself is taken by k_offsets (log_q)
        st->s_hi = S.hi;
        st->s_lo = S.lo;
        st->kmin_step = kmin;  // k_offsets resets st->kmin while its jackknife blocks run
    }
    bool amb = false;
    const double R2_32 = ldexp((double)rd.R, 32);
    for (int l = threadIdx.x; l < nlev; l += blockDim.x) {
        uint64_t z = 0;
        if (rd.resample == PA_RESAMPLE_POISSON) {
            const dd w{rd.wlev[2 * l], rd.wlev[2 * l + 1]};
            dd lam{0.0, 0.0}, m{1.0, 0.0};  // w_l = 0: tau_hat < 2^-900, no copies
            int e = 0;
            if (exact)
                lam = dd_div_d(dd{(double)rd.R, 0.0}, (double)Rp);
            else if (w.hi != 0.0)
                lam = dd_div(dd_mul_d(w, (double)rd.R), S);
            if (lam.hi != 0.0) m = dd_exp_neg_split(lam, &e);
            if (!(lam.hi <= kPoissonMaxMean) && rd.hist[kmin + l] != 0) amb = true;
            double *p = rd.plev + 6 * l;
            p[0] = lam.hi;
            p[1] = lam.lo;
            p[2] = m.hi;
            p[3] = m.lo;
            p[4] = (double)e;
        } else if (rd.resample == PA_RESAMPLE_MULTINOMIAL) {
            if (exact || l == 0) {
                z = 1ull << 40;
            } else {
                dd w{rd.wlev[2 * l], rd.wlev[2 * l + 1]};
                z = (w.hi == 0.0) ? 0ull : dd_floor_decided(dd_ldexp(w, 40), &amb);
            }
        } else {
            if (exact) {  // tau_hat = R / R_{i-1} exactly
                unsigned __int128 num = ((unsigned __int128)(uint64_t)rd.R << 32) + (uint64_t)(Rp - 1);
                z = (uint64_t)(num / (uint64_t)Rp);
            } else {
                dd w{rd.wlev[2 * l], rd.wlev[2 * l + 1]};
                if (w.hi == 0.0) {
                    z = 1;  // 0 < tau_hat < 2^-900
                } else {
                    z = dd_ceil_decided(dd_div(dd_mul_d(w, R2_32), S), &amb);
                }
            }
        }
        rd.zlev[l] = z;
    }
    if (amb) atomicOr(&amb_any, 1);
    __syncthreads();
    if (threadIdx.x == 0 && amb_any) {
        st->err = PA_ERR_NUMERIC;
        st->err_step = i;
    }
}

__global__ void __launch_bounds__(256) k_norm(const RunDesc *runs) { norm_run(runs[blockIdx.x]); }

// ------------------------------------------------------------------ free-energy jackknife

// ln Q_i = -dB E_min + ln(S / R_{i-1}) (Eq. Q) from the S of k_norm, taken
// off k_norm's critical path by one thread of a k_offsets block; dB = 0 gives
// exactly 0, and so does a single occupied level (S = R_{i-1}).
__device__ void log_q(const RunDesc &rd) {
    RunState *st = rd.st;
    const int i = st->step + 1;
    const dd db = two_sum(rd.betas[i], -rd.betas[i - 1]);
    dd lnq{0.0, 0.0};
    if (db.hi != 0.0) {
        const double e_min = -2.0 * rd.N + 4.0 * st->kmin_step;
        lnq = dd_add(dd_mul_d(db, -e_min), dd_log(dd_div_d(dd{st->s_hi, st->s_lo}, (double)st->R_cur)));
    }
    st->lnq_hi = lnq.hi;
    st->lnq_lo = lnq.lo;
}


// Sec. "Conclusions" (last guideline) with Eq. free-emergy-estimator: sample k
// of the jackknife of -beta F leaves block k of every parent population out
// of every Q.  Block k of the population entering step i is the slot range
// [floor(k R_{i-1} / n_F), floor((k + 1) R_{i-1} / n_F)) of the tree-ordered
// population, n_F = min(kBlocks, R) for the whole run.  One workgroup per
// (run, block) -- extra blocks of the k_offsets launch -- sums the parents'
// weights w = e^{-dbeta (E - E_min)} of its block (the level weights of
// k_norm) in a fixed order; the record turns the sums into ln Q^(k) - ln Q =
// ln(1 - W_k / S) - ln(1 - B_k / R_{i-1}).
__device__ void jack_weights(const RunDesc &rd, int k) {
    RunState *st = rd.st;
    const int nF = min(kBlocks, rd.R);
    if (st->err || k >= nF) return;
    if (k == 0 && threadIdx.x == 0) log_q(rd);
    __shared__ double shd[16];
    const int Rp = st->R_cur, kmin = st->kmin_step;
    const int lo = (int)((int64_t)k * Rp / nF), hi = (int)((int64_t)(k + 1) * Rp / nF);
    double s = 0.0;
    for (int j = lo + (int)threadIdx.x; j < hi; j += blockDim.x) {
        const int l = ((rd.E[j] + 2 * rd.N) >> 2) - kmin;
        s += rd.wlev[2 * l];
    }
    const double t = block_sum_f64(s, shd);
    if (threadIdx.x == 0) rd.jkw[k] = t;
}

// ------------------------------------------------------------------ copy counts
// Per-slot kernels write one partial sum per block of kSlotBlock slots into
// part[b * 8 + k]; the next kernel derives block bases and totals by summing
// those partials itself (no cross-block fences).


// Nearest-integer rule (Eq. resampling-factors, strict "<"): with
// Z = ceil(2^32 tau_hat) and the parent's uniform u32 (RESAMPLE stream),
// r_j = floor(tau_hat) + [u32 < 2^32 frac(tau_hat)] = ceil((Z - u32) / 2^32).
// PA_RESAMPLE_NONE runs get r_j = 1.
__global__ void __launch_bounds__(256) k_counts_nearest(const RunDesc *runs, WorkMap map) {
    int b;
    const RunDesc &rd = runs[map_block(map, blockIdx.x, &b)];
    RunState *st = rd.st;
    if (st->err || rd.resample == PA_RESAMPLE_MULTINOMIAL || rd.resample == PA_RESAMPLE_POISSON)
        return;
    __shared__ int64_t sh[32];
    const int Rp = st->R_cur, i = st->step + 1, kmin = st->kmin;
    const int j = b * kSlotBlock + 4 * (int)threadIdx.x;
    int64_t s = 0, s2 = 0;
    if (j < Rp) {
        uint32_t u[4] = {0, 0, 0, 0};
        if (rd.resample == PA_RESAMPLE_NEAREST) {
            U4 x = philox(rd.key0, rd.key1, (uint32_t)(j >> 2), (uint32_t)i, 0u, kTagResample);
            u[0] = x.x; u[1] = x.y; u[2] = x.z; u[3] = x.w;
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int jj = j + m;
            if (jj < Rp) {
                int c = 1;
                if (rd.resample == PA_RESAMPLE_NEAREST) {
                    const uint64_t z = rd.zlev[((rd.E[jj] + 2 * rd.N) >> 2) - kmin];
                    c = (int)((z + 0xFFFFFFFFull - u[m]) >> 32);
                }
                rd.cnt[jj] = c;
                s += c;
                s2 += (int64_t)c * c;
            }
        }
    }
    int64_t v[2] = {s, s2};
    block_sum_i64v(v, sh);
    if (threadIdx.x == 0) {
        rd.part[b * 8 + 0] = v[0];
        rd.part[b * 8 + 1] = v[1];
    }
}

// Poisson rule (Sec. "Algorithm", fluctuating population): r_j is the
// smallest k with U_j < 2^64 F(k), F the CDF of Poisson(lambda) with lambda =
// tau_hat of the parent's level and U_j its 64-bit uniform (POISSON stream:
// counter j/2, words 0-1 for even j, 2-3 for odd j, low word first).  F(k) =
// e^-lambda sum_{m<=k} lambda^m / m! in double-double: relative error below
// 2^-80 for lambda <= kPoissonMaxMean (from lambda's own error, ~lambda 2^-98,
// and k 2^-104 over the recursion), i.e. below 2^-16 in units of U; a
// comparison closer than kPoissonMargin, or no decision by kPoissonMax, fails
// with PA_ERR_NUMERIC.
// F(k) = G 2^-e: G starts as the mantissa of e^-lambda and is scaled down by
// 2^512 whenever it passes 2^512, so that neither a tiny e^-lambda nor the
// growing terms leave the binary64 range.
__device__ inline int poisson_invert(dd lam, dd G, int e, uint64_t U, bool *amb) {
    const dd Ud = dd_add(dd{(double)(U >> 32) * 4294967296.0, 0.0}, dd{(double)(uint32_t)U, 0.0});
    dd term = G;
    for (int k = 0; k < kPoissonMax; ++k) {
        const dd gap = dd_sub(dd_ldexp(G, 64 - e), Ud);
        if (gap.hi > kPoissonMargin) return k;  // U < 2^64 F(k)
        if (gap.hi > -kPoissonMargin) {
            *amb = true;
            return k;
        }
        term = dd_div_d(dd_mul(term, lam), (double)(k + 1));
        G = dd_add(G, term);
        if (G.hi > 0x1p512) {
            G = dd_ldexp(G, -512);
            term = dd_ldexp(term, -512);
            e -= 512;
        }
    }
    *amb = true;
    return kPoissonMax;
}

// The same inversion in binary64 first.  For lambda <= kPoissonFastMean and
// k <= kPoissonFastMax the computed 2^64 F(k) has a relative error below
// (lambda + 4k + 10) 2^-53 < 2^-39 (lambda's own rounding and e^-lambda, two
// roundings per step of the term recursion, one per addition of the sum),
// i.e. below 2^25 in units of U, and U converts to binary64 within 2^11; a
// comparison is taken only with a gap above 2^36.  Returns -1 when it cannot
// decide (then the double-double inversion runs).
constexpr double kPoissonFastMean = 600.0;
constexpr int kPoissonFastMax = 2000;
__device__ inline int poisson_invert_fast(double lam, uint64_t U) {
    if (!(lam <= kPoissonFastMean)) return -1;
    const double Ud = (double)U, gap_min = 0x1p36;
    double term = exp(-lam), F = term;
    for (int k = 0; k < kPoissonFastMax; ++k) {
        const double gap = ldexp(F, 64) - Ud;
        if (gap > gap_min) return k;  // U < 2^64 F(k)
        if (gap > -gap_min) return -1;
        term = term * lam / (double)(k + 1);
        F += term;
    }
    return -1;
}

__global__ void __launch_bounds__(256) k_counts_poisson(const RunDesc *runs, WorkMap map) {
    int b;
    const RunDesc &rd = runs[map_block(map, blockIdx.x, &b)];
    RunState *st = rd.st;
    if (st->err || rd.resample != PA_RESAMPLE_POISSON) return;
    __shared__ int64_t sh[32];
    __shared__ int amb_any;
    if (threadIdx.x == 0) amb_any = 0;
    const int Rp = st->R_cur, i = st->step + 1, kmin = st->kmin;
    const int j = b * kSlotBlock + 4 * (int)threadIdx.x;
    int64_t s = 0, s2 = 0;
    bool amb = false;
    if (j < Rp) {
        const U4 x0 = philox(rd.key0, rd.key1, (uint32_t)(j >> 1), (uint32_t)i, 0u, kTagPoisson);
        const U4 x1 = philox(rd.key0, rd.key1, (uint32_t)(j >> 1) + 1u, (uint32_t)i, 0u, kTagPoisson);
        const uint64_t U[4] = {((uint64_t)x0.y << 32) | x0.x, ((uint64_t)x0.w << 32) | x0.z,
                               ((uint64_t)x1.y << 32) | x1.x, ((uint64_t)x1.w << 32) | x1.z};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int jj = j + m;
            if (jj < Rp) {
                const double *p = rd.plev + 6 * (((rd.E[jj] + 2 * rd.N) >> 2) - kmin);
                int c = poisson_invert_fast(p[0] + p[1], U[m]);
                if (c < 0) c = poisson_invert(dd{p[0], p[1]}, dd{p[2], p[3]}, (int)p[4], U[m], &amb);
                rd.cnt[jj] = c;
                s += c;
                s2 += (int64_t)c * c;
            }
        }
    }
    __syncthreads();
    if (amb) atomicOr(&amb_any, 1);
    int64_t v[2] = {s, s2};
    block_sum_i64v(v, sh);  // its barriers also order amb_any
    if (threadIdx.x == 0) {
        rd.part[b * 8 + 0] = v[0];
        rd.part[b * 8 + 1] = v[1];
        if (amb_any) {
            st->err = PA_ERR_NUMERIC;
            st->err_step = i;
        }
    }
}

// Multinomial, pass 1: quantised weight q_j of each parent, its inclusive
// prefix within the block of kSlotBlock parents (cum[j]), that prefix at the
// last parent of each stretch of 64 and of each eighth of a stretch once more
// in dense arrays (send[s], read whole by every block of the draws, and
// e8[j / 8], whose eight entries for a stretch share one 64-byte segment), the
// block's total (part[b*8 + 3]), zeroed counts and a zeroed per-block count
// (part[b*8 + 0], which the draws increment).
__global__ void __launch_bounds__(256) k_multi_weights(const RunDesc *runs, WorkMap map) {
    int b;
    const RunDesc &rd = runs[map_block(map, blockIdx.x, &b)];
    RunState *st = rd.st;
    __shared__ int64_t sh[32];
    const int j = b * kSlotBlock + 4 * (int)threadIdx.x;
    // the parents' energies (up to the capacity) load alongside the run's state
    int32_t e[4] = {0, 0, 0, 0};
#pragma unroll
    for (int m = 0; m < 4; ++m)
        if (j + m < rd.C) e[m] = rd.E[j + m];
    if (st->err || rd.resample != PA_RESAMPLE_MULTINOMIAL) return;
    const int Rp = st->R_cur, kmin = st->kmin;
    uint64_t q[4] = {0, 0, 0, 0};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        if (j + m < Rp) {
            q[m] = rd.zlev[((e[m] + 2 * rd.N) >> 2) - kmin];
            rd.cnt[j + m] = 0;
        }
    }
    int64_t tot;
    uint64_t run = (uint64_t)block_exclusive_scan((int64_t)(q[0] + q[1] + q[2] + q[3]), sh, &tot);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        run += q[m];
        if (j + m < Rp) {
            rd.cum[j + m] = run;
            if (((j + m) & 7) == 7 || j + m == Rp - 1) rd.e8[(j + m) >> 3] = run;
            if (((j + m) & 63) == 63 || j + m == Rp - 1) rd.send[(j + m) >> 6] = run;
        }
    }
    if (threadIdx.x == 0) {
        rd.part[b * 8 + 3] = tot;
        rd.part[b * 8 + 0] = 0;
    }
}

// Multinomial, pass 1 with the step's normalisation in the same launch, for
// batches whose runs all resample multinomially at L <= 64: one extra block
// per run does the whole of k_norm (thresholds, S, ln Q's inputs, the checks
// that end a run), while every block of parents forms the quantised level
// weights it needs itself in LDS, with k_norm's operations in k_norm's order
// (so the integers are the same), and then proceeds as k_multi_weights.  A
// step that k_norm stops (no further temperature, a bad schedule, an
// undecidable weight) is recognised by every block on its own, and leaves
// the previous step's counts untouched.
constexpr int kFusedMaxLevels = 64 * 64 + 1;
__global__ void __launch_bounds__(256) k_multi_norm_weights(const RunDesc *runs, WorkMap map,
                                                            int slot_blocks) {
    if ((int)blockIdx.x >= slot_blocks) {
        norm_run(runs[(int)blockIdx.x - slot_blocks]);
        return;
    }
    int b;
    const RunDesc &rd = runs[map_block(map, blockIdx.x, &b)];
    RunState *st = rd.st;
    __shared__ uint64_t zl[kFusedMaxLevels];
    __shared__ double sh_hi[2], sh_lo[2];
    __shared__ int64_t sh[32];
    __shared__ int amb_any;
    const int j = b * kSlotBlock + 4 * (int)threadIdx.x;
    int32_t e[4] = {0, 0, 0, 0};
#pragma unroll
    for (int m = 0; m < 4; ++m)
        if (j + m < rd.C) e[m] = rd.E[j + m];
    if (st->err || rd.resample != PA_RESAMPLE_MULTINOMIAL) return;
    const int i = st->step + 1;
    if (i > rd.max_steps) return;
    const double b0 = rd.betas[i - 1], b1 = rd.betas[i];
    if (!(b1 >= b0) || !(b1 <= 1e300)) return;
    const int Rp = st->R_cur, kmin = st->kmin, kmax = st->kmax;
    const int nlev = kmax - kmin + 1;
    const dd db = two_sum(b1, -b0);
    const bool exact = (db.hi == 0.0) || (nlev == 1);
    if (threadIdx.x == 0) amb_any = 0;
    // k_norm's level weights: thread t's first w_t = e^{-4 dbeta t} (w_0 = 1),
    // then products with e^{-4 dbeta blockDim} = w_1 w_{blockDim-1}
    dd w{1.0, 0.0};
    if (threadIdx.x != 0 && !exact) dd_exp_neg(dd_mul_d(db, 4.0 * threadIdx.x), &w);
    dd stride{1.0, 0.0};
    if (!exact && nlev > (int)blockDim.x) {
        if (threadIdx.x == 1 || threadIdx.x == blockDim.x - 1) {
            sh_hi[threadIdx.x == 1 ? 0 : 1] = w.hi;
            sh_lo[threadIdx.x == 1 ? 0 : 1] = w.lo;
        }
        __syncthreads();
        stride = dd_mul(dd{sh_hi[0], sh_lo[0]}, dd{sh_hi[1], sh_lo[1]});
    }
    bool amb = false;
    for (int l = threadIdx.x; l < nlev; l += blockDim.x) {
        uint64_t z;
        if (exact || l == 0)
            z = 1ull << 40;
        else
            z = (w.hi == 0.0) ? 0ull : dd_floor_decided(dd_ldexp(w, 40), &amb);
        zl[l] = z;
        if (!exact) w = dd_mul(w, stride);
    }
    if (amb) atomicOr(&amb_any, 1);
    __syncthreads();
    if (amb_any) return;  // k_norm's block reports the step as undecidable
    uint64_t q[4] = {0, 0, 0, 0};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        if (j + m < Rp) {
            q[m] = zl[((e[m] + 2 * rd.N) >> 2) - kmin];
            rd.cnt[j + m] = 0;
        }
    }
    int64_t tot;
    uint64_t run = (uint64_t)block_exclusive_scan((int64_t)(q[0] + q[1] + q[2] + q[3]), sh, &tot);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        run += q[m];
        if (j + m < Rp) {
            rd.cum[j + m] = run;
            if (((j + m) & 7) == 7 || j + m == Rp - 1) rd.e8[(j + m) >> 3] = run;
            if (((j + m) & 63) == 63 || j + m == Rp - 1) rd.send[(j + m) >> 6] = run;
        }
    }
    if (threadIdx.x == 0) {
        rd.part[b * 8 + 3] = tot;
        rd.part[b * 8 + 0] = 0;
    }
}

// Multinomial, pass 2: draw d (of R) picks the first parent whose global
// cumulative weight exceeds floor(U64_d * W / 2^64).  Every block first forms
// the exclusive prefix of the parent blocks' totals in LDS (the block bases;
// W is their sum), finds a draw's parent block there, and then the parent
// inside the block from the in-block prefix: sixteen stretches of 64, their
// eighths, then single parents, each level by independent loads.  Counts
// accumulate atomically (order-free); so does each parent block's count of
// children (part[b*8 + 0], for k_offsets), gathered in LDS first so that a
// block adds each parent block's share once.  A block of kSlotBlock threads
// makes the kSlotBlock draws of one slot block (one draw per thread), so that
// the LDS index and the shares are built and added once per 1024 draws.

// One multinomial draw d: its uniform, the stretch of 64 parents that holds
// its target (from the LDS index of every 64th global cumulative weight, or,
// for populations too large for that index, from the LDS block bases and the
// ends of the block's sixteen stretches), then the eighth and the parent by
// independent loads of the in-block prefix; its count and the block's LDS
// count are incremented.
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));  // 16-byte loads

__device__ __forceinline__ void draw_one(const RunDesc &rd, int d, int i, uint64_t W,
                                         const uint64_t *base, const uint64_t *coarse, int nc,
                                         int nbp, int Rp, int32_t *bcnt) {
    const U4 x = philox(rd.key0, rd.key1, (uint32_t)(d >> 1), (uint32_t)i, 0u, kTagMulti);
    const uint64_t U = (d & 1) ? ((uint64_t)x.w << 32) | x.z : ((uint64_t)x.y << 32) | x.x;
    const uint64_t target = mulhi64(U, W);
    const gptr<const uint64_t> cum = global(static_cast<const uint64_t *>(rd.cum));
    int s0, pb;
    if (coarse) {  // the first stretch whose last global cumulative weight exceeds target
        int lo = 0, hi = nc - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (coarse[mid] > target) hi = mid; else lo = mid + 1;
        }
        s0 = 64 * lo;
        pb = s0 / kSlotBlock;
    } else {
        int lo = 0, hi = nbp - 1;  // the last block whose base is <= target
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (base[mid] <= target) lo = mid; else hi = mid - 1;
        }
        pb = lo;
        const uint64_t t = target - base[pb];
        const int s_first = pb * (kSlotBlock / 64), s_last = (min(pb * kSlotBlock + kSlotBlock, Rp) - 1) >> 6;
        const gptr<const uint64_t> send = global(static_cast<const uint64_t *>(rd.send));
        int e = 0;  // stretches of 64 whose last prefix is <= t
#pragma unroll
        for (int k = 0; k < kSlotBlock / 64 - 1; ++k) e += send[min(s_first + k, s_last)] <= t ? 1 : 0;
        s0 = pb * kSlotBlock + 64 * e;
    }
    const uint64_t t = target - base[pb];  // below the block's total
    const int last = min(pb * kSlotBlock + kSlotBlock, Rp) - 1;
    // Each level reads one aligned 64-byte segment in four 16-byte loads: the
    // eight eighth-ends of the stretch (e8), then the eight prefixes of the
    // eighth (cum).  Entries past the block's last parent (a short final
    // stretch) are stale and are not compared: the target lies below them.
    const gptr<const u64x2> e8v = global(reinterpret_cast<const u64x2 *>(rd.e8 + (s0 >> 3)));
    u64x2 q[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = e8v[k];
    int e2 = 0;  // eighths of the stretch whose end is <= t
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        const uint64_t v = (k & 1) ? q[k >> 1].y : q[k >> 1].x;
        e2 += s0 + 8 * k <= last && v <= t ? 1 : 0;
    }
    const int b0 = s0 + 8 * e2;
    const gptr<const u64x2> cv = global(reinterpret_cast<const u64x2 *>(rd.cum + b0));
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = cv[k];
    int f = 0;
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        const uint64_t v = (k & 1) ? q[k >> 1].y : q[k >> 1].x;
        f += b0 + k <= last && v <= t ? 1 : 0;
    }
    atomicAdd(&rd.cnt[b0 + f], 1);
    atomicAdd(&bcnt[pb], 1);
}

// LDS of the draws: block bases (8 bytes per parent block), their counts (4
// bytes) and, while the population has at most kCoarse stretches of 64, the
// index of every 64th global cumulative weight (8 bytes per stretch).
constexpr int kCoarse = 4096;
// the most any run with at most max_nblk parent blocks uses: 12 bytes per block,
// plus 8 per stretch for runs of at most kCoarse / 16 blocks
inline size_t draw_lds_bytes(int max_nblk) {
    const size_t small = (size_t)std::min(max_nblk, kCoarse / (kSlotBlock / 64));
    return std::max((size_t)max_nblk * 12, small * (12 + 8 * (kSlotBlock / 64)));
}

__global__ void __launch_bounds__(kSlotBlock) k_multi_draw(const RunDesc *runs, WorkMap map) {
    int b;
    const RunDesc &rd = runs[map_block(map, blockIdx.x, &b)];
    RunState *st = rd.st;
    extern __shared__ uint64_t base[];  // [nbp] bases, [nc] coarse index if used, [nbp] int32 counts
    __shared__ int64_t sh[32];
    // Loads bounded by the capacity, issued before the run's state is known
    // so that their latencies overlap: the parent-block total of this thread
    // (one per thread while the capacity has at most blockDim blocks) and the
    // stretch ends of the coarse index (at most kCoarse / blockDim each).
    const int tid = (int)threadIdx.x;
    const gptr<const uint64_t> send = global(static_cast<const uint64_t *>(rd.send));
    const uint64_t part0 = tid < rd.nblk ? (uint64_t)rd.part[tid * 8 + 3] : 0;
    constexpr int kSendPer = kCoarse / kSlotBlock;
    uint64_t se[kSendPer];
#pragma unroll
    for (int m = 0; m < kSendPer; ++m) {
        const int k = tid + m * kSlotBlock;
        se[m] = k < min(rd.G, kCoarse) ? send[k] : 0;
    }
    if (st->err || rd.resample != PA_RESAMPLE_MULTINOMIAL) return;
    const int Rp = st->R_cur, i = st->step + 1;
    const int nbp = (Rp + kSlotBlock - 1) / kSlotBlock;
    const int nc = (Rp + 63) >> 6;
    uint64_t *coarse = nc <= kCoarse ? base + nbp : nullptr;
    int32_t *bcnt = reinterpret_cast<int32_t *>(base + nbp + (coarse ? nc : 0));
    const int per = (nbp + kSlotBlock - 1) / kSlotBlock;  // blocks per thread
    const int kb = tid * per, ke = min(kb + per, nbp);
    uint64_t s = 0;
    if (per == 1) {
        s = kb < nbp ? part0 : 0;
    } else {
        for (int k = kb; k < ke; ++k) s += (uint64_t)rd.part[k * 8 + 3];
    }
    int64_t total;
    uint64_t acc = (uint64_t)block_exclusive_scan((int64_t)s, sh, &total);
    for (int k = kb; k < ke; ++k) {
        base[k] = acc;
        bcnt[k] = 0;
        acc += per == 1 ? part0 : (uint64_t)rd.part[k * 8 + 3];
    }
    __syncthreads();
    if (coarse) {
#pragma unroll
        for (int m = 0; m < kSendPer; ++m) {
            const int k = tid + m * kSlotBlock;
            if (k < nc) coarse[k] = base[k / (kSlotBlock / 64)] + se[m];
        }
        __syncthreads();
    }
    const uint64_t W = (uint64_t)total;
    const int d = b * kSlotBlock + (int)threadIdx.x;
    if (d < rd.R) draw_one(rd, d, i, W, base, coarse, nc, nbp, Rp, bcnt);
    __syncthreads();
    for (int k = threadIdx.x; k < nbp; k += blockDim.x)
        if (bcnt[k]) atomicAdd(reinterpret_cast<unsigned long long *>(&rd.part[k * 8 + 0]),
                               (unsigned long long)bcnt[k]);
}

// off[j] = sum_{l<j} r_l (children of parent j occupy [off[j], off[j] + r_j)),
// off[R_{i-1}] = R_i, and par[c] = j for those children.  Block 0 records R_i (or PA_ERR_CAPACITY,
// PA_ERR_EXTINCT) and
// sum r_j^2.  The histogram, consumed by k_norm, is cleared here so that the
// reduction at the end of the step can build the next one.
__global__ void __launch_bounds__(256) k_offsets(const RunDesc *runs, WorkMap map, int slot_blocks) {
    if ((int)blockIdx.x >= slot_blocks) {  // the free-energy jackknife's weight sums
        const int q = (int)blockIdx.x - slot_blocks;
        jack_weights(runs[q / kBlocks], q % kBlocks);
        return;
    }
    int b;
    const RunDesc &rd = runs[map_block(map, blockIdx.x, &b)];
    RunState *st = rd.st;
    __shared__ int64_t sh[32];
    __shared__ int64_t base_sh;
    // this thread's four counts and the parent blocks' child counts, loaded
    // (up to the capacity) before the run's state, whose latency they share
    const int j = b * kSlotBlock + 4 * (int)threadIdx.x;
    int c[4] = {0, 0, 0, 0};
    for (int m = 0; m < 4; ++m)
        if (j + m < rd.C) c[m] = rd.cnt[j + m];
    // children of the blocks before this one and of all blocks (one pass)
    int64_t v[3] = {0, 0, 0};
    for (int k = threadIdx.x; k < rd.nblk; k += blockDim.x) {
        const int64_t r = rd.part[k * 8 + 0];
        v[0] += k < b ? r : 0;
        v[1] += r;
    }
    if (st->err) return;
    const int Rp = st->R_cur;
    for (int m = 0; m < 4; ++m)
        if (j + m >= Rp) c[m] = 0;
    // the block's sum of r_j^2 goes to the step's total
    v[2] = (int64_t)c[0] * c[0] + (int64_t)c[1] * c[1] + (int64_t)c[2] * c[2] + (int64_t)c[3] * c[3];
    block_sum_i64v(v, sh);
    if (threadIdx.x == 0) {
        base_sh = v[0];
        if (v[2]) atomicAdd(reinterpret_cast<unsigned long long *>(&st->sum_cnt2), (unsigned long long)v[2]);
    }
    if (b == 0) {
        const int64_t total = v[1];
        if (threadIdx.x == 0) {
            if (total > rd.C || total == 0) {
                st->err = total ? PA_ERR_CAPACITY : PA_ERR_EXTINCT;
                st->err_step = st->step + 1;
            } else {
                st->R_new = (int32_t)total;
                rd.off[Rp] = (int32_t)total;
            }
            st->kmin = INT_MAX;
            st->kmax = -1;
        }
    }
    for (int k = b * (int)blockDim.x + (int)threadIdx.x; k < rd.K; k += rd.nblk * (int)blockDim.x)
        rd.hist[k] = 0;
    __syncthreads();
    int64_t tot;
    int64_t run = base_sh + block_exclusive_scan(c[0] + c[1] + c[2] + c[3], sh, &tot);
    for (int m = 0; m < 4; ++m) {
        if (j + m < Rp) {
            rd.off[j + m] = (int32_t)run;
            // the parent of each child slot (past the capacity the step fails anyway)
            const gptr<int32_t> par = global(rd.par);
            for (int64_t k = run; k < run + c[m] && k < rd.C; ++k) par[k] = j + m;
        }
        run += c[m];
    }
}

// ------------------------------------------------------------------ copy / compaction

// Bit networks of the multispin gather.  Both run as six stages of the form
// x = (x & ~g) | (y & g), y = x shifted by 2^i: one shift and one three-input
// bitwise operation per 32-bit half, with the stage masks g computed once per
// child group on the scalar unit (they depend only on the parents) and no
// branches between the stages.
//
// Compress (the selected bits of x moved to the low end in order, Hacker's
// Delight Sec. 7-4): the book's move masks mv_i, taken in gather form -- the
// positions mv_i >> 2^i receive a moved bit at stage i.  Positions that a bit
// leaves keep a stale copy, which no later stage reads (they only read
// positions holding selected bits); the low popcount(m) bits are exact.
struct Compress {
    uint64_t g[6];
    uint64_t low;  // the low popcount(m) bits
};
__device__ __forceinline__ Compress compress_masks(uint64_t m) {
    Compress n;
    const int cnt = __popcll(m);
    n.low = cnt == 64 ? ~0ull : (1ull << cnt) - 1;
    uint64_t mk = ~m << 1;  // marks the zeros of m to the right of each bit
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        uint64_t mp = mk ^ (mk << 1);  // parallel suffix (prefix xor from the right)
        mp ^= mp << 2;
        mp ^= mp << 4;
        mp ^= mp << 8;
        mp ^= mp << 16;
        mp ^= mp << 32;
        const uint64_t mv = mp & m;
        m = (m ^ mv) | (mv >> (1 << i));
        n.g[i] = mv >> (1 << i);
        mk &= ~mp;
    }
    return n;
}
// A three-input bitwise function (table as for xor3) on the halves of 64-bit
// words; the builtin returns a signed int, so each half is taken as unsigned
// before it is widened
template <int TABLE>
__device__ __forceinline__ uint64_t bitop3_64(uint64_t a, uint64_t b, uint64_t c) {
    const uint32_t hi = (uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), (uint32_t)(b >> 32),
                                                              (uint32_t)(c >> 32), TABLE);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)a, (uint32_t)b, (uint32_t)c, TABLE);
    return ((uint64_t)hi << 32) | lo;
}
// (a & ~b) | (c & b)
__device__ __forceinline__ uint64_t select_bits(uint64_t a, uint64_t b, uint64_t c) { return bitop3_64<0xB8>(a, b, c); }
// Compressed bits of x, not yet cut to the low popcount(m) bits.
__device__ __forceinline__ uint64_t net_compress(uint64_t x, const Compress &n) {
#pragma unroll
    for (int i = 0; i < 6; ++i) x = select_bits(x, n.g[i], x >> (1 << i));
    return x;
}
// Spread with copies: child c (bit c of the child word) takes bit h(c) of the
// distinct parents' bits S, where h(c) is the rank of c's parent among them.
// The left shift d(c) = c - h(c) is the number of copies (children that repeat
// the previous child's parent) at positions <= c: it never decreases and grows
// by at most one per position.  Applying the shifts by 32, 16, ..., 1 in turn,
// each where bit i of d is set at the stage's output position, then delivers
// bit c - d(c) to every c: the value bound for c sits, before the stage of bit
// i, at q = c - (d(c) mod 2^i), and d(q) lies in [d(c) - (c - q), d(c)], so
// d(q) and d(c) agree in every bit from i up.
struct Spread {
    uint64_t s[6];  // s[i]: the children with bit i of d set
    uint64_t live;  // the children that exist
};
// Dead children (past the population) come out unspecified.
__device__ __forceinline__ uint64_t net_spread(uint64_t x, const Spread &n) {
#pragma unroll
    for (int i = 5; i >= 0; --i) x = select_bits(x, n.s[i], x << (1 << i));
    return x;
}

// Child c of destination group gd takes the spins and family label of parent
// p(c) = the last j with off[j] <= c; parents stay in ascending order, so the
// copies of one parent are adjacent (tree order).  Every wavefront finds the
// parents of the group's 64 children (lane = child) and then:
//  - multispin: the child word of a site is a monotone bit map of at most a
//    few parent words.  Per parent group pg the surviving parents that feed
//    this child group form a selector P_pg; compressing each parent word by
//    P_pg and concatenating gives the distinct parents' bits S in order;
//    spreading S over the children with their copies gives the child word.
//    Lane = four consecutive sites.
//  - int8: the parents' rows of kGatherSites sites at a time are staged in LDS
//    (16-byte loads); thread = one dword (four children) of every 16th row.
constexpr int kGatherPg = 4;      // int8: parent groups staged per pass
constexpr int kGatherSites = 256;  // int8: site rows per pass (64 and 128 were slower)
constexpr int kGather8Threads = 4 * kGatherSites;  // int8: one 16-byte stage element per thread
constexpr int kGather8Step = kGather8Threads / 16;   // int8: site rows a pass step covers
constexpr int kGather8Out = kGatherSites / kGather8Step;  // int8: output dwords per thread and pass

// Shared start of both gathers: the destination group of the block, the
// parent of each lane's child and the family labels; false if there is no
// work (error, or the group lies past the new population).
struct GatherJob {
    const RunDesc *rd;
    int gd, Rn, Rp, cur, nb, N, p, nv, g_first, g_last;
};
__device__ __forceinline__ bool gather_start(const RunDesc *runs, const WorkMap &map, int layout,
                                             GatherJob *j) {
    int gd;
    const RunDesc &rd = runs[map_block(map, xcd_swizzle(blockIdx.x, gridDim.x), &gd)];
    RunState *st = rd.st;
    if (st->err || rd.layout != layout) return false;
    const int Rn = st->R_new, Rp = st->R_cur;
    if (gd * kLanes >= Rn) return false;
    const int cur = st->cur, nb = cur ^ 1;
    const int lane = threadIdx.x & 63;
    const int c = gd * kLanes + lane;
    const int p = c < Rn ? rd.par[c] : -1;  // the last j with off[j] <= c
    if ((threadIdx.x >> 6) == 0 && c < rd.C) rd.fam[nb][c] = p >= 0 ? rd.fam[cur][p] : 0;
    const int nv = __builtin_amdgcn_readfirstlane(min(kLanes, Rn - gd * kLanes));
    *j = GatherJob{&rd, gd, Rn, Rp, cur, nb, rd.N, p, nv,
                   __builtin_amdgcn_readlane(p, 0) >> 6, __builtin_amdgcn_readlane(p, nv - 1) >> 6};
    return true;
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(v >> 32), l) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
}

constexpr int kGatherPass = 256;  // multispin: sites of one wavefront pass (four per lane)
constexpr int kGatherPasses = 2;  // multispin: passes whose loads are in flight together
constexpr int kGatherThreads = 512;  // multispin: eight wavefronts, one 512-site chunk each at L = 64

__global__ void __launch_bounds__(kGatherThreads) k_gather_msc64(const RunDesc *runs, WorkMap map) {
    GatherJob jb;
    if (!gather_start(runs, map, PA_LAYOUT_MSC64, &jb)) return;
    const RunDesc &rd = *jb.rd;
    const int N = jb.N, p = jb.p, nv = jb.nv;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const gptr<const u32x4> src = global(reinterpret_cast<const u32x4 *>(rd.ms[jb.cur]));
    const gptr<u32x4> dst = global(reinterpret_cast<u32x4 *>(rd.ms[jb.nb] + (size_t)jb.gd * N));
    const int p_prev = __shfl_up(p, 1, 64);
    const bool live = lane < nv;
    // copies: children whose parent is the previous child's
    const uint64_t F = __ballot(live && lane > 0 && p == p_prev);
    Spread SP;
    {
        const int d = __popcll(F & ((2ull << lane) - 1));  // copies at lanes <= this one
#pragma unroll
        for (int i = 0; i < 6; ++i) SP.s[i] = __ballot(live && ((d >> i) & 1));
        SP.live = __ballot(live);
    }
    // the selector of parent group pg (its parents with a child in this group)
    // from the children's parents: an OR-scan of the bits 1 << (p mod 64) over
    // the lanes whose parent lies in the same group leaves it in the last such
    // lane (the parents ascend with the lane)
    const int pgl = live ? p >> 6 : INT_MAX;
    uint64_t sel = live ? 1ull << (p & 63) : 0ull;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t o = __shfl_up(sel, d, 64);
        const int og = __shfl_up(pgl, d, 64);
        if (lane >= d && og == pgl) sel |= o;
    }
    const int pg_next = __shfl_down(pgl, 1, 64);
    const uint64_t ends = __ballot(live && (lane == nv - 1 || pg_next != pgl));
    // chunks of kGatherPasses passes of a wavefront: per feeding parent group
    // (ascending), its network once and the compressed parent words of every
    // pass, concatenated in S.  Bits of S above the distinct parents may hold
    // stale bits of the compress stages: the spread reads only bits h(c) of
    // live children, and dead children are cleared at the end.
    for (int c0 = wave * kGatherPass * kGatherPasses; c0 < N; c0 += nw * kGatherPass * kGatherPasses) {
        uint64_t S[kGatherPasses][4];
        // per feeding group, the compressed words of the chunk's passes; past
        // the last site the loads repeat the last four words (never stored)
        int shift = 0;
        for (uint64_t m = ends; m; m &= m - 1) {  // uniform
            const int l = __builtin_ctzll(m);
            const Compress NP = compress_masks(readlane64(sel, l));
            const uint64_t keep = NP.low << shift;  // where this group's parents land in S
            const gptr<const u32x4> sp = src + (size_t)__builtin_amdgcn_readlane(pgl, l) * (N / 2);
#pragma unroll
            for (int k = 0; k < kGatherPasses; ++k) {
                const int sb = min(c0 + k * kGatherPass + 4 * lane, N - 4);
                const u32x4 v0 = sp[sb / 2], v1 = sp[sb / 2 + 1];
                const uint64_t x[4] = {net_compress(((uint64_t)v0.y << 32) | v0.x, NP),
                                       net_compress(((uint64_t)v0.w << 32) | v0.z, NP),
                                       net_compress(((uint64_t)v1.y << 32) | v1.x, NP),
                                       net_compress(((uint64_t)v1.w << 32) | v1.z, NP)};
                if (shift == 0) {  // uniform: the first group
#pragma unroll
                    for (int q = 0; q < 4; ++q) S[k][q] = x[q];
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) S[k][q] = select_bits(S[k][q], keep, x[q] << shift);
                }
            }
            shift += __popcll(NP.low);
        }
#pragma unroll
        for (int k = 0; k < kGatherPasses; ++k) {
            uint64_t o[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) o[q] = net_spread(S[k][q], SP);
            if (nv < 64) {  // uniform: the last, partial child group
#pragma unroll
                for (int q = 0; q < 4; ++q) o[q] &= SP.live;
            }
            const int sb = c0 + k * kGatherPass + 4 * lane;
            if (sb < N) {
                dst[sb / 2] = u32x4{(uint32_t)o[0], (uint32_t)(o[0] >> 32), (uint32_t)o[1],
                                    (uint32_t)(o[1] >> 32)};
                dst[sb / 2 + 1] = u32x4{(uint32_t)o[2], (uint32_t)(o[2] >> 32), (uint32_t)o[3],
                                        (uint32_t)(o[3] >> 32)};
            }
        }
    }
}

__global__ void __launch_bounds__(kGather8Threads) k_gather_int8(const RunDesc *runs, WorkMap map) {
    __shared__ u32x4 stage[kGatherPg * kGatherSites * 4];  // groups x rows x 64 bytes
    GatherJob jb;
    if (!gather_start(runs, map, PA_LAYOUT_INT8, &jb)) return;
    const RunDesc &rd = *jb.rd;
    const int N = jb.N, p = jb.p, g_first = jb.g_first, g_last = jb.g_last;
    const int cur = jb.cur, nb = jb.nb, gd = jb.gd;
    {
        // thread -> dword k (children 4k .. 4k + 3) of site rows sl, sl + kGather8Step, ...
        // of a chunk of kGatherSites rows
        const gptr<const u32x4> src = global(reinterpret_cast<const u32x4 *>(rd.s8[cur]));
        const gptr<uint32_t> dst = global(reinterpret_cast<uint32_t *>(rd.s8[nb] + (size_t)gd * N * kLanes));
        const int k = threadIdx.x & 15, sl = threadIdx.x >> 4;
        int pc[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) pc[m] = __shfl(p, 4 * k + m, 64);
        const uint8_t *st8 = reinterpret_cast<const uint8_t *>(stage);
        constexpr int kPass = kGatherSites * 4;  // 16-byte elements per parent group and pass
        if (g_last - g_first < kGatherPg) {
            // all parent groups fit one pass: the next pass's rows are loaded
            // into registers while the current one is picked from LDS
            const int ngb = g_last - g_first + 1;
            u32x4 pre[kGatherPg];
            auto load = [&](int s0) {
#pragma unroll
                for (int b = 0; b < kGatherPg; ++b) {
                    const int srow = s0 + ((int)threadIdx.x >> 2);
                    if (b < ngb && srow < N)
                        pre[b] = src[((size_t)(g_first + b) * N + srow) * 4 + (threadIdx.x & 3)];
                }
            };
            load(0);
            for (int s0 = 0; s0 < N; s0 += kGatherSites) {
                __syncthreads();  // the previous pass's readers are done
#pragma unroll
                for (int b = 0; b < kGatherPg; ++b)
                    if (b < ngb) stage[b * kPass + threadIdx.x] = pre[b];
                __syncthreads();
                if (s0 + kGatherSites < N) load(s0 + kGatherSites);
                uint32_t out[kGather8Out];
#pragma unroll
                for (int r = 0; r < kGather8Out; ++r) {
                    out[r] = 0;
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        if (pc[m] < 0) {
                            out[r] |= 0xFFu << (8 * m);  // past the population: spin -1
                        } else {
                            const uint8_t *row = st8 + ((pc[m] >> 6) - g_first) * (kGatherSites * 64) +
                                                 (pc[m] & 63);
                            out[r] |= (uint32_t)row[(sl + kGather8Step * r) * 64] << (8 * m);
                        }
                    }
                }
#pragma unroll
                for (int r = 0; r < kGather8Out; ++r) {
                    const int site = s0 + sl + kGather8Step * r;
                    if (site < N) dst[(size_t)site * 16 + k] = out[r];
                }
            }
            return;
        }
        for (int s0 = 0; s0 < N; s0 += kGatherSites) {
            uint32_t out[kGather8Out];
#pragma unroll
            for (int r = 0; r < kGather8Out; ++r) {
                out[r] = 0;
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    if (pc[m] < 0) out[r] |= 0xFFu << (8 * m);  // past the population: spin -1
            }
            for (int gb = g_first; gb <= g_last; gb += kGatherPg) {
                const int ngb = min(kGatherPg, g_last - gb + 1);
                __syncthreads();  // the previous pass's readers are done
                // ngb groups x kGatherSites rows x 4 uint4, spread over the block
                for (int e = threadIdx.x; e < ngb * kPass; e += blockDim.x) {
                    const int b = e / kPass, r = e - b * kPass;
                    const int srow = s0 + (r >> 2);
                    if (srow < N) stage[e] = src[((size_t)(gb + b) * N + srow) * 4 + (r & 3)];
                }
                __syncthreads();
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int rel = (pc[m] >> 6) - gb;
                    if (pc[m] >= 0 && rel >= 0 && rel < ngb) {
                        const uint8_t *row = st8 + rel * (kGatherSites * 64) + (pc[m] & 63);
#pragma unroll
                        for (int r = 0; r < kGather8Out; ++r)
                            out[r] |= (uint32_t)row[(sl + kGather8Step * r) * 64] << (8 * m);
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < kGather8Out; ++r) {
                const int site = s0 + sl + kGather8Step * r;
                if (site < N) dst[(size_t)site * 16 + k] = out[r];
            }
        }
    }
}

// ------------------------------------------------------------------ Metropolis sweeps

// Bit-sliced Metropolis classes of one word (64 replicas of one site): with
// a_k = s XOR n_k (antiparallel neighbours), A = sum a_k and dE = 8 - 4A,
// A >= 2 (dE <= 0) always flips, A = 1 is dE = 4, A = 0 is dE = 8.
// The same classes per 32-bit half with three-input operations: with m =
// maj(a1, a2, a3) and o = a1 | a2 | a3, A >= 2 is m | (a4 & o) and A = 1 is
// (o | a4) & ~(A >= 2).
struct WordClass2 {
    uint64_t ge2, eq1;
};
__device__ __forceinline__ uint32_t ge2_half(uint32_t a1, uint32_t a2, uint32_t a3, uint32_t a4,
                                             uint32_t *eq1) {
    const uint32_t m = __builtin_amdgcn_bitop3_b32(a1, a2, a3, 0xE8);   // maj
    const uint32_t o = __builtin_amdgcn_bitop3_b32(a1, a2, a3, 0xFE);   // or
    const uint32_t g = __builtin_amdgcn_bitop3_b32(m, a4, o, 0xF8);     // m | (a4 & o)
    *eq1 = __builtin_amdgcn_bitop3_b32(o, a4, g, 0x54);                 // (o | a4) & ~g
    return g;
}
__device__ __forceinline__ WordClass2 classes(uint64_t a1, uint64_t a2, uint64_t a3, uint64_t a4) {
    uint32_t e_lo, e_hi;
    const uint32_t g_lo = ge2_half((uint32_t)a1, (uint32_t)a2, (uint32_t)a3, (uint32_t)a4, &e_lo);
    const uint32_t g_hi = ge2_half((uint32_t)(a1 >> 32), (uint32_t)(a2 >> 32), (uint32_t)(a3 >> 32),
                                   (uint32_t)(a4 >> 32), &e_hi);
    return WordClass2{((uint64_t)g_hi << 32) | g_lo, ((uint64_t)e_hi << 32) | e_lo};
}

// One bit plane of the lazy comparison u32 < T, from the most significant
// plane down, on one 32-bit half of a word: a lane still tied with its
// threshold (und) is decided by the first plane where its bit differs from
// T's bit (T4's for the dE = 4 lanes, T8's for the dE = 8 lanes; on the lanes
// still tied the dE = 8 lanes are those not in eq1); it is accepted (flip) when
// the plane bit is 0 and T's is 1.  The threshold bits b4, b8 of a plane are
// the same for every lane, so each of their four combinations has its own
// three-input form: t = 0 only rejects (und &= ~pl), t = 1 only accepts
// (flip |= und & ~pl, und &= pl), and t = eq1 or ~eq1 does both.
template <int B4, int B8>
__device__ __forceinline__ void plane_half(uint32_t &und, uint32_t &flip, uint32_t eq1, uint32_t pl) {
    if (!B4 && !B8) {  // t = 0
        und = __builtin_amdgcn_bitop3_b32(und, pl, pl, 0x30);  // und & ~pl
    } else if (B4 && B8) {  // t = 1
        flip = __builtin_amdgcn_bitop3_b32(flip, und, pl, 0xF4);  // flip | (und & ~pl)
        und &= pl;
    } else if (B4) {  // t = eq1
        const uint32_t acc = __builtin_amdgcn_bitop3_b32(und, eq1, pl, 0x40);  // und & eq1 & ~pl
        und = __builtin_amdgcn_bitop3_b32(und, eq1, pl, 0x90);                 // und & ~(eq1 ^ pl)
        flip |= acc;
    } else {  // t = ~eq1
        const uint32_t acc = __builtin_amdgcn_bitop3_b32(und, eq1, pl, 0x10);  // und & ~eq1 & ~pl
        und = __builtin_amdgcn_bitop3_b32(und, eq1, pl, 0x60);                 // und & (eq1 ^ pl)
        flip |= acc;
    }
}

// Planes 2p and 2p + 1 (one Philox call x: plane 2p = x.x | x.y << 32, plane
// 2p + 1 = x.z | x.w << 32) on a word's four 32-bit halves; one branch per
// call picks the straight-line form for the four threshold bits.
struct Lanes {
    uint32_t ul, uh, fl, fh;  // undecided and accepted lanes, low and high halves
};
template <int C, int K>
__device__ __forceinline__ void plane_pair_case(Lanes *s, const uint32_t *el, const uint32_t *eh,
                                                const U4 *x) {
    constexpr int A4 = (C >> 3) & 1, A8 = (C >> 2) & 1, B4 = (C >> 1) & 1, B8 = C & 1;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        plane_half<A4, A8>(s[k].ul, s[k].fl, el[k], x[k].x);
        plane_half<A4, A8>(s[k].uh, s[k].fh, eh[k], x[k].y);
        plane_half<B4, B8>(s[k].ul, s[k].fl, el[k], x[k].z);
        plane_half<B4, B8>(s[k].uh, s[k].fh, eh[k], x[k].w);
    }
}
// K words at once (their threshold bits are the same)
template <int K>
__device__ __forceinline__ void plane_pair(Lanes *s, const uint32_t *el, const uint32_t *eh,
                                           uint32_t T4, uint32_t T8, uint32_t p, const U4 *x) {
    const uint32_t sa = 31u - 2u * p, sb = 30u - 2u * p;
    const uint32_t c = (((T4 >> sa) & 1u) << 3) | (((T8 >> sa) & 1u) << 2) |
                       (((T4 >> sb) & 1u) << 1) | ((T8 >> sb) & 1u);
    switch (c) {
    case 0: plane_pair_case<0, K>(s, el, eh, x); break;
    case 1: plane_pair_case<1, K>(s, el, eh, x); break;
    case 2: plane_pair_case<2, K>(s, el, eh, x); break;
    case 3: plane_pair_case<3, K>(s, el, eh, x); break;
    case 4: plane_pair_case<4, K>(s, el, eh, x); break;
    case 5: plane_pair_case<5, K>(s, el, eh, x); break;
    case 6: plane_pair_case<6, K>(s, el, eh, x); break;
    case 7: plane_pair_case<7, K>(s, el, eh, x); break;
    case 8: plane_pair_case<8, K>(s, el, eh, x); break;
    case 9: plane_pair_case<9, K>(s, el, eh, x); break;
    case 10: plane_pair_case<10, K>(s, el, eh, x); break;
    case 11: plane_pair_case<11, K>(s, el, eh, x); break;
    case 12: plane_pair_case<12, K>(s, el, eh, x); break;
    case 13: plane_pair_case<13, K>(s, el, eh, x); break;
    case 14: plane_pair_case<14, K>(s, el, eh, x); break;
    default: plane_pair_case<15, K>(s, el, eh, x); break;
    }
}

// Ties after the planes: the lanes whose top six uniform bits equal their
// threshold's take fresh low 26 bits (the top 26 bits of a Philox output
// word), four per call, in ascending lane order (call kTagTie | (k >> 2),
// output word k & 3 for the k-th tie).  One such comparison decides a tie:
// u < T iff low26(u) < low26(T).
constexpr uint32_t kPlanePairs = 3;            // Philox calls of bit planes: the top six bits
constexpr uint32_t kTagTie = kTagSweep | 0x100u;

// S4 = T4 << 6, S8 = T8 << 6 (32-bit): low26(u) < low26(T) iff (u >> 6) < low26(T)
// iff u < low26(T) << 6, so the tie's fresh word is compared as it is.
__device__ __forceinline__ void tie_one(uint64_t &und, uint64_t eq1, uint32_t S4, uint32_t S8,
                                        uint32_t v, uint64_t &flip) {
    const uint64_t bit = und & (0ull - und);  // lowest tied lane; 0 when none is left
    und ^= bit;
    // the lanes this slot would accept: class dE = 4 (eq1) if v < S4, dE = 8 if v < S8
    const uint32_t m4 = v < S4 ? ~0u : 0u, m8 = v < S8 ? ~0u : 0u;
    const uint32_t ahi = (uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)(eq1 >> 32), m4, m8, 0xCA);
    const uint32_t alo = (uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)eq1, m4, m8, 0xCA);
    flip = ((uint64_t)(uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)(flip >> 32), (uint32_t)(bit >> 32),
                                                             ahi, 0xF8) << 32) |
           (uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)flip, (uint32_t)bit, alo, 0xF8);  // flip | (bit & a)
}

// most tied words have one tie: the later slots are skipped once none is left
__device__ __forceinline__ void tie_call(uint64_t &und, uint64_t eq1, uint32_t S4, uint32_t S8,
                                         const U4 &x, uint64_t &flip) {
    tie_one(und, eq1, S4, S8, x.x, flip);
    if (und == 0) return;
    tie_one(und, eq1, S4, S8, x.y, flip);
    if (und == 0) return;
    tie_one(und, eq1, S4, S8, x.z, flip);
    tie_one(und, eq1, S4, S8, x.w, flip);
}

// The whole comparison of one word (64 replicas of one site) in one lane.  With
// a_k = s XOR n_k (antiparallel neighbours), A = sum a_k and dE = 8 - 4A:
// A >= 2 (dE <= 0) always flips; A = 1 (dE = 4) and A = 0 (dE = 8) flip iff
// u32 < t4 / t8.  The top six bits of u32 are compared bit plane by bit plane
// from the most significant one; the lanes still tied with their threshold
// after six planes are decided by one comparison of fresh low bits each.
// This equals the full 32-bit comparison.  All three plane calls are made:
// a word has some twenty lanes with dE > 0, so a wavefront nearly always has
// a word that needs the third, and a loop that stops early costs more than it
// saves.  With count, the calls the word needs (plane pairs while a lane is
// still tied, and tie calls) are added: plane calls to *wcalls (the same in
// every lane: the wavefront's total), tie calls to *calls.
__device__ __forceinline__ uint64_t metropolis_word(uint64_t a1, uint64_t a2, uint64_t a3,
                                                    uint64_t a4, uint64_t valid, uint32_t T4,
                                                    uint32_t T8, bool all4, bool all8,
                                                    uint32_t k0, uint32_t k1, uint32_t w,
                                                    uint32_t g, uint32_t h, bool count,
                                                    uint32_t *calls, uint32_t *wcalls) {
    const WordClass2 c = classes(a1, a2, a3, a4);
    const uint64_t eq1 = c.eq1;
    uint64_t flip = c.ge2 & valid;
    uint64_t und = valid & ~c.ge2;
    if (all4 || all8) {  // beta <= 0: a threshold of 2^32 accepts its whole class
        const uint64_t e1 = und & eq1, e0 = und & ~eq1;
        if (all4) { flip |= e1; und &= ~e1; }
        if (all8) { flip |= e0; und &= ~e0; }
    }
    Lanes s{(uint32_t)und, (uint32_t)(und >> 32), (uint32_t)flip, (uint32_t)(flip >> 32)};
    const uint32_t el = (uint32_t)eq1, eh = (uint32_t)(eq1 >> 32);
#pragma unroll
    for (uint32_t p = 0; p < kPlanePairs; ++p) {
        if (count) *wcalls += (uint32_t)__popcll(__ballot((s.ul | s.uh) != 0));
        const U4 x = philox(k0, k1, w, g, h, kTagSweep | p);
        plane_pair<1>(&s, &el, &eh, T4, T8, p, &x);
    }
    und = ((uint64_t)s.uh << 32) | s.ul;
    flip = ((uint64_t)s.fh << 32) | s.fl;
    uint32_t q = 0;
    for (; und != 0; ++q) {
        const U4 x = philox(k0, k1, w, g, h, kTagTie | q);
        tie_call(und, eq1, T4 << 6, T8 << 6, x, flip);
    }
    *calls += q;  // read only when counting
    return flip;
}

// The same comparison for K words in one lane at once: their Philox chains
// are independent instruction streams (for launches too large for more than
// one block per CU, where few wavefronts share a SIMD).  Calls are counted as
// in metropolis_word.
// In: nb[k][0..3] the neighbour words and s0[k] the site word; out: flip[k].
template <int K>
__device__ __forceinline__ void metropolis_words(const uint64_t (*nbr)[4], const uint64_t *s0,
                                                 const uint64_t *valid, uint32_t T4, uint32_t T8,
                                                 bool all4, bool all8, uint32_t k0, uint32_t k1,
                                                 const uint32_t *w, const uint32_t *g, uint32_t h,
                                                 uint64_t *flip, bool count, uint32_t *calls,
                                                 uint32_t *wcalls) {
    Lanes s[K];
    uint32_t el[K], eh[K];
    uint64_t eq1[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const WordClass2 c = classes(s0[k] ^ nbr[k][0], s0[k] ^ nbr[k][1], s0[k] ^ nbr[k][2],
                                     s0[k] ^ nbr[k][3]);
        eq1[k] = c.eq1;
        uint64_t f = c.ge2 & valid[k];
        uint64_t und = valid[k] & ~c.ge2;
        if (all4 || all8) {  // beta <= 0: a threshold of 2^32 accepts its whole class
            const uint64_t e1 = und & c.eq1, e0 = und & ~c.eq1;
            if (all4) { f |= e1; und &= ~e1; }
            if (all8) { f |= e0; und &= ~e0; }
        }
        s[k] = Lanes{(uint32_t)und, (uint32_t)(und >> 32), (uint32_t)f, (uint32_t)(f >> 32)};
        el[k] = (uint32_t)c.eq1;
        eh[k] = (uint32_t)(c.eq1 >> 32);
    }
#pragma unroll
    for (uint32_t p = 0; p < kPlanePairs; ++p) {
        U4 x[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (count) *wcalls += (uint32_t)__popcll(__ballot((s[k].ul | s[k].uh) != 0));
            x[k] = philox(k0, k1, w[k], g[k], h, kTagSweep | p);
        }
        plane_pair<K>(s, el, eh, T4, T8, p, x);
    }
    uint64_t und[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        und[k] = ((uint64_t)s[k].uh << 32) | s[k].ul;
        flip[k] = ((uint64_t)s[k].fh << 32) | s[k].fl;
    }
    for (uint32_t q = 0;; ++q) {
        bool any = false;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            any |= und[k] != 0;
            *calls += und[k] != 0 ? 1u : 0u;  // read only when counting
        }
        if (!any) break;
        U4 x[K];
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] = philox(k0, k1, w[k], g[k], h, kTagTie | q);
#pragma unroll
        for (int k = 0; k < K; ++k) tie_call(und[k], eq1[k], T4 << 6, T8 << 6, x[k], flip[k]);
    }
}

// ------------------------------------------------------------------ heatbath

// Heatbath (Sec. "Spin updates"): every move flips with probability
// p(dE) = 1 / (1 + e^{beta dE}), i.e. iff u32 < T(dE) = ceil(2^32 p(dE)), for
// the five classes dE = 8 - 4A (A antiparallel neighbours, 0..4).  For
// beta > 0, 2^32 p is never an integer and p(-dE) = 1 - p(dE), so with
// T' = T(|dE|) - 1 = floor(2^32 p(|dE|)):
//   dE > 0: u < T(dE)   iff  u <= T'
//   dE < 0: u < T(dE) = 2^32 + 1 - T(|dE|)   iff  ~u >= T'
//   dE = 0: u < 2^31    iff  the top bit of u is 0.
// The dE = +-4 classes share T'_4 and the +-8 classes T'_8, so a plane step
// compares the plane bit with t* = t ^ neg, t = T'_4's or T'_8's bit by the
// lane's |dE| and neg the dE < 0 lanes: the lane is decided where its bit
// differs from t*, and flips iff that bit is 0 (for dE > 0 a 0 below a 1 of
// T' means u < T'; for dE < 0 a 0 of u is a 1 of ~u above a 0 of T').
// A lane whose top six bits leave its comparison open draws 26 fresh bits
// (ties as in the Metropolis comparison); "open" is a property of the
// comparison itself, so it is the same set whichever way it is written.
// Classes per 32-bit half: x = a1 ^ a2 ^ a3, m = maj(a1, a2, a3), A = x + a4 + 2m:
//   |dE| = 4 (A odd): x ^ a4;  dE < 0 (A >= 3): m & (x | a4);  dE = 0 (A = 2):
//   (m & ~x & ~a4) | (~m & x & a4).
struct HbClass {
    uint32_t mag4, neg, x4, zero;
};
__device__ __forceinline__ HbClass hb_class(uint32_t a1, uint32_t a2, uint32_t a3, uint32_t a4) {
    const uint32_t x = __builtin_amdgcn_bitop3_b32(a1, a2, a3, 0x96);  // xor3
    const uint32_t m = __builtin_amdgcn_bitop3_b32(a1, a2, a3, 0xE8);  // maj
    HbClass c;
    c.mag4 = x ^ a4;
    c.neg = __builtin_amdgcn_bitop3_b32(m, x, a4, 0xE0);   // m & (x | a4)
    c.zero = __builtin_amdgcn_bitop3_b32(m, x, a4, 0x18);  // A = 2
    c.x4 = c.mag4 ^ c.neg;
    return c;
}

// One plane on one half: t* = neg (threshold bits 0, 0), ~neg (1, 1), x4 =
// mag4 ^ neg (T'_4 bit 1, T'_8 bit 0) or ~x4 (0, 1).
template <int B4, int B8>
__device__ __forceinline__ void hb_plane_half(uint32_t &und, uint32_t &flip, uint32_t neg, uint32_t x4,
                                              uint32_t pl) {
    constexpr bool same = B4 == B8;
    constexpr bool inv = same ? (B4 != 0) : (B4 == 0);
    const uint32_t X = same ? neg : x4;
    const uint32_t acc = __builtin_amdgcn_bitop3_b32(und, X, pl, inv ? 0x10 : 0x40);  // und & t* & ~pl
    und = __builtin_amdgcn_bitop3_b32(und, X, pl, inv ? 0x60 : 0x90);                // und & ~(t* ^ pl)
    flip |= acc;
}
struct HbLanes {
    uint32_t ul, uh, fl, fh;  // undecided and flipped lanes, low and high halves
    HbClass cl, ch;
};
template <int C, int K>
__device__ __forceinline__ void hb_pair_case(HbLanes *s, const U4 *x) {
    constexpr int A4 = (C >> 3) & 1, A8 = (C >> 2) & 1, B4 = (C >> 1) & 1, B8 = C & 1;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        hb_plane_half<A4, A8>(s[k].ul, s[k].fl, s[k].cl.neg, s[k].cl.x4, x[k].x);
        hb_plane_half<A4, A8>(s[k].uh, s[k].fh, s[k].ch.neg, s[k].ch.x4, x[k].y);
        hb_plane_half<B4, B8>(s[k].ul, s[k].fl, s[k].cl.neg, s[k].cl.x4, x[k].z);
        hb_plane_half<B4, B8>(s[k].uh, s[k].fh, s[k].ch.neg, s[k].ch.x4, x[k].w);
    }
}
template <int K>
__device__ __forceinline__ void hb_pair(HbLanes *s, uint32_t T4, uint32_t T8, uint32_t p, const U4 *x) {
    const uint32_t sa = 31u - 2u * p, sb = 30u - 2u * p;
    const uint32_t c = (((T4 >> sa) & 1u) << 3) | (((T8 >> sa) & 1u) << 2) |
                       (((T4 >> sb) & 1u) << 1) | ((T8 >> sb) & 1u);
    switch (c) {
    case 0: hb_pair_case<0, K>(s, x); break;
    case 1: hb_pair_case<1, K>(s, x); break;
    case 2: hb_pair_case<2, K>(s, x); break;
    case 3: hb_pair_case<3, K>(s, x); break;
    case 4: hb_pair_case<4, K>(s, x); break;
    case 5: hb_pair_case<5, K>(s, x); break;
    case 6: hb_pair_case<6, K>(s, x); break;
    case 7: hb_pair_case<7, K>(s, x); break;
    case 8: hb_pair_case<8, K>(s, x); break;
    case 9: hb_pair_case<9, K>(s, x); break;
    case 10: hb_pair_case<10, K>(s, x); break;
    case 11: hb_pair_case<11, K>(s, x); break;
    case 12: hb_pair_case<12, K>(s, x); break;
    case 13: hb_pair_case<13, K>(s, x); break;
    case 14: hb_pair_case<14, K>(s, x); break;
    default: hb_pair_case<15, K>(s, x); break;
    }
}

// Tie thresholds on the fresh word v (its top 26 bits are the lane's low 26):
// dE > 0 flips iff (v >> 6) <= low26(T'), i.e. v < (low26(T') + 1) << 6;
// dE < 0 flips iff (v >> 6) <= 2^26 - 1 - low26(T'), i.e. v < (2^26 - low26(T')) << 6.
// A class whose bound would be 2^32 (low26(T') = 2^26 - 1 for dE > 0, 0 for
// dE < 0) never ties: equal top bits already decide it (hb_settle).
struct HbTie {
    uint32_t p4, n4, p8, n8;
};
__device__ __forceinline__ HbTie hb_tie_bounds(uint32_t T4, uint32_t T8) {
    const uint32_t l4 = T4 & 0x3FFFFFFu, l8 = T8 & 0x3FFFFFFu;
    return HbTie{(l4 + 1u) << 6, (0x4000000u - l4) << 6, (l8 + 1u) << 6, (0x4000000u - l8) << 6};
}
// Lanes still tied after six planes whose comparison those bits already
// decide (see HbTie) flip now; only needed when hb_needs_settle.
__device__ __forceinline__ bool hb_needs_settle(uint32_t T4, uint32_t T8) {
    const uint32_t l4 = T4 & 0x3FFFFFFu, l8 = T8 & 0x3FFFFFFu;
    return l4 == 0x3FFFFFFu || l4 == 0u || l8 == 0x3FFFFFFu || l8 == 0u;
}
__device__ __forceinline__ void hb_settle(uint64_t &und, uint64_t &flip, uint64_t mag4, uint64_t neg,
                                          uint32_t T4, uint32_t T8) {
    const uint32_t l4 = T4 & 0x3FFFFFFu, l8 = T8 & 0x3FFFFFFu;
    uint64_t sel = 0;
    if (l4 == 0x3FFFFFFu) sel |= mag4 & ~neg;
    if (l4 == 0u) sel |= mag4 & neg;
    if (l8 == 0x3FFFFFFu) sel |= ~mag4 & ~neg;
    if (l8 == 0u) sel |= ~mag4 & neg;
    sel &= und;
    flip |= sel;
    und &= ~sel;
}
__device__ __forceinline__ void hb_tie_one(uint64_t &und, uint64_t mag4, uint64_t neg, const HbTie &b,
                                           uint32_t v, uint64_t &flip) {
    const uint64_t bit = und & (0ull - und);  // lowest tied lane; 0 when none is left
    und ^= bit;
    const uint32_t mp4 = v < b.p4 ? ~0u : 0u, mn4 = v < b.n4 ? ~0u : 0u;
    const uint32_t mp8 = v < b.p8 ? ~0u : 0u, mn8 = v < b.n8 ? ~0u : 0u;
    uint32_t a[2];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
        const uint32_t m4 = (uint32_t)(mag4 >> (32 * hh)), ng = (uint32_t)(neg >> (32 * hh));
        const uint32_t ap = __builtin_amdgcn_bitop3_b32(m4, mp4, mp8, 0xCA);  // mag4 ? mp4 : mp8
        const uint32_t an = __builtin_amdgcn_bitop3_b32(m4, mn4, mn8, 0xCA);
        a[hh] = __builtin_amdgcn_bitop3_b32(ng, an, ap, 0xCA);
    }
    flip = ((uint64_t)(uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)(flip >> 32), (uint32_t)(bit >> 32),
                                                             a[1], 0xF8) << 32) |
           (uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)flip, (uint32_t)bit, a[0], 0xF8);
}
__device__ __forceinline__ void hb_tie_call(uint64_t &und, uint64_t mag4, uint64_t neg, const HbTie &b,
                                            const U4 &x, uint64_t &flip) {
    hb_tie_one(und, mag4, neg, b, x.x, flip);
    if (und == 0) return;
    hb_tie_one(und, mag4, neg, b, x.y, flip);
    if (und == 0) return;
    hb_tie_one(und, mag4, neg, b, x.z, flip);
    hb_tie_one(und, mag4, neg, b, x.w, flip);
}

// K words of one lane (as metropolis_words).  T4, T8: T'_4, T'_8; coin: beta
// = 0, where every move flips iff the top bit of u is 0; settle:
// hb_needs_settle(T4, T8) (uniform).  Calls are counted as in metropolis_word.
template <int K>
__device__ __forceinline__ void heatbath_words(const uint64_t (*nbr)[4], const uint64_t *s0,
                                               const uint64_t *valid, uint32_t T4, uint32_t T8,
                                               bool coin, bool settle, uint32_t k0, uint32_t k1,
                                               const uint32_t *w, const uint32_t *g, uint32_t h,
                                               uint64_t *flip, bool count, uint32_t *calls,
                                               uint32_t *wcalls) {
    HbLanes s[K];
    uint32_t zl[K], zh[K];  // dE = 0 lanes (every lane when coin), decided by plane 0
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint64_t a1 = s0[k] ^ nbr[k][0], a2 = s0[k] ^ nbr[k][1], a3 = s0[k] ^ nbr[k][2],
                       a4 = s0[k] ^ nbr[k][3];
        s[k].cl = hb_class((uint32_t)a1, (uint32_t)a2, (uint32_t)a3, (uint32_t)a4);
        s[k].ch = hb_class((uint32_t)(a1 >> 32), (uint32_t)(a2 >> 32), (uint32_t)(a3 >> 32),
                           (uint32_t)(a4 >> 32));
        const uint32_t vl = (uint32_t)valid[k], vh = (uint32_t)(valid[k] >> 32);
        zl[k] = coin ? vl : vl & s[k].cl.zero;
        zh[k] = coin ? vh : vh & s[k].ch.zero;
        s[k].ul = vl & ~zl[k];
        s[k].uh = vh & ~zh[k];
        s[k].fl = s[k].fh = 0;
    }
#pragma unroll
    for (uint32_t p = 0; p < kPlanePairs; ++p) {
        U4 x[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (count) {
                const uint32_t need = p == 0 ? (s[k].ul | s[k].uh | zl[k] | zh[k]) : (s[k].ul | s[k].uh);
                *wcalls += (uint32_t)__popcll(__ballot(need != 0));
            }
            x[k] = philox(k0, k1, w[k], g[k], h, kTagSweep | p);
            if (p == 0) {  // dE = 0: u < 2^31
                s[k].fl |= zl[k] & ~x[k].x;
                s[k].fh |= zh[k] & ~x[k].y;
            }
        }
        hb_pair<K>(s, T4, T8, p, x);
    }
    const HbTie tb = hb_tie_bounds(T4, T8);
    uint64_t und[K], mag4[K], neg[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        und[k] = ((uint64_t)s[k].uh << 32) | s[k].ul;
        flip[k] = ((uint64_t)s[k].fh << 32) | s[k].fl;
        mag4[k] = ((uint64_t)s[k].ch.mag4 << 32) | s[k].cl.mag4;
        neg[k] = ((uint64_t)s[k].ch.neg << 32) | s[k].cl.neg;
        if (settle) {
            // a real (uniform) branch: the compiler would otherwise evaluate
            // the rarely needed selection for every word
            asm volatile("");
            hb_settle(und[k], flip[k], mag4[k], neg[k], T4, T8);
        }
    }
    for (uint32_t q = 0;; ++q) {
        bool any = false;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            any |= und[k] != 0;
            *calls += und[k] != 0 ? 1u : 0u;  // read only when counting
        }
        if (!any) break;
        U4 x[K];
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] = philox(k0, k1, w[k], g[k], h, kTagTie | q);
#pragma unroll
        for (int k = 0; k < K; ++k) hb_tie_call(und[k], mag4[k], neg[k], tb, x[k], flip[k]);
    }
}

// The block's lattices in LDS carry a halo: group gl's site (x, y) is word
// gl A + (y + 1) P + x + 1 with row pitch P = L + 2 and A = (L + 2) P words
// per group, and the ghost columns x = -1, L and rows y = -1, L hold copies
// of the opposite edge (periodic boundaries), so that the four neighbours of
// every site sit at -1, +1, -P and +P.
struct Halo {
    int L, P, A;
    __device__ __forceinline__ int at(int gl, int x, int y) const { return gl * A + (y + 1) * P + x + 1; }
};
__device__ __forceinline__ Halo halo(int L) { return Halo{L, L + 2, (L + 2) * (L + 2)}; }

// Copy the edges of every group's lattice into its ghost cells: item k of
// ng 4L items copies edge site src into ghost dst.  A thread's items are fixed
// for the whole kernel; the first one is kept in registers (HaloItem), the
// rest (only when 4 L ng exceeds the block) are recomputed.
struct HaloItem {
    int src, dst;  // -1: none
};
__device__ __forceinline__ HaloItem halo_item(const Halo &hl, int k) {
    const int L = hl.L, gl = k / (4 * L), r = k - gl * 4 * L, side = r / L, t = r - side * L;
    if (side == 0) return HaloItem{hl.at(gl, L - 1, t), hl.at(gl, -1, t)};
    if (side == 1) return HaloItem{hl.at(gl, 0, t), hl.at(gl, L, t)};
    if (side == 2) return HaloItem{hl.at(gl, t, L - 1), hl.at(gl, t, -1)};
    return HaloItem{hl.at(gl, t, 0), hl.at(gl, t, L)};
}
__device__ __forceinline__ void fill_halo(uint64_t *lat, const Halo &hl, int ng, const HaloItem &mine) {
    if (mine.src >= 0) lat[mine.dst] = lat[mine.src];
    for (int k = threadIdx.x + blockDim.x; k < ng * 4 * hl.L; k += blockDim.x) {
        const HaloItem it = halo_item(hl, k);
        lat[it.dst] = lat[it.src];
    }
}

// Incremental walk over the words idx, idx + nt, ... of one colour: half-column
// xh = idx mod L/2 and global row r = idx div L/2 = gl L + y, kept as (xh, y,
// gl, row = the halo index of (0, y) in group gl) and advanced by nt words
// with one carry each, so that no division is needed per word.
struct WordWalk {
    int xh, y, gl, row;
};
struct WalkStep {
    int half, L, P, dxh, dy, dgl, drow, wrap;  // stride = (dgl L + dy) half + dxh; half = units per row
};
// units = positions per row: L/2 for the words of one colour (and for pairs of
// sites), L for single sites (then xh is the column)
__device__ __forceinline__ WalkStep walk_step(int nt, const Halo &hl, int units) {
    const int dr = nt / units, dy = dr % hl.L, dgl = dr / hl.L;
    return WalkStep{units, hl.L, hl.P, nt - dr * units, dy, dgl, dgl * hl.A + dy * hl.P,
                    hl.A - hl.L * hl.P};
}
__device__ __forceinline__ WalkStep walk_step(int nt, const Halo &hl) { return walk_step(nt, hl, hl.L >> 1); }
__device__ __forceinline__ WordWalk walk_start(int idx, const Halo &hl, int units) {
    const int r = idx / units, y = r % hl.L, gl = r / hl.L;
    return WordWalk{idx - r * units, y, gl, hl.at(gl, 0, y)};
}
__device__ __forceinline__ WordWalk walk_start(int idx, const Halo &hl) { return walk_start(idx, hl, hl.L >> 1); }
__device__ __forceinline__ void walk_advance(WordWalk &w, const WalkStep &s) {
    w.xh += s.dxh;
    const int c = w.xh >= s.half ? 1 : 0;
    w.xh -= c ? s.half : 0;
    w.row += s.drow + (c ? s.P : 0);
    w.y += s.dy + c;
    w.gl += s.dgl;
    if (w.y >= s.L) {
        w.y -= s.L;
        w.gl += 1;
        w.row += s.wrap;
    }
}

// walk_advance when the stride is a whole number of rows (dxh == 0)
__device__ __forceinline__ void walk_advance_rows(WordWalk &w, const WalkStep &s) {
    w.row += s.drow;
    w.y += s.dy;
    w.gl += s.dgl;
    if (w.y >= s.L) {
        w.y -= s.L;
        w.gl += 1;
        w.row += s.wrap;
    }
}

// Bit-sliced counters for the measurement: plane k holds bit k of the 64
// replicas' counts (one 32-bit half per array).  add() takes the two bond
// bits and the spin bit of one site word: a full adder puts the two bond bits
// into the units plane and the carries ripple upwards.  kMeasSites sites per
// thread keep the bond count <= 16 (5 planes) and the up count <= 8 (4).
constexpr int kMeasSites = 8;
constexpr int kPlanesU = 5, kPlanesM = 4;

__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
}

template <int K>
__device__ __forceinline__ void ripple(uint32_t (&P)[K], uint32_t c, int from) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (k >= from) {
            const uint32_t t = P[k] & c;
            P[k] ^= c;
            c = t;
        }
    }
}

// Sum over the wavefront of a K-plane counter pair (lo: replicas 0..31, hi:
// replicas 32..63), as a reduce-scatter: the first exchange, between lanes 32
// apart, hands each lane its partner's copy of the half it keeps (lanes 0..31
// the low half, lanes 32..63 the high one), so the five butterfly levels that
// follow add one 32-bit half per lane instead of two.  After them every lane of
// a 32-lane group holds its half's sum over all 64 lanes in K + 6 planes;
// returns bit lane mod 32 of it, the count of replica `lane`.
template <int K>
__device__ __forceinline__ int wave_count(const uint32_t (&lo)[K], const uint32_t (&hi)[K], int lane) {
    const bool upper = lane >= 32;
    uint32_t a[K + 6];
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint32_t mine = upper ? hi[k] : lo[k];
        const uint32_t b = __shfl_xor(upper ? lo[k] : hi[k], 32, 64);
        const uint32_t sum = mine ^ b ^ c;
        c = maj3(mine, b, c);
        a[k] = sum;
    }
    a[K] = c;
#pragma unroll
    for (int k = K + 1; k < K + 6; ++k) a[k] = 0u;
#pragma unroll
    for (int lev = 1; lev < 6; ++lev) {
        const int off = 32 >> lev;
        c = 0;
#pragma unroll
        for (int k = 0; k < K + lev; ++k) {
            const uint32_t b = __shfl_xor(a[k], off, 64);
            const uint32_t sum = a[k] ^ b ^ c;
            c = maj3(a[k], b, c);
            a[k] = sum;
        }
        a[K + lev] = c;
    }
    const int sh = lane & 31;
    int n = 0;
#pragma unroll
    for (int k = 0; k < K + 6; ++k) n |= (int)((a[k] >> sh) & 1u) << k;
    return n;
}

struct MeasCounters {
    uint32_t ul[kPlanesU] = {}, uh[kPlanesU] = {}, ml[kPlanesM] = {}, mh[kPlanesM] = {};
    __device__ __forceinline__ void add(uint64_t a, uint64_t b, uint64_t s) {
        const uint32_t al = (uint32_t)a, ah = (uint32_t)(a >> 32);
        const uint32_t bl = (uint32_t)b, bh = (uint32_t)(b >> 32);
        uint32_t c = maj3(ul[0], al, bl);
        ul[0] = ul[0] ^ al ^ bl;
        ripple(ul, c, 1);
        c = maj3(uh[0], ah, bh);
        uh[0] = uh[0] ^ ah ^ bh;
        ripple(uh, c, 1);
        ripple(ml, (uint32_t)s, 0);
        ripple(mh, (uint32_t)(s >> 32), 0);
    }
    __device__ __forceinline__ void wave_totals(int lane, int *U, int *up) const {
        *U = wave_count<kPlanesU>(ul, uh, lane);
        *up = wave_count<kPlanesM>(ml, mh, lane);
    }
};

// One block per (run, gpb consecutive groups): the groups' L x L x 64
// lattices live in LDS (with a halo, see Halo) for all theta sweeps (colour 0
// then colour 1; a site's index within its colour w = y L/2 + floor(x/2) and
// the global half-sweep index h = 2 (theta (i-1) + sweep) + colour key its
// random bits).  Each word's whole comparison runs in one lane; a thread walks
// the words tid, tid + nt, ... of a colour.  After each half-sweep the ghost
// cells are refreshed.  Afterwards each replica's E = 2U - 2N (U antiparallel
// bonds) and M are measured.  With init != 0 no sweep is done.
// WALK: kWalkAny (general incremental walk), kWalkRows (the stride nt is a
// whole number of rows), kWalkOneGroup (also one group per block: a thread's
// column is fixed, its LDS index advances by a constant and its word index in
// the colour is the loop index).
constexpr int kMaxGroupsPerBlock = 8;
constexpr int kWalkAny = 0, kWalkRows = 1, kWalkOneGroup = 2;

// One word update of either rule (Metropolis, or heatbath when UPD; for
// heatbath all4 is the beta = 0 flag and all8 the settle flag).
template <int UPD>
__device__ __forceinline__ uint64_t update_word(uint64_t s0, uint64_t n0, uint64_t n1, uint64_t n2,
                                                uint64_t n3, uint64_t valid, uint32_t T4, uint32_t T8,
                                                bool all4, bool all8, uint32_t k0, uint32_t k1,
                                                uint32_t w, uint32_t g, uint32_t h, bool count,
                                                uint32_t *calls, uint32_t *wcalls) {
    if (UPD == PA_UPDATE_HEATBATH) {
        const uint64_t nbr[1][4] = {{n0, n1, n2, n3}};
        uint64_t f;
        heatbath_words<1>(nbr, &s0, &valid, T4, T8, all4, all8, k0, k1, &w, &g, h, &f, count, calls,
                          wcalls);
        return f;
    }
    return metropolis_word(s0 ^ n0, s0 ^ n1, s0 ^ n2, s0 ^ n3, valid, T4, T8, all4, all8, k0, k1, w, g,
                           h, count, calls, wcalls);
}

template <int LAYOUT, int WALK, int ILP, int UPD, int COUNT>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(ILP == 1 ? 8 : 4)))
k_sweep(const RunDesc *runs, WorkMap map, int init, int gpb) {
    extern __shared__ uint64_t lat[];
    __shared__ int32_t red_u[kMaxGroupsPerBlock * kLanes], red_up[kMaxGroupsPerBlock * kLanes];
    int bi;
    const RunDesc &rd = runs[map_block(map, blockIdx.x, &bi)];
    RunState *st = rd.st;
    if (rd.layout != LAYOUT || rd.update != UPD || st->err) return;
    const int Rn = st->R_new;
    const int g0 = bi * gpb;
    if (g0 * kLanes >= Rn) return;
    const int ng = min(gpb, (Rn + kLanes - 1) / kLanes - g0);  // groups with live replicas
    const int L = rd.L, N = rd.N, half = L >> 1, nb = st->cur ^ 1;
    const int tid = threadIdx.x, nt = blockDim.x;
    const Halo hl = halo(L);

    // stage the lattices in LDS: 16-byte loads (two words of one row), several
    // in flight per thread; pair w = (row, half-column) is walked like a word
    // of one colour (L is even: a pair never crosses a row)
    const WalkStep step = walk_step(nt, hl);
    if (LAYOUT == PA_LAYOUT_MSC64) {
        const gptr<const u32x4> src = global(reinterpret_cast<const u32x4 *>(rd.ms[nb] + (size_t)g0 * N));
        const int n2 = ng * N / 2;
        WordWalk wk = walk_start(tid, hl);
#pragma unroll 4
        for (int w = tid; w < n2; w += nt) {
            const u32x4 v = src[w];
            const int q = wk.row + 2 * wk.xh;
            lat[q] = ((uint64_t)v.y << 32) | v.x;
            lat[q + 1] = ((uint64_t)v.w << 32) | v.z;
            walk_advance(wk, step);
        }
    } else {
        // one site (64 bytes, four 16-byte loads) per thread and step
        const gptr<const u32x4> src = global(reinterpret_cast<const u32x4 *>(rd.s8[nb] + (size_t)g0 * N * kLanes));
        const WalkStep sstep = walk_step(nt, hl, L);
        WordWalk wk = walk_start(tid, hl, L);
#pragma unroll 2
        for (int e = tid; e < ng * N; e += nt) {
            uint64_t w = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const u32x4 v = src[4 * e + k];
                w |= (uint64_t)pack16(uint4{v.x, v.y, v.z, v.w}) << (16 * k);
            }
            lat[wk.row + wk.xh] = w;
            walk_advance(wk, sstep);
        }
    }
    const HaloItem mine = tid < ng * 4 * L ? halo_item(hl, tid) : HaloItem{-1, -1};
    for (int k = tid; k < ng * kLanes; k += nt) {
        red_u[k] = 0;
        red_up[k] = 0;
    }
    __syncthreads();
    fill_halo(lat, hl, ng, mine);
    __syncthreads();

    const int theta = init ? 0 : rd.theta;
    const int i = st->step + 1;
    const uint64_t t4 = st->t4, t8 = st->t8;
    // heatbath: all4 marks beta = 0 (fair coins) and all8 the settle flag
    const bool all4 = t4 >= (1ull << 32);
    const bool all8 = UPD == PA_UPDATE_HEATBATH ? hb_needs_settle((uint32_t)t4, (uint32_t)t8)
                                                : t8 >= (1ull << 32);
    // the thresholds are the same for every lane: keep their bits in scalar registers
    const uint32_t T4 = __builtin_amdgcn_readfirstlane((uint32_t)t4);
    const uint32_t T8 = __builtin_amdgcn_readfirstlane((uint32_t)t8);
    const int words = ng * (N >> 1);  // sites of one colour, all groups of the block
    const uint64_t last_valid = lane_mask(Rn - (g0 + ng - 1) * kLanes);
    const int P = hl.P;
    const uint32_t k0 = rd.key0, k1 = rd.key1;
    constexpr bool count = COUNT != 0;  // profiling builds of the kernel count Philox calls
    // kWalkOneGroup: the thread's column xh1, first row y1 and row stride dy1
    const int y1 = tid / half, xh1 = tid - y1 * half, dy1 = nt / half, dsite1 = dy1 * P;
    uint32_t calls = 0, wcalls = 0;
    for (int s = 0; s < theta; ++s) {
        for (int colour = 0; colour < 2; ++colour) {
            const uint32_t h = 2u * ((uint32_t)theta * (uint32_t)(i - 1) + (uint32_t)s) + (uint32_t)colour;
            WordWalk wk = walk_start(tid, hl);
            // next row of this thread's column (kWalkOneGroup): with dy1 odd the
            // site alternates between the two columns 2 xh1 and 2 xh1 + 1
            const int par1 = (colour + y1) & 1;
            int site1 = hl.at(0, 2 * xh1 + par1, y1), dlt1 = dsite1 + ((dy1 & 1) ? 1 - 2 * par1 : 0);
            auto advance1 = [&]() {
                site1 += dlt1;
                dlt1 = 2 * dsite1 - dlt1;
            };
            if (ILP == 1 && WALK == kWalkOneGroup) {
                for (int w = tid; w < words; w += nt) {
                    const int site = site1;
                    const uint64_t s0 = lat[site];
                    const uint64_t f = update_word<UPD>(s0, lat[site + 1], lat[site - 1], lat[site - P],
                                                        lat[site + P], last_valid, T4, T8, all4, all8,
                                                        k0, k1, (uint32_t)w, (uint32_t)g0, h, count,
                                                        &calls, &wcalls);
                    lat[site] = s0 ^ f;
                    advance1();
                }
            } else if (ILP == 1) {
                for (int idx = tid; idx < words; idx += nt) {
                    const int x = 2 * wk.xh + ((colour + wk.y) & 1);
                    const int site = wk.row + x;
                    const uint64_t s0 = lat[site];
                    const uint64_t valid = wk.gl == ng - 1 ? last_valid : ~0ull;
                    const uint64_t f = update_word<UPD>(s0, lat[site + 1], lat[site - 1], lat[site - P],
                                                        lat[site + P], valid, T4, T8, all4, all8, k0,
                                                        k1, (uint32_t)(wk.y * half + wk.xh),
                                                        (uint32_t)(g0 + wk.gl), h, count, &calls,
                                                        &wcalls);
                    lat[site] = s0 ^ f;
                    if (WALK == kWalkRows)
                        walk_advance_rows(wk, step);
                    else
                        walk_advance(wk, step);
                }
            } else {
                // the thread's words idx, idx + nt, ... taken ILP at a time
                for (int idx = tid; idx < words; idx += ILP * nt) {
                    int site[ILP];
                    uint64_t s0[ILP], nbr[ILP][4], valid[ILP], f[ILP];
                    uint32_t wi[ILP], gi[ILP];
#pragma unroll
                    for (int k = 0; k < ILP; ++k) {
                        const bool live = k == 0 || idx + k * nt < words;
                        if (WALK == kWalkOneGroup) {
                            site[k] = site1;
                            valid[k] = live ? last_valid : 0ull;
                            wi[k] = (uint32_t)(idx + k * nt);
                            gi[k] = (uint32_t)g0;
                            advance1();
                        } else {
                            site[k] = wk.row + 2 * wk.xh + ((colour + wk.y) & 1);
                            valid[k] = !live ? 0ull : (wk.gl == ng - 1 ? last_valid : ~0ull);
                            wi[k] = (uint32_t)(wk.y * half + wk.xh);
                            gi[k] = (uint32_t)(g0 + wk.gl);
                            if (WALK == kWalkRows)
                                walk_advance_rows(wk, step);
                            else
                                walk_advance(wk, step);
                        }
                        if (!live) site[k] = site[0];  // past the last word: a dummy with no lanes
                        s0[k] = lat[site[k]];
                        nbr[k][0] = lat[site[k] + 1];
                        nbr[k][1] = lat[site[k] - 1];
                        nbr[k][2] = lat[site[k] - P];
                        nbr[k][3] = lat[site[k] + P];
                    }
                    if (UPD == PA_UPDATE_HEATBATH)
                        heatbath_words<ILP>(nbr, s0, valid, T4, T8, all4, all8, k0, k1, wi, gi, h, f,
                                            count, &calls, &wcalls);
                    else
                        metropolis_words<ILP>(nbr, s0, valid, T4, T8, all4, all8, k0, k1, wi, gi, h, f,
                                              count, &calls, &wcalls);
#pragma unroll
                    for (int k = 0; k < ILP; ++k)
                        if (f[k]) lat[site[k]] = s0[k] ^ f[k];
                }
            }
            __syncthreads();
            fill_halo(lat, hl, ng, mine);
            __syncthreads();
        }
    }

    // measurement: every thread counts, for its sites of one group, the
    // antiparallel right and down bonds and the up spins of the group's 64
    // replicas in bit-sliced counters; the wavefront then sums its 64 threads'
    // counters (bit-plane butterfly) and lane r adds replica r's totals.
    {
        const int lane = tid & 63;
        const int dy = nt / L, dx = nt - dy * L;
        for (int gl = 0; gl < ng; ++gl) {
            int y = tid / L, x = tid - (tid / L) * L;
            for (int c0 = 0; c0 < N; c0 += kMeasSites * nt) {  // same trip count in every thread
                MeasCounters mc;
#pragma unroll
                for (int j = 0; j < kMeasSites; ++j) {
                    if (c0 + j * nt + tid < N) {
                        const int q = hl.at(gl, x, y);
                        const uint64_t w0 = lat[q];
                        mc.add(w0 ^ lat[q + 1], w0 ^ lat[q + P], w0);
                    }
                    x += dx;
                    y += dy;
                    if (x >= L) {
                        x -= L;
                        ++y;
                    }
                }
                int U, up;
                mc.wave_totals(lane, &U, &up);
                atomicAdd(&red_u[gl * kLanes + lane], U);
                atomicAdd(&red_up[gl * kLanes + lane], up);
            }
        }
    }
    if (count && theta > 0) {  // Philox calls of this block (one atomic per wave)
        const uint64_t c64 = (uint64_t)wave_sum_i64((int64_t)calls) + wcalls;
        if ((tid & 63) == 0) atomicAdd(&st->philox_calls, (unsigned long long)c64);
        if (tid == 0) atomicAdd(&st->sweep_words, (unsigned long long)theta * (unsigned long long)N * ng);
    }
    __syncthreads();
    for (int k = tid; k < ng * kLanes; k += nt) {
        const int c = g0 * kLanes + k;
        if (c < Rn) {
            rd.E[c] = 2 * red_u[k] - 2 * N;
            rd.M[c] = 2 * red_up[k] - N;
        }
    }
    if (theta > 0) {
        if (LAYOUT == PA_LAYOUT_MSC64) {
            const gptr<u32x4> dst = global(reinterpret_cast<u32x4 *>(rd.ms[nb] + (size_t)g0 * N));
            WordWalk wk = walk_start(tid, hl);
            for (int w = tid; w < ng * N / 2; w += nt) {
                const int q = wk.row + 2 * wk.xh;
                const uint64_t a = lat[q], b = lat[q + 1];
                dst[w] = u32x4{(uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32)};
                walk_advance(wk, step);
            }
        } else {
            const gptr<u32x4> dst = global(reinterpret_cast<u32x4 *>(rd.s8[nb] + (size_t)g0 * N * kLanes));
            const WalkStep sstep = walk_step(nt, hl, L);
            WordWalk wk = walk_start(tid, hl, L);
            for (int e = tid; e < ng * N; e += nt) {
                const uint64_t w = lat[wk.row + wk.xh];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint4 v = unpack16((uint32_t)(w >> (16 * k)) & 0xFFFFu);
                    dst[4 * e + k] = u32x4{v.x, v.y, v.z, v.w};
                }
                walk_advance(wk, sstep);
            }
        }
    }
}

// ------------------------------------------------------------------ reduction + record

// Population sums over the R_i replicas and family statistics from the
// tree-ordered labels: families are contiguous runs of equal labels.  Each
// block of kSlotBlock slots finds its runs (a block max-scan of the run starts)
// and sums f, sum len^2 and sum len ln len over the runs that lie inside it;
// a run that crosses the block's first or last slot is reported as a portion
// (first_len / last_len with continuation flags) for record_run to stitch.  The
// block also adds its slots to the energy histogram that the next step's
// k_norm reads.  Partials go to part[b*8 + k] (k = 0..7) and partd[b*2].
constexpr int64_t kRunContPrev = 1ll << 32, kRunContNext = 1ll << 33, kRunSingle = 1ll << 34;

__device__ void record_run(const RunDesc &rd);

__global__ void __launch_bounds__(256) k_reduce(const RunDesc *runs, WorkMap map) {
    int b;
    const RunDesc &rd = runs[map_block(map, blockIdx.x, &b)];
    RunState *st = rd.st;
    // the energies and magnetisations of this thread's four slots (up to the
    // capacity) load alongside the run's state; the slots past R_i are unused
    int32_t e_pre[4] = {0, 0, 0, 0}, m_pre[4] = {0, 0, 0, 0};
    {
        const int c = b * kSlotBlock + 4 * (int)threadIdx.x;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            if (c + m < rd.C) {
                e_pre[m] = rd.E[c + m];
                m_pre[m] = rd.M[c + m];
            }
        }
    }
    if (st->err) return;
    __shared__ int64_t shv[4][6];
    __shared__ double shd[4];
    __shared__ int wmax[16];
    __shared__ int64_t edge[2];
    __shared__ int64_t bsum[kBlocks * 4];  // blocking sums of the blocks this block touches
    const int Rn = st->R_new, nb = st->cur ^ 1;
    const int32_t *fam = rd.fam[nb];
    const int j0 = b * kSlotBlock, j1 = min(j0 + kSlotBlock, Rn);
    const bool cont_prev = j0 > 0 && j0 < Rn && fam[j0 - 1] == fam[j0];
    const bool cont_next = j1 > j0 && j1 < Rn && fam[j1] == fam[j1 - 1];
    if (threadIdx.x == 0) {
        edge[0] = 0;
        edge[1] = 0;
    }
    // blocking (Sec. "Effective population size", Eq. blocks): slot j lies in
    // block floor(((j + 1) n - 1) / R_i) of n = min(kBlocks, R_i) (the quotient of
    // two integers below 2^53, at least 1/R_i away from the next integer unless
    // it is one, so its binary64 floor is exact); this block's slots [j0, j1)
    // touch blocks kb0 .. kb1
    const int nbk = min(kBlocks, Rn);
    auto block_of = [&](int j) { return (int)floor((double)((int64_t)(j + 1) * nbk - 1) / (double)Rn); };
    const int kb0 = j1 > j0 ? block_of(j0) : 0, kb1 = j1 > j0 ? block_of(j1 - 1) : -1;
    for (int k = threadIdx.x; k < 4 * (kb1 - kb0 + 1); k += blockDim.x) bsum[k] = 0;
    // each thread owns 4 consecutive slots
    const int c0 = j0 + 4 * (int)threadIdx.x;
    int last_start = -1;  // start of the run containing the thread's last slot, within the thread
    bool is_start[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int c = c0 + m;
        is_start[m] = c < j1 && (c == j0 || fam[c - 1] != fam[c]);
        if (is_start[m]) last_start = c;
    }
    // exclusive max-scan of last_start over threads gives the run start entering each thread
    int x = last_start;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x = max(x, y);
    }
    if (lane == 63) wmax[wave] = x;
    __syncthreads();
    int prev = -1;
    for (int w = 0; w < wave; ++w) prev = max(prev, wmax[w]);
    const int up = __shfl_up(x, 1, 64);
    if (lane > 0) prev = max(prev, up);
    int64_t sE = 0, sE2 = 0, sM = 0, sM2 = 0, f = 0, s2 = 0;
    double cl = 0.0;
    int run_start = prev;
    int lev[4] = {-1, -1, -1, -1};  // energy levels of the slots, for the histogram
    int64_t ev[4] = {0, 0, 0, 0}, av[4] = {0, 0, 0, 0};  // E and |M| of the slots
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int c = c0 + m;
        if (c >= j1) break;
        if (is_start[m]) run_start = c;
        const int64_t e = e_pre[m], mm = m_pre[m];
        lev[m] = (int)((e + 2 * rd.N) >> 2);
        ev[m] = e;
        av[m] = mm < 0 ? -mm : mm;
        sE += e;
        sE2 += e * e;
        sM += mm < 0 ? -mm : mm;
        sM2 += mm * mm;
        if (c == j1 - 1 || fam[c + 1] != fam[c]) {  // a run ends at c
            const int64_t len = c - run_start + 1;
            const bool first = run_start == j0, last = c == j1 - 1;
            if ((first && cont_prev) || (last && cont_next)) {
                if (first) edge[0] = len | (cont_prev ? kRunContPrev : 0) |
                                     (cont_next ? kRunContNext : 0) | (last ? kRunSingle : 0);
                if (last) edge[1] = len;
            } else {
                f += 1;
                s2 += len * len;
                cl += (double)len * log((double)len);
            }
        }
    }
    {  // the thread's slots into the LDS blocking sums (one group of adds per block met)
        int kcur = -1;
        int64_t t[4] = {0, 0, 0, 0};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            if (lev[m] < 0) continue;
            const int k = block_of(c0 + m);
            if (k != kcur) {
                if (kcur >= 0)
                    for (int q = 0; q < 4; ++q) atomicAdd(reinterpret_cast<unsigned long long *>(&bsum[4 * (kcur - kb0) + q]), (unsigned long long)t[q]);
                kcur = k;
                t[0] = t[1] = t[2] = t[3] = 0;
            }
            t[0] += ev[m];
            t[1] += ev[m] * ev[m];
            t[2] += av[m];
            t[3] += av[m] * av[m];
        }
        if (kcur >= 0)
            for (int q = 0; q < 4; ++q) atomicAdd(reinterpret_cast<unsigned long long *>(&bsum[4 * (kcur - kb0) + q]), (unsigned long long)t[q]);
    }
    const int64_t v[6] = {sE, sE2, sM, sM2, f, s2};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int64_t t = wave_sum_i64(v[k]);
        if (lane == 0) shv[wave][k] = t;
    }
    const double tcl = wave_sum_f64(cl);
    if (lane == 0) shd[wave] = tcl;
    __syncthreads();
    if (threadIdx.x < 6) {
        int64_t t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += shv[w][threadIdx.x];
        rd.part[b * 8 + threadIdx.x] = t;
    } else if (threadIdx.x == 6) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += shd[w];
        rd.partd[b * 2] = t;
    } else if (threadIdx.x == 7) {
        // a first run that continues from the previous block but not past this
        // one is marked in edge[0]; an open last run in edge[1]
        rd.part[b * 8 + 6] = edge[0] | (cont_next ? kRunContNext : 0) | (cont_prev ? kRunContPrev : 0);
        rd.part[b * 8 + 7] = edge[1];
    }
    // the blocking sums to blk[] (integer atomics: the totals do not depend on the order)
    for (int k = threadIdx.x; k < 4 * (kb1 - kb0 + 1); k += blockDim.x)
        if (bsum[k]) atomicAdd(reinterpret_cast<unsigned long long *>(&rd.blk[4 * kb0 + k]), (unsigned long long)bsum[k]);
    block_histogram(rd, st, lev);
    // the run's last block to finish writes the record: every block publishes
    // its partials (release fence) before it counts itself done, and the last
    // one reads them all after an acquire fence
    __shared__ int last_sh;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last_sh = atomicAdd(&st->reduce_done, 1) == rd.nblk - 1;
    }
    __syncthreads();
    if (!last_sh) return;
    __threadfence();
    record_run(rd);
    if (threadIdx.x == 0) st->reduce_done = 0;
}

// The last k_reduce block of a run: combine the partials of all its blocks,
// write record i (Sec. "Model and observables" with N -> R_i; Eqs. rhot, rhos,
// one-step-Reff) and make the new population current.
__device__ void record_run(const RunDesc &rd) {
    RunState *st = rd.st;
    __shared__ int64_t sh[16 * 6];
    __shared__ double shd[32];
    const int Rn = st->R_new, nb = st->cur ^ 1;
    const int nblk = (Rn + kSlotBlock - 1) / kSlotBlock;
    // Everything the record reads from the run's state and schedule, loaded
    // before the first barrier so that the latencies overlap those of the
    // blocks' partials (none of it changes during the reduction).
    const int step = st->step + 1;
    const double beta = rd.betas[step];
    const int Rp = st->R_cur;  // the parents of this step
    const double S = st->s_hi + st->s_lo;
    const dd acc_prev{st->acc_hi, st->acc_lo}, lnq{st->lnq_hi, st->lnq_lo};
    const int64_t sum_cnt2 = st->sum_cnt2;
    const int nF = min(kBlocks, rd.R);
    double jkF_own = 0.0, jkw_own = 0.0;
    __shared__ double jw[kBlocks];  // the blocks' weight sums, for the complements below
    if ((int)threadIdx.x < nF) {
        jkF_own = st->jk_F[threadIdx.x];
        jkw_own = rd.jkw[threadIdx.x];
        jw[threadIdx.x] = jkw_own;
    }
    // thread k < n: the blocking sums of block k (used below), cleared for the next step
    const int nbk = min(kBlocks, Rn);
    const bool own = (int)threadIdx.x < nbk;
    int64_t bs[4] = {0, 0, 0, 0}, Bk = 0;
    if (own) {
        for (int q = 0; q < 4; ++q) bs[q] = rd.blk[4 * threadIdx.x + q];
        for (int q = 0; q < 4; ++q) rd.blk[4 * threadIdx.x + q] = 0;
        Bk = (int64_t)(threadIdx.x + 1) * Rn / nbk - (int64_t)threadIdx.x * Rn / nbk;
    }
    // runs that cross block boundaries: every block in which such a run ends
    // walks back over the blocks it spans (each lies wholly inside the run)
    // to the block where it started, and adds its length
    // T[0..5]: the partial fields; families, sum len^2 and sum len ln len also
    // take the crossing runs (one pass)
    int64_t T[6] = {0, 0, 0, 0, 0, 0};
    double c = 0.0;
    for (int k = threadIdx.x; k < nblk; k += blockDim.x) {
#pragma unroll
        for (int q = 0; q < 6; ++q) T[q] += rd.part[k * 8 + q];
        c += rd.partd[k * 2];
    }
    for (int k = threadIdx.x; k < nblk; k += blockDim.x) {
        const int64_t e0 = rd.part[k * 8 + 6];
        const bool cp = (e0 & kRunContPrev) != 0, cn = (e0 & kRunContNext) != 0;
        const bool single = (e0 & kRunSingle) != 0;
        if (!cp || (single && cn)) continue;  // no crossing run ends here
        int64_t len = e0 & 0xFFFFFFFFll;
        for (int q = k - 1; q >= 0; --q) {
            const int64_t eq = rd.part[q * 8 + 6];
            if ((eq & kRunSingle) && (eq & kRunContPrev)) {
                len += eq & 0xFFFFFFFFll;
            } else {
                len += rd.part[q * 8 + 7];
                break;
            }
        }
        T[4] += 1;
        T[5] += len * len;
        c += (double)len * log((double)len);
    }
    block_sum_i64v(T, sh);
    const double TCL = block_sum_f64(c, shd);
    const double Nd = (double)rd.N;

    // blocking and jackknife (Sec. "Effective population size", Eqs. blocks,
    // blocked_variance, neff, jackknife-blocks, jackknife-variance; Sec.
    // "Statistical errors"): thread k < n holds block k's sums (loaded above): its
    // means of E and |M|, and c_v and chi of the jackknife sample without block k,
    // whose variances n_k^2 Var come from exact integers (n_k = R_i - B_k
    // replicas).  Each enters as its difference d from the value of the whole
    // population, so that sum (x - mean x)^2 = sum d^2 - (sum d)^2 / n is formed
    // from small numbers in one pass.
    // free-energy jackknife (Sec. "Conclusions", last guideline; Eqs.
    // free-emergy-estimator, jackknife-variance, bias_covariance): thread k < n_F
    // adds this step's ln Q^(k) - ln Q to its running sum D_k; sample k of
    // beta F is beta F - D_k
    __shared__ int64_t tot_sh[4];
    __shared__ double bdev[kBlocks][16], dsum[16], dF[kBlocks];
    if ((int)threadIdx.x < nF) {
        const int k = threadIdx.x;
        double D = jkF_own;
        if (step > 0) {
            const int64_t lo = (int64_t)k * Rp / nF, hi = (int64_t)(k + 1) * Rp / nF;
            // ln of the weight outside block k over the total: log1p(-W_k / S),
            // except where the block holds most of the weight, where 1 - W_k / S
            // would cancel and the other blocks' own sum is taken instead (a
            // block holding all but e^-20 of it would otherwise lose 7 digits)
            const double x = jkw_own / S;
            double lw;
            if (x <= 0.5) {
                lw = log1p(-x);
            } else {
                double rest = 0.0, all = 0.0;
                for (int j = 0; j < nF; ++j) {
                    all += jw[j];
                    if (j != k) rest += jw[j];
                }
                lw = log(rest / all);
            }
            D += hi - lo == Rp ? __builtin_nan("") : lw - log1p(-(double)(hi - lo) / (double)Rp);
            st->jk_F[k] = D;
        }
        dF[k] = D;
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 4; ++q) tot_sh[q] = T[q];
    // mean of the D_k (fixed-order block sum, broadcast through LDS)
    __shared__ double dbar_sh;
    {
        const double t = block_sum_f64((int)threadIdx.x < nF ? dF[threadIdx.x] : 0.0, shd);
        if (threadIdx.x == 0) dbar_sh = t / nF;
    }
    __syncthreads();
    const double Dbar = dbar_sh;
    const double Rd = (double)Rn;
    const double whole[4] = {
        (double)tot_sh[0] / Rd, (double)tot_sh[2] / Rd,
        beta * beta / Nd * ((double)((__int128)Rn * tot_sh[1] - (__int128)tot_sh[0] * tot_sh[0]) / (Rd * Rd)),
        beta / Nd * ((double)((__int128)Rn * tot_sh[3] - (__int128)tot_sh[2] * tot_sh[2]) / (Rd * Rd))};
    if (own) {  // d and d^2 for E, |M|, c_v, chi
        const int k = threadIdx.x;
        const int64_t nk = Rn - Bk;
        const int64_t r1 = tot_sh[0] - bs[0], r2 = tot_sh[1] - bs[1];
        const int64_t q1 = tot_sh[2] - bs[2], q2 = tot_sh[3] - bs[3];
        const double nk2 = (double)nk * (double)nk;
        const double x[4] = {
            (double)bs[0] / (double)Bk, (double)bs[2] / (double)Bk,
            beta * beta / Nd * ((double)((__int128)nk * r2 - (__int128)r1 * r1) / nk2),
            beta / Nd * ((double)((__int128)nk * q2 - (__int128)q1 * q1) / nk2)};
        for (int q = 0; q < 4; ++q) {
            const double d = x[q] - whole[q];
            bdev[k][2 * q] = d;
            bdev[k][2 * q + 1] = d * d;
        }
        // jackknife samples of e and m less the whole population's value:
        // (T B_k - R b_k) / (R (R - B_k) N), b_k the block's sum
        const double den = Rd * (double)nk * Nd;
        const double ej = (double)((__int128)tot_sh[0] * Bk - (__int128)Rn * bs[0]) / den;
        const double mj = (double)((__int128)tot_sh[2] * Bk - (__int128)Rn * bs[2]) / den;
        // deviation of sample k of beta F from the samples' mean
        const double db = k < nF ? -(dF[k] - Dbar) : 0.0;
        bdev[k][8] = ej;
        bdev[k][9] = ej * db;
        bdev[k][10] = mj;
        bdev[k][11] = mj * db;
        bdev[k][12] = bdev[k][4] * db;
        bdev[k][13] = bdev[k][6] * db;
    }
    if ((int)threadIdx.x < nF) {
        const double db = -(dF[threadIdx.x] - Dbar);
        bdev[threadIdx.x][14] = db * db;
    }
    __syncthreads();
    {  // sums over the blocks: 16 strided partial sums per column, then their sum (fixed order)
        __shared__ double cpart[16][16];
        const int col = threadIdx.x & 15, part = threadIdx.x >> 4;
        const int n = col == 14 ? nF : nbk;
        double t = 0.0;
        for (int k = part; k < n; k += 16) t += bdev[k][col];
        cpart[part][col] = t;
        __syncthreads();
        if (threadIdx.x < 16) {
            double u = 0.0;
            for (int q = 0; q < 16; ++q) u += cpart[q][threadIdx.x];
            dsum[threadIdx.x] = u;
        }
    }
    __syncthreads();
    double ss[4];  // sums of squared deviations from the means over the n blocks
    for (int q = 0; q < 4; ++q) ss[q] = dsum[2 * q + 1] - dsum[2 * q] * dsum[2 * q] / nbk;
    if (threadIdx.x != 0) return;
    dd acc = acc_prev;
    if (step > 0) {  // -beta_i F_i = -beta_{i-1} F_{i-1} + ln Q_i, now that step i is complete
        acc = dd_add(acc_prev, lnq);
        st->acc_hi = acc.hi;
        st->acc_lo = acc.lo;
    }
    const double N = Nd, R = (double)Rn;
    pa_obs o;
    o.step = step;
    o.R_i = Rn;
    o.beta = beta;
    o.sum_E = T[0];
    o.sum_E2 = T[1];
    o.sum_absM = T[2];
    o.sum_M2 = T[3];
    const __int128 varE = (__int128)Rn * T[1] - (__int128)T[0] * T[0];
    const __int128 varM = (__int128)Rn * T[3] - (__int128)T[2] * T[2];
    o.e = (double)T[0] / (N * R);
    o.c_v = beta * beta * (double)varE / (N * R * R);
    o.m = (double)T[2] / (N * R);
    o.chi = beta * (double)varM / (N * R * R);
    o.ln_Q = step == 0 ? 0.0 : lnq.hi + lnq.lo;
    o.minus_beta_F = acc.hi + acc.lo;
    o.n_families = T[4];
    o.sum_fam2 = T[5];
    o.sum_cnt2 = step == 0 ? 0 : sum_cnt2;
    o.rho_t = (double)T[5] / R;
    o.rho_s = exp(TCL / R);
    o.rho_t_step = step == 0 ? 0.0 : (double)sum_cnt2 / R;
    if (nbk < 2) {
        o.r_eff_E = o.r_eff_absM = o.err_e = o.err_m = o.err_c_v = o.err_chi = __builtin_nan("");
    } else {
        const double nn = (double)nbk * (double)(nbk - 1), jf = (double)(nbk - 1) / (double)nbk;
        const double vE = ss[0] / nn, vM = ss[1] / nn;  // blocked variances of the means
        const double rr = R * (R - 1.0);
        o.r_eff_E = ((double)varE / rr) / vE;
        o.r_eff_absM = ((double)varM / rr) / vM;
        o.err_e = sqrt(vE) / N;
        o.err_m = sqrt(vM) / N;
        o.err_c_v = sqrt(jf * ss[2]);
        o.err_chi = sqrt(jf * ss[3]);
    }
    // the deviations of the beta F samples sum to zero, so each covariance is
    // (n - 1)/n sum_k (O_k^J - O) (beta F_k^J - mean): the offset of O drops out
    const double NaN = __builtin_nan("");
    const double jfF = (double)(nF - 1) / (double)nF;
    o.jk_var_beta_F = nF < 2 ? NaN : jfF * dsum[14];
    const bool cov = nF >= 2 && nbk == nF;
    o.jk_cov_e = cov ? jfF * dsum[9] : NaN;
    o.jk_cov_m = cov ? jfF * dsum[11] : NaN;
    o.jk_cov_c_v = cov ? jfF * dsum[12] : NaN;
    o.jk_cov_chi = cov ? jfF * dsum[13] : NaN;
    rd.records[step] = o;
    st->r_parents = step == 0 ? 0 : Rp;
    st->step = step;
    st->cur = nb;
    st->R_cur = Rn;
}

// ------------------------------------------------------------------ host access

// Current population of group g -> stage[l * N + site] as int8 +1 / -1.
__global__ void k_unpack_group(const RunDesc *runs, int r, int g) {
    const RunDesc &rd = runs[r];
    const int N = rd.N, cur = rd.st->cur;
    for (int idx = threadIdx.x + blockIdx.x * blockDim.x; idx < kLanes * N;
         idx += blockDim.x * gridDim.x) {
        const int l = idx / N, site = idx - l * N;
        int up;
        if (rd.layout == PA_LAYOUT_MSC64)
            up = (int)((rd.ms[cur][(size_t)g * N + site] >> l) & 1ull);
        else
            up = rd.s8[cur][((size_t)g * N + site) * kLanes + l] > 0;
        rd.stage[idx] = up ? 1 : -1;
    }
}

// stage[l * N + site] (int8 +1 / -1, lanes >= n_valid ignored) -> group g of buffer buf.
__global__ void k_pack_group(const RunDesc *runs, int r, int g, int buf, int n_valid) {
    const RunDesc &rd = runs[r];
    const int N = rd.N;
    for (int site = threadIdx.x + blockIdx.x * blockDim.x; site < N;
         site += blockDim.x * gridDim.x) {
        uint64_t w = 0;
        for (int l = 0; l < n_valid; ++l) w |= (uint64_t)(rd.stage[l * N + site] > 0) << l;
        size_t o = (size_t)g * N + site;
        if (rd.layout == PA_LAYOUT_MSC64) {
            rd.ms[buf][o] = w;
        } else {
            uint4 *dst = reinterpret_cast<uint4 *>(rd.s8[buf] + o * kLanes);
            for (int q = 0; q < 4; ++q) dst[q] = unpack16((uint32_t)(w >> (16 * q)) & 0xFFFFu);
        }
    }
}

// Adopt a population written into buffer 0 (R_i replicas) as the current one.
__global__ void k_adopt_begin(const RunDesc *runs, int r, int R_i) {
    RunState *st = runs[r].st;
    st->err = 0;
    st->cur = 1;
    st->R_new = R_i;
}
__global__ void k_adopt_end(const RunDesc *runs, int r, int step, double acc) {
    RunState *st = runs[r].st;
    st->step = step;
    st->cur = 0;
    st->R_cur = st->R_new;
    st->acc_hi = acc;
    st->acc_lo = 0.0;
    for (int k = 0; k < kBlocks; ++k) st->jk_F[k] = 0.0;  // the jackknife starts again here
}

// Swap the roles of the two population buffers (R_new = R_cur), so that an
// init-mode sweep launch measures E and M of the current population; a second
// call restores them.  Used to re-derive E and M of a restored snapshot.
__global__ void k_swap_buffers(const RunDesc *runs, int r) {
    RunState *st = runs[r].st;
    st->R_new = st->R_cur;
    st->cur ^= 1;
}

// Mark run r as holding no valid state (a rejected snapshot).
__global__ void k_set_error(const RunDesc *runs, int r, int status) {
    RunState *st = runs[r].st;
    st->err = status;
    st->err_step = st->step + 1;
}

__global__ void k_set_beta(const RunDesc *runs, int r, int idx, double beta) {
    const RunDesc &rd = runs[r];
    if (idx >= 0 && idx <= rd.max_steps) rd.betas[idx] = beta;
}

// ------------------------------------------------------------------ overlap / adaptive step

// alpha(dbeta) of the current population (one block).
__global__ void __launch_bounds__(256) k_overlap(const RunDesc *runs, int r, double dbeta) {
    const RunDesc &rd = runs[r];
    RunState *st = rd.st;
    __shared__ double shd[32];
    const int kmin = st->kmin, nlev = st->kmax - st->kmin + 1, R = st->R_cur;
    const double a = overlap_block(rd, kmin, nlev, R, dbeta, shd);
    if (threadIdx.x == 0) st->alpha_out = a;
}

// ------------------------------------------------------------------ workspace clear

__global__ void k_fill_zero(uint4 *p, size_t n16) {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n16;
         k += (size_t)blockDim.x * gridDim.x)
        p[k] = uint4{0u, 0u, 0u, 0u};
}

// ------------------------------------------------------------------ raw Philox

__global__ void k_philox(uint32_t k0, uint32_t k1, const uint32_t *ctr, int64_t n,
                         uint32_t *out) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)blockDim.x * gridDim.x) {
        U4 x = philox(k0, k1, ctr[4 * t], ctr[4 * t + 1], ctr[4 * t + 2], ctr[4 * t + 3]);
        out[4 * t] = x.x;
        out[4 * t + 1] = x.y;
        out[4 * t + 2] = x.z;
        out[4 * t + 3] = x.w;
    }
}

// ------------------------------------------------------------------ launchers

#define PA_LAUNCH(...)                                   \
    do {                                                 \
        hipLaunchKernelGGL(__VA_ARGS__);                 \
        hipError_t e_ = hipGetLastError();               \
        if (e_ != hipSuccess) return e_;                 \
    } while (0)

hipError_t launch_init(const LaunchCtx &c) {
    PA_LAUNCH(k_init_population, dim3(c.groups.total), dim3(256), 0, c.stream, c.runs,
              c.groups.map);
    return hipSuccess;
}

// LDS of one sweep block: gpb lattices with their halo
size_t sweep_lds_bytes(int L, int gpb) { return (size_t)gpb * (L + 2) * (L + 2) * 8; }

// k_sweep instantiation for a layout, a word walk and words per thread at once
template <int UPD, int C>
static const void *sweep_kernel_of(int layout, int walk, int ilp) {
    static const void *const fns[2][3][2] = {
        {{(const void *)k_sweep<0, kWalkAny, 1, UPD, C>, (const void *)k_sweep<0, kWalkAny, 2, UPD, C>},
         {(const void *)k_sweep<0, kWalkRows, 1, UPD, C>, (const void *)k_sweep<0, kWalkRows, 2, UPD, C>},
         {(const void *)k_sweep<0, kWalkOneGroup, 1, UPD, C>,
          (const void *)k_sweep<0, kWalkOneGroup, 2, UPD, C>}},
        {{(const void *)k_sweep<1, kWalkAny, 1, UPD, C>, (const void *)k_sweep<1, kWalkAny, 2, UPD, C>},
         {(const void *)k_sweep<1, kWalkRows, 1, UPD, C>, (const void *)k_sweep<1, kWalkRows, 2, UPD, C>},
         {(const void *)k_sweep<1, kWalkOneGroup, 1, UPD, C>,
          (const void *)k_sweep<1, kWalkOneGroup, 2, UPD, C>}}};
    return fns[layout][walk][ilp - 1];
}
static const void *sweep_kernel(int layout, int walk, int ilp, int upd, bool count) {
    if (upd == PA_UPDATE_HEATBATH)
        return count ? sweep_kernel_of<PA_UPDATE_HEATBATH, 1>(layout, walk, ilp)
                     : sweep_kernel_of<PA_UPDATE_HEATBATH, 0>(layout, walk, ilp);
    return count ? sweep_kernel_of<PA_UPDATE_METROPOLIS, 1>(layout, walk, ilp)
                 : sweep_kernel_of<PA_UPDATE_METROPOLIS, 0>(layout, walk, ilp);
}

hipError_t launch_sweeps(const LaunchCtx &c, int init) {
    const size_t nc = c.sweep_classes.size();
    const bool fork = nc > 1 && c.class_streams.size() == nc && c.class_events.size() == nc + 1;
    if (fork) {
        hipError_t e = hipEventRecord(c.class_events[0], c.stream);
        if (e != hipSuccess) return e;
    }
    for (size_t k = 0; k < nc; ++k) {
        const auto &cls = c.sweep_classes[k];
        hipStream_t stream = fork ? c.class_streams[k] : c.stream;
        if (fork) {
            hipError_t e = hipStreamWaitEvent(stream, c.class_events[0], 0);
            if (e != hipSuccess) return e;
        }
        const size_t lds = sweep_lds_bytes(cls.L, cls.gpb);
        const bool rows = cls.threads % (cls.L / 2) == 0;  // the word walk moves whole rows
        const int walk = !rows ? kWalkAny : cls.gpb == 1 ? kWalkOneGroup : kWalkRows;
        // words each thread updates at once: one unless the launch geometry asks
        // for two (their Philox chains interleaved; measured no faster at L = 64
        // or 128, where one block fills a CU's LDS)
        const int ilp = cls.words ? cls.words : 1;
        for (int layout = 0; layout < 2; ++layout) {
            if (!(layout == PA_LAYOUT_MSC64 ? cls.has_msc : cls.has_int8)) continue;
            for (int upd = 0; upd < 2; ++upd) {
                if (!c.any_update[upd]) continue;
                const void *fn = sweep_kernel(layout, walk, ilp, upd, c.count_calls);
                void *args[] = {(void *)&c.runs, (void *)&cls.map, (void *)&init, (void *)&cls.gpb};
                hipError_t e = hipLaunchKernel(fn, dim3(cls.total), dim3(cls.threads), args, lds, stream);
                if (e != hipSuccess) return e;
            }
        }
        if (fork) {
            hipError_t e = hipEventRecord(c.class_events[1 + k], stream);
            if (e != hipSuccess) return e;
        }
    }
    for (size_t k = 0; fork && k < nc; ++k) {
        hipError_t e = hipStreamWaitEvent(c.stream, c.class_events[1 + k], 0);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_reduce(const LaunchCtx &c) {
    PA_LAUNCH(k_reduce, dim3(c.slots.total), dim3(256), 0, c.stream, c.runs, c.slots.map);
    return hipSuccess;
}

// ------------------------------------------------------------------ runs combined
// One block per step i: the batch's runs combined at beta_i (the definitions
// are in include/pa.h, pa_weighted).  The weights are formed in log space
// relative to their maximum, R_i e^{x - x_max} with x = -beta_i F_i, and the
// fluctuating-size factor as exp(sum_k ln(R_{k-1} / R)); every sum runs over
// the runs in a fixed order (deterministic).
constexpr int kWSums = 17;

template <int K>
__device__ inline void block_sum_f64v(double (&v)[K], double *sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum_f64(v[k]);
    if (lane == 0)
        for (int k = 0; k < K; ++k) sh[wave * K + k] = v[k];
    __syncthreads();
    for (int k = 0; k < K; ++k) {
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += sh[w * K + k];
        v[k] = t;  // every thread
    }
    __syncthreads();
}
__device__ inline double block_max_f64(double v, double *sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double t = -INFINITY;
    for (int w = 0; w < nw; ++w) t = fmax(t, sh[w]);
    __syncthreads();
    return t;
}

constexpr int kMaxWeightedRuns = 4096;

__global__ void __launch_bounds__(256) k_weighted(const RunDesc *runs, int n_runs, int first,
                                                  pa_weighted *out) {
    __shared__ double sh[4 * kWSums], part[256], lr_sh[kMaxWeightedRuns];
    __shared__ int mixed;
    const int i = first + (int)blockIdx.x;
    const double beta = runs[0].records[i].beta;
    const int N = runs[0].N;
    if (threadIdx.x == 0) mixed = 0;
    __syncthreads();
    // the size factor of Eq. modified-weights2 in logs, lr_m = sum_{k=1}^{i}
    // ln(R_{k-1} / R^m): tpr threads per run take every tpr-th k, their
    // partial sums combined in a fixed order
    const int tpr = max(1, (int)blockDim.x / n_runs), rpp = (int)blockDim.x / tpr;
    for (int m0 = 0; m0 < n_runs; m0 += rpp) {
        const int m = m0 + (int)threadIdx.x / tpr, sub = (int)threadIdx.x % tpr;
        double s = 0.0;
        if (m < n_runs && (int)threadIdx.x < rpp * tpr) {
            const RunDesc &rd = runs[m];
            for (int k = 1 + sub; k <= i; k += tpr) s += log((double)rd.records[k - 1].R_i / (double)rd.R);
        }
        part[threadIdx.x] = s;
        __syncthreads();
        if ((int)threadIdx.x < rpp && m0 + (int)threadIdx.x < n_runs) {
            double t = 0.0;
            for (int q = 0; q < tpr; ++q) t += part[threadIdx.x * tpr + q];
            lr_sh[m0 + threadIdx.x] = t;
        }
        __syncthreads();
    }
    // pass 1: log weights (Eq. weighted-averages, and with the size factor)
    // and their maxima; a run that stopped before step i, or a different
    // beta_i, leaves the step uncombined
    double la_max = -INFINITY, lb_max = -INFINITY;
    for (int m = threadIdx.x; m < n_runs; m += blockDim.x) {
        const RunState *st = runs[m].st;
        if (st->err != 0 && st->err_step <= i) {
            atomicOr(&mixed, 1);
            continue;
        }
        const pa_obs &o = runs[m].records[i];
        if (o.beta != beta) atomicOr(&mixed, 1);
        const double la = o.minus_beta_F + log((double)o.R_i);
        la_max = fmax(la_max, la);
        lb_max = fmax(lb_max, la + lr_sh[m]);
    }
    la_max = block_max_f64(la_max, sh);
    lb_max = block_max_f64(lb_max, sh);
    // pass 2: weighted and plain moment sums, own estimates and beta F
    double v[kWSums];
    for (int k = 0; k < kWSums; ++k) v[k] = 0.0;
    for (int m = threadIdx.x; m < n_runs; m += blockDim.x) {
        const pa_obs &o = runs[m].records[i];
        const double R = (double)o.R_i;
        const double la = o.minus_beta_F + log(R);
        const double a = exp(la - la_max), b = exp(la + lr_sh[m] - lb_max);
        const double mom[4] = {(double)o.sum_E / R, (double)o.sum_E2 / R, (double)o.sum_absM / R,
                               (double)o.sum_M2 / R};
        for (int q = 0; q < 4; ++q) {
            v[q] += a * mom[q];
            v[4 + q] += b * mom[q];
            v[8 + q] += mom[q];
        }
        v[12] += a;
        v[13] += b;
        v[14] += a * a;
        v[15] += -o.minus_beta_F;  // beta_i F_i^m
        v[16] += (double)runs[m].R;
    }
    block_sum_f64v(v, sh);
    const double M = (double)n_runs, Fbar = v[15] / M;
    // pass 3: spread over the runs (centred sums)
    double c[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double obar[4] = {0.0, 0.0, 0.0, 0.0};
    {
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
        for (int m = threadIdx.x; m < n_runs; m += blockDim.x) {
            const pa_obs &o = runs[m].records[i];
            s4[0] += o.e;
            s4[1] += o.m;
            s4[2] += o.c_v;
            s4[3] += o.chi;
        }
        block_sum_f64v(s4, sh);
        for (int q = 0; q < 4; ++q) obar[q] = s4[q] / M;
    }
    for (int m = threadIdx.x; m < n_runs; m += blockDim.x) {
        const pa_obs &o = runs[m].records[i];
        const double dF = -o.minus_beta_F - Fbar;
        c[0] += dF * dF;
        c[1] += (o.e - obar[0]) * dF;
        c[2] += (o.m - obar[1]) * dF;
        c[3] += (o.c_v - obar[2]) * dF;
        c[4] += (o.chi - obar[3]) * dF;
    }
    block_sum_f64v(c, sh);
    if (threadIdx.x == 0) {
        double f[20];
        auto obs = [&](const double *mom, double norm, double *dst) {
            const double E1 = mom[0] / norm, E2 = mom[1] / norm, A1 = mom[2] / norm, A2 = mom[3] / norm;
            dst[0] = E1 / N;
            dst[1] = A1 / N;
            dst[2] = beta * beta * (E2 - E1 * E1) / N;
            dst[3] = beta * (A2 - A1 * A1) / N;
        };
        obs(v, v[12], f);           // weighted
        obs(v + 4, v[13], f + 4);   // weighted, fluctuating size
        obs(v + 8, M, f + 8);       // plain
        f[12] = 1.0 / v[12];        // the largest weight has a = 1
        f[13] = v[12] * v[12] / v[14];
        const double nan = __builtin_nan("");
        const double var = n_runs > 1 ? c[0] / (M - 1.0) : nan;
        f[14] = var;
        f[15] = v[16] / M * var;
        for (int q = 0; q < 4; ++q) f[16 + q] = n_runs > 1 ? c[1 + q] / (M - 1.0) : nan;
        if (mixed)
            for (int q = 0; q < 20; ++q) f[q] = nan;
        pa_weighted w;
        w.step = i;
        w.n_runs = mixed ? 0 : n_runs;
        w.beta = beta;
        w.e = f[0]; w.m = f[1]; w.c_v = f[2]; w.chi = f[3];
        w.e_mod = f[4]; w.m_mod = f[5]; w.c_v_mod = f[6]; w.chi_mod = f[7];
        w.e_plain = f[8]; w.m_plain = f[9]; w.c_v_plain = f[10]; w.chi_plain = f[11];
        w.omega_max = f[12];
        w.n_eff_runs = f[13];
        w.var_beta_F = f[14];
        w.rho_f = f[15];
        w.cov_e = f[16]; w.cov_m = f[17]; w.cov_c_v = f[18]; w.cov_chi = f[19];
        out[blockIdx.x] = w;
    }
}

// ------------------------------------------------------------------ overlap correlation
// C_q(d) of the current population (Eq. overlap_correlation).  On 1-bit
// words the sites where replicas i and i + d differ are the set bits of
// w_g XOR (the partner word), whose lane l holds replica 64 g + l + d: with
// d = 64 a + b it is (w_{g+a} >> b) | (w_{g+a+1} << (64 - b)).  So
//   sum_{i < R - d} sum_k s_k^(i) s_k^(i+d) = N (R - d) - 2 H(d),
// H(d) the popcount of those words over every site and group, lanes with
// i + d >= R masked off.  A block takes kCqSites sites of kCqGroups groups
// (its own words and the partner rows, staged in LDS; int8 sites are packed
// to bits on the way) and 256 distances, one per thread; a wavefront's 64
// distances read two partner rows.  Each thread adds its integer count to
// cq[d] as a double (exact: H(d) < 2^53).
constexpr int kCqSites = 8, kCqGroups = 128, kCqRows = kCqGroups + 5;

__global__ void __launch_bounds__(256) k_cq_zero(double *cq, int n) {
    const int d = blockIdx.x * 256 + threadIdx.x;
    if (d < n) cq[d] = 0.0;
}

__global__ void __launch_bounds__(256) k_cq(const RunDesc *runs, int d_max, double *cq) {
    __shared__ uint64_t own[kCqGroups][kCqSites], par[kCqRows][kCqSites];
    const RunDesc &rd = runs[0];
    const RunState *st = rd.st;
    const int R = st->R_cur, N = rd.N, G = (R + 63) >> 6;
    const int s0 = blockIdx.x * kCqSites, g0 = blockIdx.y * kCqGroups, dc = blockIdx.z;
    const int a_lo = 4 * dc;  // partner groups of this block's distances: a_lo .. a_lo + 3 (+1)
    auto word = [&](int g, int site) -> uint64_t {
        if (g >= G || site >= N) return 0ull;
        if (rd.layout == PA_LAYOUT_MSC64) return rd.ms[st->cur][(size_t)g * N + site];
        const uint4 *p = reinterpret_cast<const uint4 *>(rd.s8[st->cur] + ((size_t)g * N + site) * 64);
        uint64_t w = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) w |= (uint64_t)pack16(p[q]) << (16 * q);
        return w;
    };
    for (int e = threadIdx.x; e < kCqGroups * kCqSites; e += blockDim.x) {
        const int gi = e / kCqSites, si = e - gi * kCqSites;
        own[gi][si] = word(g0 + gi, s0 + si);
    }
    for (int e = threadIdx.x; e < kCqRows * kCqSites; e += blockDim.x) {
        const int gi = e / kCqSites, si = e - gi * kCqSites;
        par[gi][si] = word(g0 + a_lo + gi, s0 + si);
    }
    __syncthreads();
    // wavefront w takes b in [32 hb, 32 hb + 32), hb = w & 1, for the two
    // partner offsets a = a_lo + 2 (w >> 1) + (lane >> 5): the funnel shift
    // of the 128-bit (hi:lo) by b is then two 32-bit align operations on
    // halves chosen by hb alone (uniform in the wavefront)
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = (int)threadIdx.x & 63;
    const int hb = wv & 1;
    const int ar = 2 * (wv >> 1) + (lane >> 5), b = 32 * hb + (lane & 31);  // ar in 0 .. 3
    const int d = 64 * (a_lo + ar) + b;
    if (d < 1 || d > d_max) return;
    const uint32_t sh = (uint32_t)(lane & 31);
    const int ng = min(kCqGroups, G - g0), ns = min(kCqSites, N - s0);
    // every lane of group g0 + gi has its partner (i + d < R, i = 64 g + lane)
    // for gi < full; the groups after it are masked
    const int full = max(0, min(ng, (R - d) / 64 - g0));
    auto count_pairs = [&](auto upper) -> uint32_t {
        uint32_t cnt = 0;
        for (int si = 0; si < ns; ++si) {
            uint64_t lo = par[ar][si];
            auto pair = [&](int gi) -> uint64_t {
                const uint64_t hi = par[gi + ar + 1][si];
                const uint32_t x0 = (uint32_t)lo, x1 = (uint32_t)(lo >> 32), x2 = (uint32_t)hi,
                               x3 = (uint32_t)(hi >> 32);
                const uint32_t p0 = upper ? __builtin_amdgcn_alignbit(x2, x1, sh)
                                          : __builtin_amdgcn_alignbit(x1, x0, sh);
                const uint32_t p1 = upper ? __builtin_amdgcn_alignbit(x3, x2, sh)
                                          : __builtin_amdgcn_alignbit(x2, x1, sh);
                lo = hi;
                return own[gi][si] ^ (((uint64_t)p1 << 32) | p0);
            };
            int gi = 0;
            for (; gi < full; ++gi) cnt += (uint32_t)__popcll(pair(gi));
            for (; gi < ng; ++gi) cnt += (uint32_t)__popcll(pair(gi) & lane_mask(R - d - 64 * (g0 + gi)));
        }
        return cnt;
    };
    const uint32_t cnt = hb ? count_pairs(std::true_type{}) : count_pairs(std::false_type{});
    atomicAdd(&cq[d], (double)cnt);
}

__global__ void __launch_bounds__(256) k_cq_finish(const RunDesc *runs, int d_max, double *cq) {
    const int d = blockIdx.x * 256 + threadIdx.x;
    if (d > d_max) return;
    const double R = (double)runs[0].st->R_cur, N = (double)runs[0].N;
    cq[d] = d == 0 ? 1.0 : 1.0 - 2.0 * cq[d] / (N * (R - d));
}

hipError_t launch_overlap_correlation(const LaunchCtx &c, int N, int R, int d_max, double *cq) {
    const int n = d_max + 1, nb = (n + 255) / 256;
    PA_LAUNCH(k_cq_zero, dim3(nb), dim3(256), 0, c.stream, cq, n);
    const dim3 grid((N + kCqSites - 1) / kCqSites, ((R + 63) / 64 + kCqGroups - 1) / kCqGroups,
                    (d_max + 256) / 256);
    PA_LAUNCH(k_cq, grid, dim3(256), 0, c.stream, c.runs, d_max, cq);
    PA_LAUNCH(k_cq_finish, dim3(nb), dim3(256), 0, c.stream, c.runs, d_max, cq);
    return hipSuccess;
}

hipError_t launch_weighted(const LaunchCtx &c, int first, int count, pa_weighted *out) {
    PA_LAUNCH(k_weighted, dim3(count), dim3(256), 0, c.stream, c.runs, c.n_runs, first, out);
    return hipSuccess;
}

hipError_t launch_counts(const LaunchCtx &c) {
    // multinomial-only batches at L <= 64 fold the normalisation into the weights' launch
    const bool fused = c.any_multi && !c.any_nearest && !c.any_poisson && c.max_L <= 64;
    if (!fused) PA_LAUNCH(k_norm, dim3(c.n_runs), dim3(256), 0, c.stream, c.runs);
    if (c.any_nearest)
        PA_LAUNCH(k_counts_nearest, dim3(c.slots.total), dim3(256), 0, c.stream, c.runs,
                  c.slots.map);
    if (c.any_poisson)
        PA_LAUNCH(k_counts_poisson, dim3(c.slots.total), dim3(256), 0, c.stream, c.runs, c.slots.map);
    if (c.any_multi) {
        if (fused)
            PA_LAUNCH(k_multi_norm_weights, dim3(c.slots.total + c.n_runs), dim3(256), 0, c.stream,
                      c.runs, c.slots.map, c.slots.total);
        else
            PA_LAUNCH(k_multi_weights, dim3(c.slots.total), dim3(256), 0, c.stream, c.runs,
                      c.slots.map);
        PA_LAUNCH(k_multi_draw, dim3(c.slots.total), dim3(kSlotBlock), draw_lds_bytes(c.max_nblk),
                  c.stream, c.runs, c.slots.map);
    }
    PA_LAUNCH(k_offsets, dim3(c.slots.total + c.n_runs * kBlocks), dim3(256), 0, c.stream, c.runs,
              c.slots.map, c.slots.total);
    return hipSuccess;
}

hipError_t launch_copy(const LaunchCtx &c) {
    if (c.any_msc)
        PA_LAUNCH(k_gather_msc64, dim3(c.groups.total), dim3(kGatherThreads), 0, c.stream, c.runs,
                  c.groups.map);
    if (c.any_int8)
        PA_LAUNCH(k_gather_int8, dim3(c.groups.total), dim3(kGather8Threads), 0, c.stream, c.runs,
                  c.groups.map);
    return hipSuccess;
}

hipError_t launch_resample(const LaunchCtx &c) {
    hipError_t e = launch_counts(c);
    if (e != hipSuccess) return e;
    return launch_copy(c);
}

hipError_t launch_step(const LaunchCtx &c) {
    hipError_t e = launch_resample(c);
    if (e != hipSuccess) return e;
    e = launch_sweeps(c, 0);
    if (e != hipSuccess) return e;
    return launch_reduce(c);
}

hipError_t launch_hist_current(const LaunchCtx &c) {
    PA_LAUNCH(k_hist_clear, dim3(c.n_runs), dim3(256), 0, c.stream, c.runs);
    PA_LAUNCH(k_hist, dim3(c.slots.total), dim3(256), 0, c.stream, c.runs, c.slots.map);
    return hipSuccess;
}

hipError_t launch_overlap(const LaunchCtx &c, int r, double dbeta) {
    PA_LAUNCH(k_overlap, dim3(1), dim3(256), 0, c.stream, c.runs, r, dbeta);
    return hipSuccess;
}

hipError_t launch_swap_buffers(const LaunchCtx &c, int r) {
    PA_LAUNCH(k_swap_buffers, dim3(1), dim3(1), 0, c.stream, c.runs, r);
    return hipSuccess;
}

hipError_t launch_set_error(const LaunchCtx &c, int r, int status) {
    PA_LAUNCH(k_set_error, dim3(1), dim3(1), 0, c.stream, c.runs, r, status);
    return hipSuccess;
}

hipError_t launch_set_beta(const LaunchCtx &c, int r, int idx, double beta) {
    PA_LAUNCH(k_set_beta, dim3(1), dim3(1), 0, c.stream, c.runs, r, idx, beta);
    return hipSuccess;
}

hipError_t launch_unpack_group(const LaunchCtx &c, int r, int g, int N) {
    int blocks = (kLanes * N + 255) / 256;
    PA_LAUNCH(k_unpack_group, dim3(blocks), dim3(256), 0, c.stream, c.runs, r, g);
    return hipSuccess;
}

hipError_t launch_pack_group(const LaunchCtx &c, int r, int g, int buf, int n_valid, int N) {
    int blocks = (N + 255) / 256;
    PA_LAUNCH(k_pack_group, dim3(blocks), dim3(256), 0, c.stream, c.runs, r, g, buf, n_valid);
    return hipSuccess;
}

hipError_t launch_adopt_begin(const LaunchCtx &c, int r, int R_i) {
    PA_LAUNCH(k_adopt_begin, dim3(1), dim3(1), 0, c.stream, c.runs, r, R_i);
    return hipSuccess;
}

hipError_t launch_adopt_end(const LaunchCtx &c, int r, int step, double acc) {
    PA_LAUNCH(k_adopt_end, dim3(1), dim3(1), 0, c.stream, c.runs, r, step, acc);
    return hipSuccess;
}

hipError_t launch_philox(uint32_t k0, uint32_t k1, const uint32_t *ctr, int64_t n, uint32_t *out,
                         hipStream_t stream) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    PA_LAUNCH(k_philox, dim3((unsigned)blocks), dim3(256), 0, stream, k0, k1, ctr, n, out);
    return hipSuccess;
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t stream) {
    const size_t n16 = bytes / 16;  // workspace sizes are multiples of 256 bytes
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    PA_LAUNCH(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, stream, (uint4 *)p, n16);
    return hipSuccess;
}

hipError_t configure_kernels() {
    // multinomial draws: 12 bytes of LDS per parent block, at most 8192 blocks (R < 2^23)
    {
        hipError_t e = hipFuncSetAttribute((const void *)k_multi_draw,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 8192 * 12);
        if (e != hipSuccess) return e;
    }
    // up to kMaxSweepLds bytes of lattices (with their halo) per sweep block
    for (int k = 0; k < 48; ++k) {
        const void *f = sweep_kernel((k / 6) & 1, (k / 2) % 3, k % 2 + 1, (k / 12) & 1, k >= 24);
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxSweepLds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace pa
