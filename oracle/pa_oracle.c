/*
 * Population-annealing CPU oracle: the integer core.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, single-threaded C that shares no
 * code with the HIP library.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.
 *
 * What lives here (everything else of the oracle is in pa_oracle.py):
 *   - Philox4x32-10, written from its published definition (Salmon, Moraes,
 *     Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11):
 *     ten rounds of two 32x32->64 multiplies with the round constants
 *     0xD2511F53 / 0xCD9E8D57 and a Weyl key schedule 0x9E3779B9 / 0xBB67AE85.
 *   - the random streams the method draws from (initial spins, Metropolis
 *     uniforms, resampling uniforms), each a fixed map of (seed, indices)
 *     to a Philox counter;
 *   - simple-sampling initialisation at beta_0 = 0 (Sec. "Algorithm", step 1);
 *   - checkerboard single-spin-flip Metropolis with acceptance
 *     min[1, exp(-beta dE)] (Sec. "Spin updates");
 *   - the energy and magnetisation of each replica (Sec. "Model and
 *     observables", Eq. hamiltonian with J = 1, periodic L x L).
 *
 * Spin storage is replica-major and unpacked: spins[r * N + site], each +1 or
 * -1, site = y * L + x.
 */
#include <stdint.h>
#include <stddef.h>

/* ---------------- Philox4x32-10 ---------------- */

static void philox_round(uint32_t c[4], const uint32_t k[2]) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

void oracle_philox4x32_10(uint32_t key0, uint32_t key1, const uint32_t ctr[4], uint32_t out[4]) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key0, key1};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    out[0] = c[0];
    out[1] = c[1];
    out[2] = c[2];
    out[3] = c[3];
}

/* The same generator over n counters (ctr and out hold 4n words each), for
 * comparisons over many counters without a call per counter. */
void oracle_philox4x32_10_n(uint32_t key0, uint32_t key1, int64_t n, const uint32_t *ctr,
                            uint32_t *out) {
    for (int64_t i = 0; i < n; ++i) oracle_philox4x32_10(key0, key1, ctr + 4 * i, out + 4 * i);
}

/* ---------------- random streams ----------------
 * key = (seed mod 2^32, seed div 2^32).  The fourth counter word carries a
 * stream tag in its top nibble.  Replica slot r belongs to group g = r / 64
 * and is lane r % 64 of that group.
 *   INIT     (site, g, 0, 0x2000_0000): bits x0 | x1<<32, bit lane = 1 -> +1
 *   SWEEP    (w, g, h, 0x1000_0000 | p), p = 0, 1, 2: bit planes 2p =
 *            x0 | x1<<32 and 2p+1 = x2 | x3<<32.  Bit (31 - b) of the uniform of
 *            lane l is bit l of plane b, for b < 6.  w is the site's index within
 *            its colour, h the global half-sweep index.
 *   TIE      (w, g, h, 0x1000_0100 | q): the lanes of a word whose top six
 *            bits equal those of their threshold are its ties; the k-th tie in
 *            ascending lane order takes word k & 3 of call q = k >> 2, shifted
 *            right by six, as its low 26 bits.  Other lanes' low bits are 0: their
 *            comparison is already decided by the top six.
 *   RESAMPLE (j >> 2, i, 0, 0x3000_0000): the uniform of parent j at step i
 *            is output word j & 3.
 *   MULTI    (d >> 1, i, 0, 0x4000_0000): the 64-bit uniform of draw d at
 *            step i is x0 | x1<<32 (d even) or x2 | x3<<32 (d odd).
 */
#define TAG_SWEEP 0x10000000u
#define TAG_TIE 0x10000100u
#define TAG_INIT 0x20000000u
#define TAG_RESAMPLE 0x30000000u
#define TAG_MULTI 0x40000000u
#define TAG_POISSON 0x50000000u

static void draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t out[4]) {
    uint32_t ctr[4] = {c0, c1, c2, c3};
    oracle_philox4x32_10((uint32_t)seed, (uint32_t)(seed >> 32), ctr, out);
}

/* The top six bits of lane l's Metropolis uniform in word (w, g, h). */
uint32_t oracle_sweep_top6(uint64_t seed, uint32_t w, uint32_t g, uint32_t h, uint32_t lane) {
    uint32_t top = 0;
    for (uint32_t p = 0; p < 3; ++p) {
        uint32_t x[4];
        draw(seed, w, g, h, TAG_SWEEP | p, x);
        uint64_t plane_a = (uint64_t)x[0] | ((uint64_t)x[1] << 32);
        uint64_t plane_b = (uint64_t)x[2] | ((uint64_t)x[3] << 32);
        top |= (uint32_t)((plane_a >> lane) & 1u) << (5u - 2u * p);
        top |= (uint32_t)((plane_b >> lane) & 1u) << (4u - 2u * p);
    }
    return top;
}

/*
 * The Metropolis uniforms u[l] of the 64 lanes of word (w, g, h).  needs[l]
 * says whether lane l compares a uniform with a threshold at all (a valid
 * replica with dE > 0 whose threshold thr[l] is below 2^32); u[l] is 0 for the
 * others.  For the lanes that do, the top six bits come from the planes, and a
 * lane whose top six bits equal its threshold's (a tie) gets its low 26 bits
 * from the TIE stream in ascending lane order.  Each u[l] of a comparing lane
 * is a uniform 32-bit integer as far as u[l] < thr[l] is concerned: the low
 * bits of a lane that is not tied cannot change that comparison.
 */
void oracle_word_uniforms(uint64_t seed, uint32_t w, uint32_t g, uint32_t h, const uint64_t thr[64],
                          const int needs[64], uint32_t u[64]) {
    uint32_t ties = 0;
    for (uint32_t l = 0; l < 64; ++l) {
        u[l] = 0;
        if (!needs[l])
            continue;
        uint32_t top = oracle_sweep_top6(seed, w, g, h, l);
        u[l] = top << 26;
        if (top == (uint32_t)(thr[l] >> 26)) {
            uint32_t x[4];
            draw(seed, w, g, h, TAG_TIE | (ties >> 2), x);
            u[l] |= x[ties & 3u] >> 6;
            ++ties;
        }
    }
}

/*
 * Heatbath uniforms of word (w, g, h): as oracle_word_uniforms, except that a
 * lane counts as tied only when the top six bits leave u < thr[l] undecided,
 * i.e. they equal those of thr[l] and the low 26 bits of thr[l] are not all
 * zero (with a zero low part, equal top bits already give u >= thr[l]).
 */
void oracle_word_uniforms_heatbath(uint64_t seed, uint32_t w, uint32_t g, uint32_t h,
                                   const uint64_t thr[64], const int needs[64], uint32_t u[64]) {
    uint32_t ties = 0;
    for (uint32_t l = 0; l < 64; ++l) {
        u[l] = 0;
        if (!needs[l])
            continue;
        uint32_t top = oracle_sweep_top6(seed, w, g, h, l);
        u[l] = top << 26;
        if (top == (uint32_t)(thr[l] >> 26) && (thr[l] & 0x3FFFFFFu) != 0) {
            uint32_t x[4];
            draw(seed, w, g, h, TAG_TIE | (ties >> 2), x);
            u[l] |= x[ties & 3u] >> 6;
            ++ties;
        }
    }
}

uint32_t oracle_resample_uniform(uint64_t seed, uint32_t step, uint32_t j) {
    uint32_t x[4];
    draw(seed, j >> 2, step, 0, TAG_RESAMPLE, x);
    return x[j & 3u];
}

uint64_t oracle_multinomial_uniform(uint64_t seed, uint32_t step, uint32_t d) {
    uint32_t x[4];
    draw(seed, d >> 1, step, 0, TAG_MULTI, x);
    if ((d & 1u) == 0)
        return (uint64_t)x[0] | ((uint64_t)x[1] << 32);
    return (uint64_t)x[2] | ((uint64_t)x[3] << 32);
}

/* The 64-bit uniform of parent j for Poisson resampling at step i. */
uint64_t oracle_poisson_uniform(uint64_t seed, uint32_t step, uint32_t j) {
    uint32_t x[4];
    draw(seed, j >> 1, step, 0, TAG_POISSON, x);
    if ((j & 1u) == 0)
        return (uint64_t)x[0] | ((uint64_t)x[1] << 32);
    return (uint64_t)x[2] | ((uint64_t)x[3] << 32);
}

/* ---------------- the model ---------------- */

/* Simple sampling at beta_0 = 0: every spin of every replica is +1 or -1 with
 * probability 1/2, independently. */
void oracle_init_spins(uint64_t seed, int L, int R, int8_t *spins) {
    int N = L * L;
    for (int r = 0; r < R; ++r) {
        for (int site = 0; site < N; ++site) {
            uint32_t x[4];
            draw(seed, (uint32_t)site, (uint32_t)(r / 64), 0, TAG_INIT, x);
            uint64_t bits = (uint64_t)x[0] | ((uint64_t)x[1] << 32);
            spins[(size_t)r * N + site] = ((bits >> (r % 64)) & 1u) ? (int8_t)1 : (int8_t)-1;
        }
    }
}

/* E = -sum over nearest-neighbour pairs of s_i s_j (each bond once, via the
 * right and down neighbour of every site); M = sum of spins. */
void oracle_energy_magnetisation(int L, int R, const int8_t *spins, int32_t *E, int32_t *M) {
    int N = L * L;
    for (int r = 0; r < R; ++r) {
        const int8_t *s = spins + (size_t)r * N;
        int32_t e = 0, m = 0;
        for (int y = 0; y < L; ++y) {
            for (int x = 0; x < L; ++x) {
                int here = s[y * L + x];
                int right = s[y * L + (x + 1) % L];
                int down = s[((y + 1) % L) * L + x];
                e -= here * (right + down);
                m += here;
            }
        }
        E[r] = e;
        M[r] = m;
    }
}

/* One Metropolis attempt's energy change for flipping spin s with neighbour
 * field h: dE = 2 s h. */
int oracle_delta_energy(int s, int h) { return 2 * s * h; }

/*
 * theta checkerboard sweeps at inverse temperature beta_i of step i >= 1.
 * One sweep attempts every site of colour 0 = (x + y) even, then every site of
 * colour 1.  A flip with dE <= 0 is always accepted; otherwise it is accepted
 * iff u < exp(-beta dE) with u = u32 / 2^32.  The caller passes the exact
 * integer thresholds t4 = ceil(2^32 exp(-4 beta)) and t8 = ceil(2^32
 * exp(-8 beta)) (both in [1, 2^32]); for an integer u32, u32 / 2^32 < p holds
 * exactly when u32 < ceil(2^32 p).  spins holds R replicas occupying slots
 * slot0 .. slot0 + R - 1 of the population (their slots select their
 * uniforms).  The uniforms of a 64-replica group are drawn together
 * (oracle_word_uniforms), so slot0 must be a multiple of 64 and spins must hold
 * every replica of each group it touches (the last group may end early only
 * where the population ends).
 */
void oracle_sweeps(uint64_t seed, int L, int R, int8_t *spins, int step, int theta,
                   uint64_t t4, uint64_t t8, int slot0) {
    int N = L * L;
    int half = L / 2;
    for (int sweep = 0; sweep < theta; ++sweep) {
        for (int colour = 0; colour < 2; ++colour) {
            uint32_t h = 2u * ((uint32_t)theta * (uint32_t)(step - 1) + (uint32_t)sweep) + (uint32_t)colour;
            for (int r0 = 0; r0 < R; r0 += 64) {
                int n_lanes = R - r0 < 64 ? R - r0 : 64;
                uint32_t g = (uint32_t)((slot0 + r0) / 64);
                for (int y = 0; y < L; ++y) {
                    for (int x = 0; x < L; ++x) {
                        if (((x + y) & 1) != colour)
                            continue;
                        int site = y * L + x;
                        int dE[64];
                        uint64_t thr[64];
                        int needs[64];
                        uint32_t u[64];
                        for (int l = 0; l < 64; ++l) {
                            dE[l] = 0;
                            thr[l] = 0;
                            needs[l] = 0;
                            if (l >= n_lanes)
                                continue;
                            const int8_t *s = spins + (size_t)(r0 + l) * N;
                            int field = s[y * L + (x + 1) % L] + s[y * L + (x + L - 1) % L] +
                                        s[((y + 1) % L) * L + x] + s[((y + L - 1) % L) * L + x];
                            dE[l] = oracle_delta_energy(s[site], field);
                            if (dE[l] > 0) {
                                thr[l] = (dE[l] == 4) ? t4 : t8;
                                needs[l] = thr[l] < ((uint64_t)1 << 32);
                            }
                        }
                        oracle_word_uniforms(seed, (uint32_t)(y * half + x / 2), g, h, thr, needs, u);
                        for (int l = 0; l < n_lanes; ++l) {
                            int8_t *s = spins + (size_t)(r0 + l) * N;
                            int flip;
                            if (dE[l] <= 0)
                                flip = 1;
                            else if (!needs[l])
                                flip = 1; /* threshold 2^32: every uniform is below it */
                            else
                                flip = (uint64_t)u[l] < thr[l];
                            if (flip)
                                s[site] = (int8_t)(-s[site]);
                        }
                    }
                }
            }
        }
    }
}

/*
 * theta checkerboard heatbath sweeps (Sec. "Spin updates": heatbath, the same
 * as Glauber dynamics for Ising spins) at beta_i of step i >= 1, in the order
 * of oracle_sweeps.  The spin at a site flips with probability
 * 1 / (1 + exp(beta dE)), dE the energy change of the flip, whatever its sign;
 * equivalently the new spin is +1 with probability 1 / (1 + exp(-2 beta h)),
 * h the sum of the four neighbours.  thr[c] = ceil(2^32 / (1 + exp(beta dE)))
 * for dE = 4c - 8 (c = 0..4) is passed in; the flip happens iff u < thr[c],
 * u the lane's uniform (oracle_word_uniforms_heatbath).  Every replica
 * compares, so every valid lane draws.
 */
void oracle_sweeps_heatbath(uint64_t seed, int L, int R, int8_t *spins, int step, int theta,
                            const uint64_t thr5[5], int slot0) {
    int N = L * L;
    int half = L / 2;
    for (int sweep = 0; sweep < theta; ++sweep) {
        for (int colour = 0; colour < 2; ++colour) {
            uint32_t h = 2u * ((uint32_t)theta * (uint32_t)(step - 1) + (uint32_t)sweep) + (uint32_t)colour;
            for (int r0 = 0; r0 < R; r0 += 64) {
                int n_lanes = R - r0 < 64 ? R - r0 : 64;
                uint32_t g = (uint32_t)((slot0 + r0) / 64);
                for (int y = 0; y < L; ++y) {
                    for (int x = 0; x < L; ++x) {
                        if (((x + y) & 1) != colour)
                            continue;
                        int site = y * L + x;
                        uint64_t thr[64];
                        int needs[64];
                        uint32_t u[64];
                        for (int l = 0; l < 64; ++l) {
                            thr[l] = 0;
                            needs[l] = 0;
                            if (l >= n_lanes)
                                continue;
                            const int8_t *s = spins + (size_t)(r0 + l) * N;
                            int field = s[y * L + (x + 1) % L] + s[y * L + (x + L - 1) % L] +
                                        s[((y + 1) % L) * L + x] + s[((y + L - 1) % L) * L + x];
                            int dE = oracle_delta_energy(s[site], field);
                            thr[l] = thr5[(dE + 8) / 4];
                            needs[l] = 1;
                        }
                        oracle_word_uniforms_heatbath(seed, (uint32_t)(y * half + x / 2), g, h, thr,
                                                      needs, u);
                        for (int l = 0; l < n_lanes; ++l) {
                            int8_t *s = spins + (size_t)(r0 + l) * N;
                            if ((uint64_t)u[l] < thr[l])
                                s[site] = (int8_t)(-s[site]);
                        }
                    }
                }
            }
        }
    }
}
