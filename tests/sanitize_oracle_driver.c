/*
 * Host sanitizer driver for the oracle's C core (oracle/pa_oracle.c).
 *
 * Calls every exported function on small, ragged inputs: replica counts that
 * leave a partial 64-replica group, the smallest lattice the method uses,
 * populations that start at a later group, and acceptance thresholds at both
 * ends of their range.  Every buffer is a heap block of exactly the size the
 * function documents, so AddressSanitizer reports any access outside it and
 * UndefinedBehaviorSanitizer any signed overflow, bad shift or misaligned
 * access.  The driver prints one FNV-1a hash of every result; the test builds
 * it once with the sanitizers and once without and requires the same hash.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_philox4x32_10(uint32_t key0, uint32_t key1, const uint32_t ctr[4], uint32_t out[4]);
void oracle_philox4x32_10_n(uint32_t key0, uint32_t key1, int64_t n, const uint32_t *ctr,
                            uint32_t *out);
uint32_t oracle_sweep_top6(uint64_t seed, uint32_t w, uint32_t g, uint32_t h, uint32_t lane);
void oracle_word_uniforms(uint64_t seed, uint32_t w, uint32_t g, uint32_t h, const uint64_t thr[64],
                          const int needs[64], uint32_t u[64]);
void oracle_word_uniforms_heatbath(uint64_t seed, uint32_t w, uint32_t g, uint32_t h,
                                   const uint64_t thr[64], const int needs[64], uint32_t u[64]);
uint32_t oracle_resample_uniform(uint64_t seed, uint32_t step, uint32_t j);
uint64_t oracle_multinomial_uniform(uint64_t seed, uint32_t step, uint32_t d);
uint64_t oracle_poisson_uniform(uint64_t seed, uint32_t step, uint32_t j);
void oracle_init_spins(uint64_t seed, int L, int R, int8_t *spins);
void oracle_energy_magnetisation(int L, int R, const int8_t *spins, int32_t *E, int32_t *M);
int oracle_delta_energy(int s, int h);
void oracle_sweeps(uint64_t seed, int L, int R, int8_t *spins, int step, int theta, uint64_t t4,
                   uint64_t t8, int slot0);
void oracle_sweeps_heatbath(uint64_t seed, int L, int R, int8_t *spins, int step, int theta,
                            const uint64_t thr5[5], int slot0);

static uint64_t g_hash = 1469598103934665603ull;

static void mix(const void *p, size_t n) {
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) {
        g_hash ^= b[i];
        g_hash *= 1099511628211ull;
    }
}

static void *exact_alloc(size_t n) {
    void *p = malloc(n ? n : 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

/* The RNG streams: the bare generator at the ends of its key and counter
 * range, and every derived uniform over a few counters. */
static void rng_streams(void) {
    const uint32_t keys[3][2] = {{0u, 0u}, {0xFFFFFFFFu, 0xFFFFFFFFu}, {0x12345678u, 0x9ABCDEF0u}};
    const uint32_t ctrs[3][4] = {{0u, 0u, 0u, 0u}, {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu},
                                 {1u, 2u, 3u, 4u}};
    for (int k = 0; k < 3; ++k)
        for (int c = 0; c < 3; ++c) {
            uint32_t out[4];
            oracle_philox4x32_10(keys[k][0], keys[k][1], ctrs[c], out);
            mix(out, sizeof out);
        }
    /* the batched form over 0, 1 and 5 counters, each buffer exactly 4n words */
    for (int64_t n = 0; n <= 5; n += n ? 4 : 1) {
        uint32_t *ctr = (uint32_t *)exact_alloc((size_t)(4 * n) * sizeof(uint32_t));
        uint32_t *out = (uint32_t *)exact_alloc((size_t)(4 * n) * sizeof(uint32_t));
        for (int64_t i = 0; i < 4 * n; ++i) ctr[i] = (uint32_t)(0x9E3779B9u * (uint32_t)(i + 1));
        oracle_philox4x32_10_n(keys[2][0], keys[2][1], n, ctr, out);
        mix(out, (size_t)(4 * n) * sizeof(uint32_t));
        free(ctr);
        free(out);
    }
    const uint64_t seeds[3] = {0ull, 12345ull, 0xFFFFFFFFFFFFFFFFull};
    for (int s = 0; s < 3; ++s)
        for (uint32_t j = 0; j < 70; ++j) {
            uint32_t a = oracle_sweep_top6(seeds[s], j, j / 7, 2 * j + 1, j & 63u);
            uint32_t b = oracle_resample_uniform(seeds[s], j + 1, j);
            uint64_t c = oracle_multinomial_uniform(seeds[s], j + 1, j);
            uint64_t d = oracle_poisson_uniform(seeds[s], j + 1, j);
            mix(&a, sizeof a);
            mix(&b, sizeof b);
            mix(&c, sizeof c);
            mix(&d, sizeof d);
        }
}

/* Word uniforms with every mix of comparing lanes and ties: thresholds whose
 * top six bits match the lane's draw force the tie stream, thresholds of 0 and
 * 2^32 sit at the ends of the range. */
static void word_uniforms(void) {
    uint64_t *thr = (uint64_t *)exact_alloc(64 * sizeof(uint64_t));
    int *needs = (int *)exact_alloc(64 * sizeof(int));
    uint32_t *u = (uint32_t *)exact_alloc(64 * sizeof(uint32_t));
    for (int pattern = 0; pattern < 4; ++pattern) {
        for (uint32_t l = 0; l < 64; ++l) {
            uint32_t top = oracle_sweep_top6(777ull, 5u, 3u, 9u, l);
            needs[l] = pattern == 0 ? 1 : pattern == 1 ? (int)(l & 1u) : pattern == 2 ? (l < 3) : 0;
            switch ((l + (uint32_t)pattern) % 4u) {
            case 0: thr[l] = (uint64_t)top << 26; break;                 /* tie, zero low part */
            case 1: thr[l] = ((uint64_t)top << 26) | 0x155555u; break;   /* tie */
            case 2: thr[l] = 0ull; break;
            default: thr[l] = 1ull << 32; break;
            }
        }
        oracle_word_uniforms(777ull, 5u, 3u, 9u, thr, needs, u);
        mix(u, 64 * sizeof(uint32_t));
        oracle_word_uniforms_heatbath(777ull, 5u, 3u, 9u, thr, needs, u);
        mix(u, 64 * sizeof(uint32_t));
    }
    free(thr);
    free(needs);
    free(u);
}

/* The model on ragged populations: initial spins, energy and magnetisation,
 * and both sweeps over a few steps. */
static void model(void) {
    const int Ls[3] = {4, 6, 8};
    const int Rs[5] = {1, 63, 64, 65, 130};
    const int slot0s[2] = {0, 128};
    const uint64_t t48[3][2] = {{1ull << 32, 1ull << 32}, {1ull, 1ull}, {743511829ull, 128711131ull}};
    const uint64_t thr5[5] = {0ull, 1ull << 32, 2147483648ull, 3857341766ull, 1ull};
    for (int li = 0; li < 3; ++li)
        for (int ri = 0; ri < 5; ++ri)
            for (int si = 0; si < 2; ++si) {
                int L = Ls[li], R = Rs[ri], N = L * L;
                int8_t *spins = (int8_t *)exact_alloc((size_t)R * N);
                int32_t *E = (int32_t *)exact_alloc((size_t)R * sizeof(int32_t));
                int32_t *M = (int32_t *)exact_alloc((size_t)R * sizeof(int32_t));
                uint64_t seed = 1000u + 17u * (unsigned)li + 5u * (unsigned)ri + (unsigned)si;
                oracle_init_spins(seed, L, R, spins);
                for (int step = 1; step <= 3; ++step) {
                    const uint64_t *t = t48[(step + ri) % 3];
                    oracle_sweeps(seed, L, R, spins, step, 2, t[0], t[1], slot0s[si]);
                    oracle_energy_magnetisation(L, R, spins, E, M);
                    mix(spins, (size_t)R * N);
                    mix(E, (size_t)R * sizeof(int32_t));
                    mix(M, (size_t)R * sizeof(int32_t));
                }
                oracle_sweeps_heatbath(seed, L, R, spins, 4, 3, thr5, slot0s[si]);
                oracle_energy_magnetisation(L, R, spins, E, M);
                mix(spins, (size_t)R * N);
                mix(E, (size_t)R * sizeof(int32_t));
                mix(M, (size_t)R * sizeof(int32_t));
                free(spins);
                free(E);
                free(M);
            }
    for (int s = -1; s <= 1; s += 2)
        for (int h = -4; h <= 4; h += 2) {
            int d = oracle_delta_energy(s, h);
            mix(&d, sizeof d);
        }
}

int main(void) {
    rng_streams();
    word_uniforms();
    model();
    printf("%016llx\n", (unsigned long long)g_hash);
    return 0;
}
