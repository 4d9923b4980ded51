/*
 * Seeded synthetic input generators for the multiway mergesort workloads.
 *
 * This file holds input recipes only: it never compares, orders or merges
 * keys, so neither the GPU sort nor the CPU oracle depends on it for any of
 * the method's arithmetic.  Both sides receive the arrays it writes.
 *
 * Pseudo-random numbers: splitmix64 (Steele, Lea & Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), written out from its
 * published definition.  Bounded draws in [0, n) use Lemire's
 * multiply-shift reduction of a 32-bit draw ("Fast random integer generation
 * in an interval", 2019) without the rejection step: the bias is below
 * n / 2^32 and is irrelevant for input synthesis.
 *
 * Input families (the paper builds its inputs in the same ways, §1 and §6.3):
 *   uniform     keys drawn uniformly from [0, 2^32)
 *   nearly      identity permutation of 0..n-1 followed by k swaps of two
 *               independently uniform positions (the "sortedness" family)
 *   sixteen     one of 16 values v*0x11111111, v in 0..15 (tie-heavy)
 *   stride64    transpose of a 64 x (n/64) row-major matrix holding 0..n-1
 *               (each 64-chunk ascends; elements 64 apart are consecutive)
 *   permutation uniformly random permutation of 0..n-1 (Fisher-Yates), the
 *               paper's repeat-free random input
 */
#include <stdint.h>
#include <string.h>
#include <math.h>

typedef struct { uint64_t s; } sm64_t;

static inline uint64_t sm64_next(sm64_t* g) {
    uint64_t z = (g->s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* uniform in [0, n) for n <= 2^32 */
static inline uint64_t sm64_bounded(sm64_t* g, uint64_t n) {
    uint64_t r = sm64_next(g) >> 32;
    return (r * n) >> 32;
}

void mmsgen_splitmix64(uint64_t seed, uint64_t* out, uint64_t n) {
    sm64_t g = { seed };
    for (uint64_t i = 0; i < n; ++i) out[i] = sm64_next(&g);
}

void mmsgen_uniform_u32(uint64_t seed, uint32_t* out, uint64_t n) {
    sm64_t g = { seed };
    for (uint64_t i = 0; i < n; ++i) out[i] = (uint32_t)(sm64_next(&g) >> 32);
}

/* n <= 2^32; k swaps of (i, j), each uniform in [0, n), i may equal j */
void mmsgen_nearly_sorted_u32(uint64_t seed, uint32_t* out, uint64_t n, uint64_t k) {
    sm64_t g = { seed };
    for (uint64_t i = 0; i < n; ++i) out[i] = (uint32_t)i;
    if (n == 0) return;
    for (uint64_t t = 0; t < k; ++t) {
        uint64_t i = sm64_bounded(&g, n);
        uint64_t j = sm64_bounded(&g, n);
        uint32_t tmp = out[i]; out[i] = out[j]; out[j] = tmp;
    }
}

void mmsgen_sixteen_u32(uint64_t seed, uint32_t* out, uint64_t n) {
    sm64_t g = { seed };
    for (uint64_t i = 0; i < n; ++i)
        out[i] = (uint32_t)(sm64_next(&g) >> 60) * 0x11111111u;
}

/* n must be a multiple of 64: out[i] = (i mod 64) * (n/64) + floor(i/64) */
int mmsgen_stride64_u32(uint32_t* out, uint64_t n) {
    if (n % 64) return -1;
    uint64_t rows = n / 64;
    for (uint64_t i = 0; i < n; ++i) out[i] = (uint32_t)((i % 64) * rows + i / 64);
    return 0;
}

void mmsgen_permutation_u32(uint64_t seed, uint32_t* out, uint64_t n) {
    sm64_t g = { seed };
    for (uint64_t i = 0; i < n; ++i) out[i] = (uint32_t)i;
    for (uint64_t i = n; i > 1; --i) {
        uint64_t j = sm64_bounded(&g, i);
        uint32_t tmp = out[i - 1]; out[i - 1] = out[j]; out[j] = tmp;
    }
}

void mmsgen_iota_u32(uint32_t* out, uint64_t n) {
    for (uint64_t i = 0; i < n; ++i) out[i] = (uint32_t)i;
}

/* count sizes, each floor(2^(lo + (hi - lo) * u)) with u a 53-bit uniform in [0,1) */
void mmsgen_loguniform_sizes(uint64_t seed, uint64_t* out, uint64_t count, double lo_exp, double hi_exp) {
    sm64_t g = { seed };
    for (uint64_t i = 0; i < count; ++i) {
        double u = (double)(sm64_next(&g) >> 11) * (1.0 / 9007199254740992.0);
        out[i] = (uint64_t)floor(exp2(lo_exp + (hi_exp - lo_exp) * u));
    }
}

/* count uniforms in [0,1) with 53-bit resolution */
void mmsgen_unit_doubles(uint64_t seed, double* out, uint64_t count) {
    sm64_t g = { seed };
    for (uint64_t i = 0; i < count; ++i)
        out[i] = (double)(sm64_next(&g) >> 11) * (1.0 / 9007199254740992.0);
}
