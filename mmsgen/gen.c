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

/*
 * Conflict-heavy input for a pairwise merge-path mergesort whose threads
 * each merge vt consecutive outputs (§6.4's conflict-heavy inputs are built
 * against one such sort; the paper gives no recipe, so this one is ours).
 * n must be vt * 2^k.  Reading the sort's merge tree top-down, every merge
 * of two runs of h keys has 2h/vt thread windows of vt outputs, counted from
 * the start of the pair; in the first half of them a cycle of three windows
 * takes vt, vt and 2 outputs from the first run (the rest of the third from
 * the second run), in the second half the roles of the runs swap, and the
 * last windows are adjusted so each run gets exactly h keys.  Threads of a
 * cycle then read the first run at positions 2vt + 2 apart (32 for vt = 15)
 * at every merge step, which for 32 banks is the same bank.  The sorted
 * values 0..n-1 are split this way level by level down to runs of vt keys,
 * which are laid out in descending order.
 */
static int mp_from_first(uint64_t pos, uint64_t pairlen, uint64_t vt) {
    const uint64_t j = pos / vt, off = pos % vt;
    const uint64_t threads = pairlen / vt;
    const int heavy_first = j < threads / 2;
    const int c = (int)(j % 3);
    const int first = c < 2 ? 1 : (off < 2);
    return heavy_first ? first : !first;
}

int mmsgen_mergepath_adversary_u32(uint32_t* out, uint32_t* tmp, uint64_t n, uint64_t vt) {
    if (vt == 0 || n % vt) return -1;
    uint64_t q = n / vt;
    while (q > 1 && q % 2 == 0) q /= 2;
    if (q != 1) return -1;
    for (uint64_t i = 0; i < n; ++i) out[i] = (uint32_t)i;
    for (uint64_t len = n; len > vt; len /= 2) {
        const uint64_t h = len / 2;
        for (uint64_t s = 0; s < n; s += len) {
            const uint32_t* v = out + s;
            /* how many of the pair's outputs the pattern gives the first run */
            uint64_t na = 0;
            for (uint64_t p = 0; p < len; ++p) na += (uint64_t)mp_from_first(p, len, vt);
            /* balance: flip assignments from the end until na == h */
            uint64_t fix_from = len;
            uint64_t cnt = na;
            while (cnt != h && fix_from > 0) {
                --fix_from;
                const int f = mp_from_first(fix_from, len, vt);
                if (cnt > h && f) --cnt;
                else if (cnt < h && !f) ++cnt;
            }
            uint64_t ia = 0, ib = h;
            for (uint64_t p = 0; p < len; ++p) {
                int f = mp_from_first(p, len, vt);
                if (p >= fix_from) f = na > h ? 0 : 1;
                if (f && ia < h) tmp[s + ia++] = v[p];
                else tmp[s + ib++] = v[p];
            }
        }
        memcpy(out, tmp, n * sizeof(uint32_t));
    }
    for (uint64_t s = 0; s < n; s += vt)
        for (uint64_t a = s, b = s + vt - 1; a < b; ++a, --b) {
            uint32_t t = out[a]; out[a] = out[b]; out[b] = t;
        }
    return 0;
}
