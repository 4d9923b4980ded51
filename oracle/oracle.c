/*
 * CPU oracle for the multiway mergesort (Casanova, Iacono, Karsin,
 * Sitchinava, Weichert, "An Efficient Multiway Mergesort for GPU
 * Architectures", arXiv 1702.07961).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously
 * correct reference that the GPU library is checked against.  It shares no
 * code, header or table with the GPU path, and the GPU library never links,
 * loads or calls it.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg use it.
 *
 * What is computed (the plain definition):
 *   Given keys x_0..x_{n-1}, the sorted output is y_i = x_{p(i)}, where p is
 *   the unique permutation making the pairs (x_{p(i)}, p(i)) strictly
 *   increasing in lexicographic order.  Keys compare as unsigned 32-bit
 *   integers, or as signed 32-bit integers with ORACLE_KEY_I32.  For
 *   key-value pairs the output values are v_{p(i)} (a stable sort).
 *
 * How it is computed: sequential multiway mergesort as described in §4
 * (Multiway Mergesort): repeated merge rounds, each of which merges K sorted
 * lists into one, with the K-way merge done sequentially by a min-heap and an
 * output buffer.  The fan-out here is K = 5 and the initial runs have length
 * 1; the GPU path uses neither, so a planning mistake on one side cannot
 * coincide with the other.  Heap entries compare by (key, run index); runs
 * are contiguous ranges of the current array in input order, so this order
 * equals (key, input index) and the merge is stable.
 *
 * oracle_sort_u64 is the same sort for 64-bit keys and values (§6.3 also
 * sorts 8-byte integers).
 *
 * Also provided, each a direct transcription of a definition:
 *   oracle_partition  the split indices of §4.1 (parallel partitioning) by
 *                     merging K runs and counting, the brute-force way
 *   oracle_select     the i-th element of the sorted order by counting
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_KEY_I32 1u

#define ORACLE_OK 0
#define ORACLE_EINVAL -1
#define ORACLE_ENOMEM -2

#define ORACLE_FANOUT 5

/* ---- key order ----------------------------------------------------------- */

static int key_less(uint32_t a, uint32_t b, int i32) {
    if (i32) return (int32_t)a < (int32_t)b;
    return a < b;
}

/* ---- binary min-heap over (key, run) ------------------------------------ */

typedef struct {
    uint32_t key;
    uint32_t run;    /* run index inside the group being merged */
} hnode_t;

static int hnode_less(hnode_t a, hnode_t b, int i32) {
    if (key_less(a.key, b.key, i32)) return 1;
    if (key_less(b.key, a.key, i32)) return 0;
    return a.run < b.run;
}

typedef struct {
    hnode_t* v;
    int size;
    int i32;
} heap_t;

static void heap_swap(heap_t* h, int i, int j) {
    hnode_t t = h->v[i]; h->v[i] = h->v[j]; h->v[j] = t;
}

static void heap_push(heap_t* h, hnode_t x) {
    int i = h->size++;
    h->v[i] = x;
    while (i > 0) {
        int parent = (i - 1) / 2;
        if (!hnode_less(h->v[i], h->v[parent], h->i32)) break;
        heap_swap(h, i, parent);
        i = parent;
    }
}

static hnode_t heap_pop(heap_t* h) {
    hnode_t top = h->v[0];
    h->v[0] = h->v[--h->size];
    int i = 0;
    for (;;) {
        int l = 2 * i + 1, r = 2 * i + 2, m = i;
        if (l < h->size && hnode_less(h->v[l], h->v[m], h->i32)) m = l;
        if (r < h->size && hnode_less(h->v[r], h->v[m], h->i32)) m = r;
        if (m == i) break;
        heap_swap(h, i, m);
        i = m;
    }
    return top;
}

/* ---- K-way merge of consecutive runs (§4: min-heap plus output buffer) --- */

/*
 * Merge the runs src[starts[j] .. starts[j+1]) for j < nruns into
 * dst[starts[0] .. starts[nruns]).  Values (if any) travel with their keys.
 */
static void merge_runs(const uint32_t* src_k, const uint32_t* src_v,
                       uint32_t* dst_k, uint32_t* dst_v,
                       const uint64_t* starts, int nruns, int i32) {
    hnode_t hv[ORACLE_FANOUT];
    uint64_t next[ORACLE_FANOUT];   /* next unread position of each run */
    heap_t h = { hv, 0, i32 };
    for (int j = 0; j < nruns; ++j) {
        next[j] = starts[j];
        if (next[j] < starts[j + 1]) {
            hnode_t x = { src_k[next[j]], (uint32_t)j };
            heap_push(&h, x);
        }
    }
    uint64_t out = starts[0];
    while (h.size > 0) {
        hnode_t x = heap_pop(&h);
        int j = (int)x.run;
        dst_k[out] = src_k[next[j]];
        if (dst_v) dst_v[out] = src_v[next[j]];
        ++out;
        ++next[j];
        if (next[j] < starts[j + 1]) {
            hnode_t y = { src_k[next[j]], (uint32_t)j };
            heap_push(&h, y);
        }
    }
}

/* ---- the sort ------------------------------------------------------------ */

/*
 * Stable ascending sort of n keys (and values, if vals != NULL).
 * keys/vals are inputs; out_keys/out_vals receive the result (out_vals may be
 * NULL iff vals is NULL).  Inputs and outputs may alias.
 */
int oracle_sort(const uint32_t* keys, const uint32_t* vals,
                uint32_t* out_keys, uint32_t* out_vals,
                uint64_t n, uint32_t flags) {
    if ((vals == NULL) != (out_vals == NULL)) return ORACLE_EINVAL;
    if (n == 0) return ORACLE_OK;
    if (!keys || !out_keys) return ORACLE_EINVAL;
    int i32 = (flags & ORACLE_KEY_I32) != 0;

    uint32_t* a_k = (uint32_t*)malloc(n * sizeof(uint32_t));
    uint32_t* b_k = (uint32_t*)malloc(n * sizeof(uint32_t));
    uint32_t* a_v = vals ? (uint32_t*)malloc(n * sizeof(uint32_t)) : NULL;
    uint32_t* b_v = vals ? (uint32_t*)malloc(n * sizeof(uint32_t)) : NULL;
    if (!a_k || !b_k || (vals && (!a_v || !b_v))) {
        free(a_k); free(b_k); free(a_v); free(b_v);
        return ORACLE_ENOMEM;
    }
    memcpy(a_k, keys, n * sizeof(uint32_t));
    if (vals) memcpy(a_v, vals, n * sizeof(uint32_t));

    /* runs of length 1 are sorted; each round multiplies the run length by K */
    for (uint64_t len = 1; len < n; len *= ORACLE_FANOUT) {
        for (uint64_t g = 0; g < n; g += len * ORACLE_FANOUT) {
            uint64_t starts[ORACLE_FANOUT + 1];
            int nruns = 0;
            for (int j = 0; j <= ORACLE_FANOUT; ++j) {
                uint64_t s = g + (uint64_t)j * len;
                starts[j] = s < n ? s : n;
            }
            for (int j = 0; j < ORACLE_FANOUT; ++j)
                if (starts[j] < starts[j + 1]) nruns = j + 1;
            merge_runs(a_k, a_v, b_k, b_v, starts, nruns, i32);
        }
        uint32_t* t = a_k; a_k = b_k; b_k = t;
        t = a_v; a_v = b_v; b_v = t;
    }

    memcpy(out_keys, a_k, n * sizeof(uint32_t));
    if (vals) memcpy(out_vals, a_v, n * sizeof(uint32_t));
    free(a_k); free(b_k); free(a_v); free(b_v);
    return ORACLE_OK;
}

/*
 * Sort each segment [offsets[s], offsets[s+1]) independently (the batched
 * form: every segment is its own sort).  offsets has nseg+1 entries and must
 * be non-decreasing.
 */
int oracle_sort_segments(const uint32_t* keys, const uint32_t* vals,
                         uint32_t* out_keys, uint32_t* out_vals,
                         const uint64_t* offsets, uint64_t nseg, uint32_t flags) {
    for (uint64_t s = 0; s < nseg; ++s) {
        if (offsets[s + 1] < offsets[s]) return ORACLE_EINVAL;
        uint64_t b = offsets[s], m = offsets[s + 1] - offsets[s];
        int rc = oracle_sort(keys + b, vals ? vals + b : NULL,
                             out_keys + b, out_vals ? out_vals + b : NULL, m, flags);
        if (rc) return rc;
    }
    return ORACLE_OK;
}

/*
 * §4.1 (parallel partitioning): for K sorted runs, the rank-r split is the
 * vector c_0..c_{K-1} such that the prefixes run_k[0 .. c_k) together hold
 * exactly the first r elements of the merged order.  With duplicate keys the
 * order is (key, run index, position), which makes the split unique.
 * Computed by brute force: merge with the min-heap and count where each of
 * the first r outputs came from.
 *   keys        concatenated runs; run k is keys[run_off[k] .. run_off[k+1])
 *   run_off     K+1 non-decreasing offsets
 *   c_out       K outputs, c_out[k] in [0, len_k]
 */
int oracle_partition(const uint32_t* keys, const uint64_t* run_off, uint32_t K,
                     uint64_t r, uint32_t flags, uint64_t* c_out) {
    int i32 = (flags & ORACLE_KEY_I32) != 0;
    uint64_t total = 0;
    for (uint32_t k = 0; k < K; ++k) {
        if (run_off[k + 1] < run_off[k]) return ORACLE_EINVAL;
        total += run_off[k + 1] - run_off[k];
    }
    if (r > total) return ORACLE_EINVAL;
    hnode_t* hv = (hnode_t*)malloc((K ? K : 1) * sizeof(hnode_t));
    uint64_t* next = (uint64_t*)malloc((K ? K : 1) * sizeof(uint64_t));
    if (!hv || !next) { free(hv); free(next); return ORACLE_ENOMEM; }
    heap_t h = { hv, 0, i32 };
    for (uint32_t k = 0; k < K; ++k) {
        next[k] = run_off[k];
        if (next[k] < run_off[k + 1]) {
            hnode_t x = { keys[next[k]], k };
            heap_push(&h, x);
        }
    }
    for (uint64_t t = 0; t < r; ++t) {
        hnode_t x = heap_pop(&h);
        uint32_t k = x.run;
        ++next[k];
        if (next[k] < run_off[k + 1]) {
            hnode_t y = { keys[next[k]], k };
            heap_push(&h, y);
        }
    }
    for (uint32_t k = 0; k < K; ++k) c_out[k] = next[k] - run_off[k];
    free(hv); free(next);
    return ORACLE_OK;
}

/*
 * The element at position i of the stable sorted order, found by counting
 * rather than sorting: its key is the smallest v with #{x <= v} > i, and its
 * input index is that of the (i - #{x < v})-th occurrence of v in input
 * order.  Counting goes by the upper, then the lower 16 bits of the key in
 * the order-preserving unsigned form (sign bit flipped for signed keys).
 */
int oracle_select(const uint32_t* keys, uint64_t n, uint64_t i, uint32_t flags,
                  uint32_t* key_out, uint64_t* index_out) {
    if (i >= n) return ORACLE_EINVAL;
    uint32_t flip = (flags & ORACLE_KEY_I32) ? 0x80000000u : 0u;
    uint64_t* cnt = (uint64_t*)calloc(65536, sizeof(uint64_t));
    if (!cnt) return ORACLE_ENOMEM;

    for (uint64_t j = 0; j < n; ++j) cnt[(keys[j] ^ flip) >> 16]++;
    uint64_t below = 0;
    uint32_t hi = 0;
    while (below + cnt[hi] <= i) below += cnt[hi++];

    memset(cnt, 0, 65536 * sizeof(uint64_t));
    for (uint64_t j = 0; j < n; ++j) {
        uint32_t u = keys[j] ^ flip;
        if ((u >> 16) == hi) cnt[u & 0xFFFFu]++;
    }
    uint32_t lo = 0;
    while (below + cnt[lo] <= i) below += cnt[lo++];
    free(cnt);

    uint32_t v = ((hi << 16) | lo) ^ flip;
    uint64_t want = i - below;     /* occurrences of v to skip */
    for (uint64_t j = 0; j < n; ++j) {
        if (keys[j] == v) {
            if (want == 0) { *key_out = v; *index_out = j; return ORACLE_OK; }
            --want;
        }
    }
    return ORACLE_EINVAL;   /* unreachable for consistent input */
}

/* ======================================================================== */
/* 64-bit keys.  §6.3 also sorts 8-byte integers; the definition is the same
 * with 64-bit keys and values: the output is the unique permutation p making
 * (x_{p(i)}, p(i)) strictly increasing, keys compared as unsigned 64-bit
 * integers, or as signed ones with ORACLE_KEY_I64.  Same method as the 32-bit
 * sort above (runs of 1, fan-out 5, a min-heap over (key, run) per group),
 * written out again for 64-bit keys rather than shared, so a slip in one
 * width cannot hide behind the other.                                      */
/* ======================================================================== */

#define ORACLE_KEY_I64 2u

static int key64_less(uint64_t a, uint64_t b, int i64) {
    if (i64) return (int64_t)a < (int64_t)b;
    return a < b;
}

typedef struct {
    uint64_t key;
    uint32_t run;
} hnode64_t;

static int hnode64_less(hnode64_t a, hnode64_t b, int i64) {
    if (key64_less(a.key, b.key, i64)) return 1;
    if (key64_less(b.key, a.key, i64)) return 0;
    return a.run < b.run;
}

typedef struct {
    hnode64_t* v;
    int size;
    int i64;
} heap64_t;

static void heap64_push(heap64_t* h, hnode64_t x) {
    int i = h->size++;
    h->v[i] = x;
    while (i > 0) {
        int parent = (i - 1) / 2;
        if (!hnode64_less(h->v[i], h->v[parent], h->i64)) break;
        hnode64_t t = h->v[i]; h->v[i] = h->v[parent]; h->v[parent] = t;
        i = parent;
    }
}

static hnode64_t heap64_pop(heap64_t* h) {
    hnode64_t top = h->v[0];
    h->v[0] = h->v[--h->size];
    int i = 0;
    for (;;) {
        int l = 2 * i + 1, r = 2 * i + 2, m = i;
        if (l < h->size && hnode64_less(h->v[l], h->v[m], h->i64)) m = l;
        if (r < h->size && hnode64_less(h->v[r], h->v[m], h->i64)) m = r;
        if (m == i) break;
        hnode64_t t = h->v[i]; h->v[i] = h->v[m]; h->v[m] = t;
        i = m;
    }
    return top;
}

static void merge_runs64(const uint64_t* src_k, const uint64_t* src_v,
                         uint64_t* dst_k, uint64_t* dst_v,
                         const uint64_t* starts, int nruns, int i64) {
    hnode64_t hv[ORACLE_FANOUT];
    uint64_t next[ORACLE_FANOUT];
    heap64_t h = { hv, 0, i64 };
    for (int j = 0; j < nruns; ++j) {
        next[j] = starts[j];
        if (next[j] < starts[j + 1]) {
            hnode64_t x = { src_k[next[j]], (uint32_t)j };
            heap64_push(&h, x);
        }
    }
    uint64_t out = starts[0];
    while (h.size > 0) {
        hnode64_t x = heap64_pop(&h);
        int j = (int)x.run;
        dst_k[out] = src_k[next[j]];
        if (dst_v) dst_v[out] = src_v[next[j]];
        ++out;
        ++next[j];
        if (next[j] < starts[j + 1]) {
            hnode64_t y = { src_k[next[j]], (uint32_t)j };
            heap64_push(&h, y);
        }
    }
}

/*
 * Stable ascending sort of n 64-bit keys (and 64-bit values, if vals !=
 * NULL); same conventions as oracle_sort.
 */
int oracle_sort_u64(const uint64_t* keys, const uint64_t* vals,
                    uint64_t* out_keys, uint64_t* out_vals,
                    uint64_t n, uint32_t flags) {
    if ((vals == NULL) != (out_vals == NULL)) return ORACLE_EINVAL;
    if (n == 0) return ORACLE_OK;
    if (!keys || !out_keys) return ORACLE_EINVAL;
    int i64 = (flags & ORACLE_KEY_I64) != 0;

    uint64_t* a_k = (uint64_t*)malloc(n * sizeof(uint64_t));
    uint64_t* b_k = (uint64_t*)malloc(n * sizeof(uint64_t));
    uint64_t* a_v = vals ? (uint64_t*)malloc(n * sizeof(uint64_t)) : NULL;
    uint64_t* b_v = vals ? (uint64_t*)malloc(n * sizeof(uint64_t)) : NULL;
    if (!a_k || !b_k || (vals && (!a_v || !b_v))) {
        free(a_k); free(b_k); free(a_v); free(b_v);
        return ORACLE_ENOMEM;
    }
    memcpy(a_k, keys, n * sizeof(uint64_t));
    if (vals) memcpy(a_v, vals, n * sizeof(uint64_t));

    for (uint64_t len = 1; len < n; len *= ORACLE_FANOUT) {
        for (uint64_t g = 0; g < n; g += len * ORACLE_FANOUT) {
            uint64_t starts[ORACLE_FANOUT + 1];
            int nruns = 0;
            for (int j = 0; j <= ORACLE_FANOUT; ++j) {
                uint64_t s = g + (uint64_t)j * len;
                starts[j] = s < n ? s : n;
            }
            for (int j = 0; j < ORACLE_FANOUT; ++j)
                if (starts[j] < starts[j + 1]) nruns = j + 1;
            merge_runs64(a_k, a_v, b_k, b_v, starts, nruns, i64);
        }
        uint64_t* t = a_k; a_k = b_k; b_k = t;
        t = a_v; a_v = b_v; b_v = t;
    }

    memcpy(out_keys, a_k, n * sizeof(uint64_t));
    if (vals) memcpy(out_vals, a_v, n * sizeof(uint64_t));
    free(a_k); free(b_k); free(a_v); free(b_v);
    return ORACLE_OK;
}
