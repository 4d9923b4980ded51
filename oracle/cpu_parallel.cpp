// Multi-core CPU sort timed as CONTEXT beside the GPU numbers.
//
// BENCHMARK INFRASTRUCTURE ONLY, and not the oracle: no parity check uses
// it.  It is libstdc++'s parallel mode (__gnu_parallel::stable_sort over
// OpenMP threads), the strongest CPU comparison sort available in this
// image, run on all host cores the process may use.  Only the benchmark's
// CPU-baseline leg calls it; the GPU library never loads it.
//
// Key orders match the oracle's: unsigned 32-bit keys, or signed 32-bit keys
// (flag 1); pairs are sorted stably by key.
#include <parallel/algorithm>

#include <omp.h>
#include <stdint.h>

#include <vector>

extern "C" {

int cpu_parallel_threads(void) { return omp_get_max_threads(); }

// keys in place
int cpu_parallel_sort_u32(uint32_t* keys, uint64_t n, uint32_t flags) {
    if (flags & 1u) {
        int32_t* k = reinterpret_cast<int32_t*>(keys);
        __gnu_parallel::stable_sort(k, k + n);
    } else {
        __gnu_parallel::stable_sort(keys, keys + n);
    }
    return 0;
}

// (key, value) pairs in place, stable by key: sorts (order-preserving key,
// input index) composites, then gathers the values
int cpu_parallel_sort_pairs_u32(uint32_t* keys, uint32_t* vals, uint64_t n, uint32_t flags) {
    const uint32_t flip = (flags & 1u) ? 0x80000000u : 0u;
    std::vector<uint64_t> c(n);
    std::vector<uint32_t> v(vals, vals + n);
#pragma omp parallel for
    for (int64_t i = 0; i < (int64_t)n; ++i) c[i] = ((uint64_t)(keys[i] ^ flip) << 32) | (uint64_t)i;
    __gnu_parallel::sort(c.begin(), c.end());
#pragma omp parallel for
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        keys[i] = (uint32_t)(c[i] >> 32) ^ flip;
        vals[i] = v[(uint32_t)c[i]];
    }
    return 0;
}

// 64-bit keys in place (unsigned)
int cpu_parallel_sort_u64(uint64_t* keys, uint64_t n) {
    __gnu_parallel::stable_sort(keys, keys + n);
    return 0;
}

}  // extern "C"
