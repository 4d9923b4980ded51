// Element kinds of the 64-bit sorts (§6.3 also sorts 8-byte integers) for
// the generic networks of mms_device.h: the bitonic wave sort, the bitonic
// merge of a block and the LDS block merge of two runs.
//
//   E64   a 64-bit key (unsigned order; signed keys are mapped with
//         key ^ 2^63 on the way in and back on the way out)
//   E64T  key and tag.  The tag is the element's slot in the tile as loaded
//         (the runs sit in LDS in run order), so (key, tag) is the stable
//         order and every network sorts stably; the values stay in LDS where
//         they were loaded and are gathered by tag when a tile is stored.
//
// Every LDS access of the networks moves one element per lane at
// consecutive element positions (a fixed function of lane and step plus a
// wave-uniform base), so their traffic is free of bank conflicts whatever
// the keys; only the final gather of values by tag reads data-dependent
// addresses.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mms_device.h"

namespace mms {

constexpr uint64_t kSentKey64 = ~0ull;
constexpr uint32_t kSentTag = 0xFFFFFFFFu;   // above every tag
constexpr uint64_t kSignFlip64 = 0x8000000000000000ull;

typedef __attribute__((address_space(1))) uint64_t gu64;
typedef const __attribute__((address_space(1))) uint64_t cgu64;
__device__ __forceinline__ gu64* gptr64(uint64_t* p) { return (gu64*)p; }
__device__ __forceinline__ cgu64* gptr64(const uint64_t* p) { return (cgu64*)p; }

struct E64 {
    uint64_t k;
    __device__ static E64 sentinel() { return {kSentKey64}; }
};
struct E64T {
    uint64_t k;
    uint32_t t;
    __device__ static E64T sentinel() { return {kSentKey64, kSentTag}; }
};

__device__ __forceinline__ bool before(const E64& a, const E64& b) { return a.k < b.k; }
__device__ __forceinline__ bool before(const E64T& a, const E64T& b) {
    return a.k < b.k || (a.k == b.k && a.t < b.t);
}

__device__ __forceinline__ void cex(E64& lo, E64& hi) {
    const uint64_t a = lo.k, b = hi.k;
    const bool sw = b < a;
    lo.k = sw ? b : a;
    hi.k = sw ? a : b;
}
__device__ __forceinline__ void cex(E64T& lo, E64T& hi) {
    const bool sw = before(hi, lo);
    const E64T a = lo, b = hi;
    lo.k = sw ? b.k : a.k; lo.t = sw ? b.t : a.t;
    hi.k = sw ? a.k : b.k; hi.t = sw ? a.t : b.t;
}

// keep the earlier (want_first) or the later of `mine` and `other`
__device__ __forceinline__ E64 pick(const E64& mine, const E64& other, bool want_first) {
    const bool other_first = other.k < mine.k;
    return {(want_first ? other_first : !other_first) ? other.k : mine.k};
}
__device__ __forceinline__ E64T pick(const E64T& mine, const E64T& other, bool want_first) {
    const bool other_first = before(other, mine);
    const bool take = want_first ? other_first : !other_first;
    return {take ? other.k : mine.k, take ? other.t : mine.t};
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int m) {
    const uint32_t lo = shfl_xor_u32((uint32_t)x, m);
    const uint32_t hi = shfl_xor_u32((uint32_t)(x >> 32), m);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ E64 shfl_xor(const E64& e, int m) { return {shfl_xor_u64(e.k, m)}; }
__device__ __forceinline__ E64T shfl_xor(const E64T& e, int m) {
    return {shfl_xor_u64(e.k, m), shfl_xor_u32(e.t, m)};
}

// LDS views of a 64-bit key-value merge buffer: key(i) and get(i) read
// slot i, put(i, e) writes it (the interface merge_level reads and writes
// through).
// Key-value merge levels: level 0 reads the keys as loaded, each element's
// tag being its own slot; later levels read keys and 16-bit tags written by
// the level before (tile slots stay below 2^16).
struct LdsKT64Loaded {
    using El = E64T;
    uint64_t* k;
    __device__ __forceinline__ uint64_t key(uint32_t i) const { return k[i]; }
    __device__ __forceinline__ El get(uint32_t i) const { return {k[i], i}; }
};
struct LdsKT64 {
    using El = E64T;
    uint64_t* k;
    uint16_t* t;
    __device__ __forceinline__ uint64_t key(uint32_t i) const { return k[i]; }
    __device__ __forceinline__ El get(uint32_t i) const { return {k[i], t[i]}; }
    __device__ __forceinline__ void put(uint32_t i, const El& e) const {
        k[i] = e.k;
        t[i] = (uint16_t)e.t;
    }
};

// Memory sink of a tile's last key-value merge level: position i < lim is
// stored (with the signed-key mapping undone, the value gathered by tag),
// positions past it are sentinels.
struct GlobalSinkKT64 {
    uint64_t* k;
    uint64_t* v;
    const uint64_t* V;   // LDS values, by slot as loaded
    uint64_t flip;
    uint32_t lim;
    __device__ __forceinline__ void put(uint32_t i, const E64T& e) const {
        if (i < lim) {
            gptr64(k)[i] = e.k ^ flip;
            gptr64(v)[i] = V[e.t];
        }
    }
};

}  // namespace mms
