// Element kinds of the 64-bit sorts (§6.3 also sorts 8-byte integers) for
// the generic networks of mms_device.h: the bitonic wave sort, the bitonic
// merge of a block and the LDS block merge of two runs.
//
//   E64   a 64-bit key (unsigned order; signed keys are mapped with
//         key ^ 2^63 on the way in and back on the way out)
//   E64V  key, tag, 64-bit value.  The tag is the element's position in the
//         array (or LDS buffer) the pass reads, so (key, tag) is the stable
//         order and every network sorts stably.
//
// Every LDS access below moves one element per lane at consecutive element
// positions (a fixed function of lane and step plus a wave-uniform base), so
// the 64-bit traffic is free of bank conflicts whatever the keys.
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
struct E64V {
    uint64_t k;
    uint32_t t;
    uint64_t v;
    __device__ static E64V sentinel() { return {kSentKey64, kSentTag, 0ull}; }
};

__device__ __forceinline__ bool before(const E64& a, const E64& b) { return a.k < b.k; }
__device__ __forceinline__ bool before(const E64V& a, const E64V& b) {
    return a.k < b.k || (a.k == b.k && a.t < b.t);
}

__device__ __forceinline__ void cex(E64& lo, E64& hi) {
    const uint64_t a = lo.k, b = hi.k;
    const bool sw = b < a;
    lo.k = sw ? b : a;
    hi.k = sw ? a : b;
}
__device__ __forceinline__ void cex(E64V& lo, E64V& hi) {
    const bool sw = before(hi, lo);
    const E64V a = lo, b = hi;
    lo.k = sw ? b.k : a.k; lo.t = sw ? b.t : a.t; lo.v = sw ? b.v : a.v;
    hi.k = sw ? a.k : b.k; hi.t = sw ? a.t : b.t; hi.v = sw ? a.v : b.v;
}

// keep the earlier (want_first) or the later of `mine` and `other`
__device__ __forceinline__ E64 pick(const E64& mine, const E64& other, bool want_first) {
    const bool other_first = other.k < mine.k;
    return {(want_first ? other_first : !other_first) ? other.k : mine.k};
}
__device__ __forceinline__ E64V pick(const E64V& mine, const E64V& other, bool want_first) {
    const bool other_first = before(other, mine);
    const bool take = want_first ? other_first : !other_first;
    return {take ? other.k : mine.k, take ? other.t : mine.t, take ? other.v : mine.v};
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int m) {
    const uint32_t lo = shfl_xor_u32((uint32_t)x, m);
    const uint32_t hi = shfl_xor_u32((uint32_t)(x >> 32), m);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ E64 shfl_xor(const E64& e, int m) { return {shfl_xor_u64(e.k, m)}; }
__device__ __forceinline__ E64V shfl_xor(const E64V& e, int m) {
    return {shfl_xor_u64(e.k, m), shfl_xor_u32(e.t, m), shfl_xor_u64(e.v, m)};
}

// LDS views of a 64-bit merge buffer (see LdsKV32)
struct LdsK64 {
    using El = E64;
    uint64_t* k;
    __device__ __forceinline__ uint64_t key(uint32_t i) const { return k[i]; }
    __device__ __forceinline__ El get(uint32_t i) const { return {k[i]}; }
    __device__ __forceinline__ void put(uint32_t i, const El& e) const { k[i] = e.k; }
};
struct LdsKV64 {
    using El = E64V;
    uint64_t* k;
    uint64_t* v;
    __device__ __forceinline__ uint64_t key(uint32_t i) const { return k[i]; }
    __device__ __forceinline__ El get(uint32_t i) const { return {k[i], i, v[i]}; }
    __device__ __forceinline__ void put(uint32_t i, const El& e) const {
        k[i] = e.k;
        v[i] = e.v;
    }
};

// Memory sinks of a tile's last merge level: position i < lim is stored
// (with the signed-key mapping undone), positions past it are sentinels.
struct GlobalSinkK64 {
    uint64_t* k;
    uint64_t flip;
    uint32_t lim;
    __device__ __forceinline__ void put(uint32_t i, const E64& e) const {
        if (i < lim) gptr64(k)[i] = e.k ^ flip;
    }
};
struct GlobalSinkKV64 {
    uint64_t* k;
    uint64_t* v;
    uint64_t flip;
    uint32_t lim;
    __device__ __forceinline__ void put(uint32_t i, const E64V& e) const {
        if (i < lim) {
            gptr64(k)[i] = e.k ^ flip;
            gptr64(v)[i] = e.v;
        }
    }
};

}  // namespace mms
