// 64-bit words in the transposed block merge: a (key, tag) pair packed into
// one word for the key-value sorts, or a 64-bit key.
//
// The merge and base case of the key-value sort order the pairs (key, tag),
// tag being an element's slot in the tile as loaded, which is the stable
// order (§4.2 sorts blocks with bitonic networks, which are not stable on
// keys alone); the values stay in LDS where they were loaded and are
// gathered by tag when a tile is stored.  The pair is packed into the
// mantissa of a positive normal double with a fixed exponent:
//   bits 63..52  0x400 (sign 0, biased exponent 1024)
//   bits 51..20  key
//   bits 19..0   tag (< 2^16 here; the sentinel's is 0xFFFFF)
// Doubles of one sign and exponent order like their mantissas, so the 64-bit
// float min and max (one full-rate instruction each, exact, no rounding) are
// the compare-exchange of the pairs, and the sentinel (key 0xFFFFFFFF, tag
// 0xFFFFF) is above every real element.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mms_device.h"
#include "mms_tile_plan.h"

namespace mms {

constexpr uint32_t kKtExp = 0x400u << 20;   // sign and exponent in the high word

__device__ __forceinline__ double kt_join(uint32_t hi, uint32_t lo) {
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ uint32_t kt_hi(double x) { return (uint32_t)(__builtin_bit_cast(uint64_t, x) >> 32); }
__device__ __forceinline__ uint32_t kt_lo(double x) { return (uint32_t)__builtin_bit_cast(uint64_t, x); }

__device__ __forceinline__ double kt_pack(uint32_t key, uint32_t tag) {
    // high word: exponent | key >> 12; low word: key << 20 | tag
    return kt_join(__builtin_amdgcn_alignbit(0x400u, key, 12u), (key << 20) | tag);
}
__device__ __forceinline__ uint32_t kt_key(double x) { return __builtin_amdgcn_alignbit(kt_hi(x), kt_lo(x), 20u); }
__device__ __forceinline__ uint32_t kt_tag(double x) { return kt_lo(x) & 0xFFFFFu; }
__device__ __forceinline__ double kt_sentinel() { return kt_join(kKtExp | 0xFFFFFu, 0xFFFFFFFFu); }

// min and max as single instructions (the library's fmin would first
// quieten possible signalling NaNs, which these values never are)
__device__ __forceinline__ double kt_min(double a, double b) {
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double kt_max(double a, double b) {
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ void cex_kt(double& lo, double& hi) {
    const double a = lo, b = hi;
    lo = kt_min(a, b);
    hi = kt_max(a, b);
}

// The transposed block merge below runs on any 64-bit word with these
// operations: packed (key, tag) doubles, or 64-bit keys (unsigned order, a
// compare and two selects per compare-exchange half).
__device__ __forceinline__ uint32_t w_hi(double x) { return kt_hi(x); }
__device__ __forceinline__ uint32_t w_lo(double x) { return kt_lo(x); }
__device__ __forceinline__ uint32_t w_hi(uint64_t x) { return (uint32_t)(x >> 32); }
__device__ __forceinline__ uint32_t w_lo(uint64_t x) { return (uint32_t)x; }
template <class T> __device__ __forceinline__ T w_join(uint32_t hi, uint32_t lo);
template <> __device__ __forceinline__ double w_join<double>(uint32_t hi, uint32_t lo) { return kt_join(hi, lo); }
template <> __device__ __forceinline__ uint64_t w_join<uint64_t>(uint32_t hi, uint32_t lo) {
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ void w_cex(double& lo, double& hi) { cex_kt(lo, hi); }
__device__ __forceinline__ void w_cex(uint64_t& lo, uint64_t& hi) {
    const uint64_t a = lo, b = hi;
    const bool sw = b < a;
    lo = sw ? b : a;
    hi = sw ? a : b;
}
__device__ __forceinline__ double w_min(double a, double b) { return kt_min(a, b); }
__device__ __forceinline__ uint64_t w_min(uint64_t a, uint64_t b) { return b < a ? b : a; }
template <class T> __device__ __forceinline__ T w_sentinel();
template <> __device__ __forceinline__ double w_sentinel<double>() { return kt_sentinel(); }
template <> __device__ __forceinline__ uint64_t w_sentinel<uint64_t>() { return ~0ull; }

template <int EM, class T>
__device__ __forceinline__ void reg_stages_kt(T (&m)[EM]) {
#pragma unroll
    for (int d = EM / 2; d >= 1; d >>= 1) {
#pragma unroll
        for (int e = 0; e < EM; ++e)
            if ((e & d) == 0) w_cex(m[e], m[e | d]);
    }
}

// One transpose step of block_sort_kt for one 32-bit half of every element:
// write the half at wr(e), read it back at rd(e).  The LDS performs a wave's
// operations in order, so the second half's writes may follow the first
// half's reads into the same scratch without a wait.
template <int EM, class Wr, class Rd>
__device__ __forceinline__ void xpose_half(uint32_t (&h)[EM], uint32_t* scr, Wr wr, Rd rd) {
#pragma unroll
    for (int e = 0; e < EM; ++e) scr[wr(e)] = h[e];
    lds_wave_sync();
#pragma unroll
    for (int e = 0; e < EM; ++e) h[e] = scr[rd(e)];
    lds_wave_sync();
}

// Sort the bitonic block of N = 64*EM pairs held in layout S (register =
// index bits above 6, lane = bits 5..0) into layout F (register 4c+j =
// position c*256 + 4*lane + j), with the index moves of block_sort_keys and
// the same conflict-free scratch pattern, each transpose done once for the
// high and once for the low words.
template <int EM, class T>
__device__ __forceinline__ void block_sort_kt(T (&m)[EM], uint32_t* scr, int lane) {
    static_assert(EM == 8, "64x8-pair blocks");
    constexpr uint32_t RS = Xpose<EM>::RS;
    const uint32_t ul = (uint32_t)lane;
    asm volatile("" ::: "memory");                       // the previous block's scratch reads come first
    reg_stages_kt<EM>(m);                                // index bits 8..6
    uint32_t hi[EM], lo[EM];
#pragma unroll
    for (int e = 0; e < EM; ++e) {
        hi[e] = w_hi(m[e]);
        lo[e] = w_lo(m[e]);
    }
    const uint32_t tb = (ul >> 3) * RS + (ul & 7u);      // lane = (bits 8..6, bits 2..0)
    auto s_at = [&](int e) { return (uint32_t)e * RS + ul; };
    auto t_at = [&](int e) { return tb + (uint32_t)e * 8u; };
    xpose_half<EM>(hi, scr, s_at, t_at);
    xpose_half<EM>(lo, scr, s_at, t_at);
#pragma unroll
    for (int e = 0; e < EM; ++e) m[e] = w_join<T>(hi[e], lo[e]);
    reg_stages_kt<EM>(m);                                // index bits 5..3
#pragma unroll
    for (int e = 0; e < EM; ++e) {
        hi[e] = w_hi(m[e]);
        lo[e] = w_lo(m[e]);
    }
    const uint32_t fb = (ul >> 4) * RS + 4u * (ul & 15u);
    auto to_f = [&](uint32_t (&h)[EM]) {
#pragma unroll
        for (int e = 0; e < EM; ++e) scr[t_at(e)] = h[e];
        lds_wave_sync();
#pragma unroll
        for (int c = 0; c < EM / 4; ++c) {
            const uint4 v = *reinterpret_cast<const uint4*>(scr + fb + (uint32_t)c * 4u * RS);
            h[4 * c + 0] = v.x;
            h[4 * c + 1] = v.y;
            h[4 * c + 2] = v.z;
            h[4 * c + 3] = v.w;
        }
        lds_wave_sync();
    };
    to_f(hi);
    to_f(lo);
    // index bit 2 = lane bit 0: lanes l and l ^ 1 meet, the odd lane keeps
    // the larger pair
    const bool keep_max = (ul & 1u) != 0;
    uint32_t oh[EM], ol[EM];
#pragma unroll
    for (int e = 0; e < EM; ++e) {
        oh[e] = (uint32_t)__builtin_amdgcn_mov_dpp((int)hi[e], 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
        ol[e] = (uint32_t)__builtin_amdgcn_mov_dpp((int)lo[e], 0xB1, 0xF, 0xF, false);
    }
#pragma unroll
    for (int e = 0; e < EM; ++e) {
        const T a = w_join<T>(hi[e], lo[e]), o = w_join<T>(oh[e], ol[e]);
        m[e] = ((o < a) != keep_max) ? o : a;   // one compare, two selects
    }
#pragma unroll
    for (int c = 0; c < EM / 4; ++c) {                   // index bits 1..0
        w_cex(m[4 * c + 0], m[4 * c + 2]);
        w_cex(m[4 * c + 1], m[4 * c + 3]);
        w_cex(m[4 * c + 0], m[4 * c + 1]);
        w_cex(m[4 * c + 2], m[4 * c + 3]);
    }
}

// A (key, tag) word as an element of the generic networks (wave_sort_blocked,
// wave_merge_tail): compare-exchange by min and max, a lane-dependent pick by
// one compare, and lane exchanges of both halves.
struct ElemKT {
    double d;
    __device__ static ElemKT sentinel() { return {kt_sentinel()}; }
};
__device__ __forceinline__ void cex(ElemKT& lo, ElemKT& hi) { cex_kt(lo.d, hi.d); }
__device__ __forceinline__ ElemKT pick(const ElemKT& mine, const ElemKT& other, bool want_first) {
    const bool other_first = other.d < mine.d;
    return (want_first == other_first) ? other : mine;
}
__device__ __forceinline__ ElemKT shfl_xor(const ElemKT& e, int m) {
    return {kt_join(shfl_xor_u32(kt_hi(e.d), m), shfl_xor_u32(kt_lo(e.d), m))};
}

// Number of block positions k with a_k < b_k (a increasing and b
// decreasing in k, so they form a prefix): the sum of the registers' ballot
// counts, with no branch, as prefix_len does for keys.
template <int EM, class T>
__device__ __forceinline__ uint32_t prefix_len_kt(const T (&a)[EM], const T (&b)[EM]) {
    uint32_t u = 0;
#pragma unroll
    for (int e = 0; e < EM; ++e) u += (uint32_t)__popcll(__ballot(a[e] < b[e]));
    return u;
}

// LDS sources of a merge level.  Level 0 reads the keys as loaded, each
// element's tag being its own slot; later levels read keys and 16-bit tags.
// from(i) gives a cursor at slot i whose at(off) reads slot i + off, so the
// reads of a block share one address register and constant offsets; raw
// returns the key and tag unpacked, so a block's reads can all be issued
// before the first is used.
struct KtSrcLoaded {
    using Word = double;
    const uint32_t* k;
    struct Cur {
        const uint32_t* k;
        uint32_t t0;
        __device__ __forceinline__ void raw(uint32_t off, uint32_t& key, uint32_t& tag) const {
            key = k[off];
            tag = t0 + off;
        }
    };
    __device__ __forceinline__ Cur from(uint32_t i) const { return {k + i, i}; }
    __device__ __forceinline__ uint32_t corank(uint32_t aA, uint32_t la, uint32_t aB, uint32_t lb, uint32_t d,
                                               int lane) const {
        return lds_corank2(k, aA, la, aB, lb, d, lane);
    }
    // pairs i .. i+3 (i a multiple of 4)
    __device__ __forceinline__ void at4(uint32_t i, double* r) const {
        const uint4 v = *reinterpret_cast<const uint4*>(k + i);
        r[0] = kt_pack(v.x, i);
        r[1] = kt_pack(v.y, i + 1u);
        r[2] = kt_pack(v.z, i + 2u);
        r[3] = kt_pack(v.w, i + 3u);
    }
};
struct KtSrcTagged {
    using Word = double;
    const uint32_t* k;
    const uint16_t* t;
    struct Cur {
        const uint32_t* k;
        const uint16_t* t;
        __device__ __forceinline__ void raw(uint32_t off, uint32_t& key, uint32_t& tag) const {
            key = k[off];
            tag = t[off];
        }
    };
    __device__ __forceinline__ Cur from(uint32_t i) const { return {k + i, t + i}; }
    __device__ __forceinline__ uint32_t corank(uint32_t aA, uint32_t la, uint32_t aB, uint32_t lb, uint32_t d,
                                               int lane) const {
        return lds_corank2(k, aA, la, aB, lb, d, lane);
    }
    __device__ __forceinline__ void at4(uint32_t i, double* r) const {
        const uint4 v = *reinterpret_cast<const uint4*>(k + i);
        const uint2 w = *reinterpret_cast<const uint2*>(t + i);
        r[0] = kt_pack(v.x, w.x & 0xFFFFu);
        r[1] = kt_pack(v.y, w.x >> 16);
        r[2] = kt_pack(v.z, w.y & 0xFFFFu);
        r[3] = kt_pack(v.w, w.y >> 16);
    }
};

// Sinks for a sorted block in layout F: block position t = c*256 + 4*lane +
// j goes to pos0 + t when t < cnt (pos0 a multiple of 4).
struct KtSinkLds {
    uint32_t* k;
    uint16_t* t;
    template <int EM>
    __device__ __forceinline__ void put_block(uint32_t pos0, uint32_t cnt, const double (&m)[EM], int lane) const {
        uint32_t* ok = k + pos0;
        uint16_t* ot = t + pos0;
        store_block<EM>(
            cnt, true, lane,
            [&](int c, uint32_t p) {
                const double* r = m + 4 * c;
                *reinterpret_cast<uint4*>(ok + p) = make_uint4(kt_key(r[0]), kt_key(r[1]), kt_key(r[2]), kt_key(r[3]));
                // two 16-bit tags per word: the low halves of the low words
                *reinterpret_cast<uint2*>(ot + p) =
                    make_uint2(__builtin_amdgcn_perm(kt_lo(r[1]), kt_lo(r[0]), 0x05040100u),
                               __builtin_amdgcn_perm(kt_lo(r[3]), kt_lo(r[2]), 0x05040100u));
            },
            [&](int c, int j, uint32_t p) {
                ok[p] = kt_key(m[4 * c + j]);
                ot[p] = (uint16_t)kt_lo(m[4 * c + j]);
            });
    }
};
// The last level: keys to memory (undoing the signed-key mapping) and each
// pair's value, gathered from the tile's value slots by its tag.
struct KtSinkGlobal {
    uint32_t* k;         // tile output base
    uint32_t* v;
    const uint32_t* V;   // LDS values, by slot
    uint32_t flip;
    uint32_t lim;        // positions >= lim are not stored
    bool vec;            // k and v are 16-byte aligned
    template <int EM>
    __device__ __forceinline__ void put_block(uint32_t pos0, uint32_t cnt, const double (&m)[EM], int lane) const {
        gu32* gk = gptr(k) + pos0;
        gu32* gv = gptr(v) + pos0;
        store_block<EM>(
            min(cnt, lim > pos0 ? lim - pos0 : 0u), vec, lane,
            [&](int c, uint32_t p) {
                const double* r = m + 4 * c;
                *reinterpret_cast<gu32x4*>(gk + p) =
                    u32x4{kt_key(r[0]) ^ flip, kt_key(r[1]) ^ flip, kt_key(r[2]) ^ flip, kt_key(r[3]) ^ flip};
                *reinterpret_cast<gu32x4*>(gv + p) =
                    u32x4{V[kt_tag(r[0])], V[kt_tag(r[1])], V[kt_tag(r[2])], V[kt_tag(r[3])]};
            },
            [&](int c, int j, uint32_t p) {
                gk[p] = kt_key(m[4 * c + j]) ^ flip;
                gv[p] = V[kt_tag(m[4 * c + j])];
            });
    }
};

// A block's candidates: a_e = A[64e] (lane's own offset in A) and b_e =
// B[64(EM-1-e)], every read issued before any is packed.
template <int EM, class Cur>
__device__ __forceinline__ void read_block(const Cur& A, const Cur& B, double (&a)[EM], double (&b)[EM]) {
    uint32_t ka[EM], ta[EM], kb[EM], tb[EM];
#pragma unroll
    for (int e = 0; e < EM; ++e) {
        A.raw((uint32_t)e * kWave, ka[e], ta[e]);
        B.raw((uint32_t)(EM - 1 - e) * kWave, kb[e], tb[e]);
    }
#pragma unroll
    for (int e = 0; e < EM; ++e) {
        a[e] = kt_pack(ka[e], ta[e]);
        b[e] = kt_pack(kb[e], tb[e]);
    }
}

// Merge outputs [d0, d1) of A = X[aA, aA+la) and B = X[aB, aB+lb) in blocks
// of N = 64*EM words, the 64-bit form of merge_pair_range_keys.  For packed
// (key, tag) pairs A holds the smaller tags, so the split on keys with A
// first on ties is the split of the pair order; for 64-bit keys a key equal
// to the sentinel stands in for it, as in the 32-bit keys merge.
// out_base + d0 must be a multiple of 4.
template <int EM, class Src, class Sink>
__device__ __forceinline__ void merge_pair_range_kt(const Src& X, uint32_t aA, uint32_t la, uint32_t aB, uint32_t lb,
                                                    uint32_t d0, uint32_t d1, const Sink& out, uint32_t out_base,
                                                    uint32_t* scr, int lane) {
    using T = typename Src::Word;
    constexpr uint32_t N = (uint32_t)kWave * EM;
    if (la == 0 || lb == 0) {
        // one run is empty: the other is already in order; move it in the
        // block layout (reads past the run stay in the caller's LDS and are
        // not stored)
        const uint32_t a0 = lb == 0 ? aA : aB;
        for (uint32_t o = d0; o < d1; o += N) {
            T m[EM];
#pragma unroll
            for (int c = 0; c < EM / 4; ++c) X.at4(a0 + o + (uint32_t)c * 256u + 4u * (uint32_t)lane, m + 4 * c);
            out.template put_block<EM>(out_base + o, min(N, d1 - o), m, lane);
        }
        return;
    }
    if (d0 == 0 && d1 == la + lb && la <= N && lb <= N && la + lb > N) {
        // the whole pair from one read, as in merge_pair_range_keys: the
        // minimum and maximum halves of the bitonic sequence of A and
        // reversed B (each padded with sentinels to N) are sorted apart; a
        // sentinel orders after every element, so the second half's
        // la + lb - N stored positions hold elements only
        const auto A = X.from(aA + (uint32_t)lane);
        const auto B = X.from(aB + (N - 1u) - (uint32_t)lane - (uint32_t)(EM - 1) * kWave);
        T lo[EM], hi[EM];
        read_block<EM>(A, B, lo, hi);
#pragma unroll
        for (int e = 0; e < EM; ++e) {
            const uint32_t k = (uint32_t)e * kWave + (uint32_t)lane;
            lo[e] = k < la ? lo[e] : w_sentinel<T>();
            hi[e] = N - 1u - k < lb ? hi[e] : w_sentinel<T>();
            w_cex(lo[e], hi[e]);
        }
        block_sort_kt<EM>(lo, scr, lane);
        out.template put_block<EM>(out_base, N, lo, lane);
        block_sort_kt<EM>(hi, scr, lane);
        out.template put_block<EM>(out_base + N, la + lb - N, hi, lane);
        return;
    }
    uint32_t p = X.corank(aA, la, aB, lb, d0, lane);
    uint32_t q = d0 - p;
    for (uint32_t o = d0; o < d1; o += N) {
        T m[EM];
        uint32_t u;
        if (p + N <= la && q + N <= lb) {
            // b's reads from its lowest position up, so every address is a
            // base plus a constant offset
            const auto A = X.from(aA + p + (uint32_t)lane);
            const auto B = X.from(aB + q + (N - 1u) - (uint32_t)lane - (uint32_t)(EM - 1) * kWave);
            T a[EM], b[EM];
            read_block<EM>(A, B, a, b);
#pragma unroll
            for (int e = 0; e < EM; ++e) m[e] = w_min(a[e], b[e]);
            u = prefix_len_kt<EM, T>(a, b);
        } else {
            // near the end of a run: the same reads, then the sentinel for
            // every position past a run's end.  Those reads stay below the
            // end of the last run plus N, inside the caller's LDS; what they
            // return is discarded.  Only positions where a is strictly below
            // b count as taken from A, so the A cursor stays inside its run
            // and the B cursor passes its end only in the range's last
            // block.
            const uint32_t pc = min(p, la), qc = min(q, lb);
            const auto A = X.from(aA + pc + (uint32_t)lane);
            const auto B = X.from(aB + qc + (N - 1u) - (uint32_t)lane - (uint32_t)(EM - 1) * kWave);
            const uint32_t ra = la - pc, rb = lb - qc;
            T a[EM], b[EM];
            read_block<EM>(A, B, a, b);
            if (ra < N) {   // one wave-uniform branch per run that ends inside the block
#pragma unroll
                for (int e = 0; e < EM; ++e)
                    a[e] = (uint32_t)e * kWave + (uint32_t)lane < ra ? a[e] : w_sentinel<T>();
            }
            if (rb < N) {
#pragma unroll
                for (int e = 0; e < EM; ++e)
                    b[e] = N - 1u - ((uint32_t)e * kWave + (uint32_t)lane) < rb ? b[e] : w_sentinel<T>();
            }
#pragma unroll
            for (int e = 0; e < EM; ++e) m[e] = w_min(a[e], b[e]);
            u = prefix_len_kt<EM, T>(a, b);
        }
        block_sort_kt<EM>(m, scr, lane);
        out.template put_block<EM>(out_base + o, min(N, d1 - o), m, lane);
        p += u;   // u is a sum of ballot counts: the cursors stay wave-uniform
        q += N - u;
    }
}

// 64-bit keys: one LDS array of words, and the sinks of a sorted block in
// layout F (block position t = c*256 + 4*lane + j, four consecutive words per
// lane and c: two 16-byte accesses).
struct U64Src {
    using Word = uint64_t;
    const uint64_t* k;
    struct Cur {
        const uint64_t* k;
    };
    __device__ __forceinline__ Cur from(uint32_t i) const { return {k + i}; }
    __device__ __forceinline__ uint64_t key(uint32_t i) const { return k[i]; }
    __device__ __forceinline__ void at4(uint32_t i, uint64_t* r) const {
        const ulonglong2 v0 = *reinterpret_cast<const ulonglong2*>(k + i);
        const ulonglong2 v1 = *reinterpret_cast<const ulonglong2*>(k + i + 2);
        r[0] = v0.x;
        r[1] = v0.y;
        r[2] = v1.x;
        r[3] = v1.y;
    }
    __device__ __forceinline__ uint32_t corank(uint32_t aA, uint32_t la, uint32_t aB, uint32_t lb, uint32_t d,
                                               int lane) const {
        return lds_corank2_view(*this, aA, la, aB, lb, d, lane);
    }
};
template <int EM>
__device__ __forceinline__ void read_block(const U64Src::Cur& A, const U64Src::Cur& B, uint64_t (&a)[EM],
                                           uint64_t (&b)[EM]) {
#pragma unroll
    for (int e = 0; e < EM; ++e) {
        a[e] = A.k[(uint32_t)e * kWave];
        b[e] = B.k[(uint32_t)(EM - 1 - e) * kWave];
    }
}
struct U64SinkLds {
    uint64_t* k;
    template <int EM>
    __device__ __forceinline__ void put_block(uint32_t pos0, uint32_t cnt, const uint64_t (&m)[EM], int lane) const {
        uint64_t* o = k + pos0;
        store_block<EM>(
            cnt, true, lane,
            [&](int c, uint32_t p) {
                const uint64_t* r = m + 4 * c;
                *reinterpret_cast<ulonglong2*>(o + p) = make_ulonglong2(r[0], r[1]);
                *reinterpret_cast<ulonglong2*>(o + p + 2) = make_ulonglong2(r[2], r[3]);
            },
            [&](int c, int j, uint32_t p) { o[p] = m[4 * c + j]; });
    }
};
struct U64SinkGlobal {
    uint64_t* k;         // tile output base
    uint64_t flip;
    uint32_t lim;        // positions >= lim are not stored
    bool vec;            // k is 16-byte aligned
    template <int EM>
    __device__ __forceinline__ void put_block(uint32_t pos0, uint32_t cnt, const uint64_t (&m)[EM], int lane) const {
        typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
        typedef __attribute__((address_space(1))) u64x2 gu64x2_t;
        typedef __attribute__((address_space(1))) uint64_t gu64_t;
        gu64_t* g = (gu64_t*)k + pos0;
        store_block<EM>(
            min(cnt, lim > pos0 ? lim - pos0 : 0u), vec, lane,
            [&](int c, uint32_t p) {
                const uint64_t* r = m + 4 * c;
                *reinterpret_cast<gu64x2_t*>(g + p) = u64x2{r[0] ^ flip, r[1] ^ flip};
                *reinterpret_cast<gu64x2_t*>(g + p + 2) = u64x2{r[2] ^ flip, r[3] ^ flip};
            },
            [&](int c, int j, uint32_t p) { g[p] = m[4 * c + j] ^ flip; });
    }
};

// One planned merge level (the plan's encoding as in the keys merge).
template <int EM, class Src, class Sink>
__device__ __forceinline__ void merge_level_kt(const Src& X, const Meta& mt, uint32_t nseg0, uint32_t lvl,
                                               const Sink& out, uint32_t* scr, int wave, int lane) {
    const uint32_t* pw = mt.plan + 2u * (lvl * 16u + (uint32_t)wave);
    const uint32_t w0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)pw[0]);
    uint32_t own = (uint32_t)__builtin_amdgcn_readfirstlane((int)pw[1]);
    auto run = [&](uint32_t i, uint32_t d0, uint32_t d1, bool whole) {
        const uint32_t g0 = min((2u * i) << lvl, nseg0);
        const uint32_t g1 = min((2u * i + 1u) << lvl, nseg0);
        const uint32_t g2 = min((2u * i + 2u) << lvl, nseg0);
        const uint32_t aA = (uint32_t)__builtin_amdgcn_readfirstlane((int)mt.sbeg[g0]);
        const uint32_t aB = (uint32_t)__builtin_amdgcn_readfirstlane((int)mt.sbeg[g1]);
        const uint32_t p0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)mt.plen[g0]);
        const uint32_t p1 = (uint32_t)__builtin_amdgcn_readfirstlane((int)mt.plen[g1]);
        const uint32_t p2 = (uint32_t)__builtin_amdgcn_readfirstlane((int)mt.plen[g2]);
        const uint32_t la = p1 - p0, lb = p2 - p1;
        if (whole) d1 = la + lb;
        if (d0 < d1) merge_pair_range_kt<EM>(X, aA, la, aB, lb, d0, d1, out, aA, scr, lane);
    };
    run(w0 & 15u, (w0 >> 4) & 0x3FFFu, w0 >> 18, false);
    while (own) {
        const uint32_t i = (uint32_t)__builtin_ctz(own);
        own &= own - 1u;
        run(i, 0u, 0u, true);
    }
}

}  // namespace mms
