// Device building blocks of the multiway mergesort on gfx950 (wave64).
//
// Everything here obeys one rule that makes the LDS traffic free of bank
// conflicts whatever the data: every LDS instruction touches addresses that
// are a fixed function of (lane, step) plus a wave-uniform base.  All
// data-dependent routing happens in registers, through compare-exchange
// networks and cross-lane exchanges (§2.2 and §4.2 of the paper explain why
// data-dependent shared-memory addressing is what costs the pairwise
// mergesorts their bank conflicts).
//
// Element kinds: Elem<false> is a 32-bit key (unsigned order; signed keys
// are mapped with key ^ 0x80000000 on the way in and back on the way out).
// Key-value sorts use the (key, tag) words of mms_device_kt.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mms {

constexpr int kWave = 64;
constexpr uint32_t kSentKey = 0xFFFFFFFFu;

// Global-memory views.  Accesses through generic pointers compile to FLAT
// instructions, which count against the LDS counter as well as the vector
// memory counter, so an LDS barrier would wait for them; through
// address-space-1 pointers they become global_* instructions.
typedef __attribute__((address_space(1))) uint32_t gu32;
typedef const __attribute__((address_space(1))) uint32_t cgu32;
// four keys at a 4-byte aligned global address
typedef uint32_t u32x4a4 __attribute__((ext_vector_type(4), aligned(4)));
typedef const __attribute__((address_space(1))) u32x4a4 cgu32x4a4;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) u32x4 gu32x4;

__device__ __forceinline__ gu32* gptr(uint32_t* p) { return (gu32*)p; }
__device__ __forceinline__ cgu32* gptr(const uint32_t* p) { return (cgu32*)p; }

template <bool P> struct Elem;
template <> struct Elem<false> {
    uint32_t k;
    __device__ static Elem sentinel() { return {kSentKey}; }
};

// strict "a comes before b"
__device__ __forceinline__ bool before(const Elem<false>& a, const Elem<false>& b) { return a.k < b.k; }

// compare-exchange: lo receives the earlier element, hi the later one
__device__ __forceinline__ void cex(Elem<false>& lo, Elem<false>& hi) {
    uint32_t a = lo.k, b = hi.k;
    lo.k = min(a, b);
    hi.k = max(a, b);
}

// Median of three unsigned values in one instruction: with c = 0 it is
// min(a, b), with c = ~0 it is max(a, b), so a lane-dependent c picks the
// lower or upper half of a compare-exchange without a select.
__device__ __forceinline__ uint32_t med3_u32(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t d;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

// keep the earlier (want_first) or the later of `mine` and `other`
__device__ __forceinline__ Elem<false> pick(const Elem<false>& mine, const Elem<false>& other, bool want_first) {
    return {med3_u32(mine.k, other.k, want_first ? 0u : ~0u)};
}

// Value of lane (lane ^ m).  When m is a constant (after loop unrolling)
// this folds to one exchange: DPP within a row of 16 lanes
// (quad permutes, row mirrors, rotate by 8), a ds_swizzle inside 32 lanes,
// and ds_bpermute across the halves of the wave.
__device__ __forceinline__ uint32_t shfl_xor_u32(uint32_t x, int m) {
    const int v = (int)x;
    // a mask only known at run time (a loop the compiler kept rolled) takes
    // the general permute rather than a branch per exchange
    if (!__builtin_constant_p(m)) return (uint32_t)__shfl_xor(v, m, kWave);
    switch (m) {
        case 1: return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);    // quad_perm [1,0,3,2]
        case 2: return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);    // quad_perm [2,3,0,1]
        case 3: return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0x1B, 0xF, 0xF, false);    // quad_perm [3,2,1,0]
        case 7: return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false);   // row_half_mirror
        case 8: return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);   // row_ror:8
        case 15: return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false);  // row_mirror
        // bit-mask swizzle inside 32 lanes: and 0x1F, or 0, xor m
        case 4: return (uint32_t)__builtin_amdgcn_ds_swizzle(v, 0x1F | (4 << 10));
        case 16: return (uint32_t)__builtin_amdgcn_ds_swizzle(v, 0x1F | (16 << 10));
        case 31: return (uint32_t)__builtin_amdgcn_ds_swizzle(v, 0x1F | (31 << 10));
        default: return (uint32_t)__shfl_xor(v, m, kWave);
    }
}
__device__ __forceinline__ Elem<false> shfl_xor(const Elem<false>& e, int m) { return {shfl_xor_u32(e.k, m)}; }

// ---------------------------------------------------------------------------
// Base case: sort the 64*E elements a wave holds, E per lane (§4.3 sorts a
// W x W grid with rows in registers and transposes; here every stage is a
// bitonic compare-exchange, in-lane for index bits below log2(E) and across
// lanes for the rest).  Result layout is "blocked": lane l holds positions
// l*E .. l*E+E-1 of the wave's sorted run.
// ---------------------------------------------------------------------------
template <int E, class El>
__device__ __forceinline__ void wave_sort_blocked(El (&r)[E], int lane) {
#pragma unroll
    for (int s = 1; s < E; s <<= 1) {
#pragma unroll
        for (int e = 0; e < E; ++e)
            if ((e & s) == 0) cex(r[e], r[e ^ (2 * s - 1)]);
#pragma unroll
        for (int d = s / 2; d >= 1; d >>= 1) {
#pragma unroll
            for (int e = 0; e < E; ++e)
                if ((e & d) == 0) cex(r[e], r[e | d]);
        }
    }
#pragma unroll
    for (int sl = 1; sl < kWave; sl <<= 1) {
        // mirror stage: (lane, e) meets (lane ^ (2sl-1), E-1-e)
        const bool lower = (lane & sl) == 0;
        El t[E];
#pragma unroll
        for (int e = 0; e < E; ++e) t[e] = pick(r[e], shfl_xor(r[E - 1 - e], 2 * sl - 1), lower);
#pragma unroll
        for (int e = 0; e < E; ++e) r[e] = t[e];
#pragma unroll
        for (int dl = sl / 2; dl >= 1; dl >>= 1) {
            const bool lo = (lane & dl) == 0;
#pragma unroll
            for (int e = 0; e < E; ++e) r[e] = pick(r[e], shfl_xor(r[e], dl), lo);
        }
#pragma unroll
        for (int d = E / 2; d >= 1; d >>= 1) {
#pragma unroll
            for (int e = 0; e < E; ++e)
                if ((e & d) == 0) cex(r[e], r[e | d]);
        }
    }
}

// The in-wave tail of a bitonic merge in the blocked layout: lane distances
// 32 .. 1, then register distances (after the cross-wave stages of a
// workgroup-wide merge).
template <int E, class El>
__device__ __forceinline__ void wave_merge_tail(El (&r)[E], int lane) {
#pragma unroll
    for (int dl = kWave / 2; dl >= 1; dl >>= 1) {
        const bool lo = (lane & dl) == 0;
#pragma unroll
        for (int e = 0; e < E; ++e) r[e] = pick(r[e], shfl_xor(r[e], dl), lo);
    }
#pragma unroll
    for (int d = E / 2; d >= 1; d >>= 1) {
#pragma unroll
        for (int e = 0; e < E; ++e)
            if ((e & d) == 0) cex(r[e], r[e | d]);
    }
}

// ---------------------------------------------------------------------------
// Bitonic merge of 64*EM elements held "striped" (lane l, register e holds
// index e*64 + l): register distances first, then lane distances 32..1.
// ---------------------------------------------------------------------------
template <int EM, class El>
__device__ __forceinline__ void bitonic_merge_striped(El (&m)[EM], int lane) {
#pragma unroll
    for (int d = EM / 2; d >= 1; d >>= 1) {
#pragma unroll
        for (int e = 0; e < EM; ++e)
            if ((e & d) == 0) cex(m[e], m[e | d]);
    }
#pragma unroll
    for (int dl = kWave / 2; dl >= 1; dl >>= 1) {
        const bool lo = (lane & dl) == 0;
#pragma unroll
        for (int e = 0; e < EM; ++e) m[e] = pick(m[e], shfl_xor(m[e], dl), lo);
    }
}

// ---------------------------------------------------------------------------
// Merge-path split inside LDS: the number p of elements of A = X[aA, aA+la)
// among the first d elements of merge(A, B = X[aB, aB+lb)), A first on ties.
// The wave probes 64 points per round, one per lane, with an odd stride, so
// the 64 reads of one round fall in 64 distinct banks (for 64-bit keys, on
// distinct bank pairs: 32 lanes are served per cycle and lane l covers words
// 2(c + l*step) and 2(c + l*step) + 1).  A range of R > 1 candidates takes
// ceil(log64 R) rounds: at most two for every merge tile here.  X is an LDS view
// (key(i)); keys are compared alone, A first on ties, which is the stable
// order of the two runs.
// ---------------------------------------------------------------------------
template <class View>
__device__ __forceinline__ uint32_t lds_corank2_view(const View& X, uint32_t aA, uint32_t la, uint32_t aB,
                                                     uint32_t lb, uint32_t d, int lane) {
    // wave-uniform bounds, kept in scalar registers
    uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(d > lb ? d - lb : 0u));
    uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)min(d, la));
    while (lo < hi) {
        // probe lane sits at lo + lane*step; a probe past hi reads the last
        // valid position instead (every index stays inside both runs) and
        // does not count
        const uint32_t R = hi - lo;
        const uint32_t step = ((R + 63u) >> 6) | 1u;
        const uint32_t m0 = lo + (uint32_t)lane * step;
        const bool v0 = m0 < hi;
        const uint32_t c0 = v0 ? m0 : hi - 1u;
        const bool p0 = v0 && X.key(aA + c0) <= X.key(aB + d - 1u - c0);
        const uint32_t t = (uint32_t)__popcll(__ballot(p0));
        const uint32_t nvalid = (uint32_t)__popcll(__ballot(v0));
        const uint32_t nlo = t > 0 ? lo + (t - 1u) * step + 1u : lo;
        const uint32_t nhi = t < nvalid ? lo + t * step : hi;
        lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)nlo);
        hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)nhi);
    }
    return lo;
}

// lds_corank2_view over a plain array of 32-bit keys.
struct KeysView {
    const uint32_t* k;
    __device__ __forceinline__ uint32_t key(uint32_t i) const { return k[i]; }
};
__device__ __forceinline__ uint32_t lds_corank2(const uint32_t* Xk, uint32_t aA, uint32_t la, uint32_t aB,
                                                uint32_t lb, uint32_t d, int lane) {
    return lds_corank2_view(KeysView{Xk}, aA, la, aB, lb, d, lane);
}

// ---------------------------------------------------------------------------
// Merge outputs [d0, d1) of the pair (A, B) in blocks of N = 64*EM.  Each
// block reads the next N candidates of A (ascending) and of B (descending),
// keeps the smaller of each opposing pair — the N smallest remaining
// elements, as a bitonic sequence — and sorts them with a bitonic merge.
// The number u of A elements kept advances the wave-uniform cursors.  Reads
// are 64 consecutive elements per instruction; writes likewise.
// Positions past the end of A or B read as sentinels; with keys alone a
// sentinel may stand in for an equal real maximum key, which leaves the
// output values unchanged.  X is an LDS view (key / get / put).
// ---------------------------------------------------------------------------
template <int EM, class View, class Sink>
__device__ __forceinline__ void merge_pair_range(const View& X, uint32_t aA, uint32_t la, uint32_t aB, uint32_t lb,
                                                 uint32_t d0, uint32_t d1, const Sink& out, uint32_t out_base,
                                                 int lane) {
    using El = typename View::El;
    constexpr uint32_t N = (uint32_t)kWave * EM;
    if (la == 0 || lb == 0) {   // one run is empty: the other is already in order
        const uint32_t a0 = lb == 0 ? aA : aB;
        for (uint32_t k = d0 + (uint32_t)lane; k < d1; k += (uint32_t)kWave) out.put(out_base + k, X.get(a0 + k));
        return;
    }
    uint32_t p = lds_corank2_view(X, aA, la, aB, lb, d0, lane);
    uint32_t q = d0 - p;
    for (uint32_t o = d0; o < d1; o += N) {
        El m[EM];
        uint32_t u = 0;
#pragma unroll
        for (int e = 0; e < EM; ++e) {
            const uint32_t k = (uint32_t)e * kWave + (uint32_t)lane;
            const uint32_t ia = p + k;
            const uint32_t jb = q + (N - 1u - k);
            const El a = ia < la ? X.get(aA + ia) : El::sentinel();
            const El b = jb < lb ? X.get(aB + jb) : El::sentinel();
            const bool take_a = !before(b, a);
            m[e] = take_a ? a : b;
            u += (uint32_t)__popcll(__ballot(take_a));
        }
        bitonic_merge_striped<EM>(m, lane);
        const uint32_t cnt = min(N, d1 - o);
#pragma unroll
        for (int e = 0; e < EM; ++e) {
            const uint32_t k = (uint32_t)e * kWave + (uint32_t)lane;
            if (k < cnt) out.put(out_base + o + k, m[e]);
        }
        p += u;
        q += N - u;
    }
}

// ---------------------------------------------------------------------------
// One level of the in-LDS merge tree: segments seg(i) = seg0[min(i<<lvl,
// nseg0)] are merged in adjacent pairs; wave w produces the outputs
// [w*total/nw, (w+1)*total/nw) of the whole level, so the work is balanced
// whatever the segment lengths.
// ---------------------------------------------------------------------------
template <int EM, class View, class Sink>
__device__ __forceinline__ void merge_level(const View& X, const uint32_t* seg0, uint32_t nseg0, uint32_t lvl,
                                            uint32_t total, const Sink& out, int wave, int nwaves, int lane) {
    // total < 2^20 here, so the 32-bit products cannot overflow
    const uint32_t o0 = total * (uint32_t)wave / (uint32_t)nwaves;
    const uint32_t o1 = total * (uint32_t)(wave + 1) / (uint32_t)nwaves;
    const uint32_t nseg = (nseg0 + (1u << lvl) - 1u) >> lvl;
    const uint32_t npairs = (nseg + 1u) / 2u;
    for (uint32_t i = 0; i < npairs; ++i) {
        const uint32_t s0 = seg0[min((2u * i) << lvl, nseg0)];
        const uint32_t s1 = seg0[min((2u * i + 1u) << lvl, nseg0)];
        const uint32_t s2 = seg0[min((2u * i + 2u) << lvl, nseg0)];
        const uint32_t lo = max(o0, s0), hi = min(o1, s2);
        if (lo >= hi) continue;
        merge_pair_range<EM>(X, s0, s1 - s0, s1, s2 - s1, lo - s0, hi - s0, out, s0, lane);
    }
}

// ===========================================================================
// Keys-only block merge with LDS transposes.
//
// The bitonic block of N = 64*EM keys is sorted with every compare-exchange
// inside a lane.  Index bits are moved between register and lane positions
// by two transposes through a wave-private scratch whose 64-word rows are
// padded (row stride RS), which makes every scratch access conflict-free:
//   S  (as read)   register = index bits above 6, lane = bits 5..0
//   T1             register = bits 5..2 (EM=16) or 5..3 (EM=8)
//   F  (as stored) register 4c+j = position c*256 + 4*lane + j, so each
//                  lane stores 16-byte chunks and a wave stores 1 KiB runs
// With EM = 8 index bit 2 is lane bit 0 in F and takes one DPP exchange.
// Measured gfx950 rules behind the padding: 32-bit accesses are served 32
// lanes per cycle over 32 banks, 128-bit accesses 16 lanes per cycle over 64
// banks.
// ===========================================================================
template <int EM> struct Xpose;
template <> struct Xpose<16> {
    static constexpr uint32_t RS = 68;
    static constexpr uint32_t WORDS = 16 * RS;
};
template <> struct Xpose<8> {
    static constexpr uint32_t RS = 72;
    static constexpr uint32_t WORDS = 8 * RS;
};

// floor(a / b) for b > 0, a < 2^24 and a / b < 2^22, without the integer
// division sequence.  a converts to float exactly; the reciprocal is within
// one ulp and the product rounds once, so the estimate is within
// (a / b) * 2^-22 < 1 of a / b and its truncation within one of the
// quotient; one correction step each way makes it exact (q * b <= a + b
// stays below 2^32).
__device__ __forceinline__ uint32_t udiv_small(uint32_t a, uint32_t b) {
    uint32_t q = (uint32_t)((float)a * __builtin_amdgcn_rcpf((float)b));
    if (q * b > a) --q;
    else if ((q + 1u) * b <= a) ++q;
    return q;
}

// Ordering point for a wave's own LDS traffic.  The LDS performs a wave's
// operations in the order the wave issues them, so a read issued after the
// wave's own writes returns what they wrote without waiting for them to
// complete (the compiler's memory model emits no wait for a fence at
// wavefront scope either); only the compiler must keep the order.
__device__ __forceinline__ void lds_wave_sync() { asm volatile("" ::: "memory"); }

// Wait until every vector memory operation the wave has issued (loads,
// stores, copies into LDS) is complete.
__device__ __forceinline__ void vm_drain() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Copy word `off` of the wave-uniform global array `base` into word `off` of
// the wave-uniform LDS array `lds` through the memory unit (no register
// holds it): one call per lane, lane l passing off = l, moves 64 consecutive
// words.  The copy is complete once the wave's vector memory counter drains.
__device__ __forceinline__ void dma_dword(const uint32_t* base, uint32_t off, uint32_t* lds) {
    const uint64_t a = (uint64_t)(uintptr_t)base;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32));
    const uint32_t* ub = (const uint32_t*)(uintptr_t)(((uint64_t)hi << 32) | lo);
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(ub + off),
                                     (__attribute__((address_space(3))) void*)lds, 4, 0, 0);
}

// Workgroup barrier for LDS traffic only.  Unlike __syncthreads() it does not
// wait for outstanding global loads and stores, so a prefetch into registers
// and the previous tile's stores stay in flight across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

__device__ __forceinline__ void cex_u32(uint32_t& lo, uint32_t& hi) {
    const uint32_t a = lo, b = hi;
    lo = min(a, b);
    hi = max(a, b);
}

template <int EM>
__device__ __forceinline__ void reg_stages(uint32_t (&m)[EM]) {
#pragma unroll
    for (int d = EM / 2; d >= 1; d >>= 1) {
#pragma unroll
        for (int e = 0; e < EM; ++e)
            if ((e & d) == 0) cex_u32(m[e], m[e | d]);
    }
}

// Sort the bitonic block held in layout S; the result is left in layout F.
template <int EM>
__device__ __forceinline__ void block_sort_keys(uint32_t (&m)[EM], uint32_t* scr, int lane) {
    constexpr uint32_t RS = Xpose<EM>::RS;
    const uint32_t ul = (uint32_t)lane;
    asm volatile("" ::: "memory");                       // keep the previous block's scratch reads first
    reg_stages<EM>(m);                                   // index bits 9..6 (EM=16) / 8..6 (EM=8)
#pragma unroll
    for (int e = 0; e < EM; ++e) scr[e * RS + ul] = m[e];
    lds_wave_sync();
    uint32_t tb;
    if constexpr (EM == 16) tb = (ul >> 2) * RS + (ul & 3u);   // lane = (bits 9..6, bits 1..0)
    else tb = (ul >> 3) * RS + (ul & 7u);                       // lane = (bits 8..6, bits 2..0)
    constexpr uint32_t CS = EM == 16 ? 4u : 8u;                 // stride of the register bits
#pragma unroll
    for (int e = 0; e < EM; ++e) m[e] = scr[tb + e * CS];
    reg_stages<EM>(m);                                   // index bits 5..2 / 5..3
#pragma unroll
    for (int e = 0; e < EM; ++e) scr[tb + e * CS] = m[e];
    lds_wave_sync();
    const uint32_t fb = (ul >> 4) * RS + 4u * (ul & 15u);
#pragma unroll
    for (int c = 0; c < EM / 4; ++c) {
        const uint4 v = *reinterpret_cast<const uint4*>(scr + fb + (uint32_t)c * 4u * RS);
        m[4 * c + 0] = v.x;
        m[4 * c + 1] = v.y;
        m[4 * c + 2] = v.z;
        m[4 * c + 3] = v.w;
    }
    if constexpr (EM == 8) {                             // index bit 2 = lane bit 0
        const uint32_t keep_max = (ul & 1u) ? ~0u : 0u;
        uint32_t o[EM];   // all exchanges first: no wait states between a write and its exchange
#pragma unroll
        for (int e = 0; e < EM; ++e) o[e] = (uint32_t)__builtin_amdgcn_mov_dpp((int)m[e], 0xB1, 0xF, 0xF, false);
#pragma unroll
        for (int e = 0; e < EM; ++e) m[e] = med3_u32(m[e], o[e], keep_max);
    }
#pragma unroll
    for (int c = 0; c < EM / 4; ++c) {                   // index bits 1..0
        cex_u32(m[4 * c + 0], m[4 * c + 2]);
        cex_u32(m[4 * c + 1], m[4 * c + 3]);
        cex_u32(m[4 * c + 0], m[4 * c + 1]);
        cex_u32(m[4 * c + 2], m[4 * c + 3]);
    }
}

// Store a block held in layout F: chunk c of lane l is block positions
// p = c*256 + 4l .. p+3.  put4(c, p) stores a whole chunk, put1(c, j, p + j)
// one position; positions at or past lim are not stored, and whole chunks
// only where vec allows it.  A whole block takes one wave-uniform branch.
template <int EM, class Put4, class Put1>
__device__ __forceinline__ void store_block(uint32_t lim, bool vec, int lane, const Put4& put4, const Put1& put1) {
    if (vec && lim >= (uint32_t)EM * 64u) {
#pragma unroll
        for (int c = 0; c < EM / 4; ++c) put4(c, (uint32_t)c * 256u + 4u * (uint32_t)lane);
        return;
    }
#pragma unroll
    for (int c = 0; c < EM / 4; ++c) {
        const uint32_t p = (uint32_t)c * 256u + 4u * (uint32_t)lane;
        if (vec && p + 4u <= lim) {
            put4(c, p);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (p + (uint32_t)j < lim) put1(c, j, p + (uint32_t)j);
        }
    }
}

// Sinks for a sorted block in layout F: block position t = c*256 + 4*lane + j
// goes to pos0 + t when t < cnt.  pos0 must be a multiple of 4 for the
// 16-byte path; `vec` says whether the base pointer allows it.
struct LdsSinkKeys {
    uint32_t* y;
    template <int EM>
    __device__ __forceinline__ void put_block(uint32_t pos0, uint32_t cnt, const uint32_t (&m)[EM], int lane) const {
        uint32_t* o = y + pos0;
        store_block<EM>(
            cnt, true, lane,
            [&](int c, uint32_t p) {
                *reinterpret_cast<uint4*>(o + p) = make_uint4(m[4 * c], m[4 * c + 1], m[4 * c + 2], m[4 * c + 3]);
            },
            [&](int c, int j, uint32_t p) { o[p] = m[4 * c + j]; });
    }
};
struct GlobalSinkKeys {
    uint32_t* y;     // tile output base
    uint32_t flip;
    uint32_t lim;    // positions >= lim are not stored
    bool vec;        // y is 16-byte aligned
    template <int EM>
    __device__ __forceinline__ void put_block(uint32_t pos0, uint32_t cnt, const uint32_t (&m)[EM], int lane) const {
        gu32* g = gptr(y) + pos0;
        store_block<EM>(
            min(cnt, lim > pos0 ? lim - pos0 : 0u), vec, lane,
            [&](int c, uint32_t p) {
                *reinterpret_cast<gu32x4*>(g + p) =
                    u32x4{m[4 * c] ^ flip, m[4 * c + 1] ^ flip, m[4 * c + 2] ^ flip, m[4 * c + 3] ^ flip};
            },
            [&](int c, int j, uint32_t p) { g[p] = m[4 * c + j] ^ flip; });
    }
};

// Number of block positions k = 64 e + lane with a_k <= b_k: the sum of the
// registers' ballot counts, with no branch (a is non-decreasing and b
// non-increasing in k, so the positions form a prefix of the block).
template <int EM>
__device__ __forceinline__ uint32_t prefix_len(const uint32_t (&a)[EM], const uint32_t (&b)[EM]) {
    uint32_t u = 0;
#pragma unroll
    for (int e = 0; e < EM; ++e) u += (uint32_t)__popcll(__ballot(a[e] <= b[e]));
    return u;
}

// Merge outputs [d0, d1) of A = X[aA, aA+la) and B = X[aB, aB+lb) (keys),
// blocks of N = 64*EM as in merge_pair_range; out_base + d0 must be a
// multiple of 4.
template <int EM, class Sink>
__device__ __forceinline__ void merge_pair_range_keys(const uint32_t* X, uint32_t aA, uint32_t la, uint32_t aB,
                                                      uint32_t lb, uint32_t d0, uint32_t d1, const Sink& out,
                                                      uint32_t out_base, uint32_t* scr, int lane) {
    constexpr uint32_t N = (uint32_t)kWave * EM;
    if (la == 0 || lb == 0) {
        // one run is empty (an odd run count at this level, or an empty
        // piece): the other is already in order; move it in the block layout
        // the sinks take, 16-byte reads (aA, aB, d0 and N are multiples of
        // 4; reads past the run stay in the caller's LDS and are not stored)
        const uint32_t a0 = lb == 0 ? aA : aB;
        for (uint32_t o = d0; o < d1; o += N) {
            uint32_t m[EM];
#pragma unroll
            for (int c = 0; c < EM / 4; ++c) {
                const uint4 v = *reinterpret_cast<const uint4*>(X + a0 + o + (uint32_t)c * 256u + 4u * (uint32_t)lane);
                m[4 * c] = v.x;
                m[4 * c + 1] = v.y;
                m[4 * c + 2] = v.z;
                m[4 * c + 3] = v.w;
            }
            out.template put_block<EM>(out_base + o, min(N, d1 - o), m, lane);
        }
        return;
    }
    if (d0 == 0 && d1 == la + lb && la <= N && lb <= N && la + lb > N) {
        // The whole pair in one read: A ascending and B descending, each
        // padded with sentinels to N, form a bitonic sequence of 2N whose
        // element-wise minimum and maximum halves hold the N smallest keys
        // and the other la + lb - N (then sentinels), each half bitonic:
        // two block sorts finish the pair, with no second read.  The reads
        // stay below the end of B plus N, as in the blocks below.
        const uint32_t* Ap = X + aA + (uint32_t)lane;
        const uint32_t* Bp = X + aB + (N - 1u) - (uint32_t)lane;
        uint32_t a[EM], b[EM], lo[EM], hi[EM];
#pragma unroll
        for (int e = 0; e < EM; ++e) {
            a[e] = Ap[e * kWave];
            b[e] = Bp[-(e * kWave)];
        }
#pragma unroll
        for (int e = 0; e < EM; ++e) {
            const uint32_t k = (uint32_t)e * kWave + (uint32_t)lane;
            const uint32_t ak = k < la ? a[e] : kSentKey;
            const uint32_t bk = N - 1u - k < lb ? b[e] : kSentKey;
            lo[e] = min(ak, bk);
            hi[e] = max(ak, bk);
        }
        block_sort_keys<EM>(lo, scr, lane);
        out.template put_block<EM>(out_base, N, lo, lane);
        block_sort_keys<EM>(hi, scr, lane);
        out.template put_block<EM>(out_base + N, la + lb - N, hi, lane);
        return;
    }
    uint32_t p = lds_corank2(X, aA, la, aB, lb, d0, lane);
    uint32_t q = d0 - p;
    for (uint32_t o = d0; o < d1; o += N) {
        uint32_t m[EM];
        uint32_t u = 0;
        if (p + N <= la && q + N <= lb) {
            const uint32_t* Ap = X + aA + p + (uint32_t)lane;
            const uint32_t* Bp = X + aB + q + (N - 1u) - (uint32_t)lane;
            uint32_t a[EM], b[EM];
#pragma unroll
            for (int e = 0; e < EM; ++e) {      // all reads in flight together
                a[e] = Ap[e * kWave];
                b[e] = Bp[-(e * kWave)];
            }
#pragma unroll
            for (int e = 0; e < EM; ++e) m[e] = min(a[e], b[e]);
            u = prefix_len<EM>(a, b);
        } else {
            // near the end of a run: the same reads, then the sentinel for
            // every position past the run's end, with no branch per element.
            // Those reads stay below X + (end of the last run) + N, inside
            // the caller's LDS (the layouts keep at least N words of other
            // LDS data after each buffer); what they return is discarded.
            // Keys equal to the sentinel can carry p past la (they are then
            // indistinguishable from it), so the cursors are capped first.
            const uint32_t pc = min(p, la), qc = min(q, lb);
            const uint32_t* Ap = X + aA + pc + (uint32_t)lane;
            const uint32_t* Bp = X + aB + qc + (N - 1u) - (uint32_t)lane;
            const uint32_t ra = la - pc, rb = lb - qc;   // elements left in A and B
            uint32_t a[EM], b[EM];
#pragma unroll
            for (int e = 0; e < EM; ++e) {
                a[e] = Ap[e * kWave];
                b[e] = Bp[-(e * kWave)];
            }
#pragma unroll
            for (int e = 0; e < EM; ++e) {
                const uint32_t k = (uint32_t)e * kWave + (uint32_t)lane;
                a[e] = k < ra ? a[e] : kSentKey;          // still non-decreasing in k
                b[e] = N - 1u - k < rb ? b[e] : kSentKey;  // still non-increasing in k
                m[e] = min(a[e], b[e]);
            }
            u = prefix_len<EM>(a, b);
        }
        block_sort_keys<EM>(m, scr, lane);
        out.template put_block<EM>(out_base + o, min(N, d1 - o), m, lane);
        p += u;   // u is a sum of ballot counts: the cursors stay wave-uniform
        q += N - u;
    }
}

// One merge level planned in advance: word 0 of (lvl, wave) holds the
// wave's main range (pair index in bits 0..3, outputs [d0, d1) in bits
// 4..17 and 18..31), word 1 a mask of further pairs the wave merges whole.
// Pair i of level lvl merges segments 2i and 2i+1 (indices into
// sbeg / plen, clamped to nseg0); the output of pair i starts at its first
// segment's slot.
template <int EM, class Sink>
__device__ __forceinline__ void merge_level_planned(const uint32_t* X, const uint32_t* sbeg, const uint32_t* plen,
                                                    const uint32_t* plan, uint32_t nseg0, uint32_t lvl,
                                                    const Sink& out, uint32_t* scr, int wave, int lane) {
    const uint32_t* pw = plan + 2u * (lvl * 16u + (uint32_t)wave);
    const uint32_t w0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)pw[0]);
    uint32_t own = (uint32_t)__builtin_amdgcn_readfirstlane((int)pw[1]);
    auto run = [&](uint32_t i, uint32_t d0, uint32_t d1, bool whole) {
        const uint32_t g0 = min((2u * i) << lvl, nseg0);
        const uint32_t g1 = min((2u * i + 1u) << lvl, nseg0);
        const uint32_t g2 = min((2u * i + 2u) << lvl, nseg0);
        const uint32_t aA = (uint32_t)__builtin_amdgcn_readfirstlane((int)sbeg[g0]);
        const uint32_t aB = (uint32_t)__builtin_amdgcn_readfirstlane((int)sbeg[g1]);
        const uint32_t p0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)plen[g0]);
        const uint32_t p1 = (uint32_t)__builtin_amdgcn_readfirstlane((int)plen[g1]);
        const uint32_t p2 = (uint32_t)__builtin_amdgcn_readfirstlane((int)plen[g2]);
        const uint32_t la = p1 - p0, lb = p2 - p1;
        if (whole) d1 = la + lb;
        if (d0 < d1) merge_pair_range_keys<EM>(X, aA, la, aB, lb, d0, d1, out, aA, scr, lane);
    };
    run(w0 & 15u, (w0 >> 4) & 0x3FFFu, w0 >> 18, false);
    while (own) {
        const uint32_t i = (uint32_t)__builtin_ctz(own);
        own &= own - 1u;
        run(i, 0u, 0u, true);
    }
}

}  // namespace mms
