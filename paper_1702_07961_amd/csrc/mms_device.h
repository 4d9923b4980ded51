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
// Element kinds:
//   Elem<false>  a 32-bit key (unsigned order; signed keys are mapped with
//                key ^ 0x80000000 on the way in and back on the way out)
//   Elem<true>   key, tag, value.  The tag is the element's position in the
//                array the current pass reads, so (key, tag) order is the
//                stable order and every network sorts stably.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mms {

constexpr int kWave = 64;
constexpr uint32_t kSentKey = 0xFFFFFFFFu;
constexpr uint32_t kSentTag = 0xFFFFFFFFu;

template <bool P> struct Elem;
template <> struct Elem<false> {
    uint32_t k;
    __device__ static Elem sentinel() { return {kSentKey}; }
};
template <> struct Elem<true> {
    uint32_t k, t, v;
    __device__ static Elem sentinel() { return {kSentKey, kSentTag, 0u}; }
};

// strict "a comes before b"
__device__ __forceinline__ bool before(const Elem<false>& a, const Elem<false>& b) { return a.k < b.k; }
__device__ __forceinline__ bool before(const Elem<true>& a, const Elem<true>& b) {
    uint64_t x = ((uint64_t)a.k << 32) | a.t, y = ((uint64_t)b.k << 32) | b.t;
    return x < y;
}

// compare-exchange: lo receives the earlier element, hi the later one
__device__ __forceinline__ void cex(Elem<false>& lo, Elem<false>& hi) {
    uint32_t a = lo.k, b = hi.k;
    lo.k = min(a, b);
    hi.k = max(a, b);
}
__device__ __forceinline__ void cex(Elem<true>& lo, Elem<true>& hi) {
    bool sw = before(hi, lo);
    Elem<true> a = lo, b = hi;
    lo.k = sw ? b.k : a.k; lo.t = sw ? b.t : a.t; lo.v = sw ? b.v : a.v;
    hi.k = sw ? a.k : b.k; hi.t = sw ? a.t : b.t; hi.v = sw ? a.v : b.v;
}

// keep the earlier (want_first) or the later of `mine` and `other`
__device__ __forceinline__ Elem<false> pick(const Elem<false>& mine, const Elem<false>& other, bool want_first) {
    return {want_first ? min(mine.k, other.k) : max(mine.k, other.k)};
}
__device__ __forceinline__ Elem<true> pick(const Elem<true>& mine, const Elem<true>& other, bool want_first) {
    bool other_first = before(other, mine);
    bool take = want_first ? other_first : !other_first;
    Elem<true> r;
    r.k = take ? other.k : mine.k;
    r.t = take ? other.t : mine.t;
    r.v = take ? other.v : mine.v;
    return r;
}

__device__ __forceinline__ uint32_t shfl_xor_u32(uint32_t x, int m) {
    return (uint32_t)__shfl_xor((int)x, m, kWave);
}
__device__ __forceinline__ Elem<false> shfl_xor(const Elem<false>& e, int m) { return {shfl_xor_u32(e.k, m)}; }
__device__ __forceinline__ Elem<true> shfl_xor(const Elem<true>& e, int m) {
    return {shfl_xor_u32(e.k, m), shfl_xor_u32(e.t, m), shfl_xor_u32(e.v, m)};
}

// ---------------------------------------------------------------------------
// Base case: sort the 64*E elements a wave holds, E per lane (§4.3 sorts a
// W x W grid with rows in registers and transposes; here every stage is a
// bitonic compare-exchange, in-lane for index bits below log2(E) and across
// lanes for the rest).  Result layout is "blocked": lane l holds positions
// l*E .. l*E+E-1 of the wave's sorted run.
// ---------------------------------------------------------------------------
template <int E, bool P>
__device__ __forceinline__ void wave_sort_blocked(Elem<P> (&r)[E], int lane) {
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
        Elem<P> t[E];
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

// ---------------------------------------------------------------------------
// Bitonic merge of 64*EM elements held "striped" (lane l, register e holds
// index e*64 + l): register distances first, then lane distances 32..1.
// ---------------------------------------------------------------------------
template <int EM, bool P>
__device__ __forceinline__ void bitonic_merge_striped(Elem<P> (&m)[EM], int lane) {
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

// LDS element access: tags are LDS positions (the pass's stable order)
template <bool P> __device__ __forceinline__ Elem<P> lds_get(const uint32_t* Xk, const uint32_t* Xv, uint32_t i);
template <> __device__ __forceinline__ Elem<false> lds_get<false>(const uint32_t* Xk, const uint32_t*, uint32_t i) {
    return {Xk[i]};
}
template <> __device__ __forceinline__ Elem<true> lds_get<true>(const uint32_t* Xk, const uint32_t* Xv, uint32_t i) {
    return {Xk[i], i, Xv[i]};
}

// ---------------------------------------------------------------------------
// Merge-path split inside LDS: the number p of elements of A = X[aA, aA+la)
// among the first d elements of merge(A, B = X[aB, aB+lb)), A first on ties.
// The wave probes 64 points per round with an odd stride, so the 64 reads of
// one round fall in 64 distinct banks.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lds_corank2(const uint32_t* Xk, uint32_t aA, uint32_t la, uint32_t aB,
                                                uint32_t lb, uint32_t d, int lane) {
    uint32_t lo = d > lb ? d - lb : 0u;
    uint32_t hi = min(d, la);
    while (lo < hi) {
        const uint32_t R = hi - lo;
        const uint32_t step = ((R + 63u) >> 6) | 1u;
        const uint32_t m = lo + (uint32_t)lane * step;
        bool pred = false;
        if (m < hi) pred = Xk[aA + m] <= Xk[aB + d - 1u - m];
        const uint32_t t = (uint32_t)__popcll(__ballot(pred));
        const uint32_t nvalid = min(64u, (R + step - 1u) / step);
        const uint32_t nlo = t > 0 ? lo + (t - 1u) * step + 1u : lo;
        const uint32_t nhi = t < nvalid ? lo + t * step : hi;
        lo = nlo;
        hi = nhi;
    }
    return lo;
}

// Output sinks for a merged range
template <bool P> struct LdsSink {
    uint32_t* k;
    uint32_t* v;
    __device__ __forceinline__ void put(uint32_t i, const Elem<P>& e) const {
        k[i] = e.k;
        if constexpr (P) v[i] = e.v;
    }
};
// Writes to memory, undoing the signed-key mapping; positions >= lim are
// dropped (they hold the sentinels of a ragged tile).
template <bool P> struct GlobalSinkLim {
    uint32_t* k;
    uint32_t* v;
    uint32_t flip;
    uint32_t lim;
    __device__ __forceinline__ void put(uint32_t i, const Elem<P>& e) const {
        if (i < lim) {
            k[i] = e.k ^ flip;
            if constexpr (P) v[i] = e.v;
        }
    }
};

// ---------------------------------------------------------------------------
// Merge outputs [d0, d1) of the pair (A, B) in blocks of N = 64*EM.  Each
// block reads the next N candidates of A (ascending) and of B (descending),
// keeps the smaller of each opposing pair — the N smallest remaining
// elements, as a bitonic sequence — and sorts them with a bitonic merge.
// The number u of A elements kept advances the wave-uniform cursors.  Reads
// are 64 consecutive words per instruction; writes likewise.
// Positions past the end of A or B read as sentinels; with keys alone a
// sentinel may stand in for an equal real maximum key, which leaves the
// output values unchanged.
// ---------------------------------------------------------------------------
template <int EM, bool P, class Sink>
__device__ __forceinline__ void merge_pair_range(const uint32_t* Xk, const uint32_t* Xv, uint32_t aA, uint32_t la,
                                                 uint32_t aB, uint32_t lb, uint32_t d0, uint32_t d1,
                                                 const Sink& out, uint32_t out_base, int lane) {
    constexpr uint32_t N = (uint32_t)kWave * EM;
    uint32_t p = lds_corank2(Xk, aA, la, aB, lb, d0, lane);
    uint32_t q = d0 - p;
    for (uint32_t o = d0; o < d1; o += N) {
        Elem<P> m[EM];
        uint32_t u = 0;
#pragma unroll
        for (int e = 0; e < EM; ++e) {
            const uint32_t k = (uint32_t)e * kWave + (uint32_t)lane;
            const uint32_t ia = p + k;
            const uint32_t jb = q + (N - 1u - k);
            const Elem<P> a = ia < la ? lds_get<P>(Xk, Xv, aA + ia) : Elem<P>::sentinel();
            const Elem<P> b = jb < lb ? lds_get<P>(Xk, Xv, aB + jb) : Elem<P>::sentinel();
            const bool take_a = !before(b, a);
            m[e] = take_a ? a : b;
            u += (uint32_t)__popcll(__ballot(take_a));
        }
        bitonic_merge_striped<EM, P>(m, lane);
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
template <int EM, bool P, class Sink>
__device__ __forceinline__ void merge_level(const uint32_t* Xk, const uint32_t* Xv, const uint32_t* seg0,
                                            uint32_t nseg0, uint32_t lvl, uint32_t total, const Sink& out,
                                            int wave, int nwaves, int lane) {
    const uint32_t o0 = (uint32_t)(((uint64_t)total * (uint32_t)wave) / (uint32_t)nwaves);
    const uint32_t o1 = (uint32_t)(((uint64_t)total * (uint32_t)(wave + 1)) / (uint32_t)nwaves);
    const uint32_t nseg = (nseg0 + (1u << lvl) - 1u) >> lvl;
    const uint32_t npairs = (nseg + 1u) / 2u;
    for (uint32_t i = 0; i < npairs; ++i) {
        const uint32_t s0 = seg0[min((2u * i) << lvl, nseg0)];
        const uint32_t s1 = seg0[min((2u * i + 1u) << lvl, nseg0)];
        const uint32_t s2 = seg0[min((2u * i + 2u) << lvl, nseg0)];
        const uint32_t lo = max(o0, s0), hi = min(o1, s2);
        if (lo >= hi) continue;
        merge_pair_range<EM, P>(Xk, Xv, s0, s1 - s0, s1, s2 - s1, lo - s0, hi - s0, out, s0, lane);
    }
}

}  // namespace mms
