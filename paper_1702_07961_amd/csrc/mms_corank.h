// Partition (§4.1) device code shared by the 32-bit and 64-bit kernels: the
// exact split of K sorted runs at a rank, one wave per query.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mms_device.h"

namespace mms {

// ===========================================================================
// Partition (§4.1): split indices c_0..c_{K-1} of K sorted runs at rank r.
//
// Exact, with O(log L) dependent probe rounds.  At resolution h (a power of
// two) call block j of run k its elements [j*h, (j+1)*h) and represent a full
// block by its last element.  The number of run-k full blocks inside the
// first r merged elements is floor(c_k / h), and the blocks inside form the
// smallest such representatives overall (the first r elements are closed
// downwards).  Their total t_h = sum_k floor(c_k/h) lies in
// [ceil((r - K(h-1))/h), floor(r/h)], an interval narrower than K.
// Going from resolution 2h to h, run k can only gain half-blocks of the
// blocks the previous level left undecided; every such candidate is probed
// once, the candidates are ranked in the wave, and the bounds on t_h turn
// into bounds [lo_k, hi_k] on floor(c_k/h) whose widths sum to less than K.
// So at most 3K-2 candidates exist per level (one per lane for K <= 16), and
// at h = 1 the bounds meet: c_k = lo_k = hi_k.  Ties are ordered by (key,
// run, position), the stable order.
// ===========================================================================
// Inclusive sum over the 16 lanes of each row (DPP row shifts).
__device__ __forceinline__ uint32_t row16_incl_sum(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);   // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);   // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);   // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);   // row_shr:8
    return x;
}

// Inclusive maximum over all 64 lanes: row shifts, then the row broadcasts of
// lanes 15 and 31 carry it across rows.
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t x) {
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false));   // row_shr:1
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false));   // row_shr:2
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false));   // row_shr:4
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false));   // row_shr:8
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false));   // row_bcast:15
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false));   // row_bcast:31
    return x;
}

// Set bits of mask at positions [off, off + cnt), off < 64, cnt <= 64 - off.
__device__ __forceinline__ uint32_t bits_in(uint64_t mask, uint32_t off, uint32_t cnt) {
    const uint64_t x = mask >> off;
    return cnt ? (uint32_t)__popcll(x << (64u - cnt)) : 0u;
}

// A wave's LDS scratch for corank_wave: the candidate of every lane, read
// back as broadcasts (32-bit keys: the composite (key, lane); 64-bit keys:
// the key, the lane being its slot), and the level tag | run + 1 at the lane
// where a run's candidates start.
template <class KeyT> struct CorankLdsT;
template <> struct CorankLdsT<uint32_t> {
    uint64_t comp[64];
    uint32_t head[64];
};
template <> struct CorankLdsT<uint64_t> {
    uint64_t comp[64];
    uint32_t head[64];
};
using CorankLds = CorankLdsT<uint32_t>;

// Returns c_k in lane k (k < Kg <= 16); other lanes return 0.  All 64 lanes
// call with the same arguments; positions inside a run are below 2^32.
//
// Each round refines the resolution by 2^s: s = 1 in general, s = 2 when at
// most 9 runs take part.  With bounds lo_k <= floor(c_k/h) <= hi_k and
// sum(hi - lo) < K, the sub-blocks of h' = h/2^s that can still be inside
// are [2^s lo, 2^s hi + 2^s - 2] (sub-block 2^s(hi+1) - 1 being inside would
// put c_k past block hi), at most (2^(s+1) - 1)K - 2^s in all: 3K - 2 <= 46
// for K <= 16, 7K - 4 <= 59 for K <= 9, one per lane either way.  The first
// round starts from lo = hi = 0, so only (2^s - 1)K candidates exist and it
// takes the largest s with (2^s - 1)K <= 64 (2 for K <= 16, 3 for K <= 9,
// 4 for K <= 4, 5 for K <= 2): one dependent round fewer, or more.
//
// The candidates of a round sit in lanes run by run (run k's in lanes off_k ..
// off_k + cnt_k - 1, in block order), so lane order is (run, block) order and
// the stable order of candidates is (key, lane).  A lane finds its run from
// the heads the runs write into LDS (prefix maximum over the lanes; tags grow
// with the round, so stale heads of earlier rounds lose), ranks its candidate
// against all others read back from LDS as broadcasts, and the runs count
// their inside candidates from two ballots.  The sum of the lower bounds is
// kept as a scalar, so the bounds on t_h need no reduction.
template <int STEP, class KeyT>
__device__ uint32_t corank_rounds(const KeyT* __restrict__ keys, uint64_t gb, uint64_t glen, uint64_t L,
                                  uint32_t Kg, uint32_t r, KeyT flip, int lane, CorankLdsT<KeyT>* sh) {
    const uint32_t nk = (uint32_t)lane < Kg ? (uint32_t)min(L, glen - (uint64_t)lane * L) : 0u;
    const uint64_t maxlen = Kg > 1 ? L : glen;
    const __attribute__((address_space(1))) KeyT* kp = (const __attribute__((address_space(1))) KeyT*)keys + gb;
    sh->head[lane] = 0u;
    // resolution 2^l with 2^l > every run: lo = hi = 0 bound floor(c_k / 2^l)
    int l = maxlen ? 64 - __builtin_clzll(maxlen) : 0;
    uint32_t lo = 0, hi = 0;   // lane k
    uint32_t slo = 0;          // sum of lo over the runs
    uint32_t tag = 0;
    int s = min(l, Kg <= 2u ? 5 : Kg <= 4u ? 4 : Kg <= 9u ? 3 : 2);   // the first round's step
    while (l > 0) {
        l -= s;
        tag += 256u;
        const uint32_t nb = nk >> l;   // full blocks of run k at resolution 2^l
        const uint32_t jlo = lo << s;
        const uint32_t jmax = (hi << s) + (1u << s) - 2u;
        const uint32_t cnt = nb > jlo ? min(jmax, nb - 1u) - jlo + 1u : 0u;
        const uint32_t incl = row16_incl_sum(cnt);
        const uint32_t off = incl - cnt;
        const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 15);
        if (cnt) sh->head[off] = tag | (uint32_t)(lane + 1);
        lds_wave_sync();
        const uint32_t kk = (wave_incl_max(sh->head[lane]) & 0xFFu) - 1u;
        const bool valid = (uint32_t)lane < total;
        // block index of this lane's candidate = lane + (jlo - off) of its run
        const uint32_t d = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(kk << 2), (int)(jlo - off));
        // the candidate's stable position is (key, lane); 32-bit keys pack
        // it into one 64-bit word, 64-bit keys compare the lane on ties
        uint64_t comp = ~0ull;
        if (valid) {
            const uint32_t pos = (((uint32_t)lane + d + 1u) << l) - 1u;
            const KeyT key = kp[(uint64_t)kk * L + pos] ^ flip;
            if constexpr (sizeof(KeyT) == 4) comp = ((uint64_t)key << 32) | (uint32_t)lane;
            else comp = (uint64_t)key;
        }
        sh->comp[lane] = comp;
        lds_wave_sync();
        uint32_t rank = 0;
        if constexpr (sizeof(KeyT) == 4) {
            // two trips' reads in flight: at most 64 VGPRs, eight waves per SIMD
#pragma unroll 2
            for (uint32_t m = 0; m < total; m += 8) {
#pragma unroll
                for (uint32_t e = 0; e < 8; ++e) rank += sh->comp[m + e] < comp ? 1u : 0u;
            }
        } else {
#pragma unroll 2
            for (uint32_t m = 0; m < total; m += 8) {
#pragma unroll
                for (uint32_t e = 0; e < 8; ++e) {
                    const uint64_t c = sh->comp[m + e];
                    rank += (c < comp || (c == comp && m + e < (uint32_t)lane)) ? 1u : 0u;
                }
            }
        }

        // t_h in [ceil((r - Kg(h-1)) / h), floor(r / h)]; all wave-uniform
        const uint64_t hm1 = (1ull << l) - 1u;
        const uint64_t kh = (uint64_t)Kg * hm1;
        const uint32_t tlo = (uint64_t)r > kh ? (uint32_t)(((uint64_t)r - kh + hm1) >> l) : 0u;
        const uint32_t thi = r >> l;
        const uint32_t sj = slo << s;   // sum of jlo
        const uint32_t dlo = tlo > sj ? tlo - sj : 0u;
        const uint32_t dhi = thi > sj ? thi - sj : 0u;
        const uint32_t mlo = dlo < total ? dlo : total;
        const uint32_t mhi = dhi < total ? dhi : total;
        const uint64_t blo = __ballot(valid && rank < mlo);
        const uint64_t bhi = __ballot(valid && rank < mhi);
        lo = jlo + bits_in(blo, off, cnt);
        hi = jlo + bits_in(bhi, off, cnt);
        slo = sj + (uint32_t)__popcll(blo);
        s = STEP == 1 ? 1 : min(STEP, l);
    }
    return lo;
}

template <class KeyT>
__device__ uint32_t corank_wave(const KeyT* __restrict__ keys, uint64_t gb, uint64_t glen, uint64_t L, uint32_t Kg,
                                uint32_t r, KeyT flip, int lane, CorankLdsT<KeyT>* sh) {
    if (Kg <= 9) return corank_rounds<2>(keys, gb, glen, L, Kg, r, flip, lane, sh);
    return corank_rounds<1>(keys, gb, glen, L, Kg, r, flip, lane, sh);
}

}  // namespace mms
