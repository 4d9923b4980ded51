// Tile plans of the K-way merges (§4.2): where each run's piece of a merge
// tile sits in LDS and which outputs of every merge level each wave
// produces.  Shared by the keys-only and the key-value merge kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mms_device.h"
#include "mms_internal.h"

namespace mms {

// Piece table of a tile, written by one wave: src0[k] (the key in LDS slot
// P of piece k comes from position src0[k] + P of the group, modulo 2^32),
// plen[k] (prefix of piece lengths), sbeg[k] (4-aligned LDS offsets).
struct Meta {
    uint32_t* src0;
    uint32_t* plen;
    uint32_t* sbeg;
    uint32_t* plan;   // [4 levels][16 waves][2]: each wave's work per level
    uint8_t* cseg;    // piece whose LDS slots hold slot 64*c (slot coordinates)
};
constexpr uint32_t kPlanWords = 4u * 16u * 2u;

// Exclusive sum over the 16 lanes of each row (DPP row shifts; a lane
// shifted in from outside the row reads 0).
__device__ __forceinline__ uint32_t excl_scan16(uint32_t x) {
    uint32_t incl = x;
    incl += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)incl, 0x111, 0xF, 0xF, false);   // row_shr:1
    incl += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)incl, 0x112, 0xF, 0xF, false);   // row_shr:2
    incl += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)incl, 0x114, 0xF, 0xF, false);   // row_shr:4
    incl += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)incl, 0x118, 0xF, 0xF, false);   // row_shr:8
    return incl - x;
}

// Work of every wave at every merge level of the tile, one (level, wave) per
// lane (lane = 16 * level + wave).  Pair i of level l gets the waves whose
// equal shares of the level's outputs have their midpoints inside it,
// (2w+1) * total / (2W) in [plen[g0], plen[g2]), and they split it evenly at
// multiples of 4; a pair holding no midpoint goes whole to the wave whose
// share holds its start.  No quantity reaches 2^22 (udiv_small's range).
template <int W>
__device__ __forceinline__ void build_plan(const Meta& m, uint32_t Kg, int lane) {
    const uint32_t total = m.plen[Kg];
    const uint32_t l = (uint32_t)lane >> 4, w = (uint32_t)lane & 15u;
    uint32_t nlev = 0;
    while ((1u << nlev) < Kg) ++nlev;
    const bool act = w < (uint32_t)W && l < nlev;
    const uint32_t nseg = act ? (Kg + (1u << l) - 1u) >> l : 0u;
    const uint32_t npairs = (nseg + 1u) >> 1;
    const uint32_t mid2 = (2u * w + 1u) * total;           // 2W * midpoint
    // output start of pair i of the level (i <= 8), read once
    uint32_t pst[9];
#pragma unroll
    for (uint32_t i = 0; i < 9u; ++i) pst[i] = m.plen[min((2u * i) << l, Kg)];
    uint32_t iw = 0;
#pragma unroll
    for (uint32_t i = 1; i < 8u; ++i)
        if (i < npairs && 2u * (uint32_t)W * pst[i] <= mid2) iw = i;
    const uint64_t grp = 0xFFFFull << (16u * (l & 3u));
    uint32_t v0 = 0, nw = 1, own = 0;
#pragma unroll
    for (uint32_t i = 0; i < 8u; ++i) {
        const uint64_t mi = __ballot(act && i < npairs && iw == i) & grp;
        if (act && i == iw && mi) {
            v0 = (uint32_t)__builtin_ctzll(mi) - 16u * l;
            nw = (uint32_t)__popcll(mi);
        }
        if (act && i < npairs && mi == 0ull && total) {
            const uint32_t o = min(udiv_small(pst[i] * (uint32_t)W, total), (uint32_t)W - 1u);
            if (o == w) own |= 1u << i;
        }
    }
    if (act) {
        uint32_t p0 = pst[0], p2 = pst[1];
#pragma unroll
        for (uint32_t i = 1; i < 8u; ++i)
            if (iw == i) {
                p0 = pst[i];
                p2 = pst[i + 1u];
            }
        const uint32_t sz = p2 - p0, j = w - v0;
        const uint32_t d0 = total ? udiv_small(sz * j, nw) & ~3u : 0u;
        const uint32_t d1 = !total ? 0u : (j + 1u == nw ? sz : udiv_small(sz * (j + 1u), nw) & ~3u);
        m.plan[2u * (uint32_t)lane] = iw | (d0 << 4) | (d1 << 18);
        m.plan[2u * (uint32_t)lane + 1u] = own;
    }
}

// The plan entry a wave merges.  Waves w and w+4 share a SIMD, which serves
// the older one first, and an entry costs more the later its outputs lie in
// its pair (those blocks reach the runs' ends and mask the positions past
// them), at every level from the second on.  With eight waves, SIMD s runs
// entries 7-s (on its older wave) and s, so each SIMD gets one later and one
// earlier entry.
template <int W>
__device__ __forceinline__ int plan_entry(int wave) {
    return W == 8 ? (wave < 4 ? 7 - wave : wave - 4) : wave;
}

// Piece layout of a tile of cnt outputs from Kg runs, in registers: lane
// k < Kg, holding run k's split indices s <= e, gets its piece's length, its
// first output (plen) and its 4-aligned first LDS slot (sbeg).
struct PieceLayout {
    uint32_t len, pl, sb;
};
__device__ __forceinline__ PieceLayout piece_layout(uint32_t s, uint32_t e, uint32_t Kg, uint32_t cnt, int lane) {
    const bool own = (uint32_t)lane < Kg;
    uint32_t len = own ? e - s : 0u;
    uint32_t pl = excl_scan16(len);
    // guards for memory safety only: keep the pieces inside the tile
    len = pl >= cnt ? 0u : min(len, cnt - pl);
    pl = min(pl, cnt);
    const uint32_t sb = excl_scan16((len + 3u) & ~3u);
    return {len, pl, sb};
}

// The piece layout written to the tile's table: src0, plen and sbeg of
// every run (run k starts at k*L in its group) and their totals.
__device__ __forceinline__ void build_pieces(const Meta& m, uint32_t s, uint32_t e, uint32_t Kg, uint32_t cnt,
                                             uint64_t L, int lane) {
    const PieceLayout pc = piece_layout(s, e, Kg, cnt, lane);
    if ((uint32_t)lane < Kg) {
        m.src0[lane] = (uint32_t)((uint64_t)lane * L) + s - pc.sb;
        m.plen[lane] = pc.pl;
        m.sbeg[lane] = pc.sb;
    }
    const uint32_t tot_pl = (uint32_t)__builtin_amdgcn_readlane((int)(pc.pl + pc.len), (int)(Kg - 1u));
    const uint32_t tot_sb =
        (uint32_t)__builtin_amdgcn_readlane((int)(pc.sb + ((pc.len + 3u) & ~3u)), (int)(Kg - 1u));
    if (lane == 0) {
        m.plen[Kg] = tot_pl;
        m.sbeg[Kg] = tot_sb;
    }
}

}  // namespace mms
