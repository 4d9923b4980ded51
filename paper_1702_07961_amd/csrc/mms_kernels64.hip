// gfx950 kernels of the 64-bit multiway mergesort (§6.3 also sorts 8-byte
// integers): 64-bit keys alone, or stable pairs of 64-bit keys and 64-bit
// values.  The method is the one of the 32-bit path:
//
//   tile_sort64   base case (§4.3): each workgroup sorts a tile in registers
//                 (a bitonic network per wave, then bitonic merges across
//                 the waves through LDS)
//   corank64      partition (§4.1): the exact split of each output tile
//   merge64       K-way merge of one output tile through LDS (§4.2, §7),
//                 log2 K levels of pairwise block merges: keys with the
//                 transposed block step of the 32-bit merges on 64-bit words
//                 (pieces at 4-aligned slots, a per-wave level plan), pairs
//                 with lane-exchange networks on (key, tag) elements
//
// Pairs carry (key, tag) through every network, the tag being the element's
// slot in the tile as loaded, so every step is stable; the values stay in LDS
// where they were loaded and are gathered by tag when a tile is stored.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "mms_corank.h"
#include "mms_device.h"
#include "mms_device64.h"
#include "mms_device_kt.h"
#include "mms_tile_plan.h"
#include "mms_internal.h"

namespace mms {

namespace {

// LDS of one exchange buffer of the base case: keys, then (pairs) tags, for
// T elements
template <bool PAIRS> constexpr uint32_t xbuf_bytes(uint32_t T) { return T * (PAIRS ? 12u : 8u); }
// LDS of the base case: (pairs) the values as loaded, then two exchange
// buffers
template <bool PAIRS> constexpr uint32_t tile_lds_bytes(uint32_t T) {
    return (PAIRS ? 8u * T : 0u) + 2u * xbuf_bytes<PAIRS>(T);
}

}  // namespace

// ===========================================================================
// Base case.  Wave w loads positions w*CH + e*64 + lane (coalesced) and sorts
// them in registers; lane l then holds positions l*E .. l*E+E-1 of its wave's
// run.  Level lvl merges runs of 2^lvl waves: a mirror stage pairs element
// (lane, e) of wave w with element (63-lane, E-1-e) of wave w ^ (2^(lvl+1)-1),
// then wave-distance stages pair equal slots, each through LDS, and the
// in-wave tail finishes.  In LDS element (lane, e) of wave w sits at slot
// w*CH + e*64 + lane, so every exchange access is 64 consecutive elements.
// ===========================================================================
template <int E, int W, bool PAIRS>
__global__ __launch_bounds__(W * 64) void k_tile_sort64(Phase64 ph, Bufs64 b, uint64_t flip) {
    using El = std::conditional_t<PAIRS, E64T, E64>;
    constexpr uint32_t CH = 64u * E;
    constexpr uint32_t T = CH * W;
    extern __shared__ __align__(16) uint64_t smem64[];
    uint64_t* V = smem64;                                       // pairs: values by slot
    uint8_t* xbase = reinterpret_cast<uint8_t*>(smem64 + (PAIRS ? T : 0u));

    const int lane = threadIdx.x & 63;
    const uint32_t ul = (uint32_t)lane;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint64_t base = (uint64_t)blockIdx.x * T;
    const uint32_t cnt = (uint32_t)min<uint64_t>(T, ph.n - base);
    uint64_t* out_k = (ph.dst_out ? b.out_k : b.ws_k) + base;
    uint64_t* out_v = PAIRS ? (ph.dst_out ? b.out_v : b.ws_v) + base : nullptr;
    const uint64_t flip_out = ph.final_pass ? flip : 0ull;

    // the wave sorts any arrangement of its keys, so each lane loads two
    // consecutive elements per 16-byte load (chunk c: positions c*128 +
    // 2*lane, +1); a pair's tag is its own tile position
    typedef uint64_t v2u64 __attribute__((ext_vector_type(2)));
    typedef const __attribute__((address_space(1))) v2u64 cgv2u64;
    El r[E];
    const uint64_t* in_k = b.in_k + base;
    const uint64_t* in_v = PAIRS ? b.in_v + base : b.in_k + base;
    const bool vec_in = ((((uintptr_t)in_k) | (uintptr_t)in_v) & 15u) == 0;
#pragma unroll
    for (uint32_t c = 0; c < (uint32_t)E / 2u; ++c) {
        const uint32_t j = (uint32_t)wave * CH + c * 128u + 2u * ul;
        if (vec_in && j + 2u <= cnt) {
            const v2u64 k = *reinterpret_cast<cgv2u64*>(gptr64(in_k) + j);
            if constexpr (PAIRS) {
                const v2u64 v = *reinterpret_cast<cgv2u64*>(gptr64(in_v) + j);
                r[2 * c] = El{k[0] ^ flip, j};
                r[2 * c + 1] = El{k[1] ^ flip, j + 1u};
                V[j] = v[0];
                V[j + 1] = v[1];
            } else {
                r[2 * c] = El{k[0] ^ flip};
                r[2 * c + 1] = El{k[1] ^ flip};
            }
        } else {
#pragma unroll
            for (uint32_t q = 0; q < 2u; ++q) {
                const uint32_t jq = j + q;
                if (jq < cnt) {
                    if constexpr (PAIRS) {
                        r[2 * c + q] = El{gptr64(in_k)[jq] ^ flip, jq};
                        V[jq] = gptr64(in_v)[jq];
                    } else {
                        r[2 * c + q] = El{gptr64(in_k)[jq] ^ flip};
                    }
                } else {
                    r[2 * c + q] = El::sentinel();
                }
            }
        }
    }
    wave_sort_blocked<E>(r, lane);

    uint32_t buf = 0;
    auto exchange = [&](int pw, bool mirror, bool want_first) {
        uint8_t* X = xbase + buf * xbuf_bytes<PAIRS>(T);
        buf ^= 1u;
        uint64_t* xk = reinterpret_cast<uint64_t*>(X);
        uint32_t* xt = reinterpret_cast<uint32_t*>(xk + T);
        const uint32_t me = (uint32_t)wave * CH;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t slot = me + (uint32_t)e * 64u + ul;
            xk[slot] = r[e].k;
            if constexpr (PAIRS) xt[slot] = r[e].t;
        }
        lds_barrier();
        const uint32_t them = (uint32_t)pw * CH;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t slot = them + (mirror ? (uint32_t)(E - 1 - e) * 64u + (63u - ul) : (uint32_t)e * 64u + ul);
            El o;
            if constexpr (PAIRS) o = El{xk[slot], xt[slot]};
            else o = El{xk[slot]};
            r[e] = pick(r[e], o, want_first);
        }
    };
#pragma unroll
    for (int lvl = 0; (1 << lvl) < W; ++lvl) {
        const int gw = 1 << lvl;
        exchange(wave ^ (2 * gw - 1), true, (wave & gw) == 0);
#pragma unroll
        for (int dw = gw >> 1; dw >= 1; dw >>= 1) exchange(wave ^ dw, false, (wave & dw) == 0);
        wave_merge_tail<E>(r, lane);
    }

    // lane l holds tile positions wave*CH + l*E .. + E-1: pairs of 16 bytes
    const uint32_t p0 = (uint32_t)wave * CH + ul * (uint32_t)E;
    const bool vec = ((((uintptr_t)out_k) | (uintptr_t)(PAIRS ? out_v : out_k)) & 15u) == 0;
    typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(1))) u64x2 gu64x2;
#pragma unroll
    for (int e = 0; e < E; e += 2) {
        const uint32_t pos = p0 + (uint32_t)e;
        if (vec && pos + 2u <= cnt) {
            *reinterpret_cast<gu64x2*>(gptr64(out_k) + pos) = u64x2{r[e].k ^ flip_out, r[e + 1].k ^ flip_out};
            if constexpr (PAIRS) *reinterpret_cast<gu64x2*>(gptr64(out_v) + pos) = u64x2{V[r[e].t], V[r[e + 1].t]};
        } else {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if (pos + (uint32_t)j < cnt) {
                    gptr64(out_k)[pos + j] = r[e + j].k ^ flip_out;
                    if constexpr (PAIRS) gptr64(out_v)[pos + j] = V[r[e + j].t];
                }
            }
        }
    }
}

// ===========================================================================
// Partition (§4.1): one wave per output tile of a merge round, the split at
// the tile's first output.  The round reads the buffer it does not write.
// ===========================================================================
__global__ __launch_bounds__(256) void k_corank_tiles64(Phase64 ph, Bufs64 b, RoundArgs ra,
                                                        uint32_t* __restrict__ table) {
    __shared__ CorankLdsT<uint64_t> sh[4];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint64_t t = (uint64_t)blockIdx.x * 4u + (uint64_t)wave;
    if (t >= ph.tiles) return;
    const uint64_t* src = ph.dst_out ? b.ws_k : b.out_k;
    const uint64_t grp = t / ra.tpg;
    const uint64_t i = t - grp * ra.tpg;
    const uint64_t span = (uint64_t)ra.K * ra.L;
    const uint64_t gb = grp * span;
    const uint64_t glen = min(span, ph.n - gb);
    const uint32_t Kg = (uint32_t)((glen + ra.L - 1) / ra.L);
    uint32_t c = 0;
    if (i > 0) c = corank_wave<uint64_t>(src, gb, glen, ra.L, Kg, (uint32_t)(i * ra.Tout), 0ull, lane, &sh[wave]);
    if ((uint32_t)lane < ra.K) table[t * ra.K + (uint64_t)lane] = c;
}

// ===========================================================================
// Key-value K-way merge of one output tile (§4.2, §7): the tile's pieces of
// its group's runs, bounded by the split indices of its first and last
// output, are loaded into LDS back to back, merged pairwise level by level
// (log2 K levels, 64x4-pair blocks, every wave an equal share of each
// level's outputs), and the last level is written to memory.
// ===========================================================================
template <int W>
__global__ __launch_bounds__(W * 64) void k_merge64_pairs(Phase64 ph, Bufs64 b, RoundArgs ra,
                                                          const uint32_t* __restrict__ table, uint64_t flip) {
    constexpr int EM = 4;   // a wave's share of a level: 256 pairs
    constexpr uint32_t NT = W * 64u;
    const uint32_t Tout = ra.Tout, K = ra.K;
    const uint64_t L = ra.L;
    extern __shared__ __align__(16) uint64_t smem64[];
    // keys of the level buffers, the values by slot as loaded and the keys'
    // 16-bit tags
    uint64_t* Xk = smem64;
    uint64_t* Yk = smem64 + Tout;
    uint64_t* V = smem64 + 2 * Tout;
    uint16_t* Xt = reinterpret_cast<uint16_t*>(smem64 + 3 * Tout);
    uint16_t* Yt = Xt + Tout;
    uint32_t* seg0 = reinterpret_cast<uint32_t*>(Yt + Tout);                             // [kMaxFanout + 1]
    uint32_t* start = seg0 + kMaxFanout + 1;                                            // [kMaxFanout]

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint64_t t = blockIdx.x;
    const uint64_t* src_k = ph.dst_out ? b.ws_k : b.out_k;
    const uint64_t* src_v = ph.dst_out ? b.ws_v : b.out_v;
    uint64_t* dst_k = ph.dst_out ? b.out_k : b.ws_k;
    uint64_t* dst_v = ph.dst_out ? b.out_v : b.ws_v;
    const uint64_t flip_out = ph.final_pass ? flip : 0ull;
    const uint64_t grp = t / ra.tpg;
    const uint64_t i = t - grp * ra.tpg;
    const uint64_t span = (uint64_t)K * L;
    const uint64_t gb = grp * span;
    const uint64_t glen = min(span, ph.n - gb);
    const uint32_t Kg = (uint32_t)((glen + L - 1) / L);
    const uint64_t obeg = i * (uint64_t)Tout;
    const uint32_t cnt = (uint32_t)min<uint64_t>(Tout, glen - obeg);
    const uint64_t obase = gb + obeg;

    if (Kg == 1) {   // a lone run: its tile is already in order
        for (uint32_t j = threadIdx.x; j < cnt; j += NT) {
            gptr64(dst_k)[obase + j] = gptr64(src_k)[obase + j] ^ flip_out;
            gptr64(dst_v)[obase + j] = gptr64(src_v)[obase + j];
        }
        return;
    }
    // Every wave reads the split indices (lane k < Kg: piece k) and lays
    // the pieces out in registers, so its loads into LDS go out at once;
    // wave 0 also writes the layout for the merge levels.
    uint32_t len = 0, st_k = 0;
    if ((uint32_t)lane < Kg) {
        const uint32_t k = (uint32_t)lane;
        const uint64_t nk = min(L, glen - (uint64_t)k * L);
        // the clamps only guard memory safety; exact splits never trigger them
        st_k = i == 0 ? 0u : min(table[t * K + k], (uint32_t)nk);
        const uint32_t e = (obeg + Tout >= glen) ? (uint32_t)nk : min(table[(t + 1) * K + k], (uint32_t)nk);
        len = e > st_k ? e - st_k : 0u;
    }
    const uint32_t incl = min(row16_incl_sum(len), cnt);   // piece k ends at seg0[k + 1]
    {
        // the pieces, concatenated, go into LDS by the memory unit: 64 words
        // (32 elements) of keys and of values per instruction, no register
        // holding them, every chunk in flight at once; chunks are dealt to
        // the waves round-robin in piece order
        uint32_t cbase = 0;
        for (uint32_t k = 0; k < Kg; ++k) {
            const uint32_t s0 = k ? (uint32_t)__builtin_amdgcn_readlane((int)incl, (int)(k - 1u)) : 0u;
            const uint32_t s1 = (uint32_t)__builtin_amdgcn_readlane((int)incl, (int)k);
            const uint32_t st = (uint32_t)__builtin_amdgcn_readlane((int)st_k, (int)k);
            const uint32_t w0 = 2u * s0, w1 = s1 > s0 ? 2u * s1 : w0;   // LDS words of the piece
            const uint32_t nch = (w1 - w0 + 63u) >> 6;
            const uint64_t run0 = 2u * (gb + (uint64_t)k * L + st);   // the piece's first word
            for (uint32_t c = ((uint32_t)wave + W - cbase % W) % W; c < nch; c += W) {
                const uint32_t j0 = w0 + 64u * c;
                if (j0 + (uint32_t)lane < w1) {
                    dma_dword(reinterpret_cast<const uint32_t*>(src_k) + run0 + 64u * c, (uint32_t)lane,
                              reinterpret_cast<uint32_t*>(Xk) + j0);
                    dma_dword(reinterpret_cast<const uint32_t*>(src_v) + run0 + 64u * c, (uint32_t)lane,
                              reinterpret_cast<uint32_t*>(V) + j0);
                }
            }
            cbase += nch;
        }
    }
    if (wave == 0) {
        if ((uint32_t)lane < Kg) {
            start[lane] = st_k;
            seg0[lane + 1] = incl;
        }
        if (lane == 0) seg0[0] = 0;
    }
    vm_drain();
    lds_barrier();

    for (uint32_t lvl = 0; (1u << lvl) < Kg; ++lvl) {
        const bool last = (2u << lvl) >= Kg;
        const GlobalSinkKT64 gout{dst_k + obase, dst_v + obase, V, flip_out, cnt};
        if (lvl == 0) {
            const LdsKT64Loaded X{Xk};
            if (last) merge_level<EM>(X, seg0, Kg, lvl, cnt, gout, wave, W, lane);
            else merge_level<EM>(X, seg0, Kg, lvl, cnt, LdsKT64{Yk, Yt}, wave, W, lane);
        } else {
            const LdsKT64 X{Xk, Xt};
            if (last) merge_level<EM>(X, seg0, Kg, lvl, cnt, gout, wave, W, lane);
            else merge_level<EM>(X, seg0, Kg, lvl, cnt, LdsKT64{Yk, Yt}, wave, W, lane);
        }
        lds_barrier();
        uint64_t* tmp = Xk; Xk = Yk; Yk = tmp;
        uint16_t* tt = Xt; Xt = Yt; Yt = tt;
    }
}

// ===========================================================================
// Keys-only K-way merge of one output tile (§4.2, §7) with the transposed
// block step of the 32-bit merges on 64-bit words: every wave lays the
// tile's pieces out at 4-aligned slots from the split rows and issues its
// LDS copies at once, wave 0 plans each level's work per wave, and the
// levels merge 64x8-key blocks sorted in registers through two transposes
// of the words' halves.  LDS: two level buffers of cap = Tout + 4K keys, the
// waves' transpose scratch, the piece table and plan (two workgroups per CU
// at 3840-key tiles).
// ===========================================================================
constexpr uint32_t kMetaWords64 = 3u * 17u + kPlanWords;

template <int W>
__global__ __launch_bounds__(W * 64, 4) void k_merge64_keys(Phase64 ph, Bufs64 b, RoundArgs ra,
                                                            const uint32_t* __restrict__ table, uint64_t flip) {
    constexpr int EM = 8;
    const uint32_t Tout = ra.Tout, K = ra.K;
    const uint64_t L = ra.L;
    const uint32_t cap = Tout + 4u * K;
    extern __shared__ __align__(16) uint64_t smem64[];
    uint64_t* X = smem64;
    uint64_t* Y = smem64 + cap;
    uint32_t* scr = reinterpret_cast<uint32_t*>(Y + cap);
    uint32_t* mb = scr + W * Xpose<EM>::WORDS;
    const Meta mt{mb, mb + 17, mb + 34, mb + 51, nullptr};

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    uint32_t* wscr = scr + (uint32_t)wave * Xpose<EM>::WORDS;
    const uint64_t t = blockIdx.x;
    const uint64_t* src = ph.dst_out ? b.ws_k : b.out_k;
    uint64_t* dst = ph.dst_out ? b.out_k : b.ws_k;
    const uint64_t flip_out = ph.final_pass ? flip : 0ull;
    const uint64_t grp = t / ra.tpg;
    const uint64_t i = t - grp * ra.tpg;
    const uint64_t span = (uint64_t)K * L;
    const uint64_t gb = grp * span;
    const uint64_t glen = min(span, ph.n - gb);
    const uint32_t Kg = (uint32_t)((glen + L - 1) / L);
    const uint64_t obeg = i * (uint64_t)Tout;
    const uint32_t cnt = (uint32_t)min<uint64_t>(Tout, glen - obeg);
    const uint64_t obase = gb + obeg;

    if (Kg == 1) {   // a lone run: its tile is already in order
        for (uint32_t j = threadIdx.x; j < cnt; j += blockDim.x) gptr64(dst)[obase + j] = gptr64(src)[obase + j] ^ flip_out;
        return;
    }
    uint32_t s = 0, e = 0;
    if ((uint32_t)lane < Kg) {
        const uint32_t k = (uint32_t)lane;
        const uint32_t nk = (uint32_t)min(L, glen - (uint64_t)k * L);
        // the clamps only guard memory safety; exact splits never trigger them
        s = i == 0 ? 0u : min(table[t * K + k], nk);
        e = (obeg + Tout >= glen) ? nk : min(max(table[(t + 1) * K + k], s), nk);
    }
    {
        // each piece's keys (two words each) go into LDS by the memory unit,
        // 64 words per instruction, chunks dealt to the waves round-robin
        const PieceLayout pc = piece_layout(s, e, Kg, cnt, lane);
        const uint32_t* src32 = reinterpret_cast<const uint32_t*>(src);
        uint32_t* X32 = reinterpret_cast<uint32_t*>(X);
        uint32_t cbase = 0;
        for (uint32_t k = 0; k < Kg; ++k) {
            const uint32_t w0 = 2u * (uint32_t)__builtin_amdgcn_readlane((int)pc.sb, (int)k);
            const uint32_t nw = 2u * (uint32_t)__builtin_amdgcn_readlane((int)pc.len, (int)k);
            const uint32_t st = (uint32_t)__builtin_amdgcn_readlane((int)s, (int)k);
            const uint32_t nch = (nw + 63u) >> 6;
            const uint64_t run0 = 2u * (gb + (uint64_t)k * L + st);   // the piece's first word
            for (uint32_t c = ((uint32_t)wave + W - cbase % W) % W; c < nch; c += W) {
                if (64u * c + (uint32_t)lane < nw) dma_dword(src32 + run0 + 64u * c, (uint32_t)lane, X32 + w0 + 64u * c);
            }
            cbase += nch;
        }
    }
    if (wave == 0) {   // the other waves wait for this plan: it issues first
        __builtin_amdgcn_s_setprio(2);
        build_pieces(mt, s, e, Kg, cnt, L, lane);
        lds_wave_sync();
        build_plan<W>(mt, Kg, lane);
        __builtin_amdgcn_s_setprio(0);
    }
    vm_drain();
    lds_barrier();

    uint32_t nlev = 0;
    while ((1u << nlev) < Kg) ++nlev;
    const bool vec = ((uintptr_t)(dst + obase) & 15u) == 0;
    const U64SinkGlobal gout{dst + obase, flip_out, cnt, vec};
    for (uint32_t lvl = 0; lvl < nlev; ++lvl) {
        const U64Src in{X};
        if (lvl + 1u == nlev) merge_level_kt<EM>(in, mt, Kg, lvl, gout, wscr, plan_entry<W>(wave), lane);
        else merge_level_kt<EM>(in, mt, Kg, lvl, U64SinkLds{Y}, wscr, plan_entry<W>(wave), lane);
        lds_barrier();
        uint64_t* tmp = X; X = Y; Y = tmp;
    }
}

// ===========================================================================
// Launchers
// ===========================================================================
static hipError_t allow_lds64(const void* f, size_t bytes) {
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_tile_sort64(bool pairs, const Phase64& ph, const Bufs64& b, uint64_t flip, hipStream_t s) {
    if (ph.tiles == 0) return hipSuccess;
    if (pairs) {
        constexpr int E = 8, W = 4;
        static_assert(64u * E * W == kT64Pairs, "pairs base tile");
        const size_t lds = tile_lds_bytes<true>(kT64Pairs);
        hipError_t e = allow_lds64((const void*)k_tile_sort64<E, W, true>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_tile_sort64<E, W, true>), dim3((unsigned)ph.tiles), dim3(W * 64), lds, s, ph, b, flip);
    } else {
        constexpr int E = 8, W = 8;
        static_assert(64u * E * W == kT64Keys, "keys base tile");
        const size_t lds = tile_lds_bytes<false>(kT64Keys);
        hipError_t e = allow_lds64((const void*)k_tile_sort64<E, W, false>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_tile_sort64<E, W, false>), dim3((unsigned)ph.tiles), dim3(W * 64), lds, s, ph, b, flip);
    }
    return hipGetLastError();
}

hipError_t launch_corank_tiles64(const Phase64& ph, const Bufs64& b, const RoundArgs& ra, uint32_t* table,
                                 hipStream_t s) {
    if (ph.tiles == 0) return hipSuccess;
    const uint64_t blocks = (ph.tiles + 3) / 4;
    hipLaunchKernelGGL(k_corank_tiles64, dim3((unsigned)blocks), dim3(256), 0, s, ph, b, ra, table);
    return hipGetLastError();
}

hipError_t launch_merge64(bool pairs, const Phase64& ph, const Bufs64& b, const RoundArgs& ra, const uint32_t* table,
                          uint64_t flip, hipStream_t s) {
    if (ph.tiles == 0) return hipSuccess;
    if (ra.K > kMaxFanout || ra.Tout > (pairs ? kTout64Pairs : kTout64Keys) || ra.Tout % 4) return hipErrorInvalidValue;
    constexpr int W = 8;
    if (!pairs) {
        const uint32_t cap = ra.Tout + 4u * ra.K;
        const size_t lds = 8u * 2u * cap + (W * Xpose<8>::WORDS + kMetaWords64) * sizeof(uint32_t);
        hipError_t e = allow_lds64((const void*)k_merge64_keys<W>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_merge64_keys<W>), dim3((unsigned)ph.tiles), dim3(W * 64), lds, s, ph, b, ra, table, flip);
        return hipGetLastError();
    }
    // keys 2 x Tout, values Tout and 16-bit tags 2 x Tout
    const size_t lds = 28u * ra.Tout + (2u * kMaxFanout + 4u) * sizeof(uint32_t);
    hipError_t e = allow_lds64((const void*)k_merge64_pairs<W>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_merge64_pairs<W>), dim3((unsigned)ph.tiles), dim3(W * 64), lds, s, ph, b, ra, table, flip);
    return hipGetLastError();
}

}  // namespace mms
