// Key-value K-way merge round (§4.2, values moving with their keys), one
// workgroup per output tile.
//
// A tile's input is the K pieces of its group's runs bounded by the split
// indices of its first and last output (§4.1).  Wave 0 lays the pieces out at
// 4-aligned LDS slots and plans every merge level's work per wave; the
// pieces' keys and values then go into LDS through the memory unit.  The
// merge tree runs on (key, tag) pairs packed into 64-bit words (tag = the
// pair's slot as loaded, which orders equal keys stably): level 0 reads the
// loaded keys, later levels read keys and 16-bit tags written by the level
// before, and the last level stores keys to memory with each value gathered
// from its slot.  LDS (words, cap = Tout + 4K slots): keys 2 x cap, tags
// 2 x cap/2, values cap, the waves' transpose scratch, the piece table and
// plan; for Tout = 3840 two workgroups share a compute unit.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mms_device.h"
#include "mms_device_kt.h"
#include "mms_internal.h"
#include "mms_tile_plan.h"

namespace mms {

namespace {

constexpr int kEMP = 8;   // 64 x 8-pair merge blocks
constexpr uint32_t kMetaWordsP = 3u * 17u + kPlanWords;

}  // namespace

template <int W>
__global__ __launch_bounds__(W * 64, 4) void k_merge_pairs(Phase ph, Bufs b, RoundArgs ra,
                                                           const uint32_t* __restrict__ table, uint32_t flip) {
    const uint32_t Tout = ra.Tout, K = ra.K;
    const uint64_t L = ra.L;
    const uint32_t cap = Tout + 4u * K;
    extern __shared__ __align__(16) uint32_t smem[];
    uint32_t* K0 = smem;
    uint32_t* K1 = K0 + cap;
    uint16_t* T0 = reinterpret_cast<uint16_t*>(K1 + cap);
    uint16_t* T1 = T0 + cap;
    uint32_t* V = reinterpret_cast<uint32_t*>(T1 + cap);
    uint32_t* scr = V + cap;
    uint32_t* mb = scr + W * Xpose<kEMP>::WORDS;
    const Meta mt{mb, mb + 17, mb + 34, mb + 51, nullptr};

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wave-uniform
    uint32_t* wscr = scr + (uint32_t)wave * Xpose<kEMP>::WORDS;
    const uint64_t t = blockIdx.x;
    const TileRef tr = tile_ref(ph, b, t);
    const uint32_t flip_out = tr.final_pass ? flip : 0u;
    const uint32_t grp = tr.local / (uint32_t)ra.tpg;
    const uint64_t i = tr.local - (uint64_t)grp * ra.tpg;
    const uint64_t span = (uint64_t)K * L;
    const uint64_t gb = (uint64_t)grp * span;
    const uint64_t glen = min(span, tr.n - gb);
    const uint32_t Kg = (uint32_t)((glen + L - 1) / L);
    const uint64_t obeg = i * (uint64_t)Tout;
    const uint32_t cnt = (uint32_t)min<uint64_t>(Tout, glen - obeg);
    const uint64_t obase = gb + obeg;

    if (Kg == 1) {   // a lone run: its tile is already in order
        for (uint32_t j = threadIdx.x; j < cnt; j += blockDim.x) {
            gptr(tr.dst_k)[obase + j] = gptr(tr.src_k)[obase + j] ^ flip_out;
            gptr(tr.dst_v)[obase + j] = gptr(tr.src_v)[obase + j];
        }
        return;
    }
    // Every wave reads the tile's split indices (lane k < Kg: run k) and
    // lays the pieces out in registers, so its loads into LDS go out at
    // once; wave 0 also writes the layout and plans the merge levels while
    // they are in flight.
    uint32_t s = 0, e = 0;
    if ((uint32_t)lane < Kg) {
        const uint32_t k = (uint32_t)lane;
        const uint32_t nk = (uint32_t)min(L, glen - (uint64_t)k * L);
        // the clamps only guard memory safety; exact splits never trigger them
        s = i == 0 ? 0u : min(table[t * K + k], nk);
        e = (obeg + Tout >= glen) ? nk : min(max(table[(t + 1) * K + k], s), nk);
    }
    {
        // The pieces' keys and values go into LDS by the memory unit, 64
        // words per instruction; chunks are dealt to the waves round-robin in
        // piece order.
        const PieceLayout pc = piece_layout(s, e, Kg, cnt, lane);
        uint32_t cbase = 0;   // chunks of the earlier pieces
        for (uint32_t k = 0; k < Kg; ++k) {
            const uint32_t s0 = (uint32_t)__builtin_amdgcn_readlane((int)pc.sb, (int)k);
            const uint32_t len = (uint32_t)__builtin_amdgcn_readlane((int)pc.len, (int)k);
            const uint32_t st = (uint32_t)__builtin_amdgcn_readlane((int)s, (int)k);
            const uint32_t nch = (len + 63u) >> 6;
            const uint64_t run0 = gb + (uint64_t)k * L + st;   // the piece's first element
            for (uint32_t c = ((uint32_t)wave + W - cbase % W) % W; c < nch; c += W) {
                if (64u * c + (uint32_t)lane < len) {
                    dma_dword(tr.src_k + run0 + 64u * c, (uint32_t)lane, K0 + s0 + 64u * c);
                    dma_dword(tr.src_v + run0 + 64u * c, (uint32_t)lane, V + s0 + 64u * c);
                }
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
    const int pe = plan_entry<W>(wave);   // balanced over the SIMDs
    uint32_t* Xk = K0;
    uint16_t* Xt = T0;
    uint32_t* Yk = K1;
    uint16_t* Yt = T1;
    const bool vec = (((uintptr_t)(tr.dst_k + obase) | (uintptr_t)(tr.dst_v + obase)) & 15u) == 0;
    const KtSinkGlobal gout{tr.dst_k + obase, tr.dst_v + obase, V, flip_out, cnt, vec};
    for (uint32_t lvl = 0; lvl < nlev; ++lvl) {
        const bool last = lvl + 1u == nlev;
        if (lvl == 0) {
            const KtSrcLoaded X{Xk};
            if (last) merge_level_kt<kEMP>(X, mt, Kg, lvl, gout, wscr, pe, lane);
            else merge_level_kt<kEMP>(X, mt, Kg, lvl, KtSinkLds{Yk, Yt}, wscr, pe, lane);
        } else {
            const KtSrcTagged X{Xk, Xt};
            if (last) merge_level_kt<kEMP>(X, mt, Kg, lvl, gout, wscr, pe, lane);
            else merge_level_kt<kEMP>(X, mt, Kg, lvl, KtSinkLds{Yk, Yt}, wscr, pe, lane);
        }
        lds_barrier();
        uint32_t* tk = Xk; Xk = Yk; Yk = tk;
        uint16_t* tt = Xt; Xt = Yt; Yt = tt;
    }
}

static hipError_t allow_lds(const void* f, size_t bytes) {
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_merge_pairs(const Phase& ph, const Bufs& b, const RoundArgs& ra, const uint32_t* table,
                              uint32_t flip, hipStream_t s) {
    if (ph.tiles == 0) return hipSuccess;
    // tags are 16-bit slots; the plan encodes outputs in 14 bits
    if (ra.Tout > kToutPairs || ra.Tout % 4 || ra.K > kMaxFanout) return hipErrorInvalidValue;
    const uint32_t cap = ra.Tout + 4u * ra.K;
    const size_t lds = (4u * cap + kW3 * Xpose<kEMP>::WORDS + kMetaWordsP) * sizeof(uint32_t);
    hipError_t e = allow_lds((const void*)k_merge_pairs<kW3>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_merge_pairs<kW3>), dim3((unsigned)ph.tiles), dim3(kW3 * 64), lds, s, ph, b, ra, table, flip);
    return hipGetLastError();
}

}  // namespace mms
