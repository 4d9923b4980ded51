// Keys-only K-way merge round (§4.2, §7) as a persistent kernel.
//
// Each workgroup walks the output tiles t = blockIdx.x, blockIdx.x + G, ...
// of a round.  A tile's input is the K pieces of its group's runs bounded by
// the split indices of its first and last output (§4.1).  The pieces are
// placed at 4-aligned offsets of LDS buffer X and merged pairwise, level by
// level, with the conflict-free block step of merge_level_keys (log2 K
// levels: X->Y->X->...); the last level stores straight to memory.
//
// Memory latency is hidden by a two-stage prefetch: while tile t is merged,
// the keys of tile t+G are loaded into registers (each thread holds
// ceil(Tout / threads) of them together with their LDS destinations), and
// wave 0 already holds the split indices of tile t+2G.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mms_device.h"
#include "mms_internal.h"

namespace mms {

namespace {

struct TileGeo {
    const uint32_t* src;  // buffer the round reads (segment start)
    uint32_t* dst;        // buffer the round writes (segment start)
    uint64_t gb;      // group start inside the segment
    uint64_t glen;    // group size
    uint64_t obeg;    // tile start inside the group
    uint32_t Kg;      // runs in the group
    uint32_t cnt;     // outputs of the tile
    bool first;       // first tile of its group
    bool last;        // last tile of its group
    bool final_pass;  // last pass of the segment
};

__device__ __forceinline__ TileGeo tile_geo(const Phase& ph, const Bufs& b, uint64_t t, const RoundArgs& ra) {
    const TileRef tr = tile_ref(ph, b, t);
    TileGeo g;
    // tile counts stay far below 2^32, so 32-bit division suffices
    const uint32_t grp = tr.local / (uint32_t)ra.tpg;
    const uint64_t i = tr.local - (uint64_t)grp * ra.tpg;
    const uint64_t span = (uint64_t)ra.K * ra.L;
    const uint64_t gb = (uint64_t)grp * span;
    g.src = tr.src_k;
    g.dst = tr.dst_k;
    g.gb = gb;
    g.glen = min(span, tr.n - gb);
    g.Kg = (uint32_t)((g.glen + ra.L - 1) / ra.L);
    g.obeg = i * (uint64_t)ra.Tout;
    g.cnt = (uint32_t)min<uint64_t>(ra.Tout, g.glen - g.obeg);
    g.first = i == 0;
    g.last = g.obeg + ra.Tout >= g.glen;
    g.final_pass = tr.final_pass;
    return g;
}

// Split indices of tile t for run `lane` (wave 0, lanes < Kg): start s, end e.
__device__ __forceinline__ void load_split(const uint32_t* __restrict__ table, uint64_t t, const TileGeo& g,
                                           uint64_t L, uint32_t K, int lane, uint32_t& s, uint32_t& e) {
    s = 0;
    e = 0;
    if ((uint32_t)lane < g.Kg) {
        const uint32_t nk = (uint32_t)min(L, g.glen - (uint64_t)lane * L);
        s = g.first ? 0u : table[t * K + (uint32_t)lane];
        e = g.last ? nk : table[(t + 1) * K + (uint32_t)lane];
        // guards for memory safety only; exact splits satisfy s <= e <= nk
        s = min(s, nk);
        e = min(max(e, s), nk);
    }
}

// Piece table of a tile, written by wave 0: start[k] (inside run k),
// plen[k] (prefix of piece lengths), sbeg[k] (4-aligned LDS offsets).
struct Meta {
    uint32_t* start;
    uint32_t* plen;
    uint32_t* sbeg;
    uint32_t* cseg;   // [kToutKeys/64]: piece holding position 64*c of the tile
};
constexpr uint32_t kMetaWords = 3u * 17u + kToutKeys / 64u;

__device__ __forceinline__ uint32_t excl_scan16(uint32_t x, int lane) {
    uint32_t incl = x;
#pragma unroll
    for (int d = 1; d < 16; d <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)incl, d, 64);
        if ((lane & 15) >= d) incl += y;
    }
    return incl - x;
}

__device__ __forceinline__ void build_meta(const Meta& m, uint32_t s, uint32_t e, const TileGeo& g, int lane) {
    const bool own = (uint32_t)lane < g.Kg;
    uint32_t len = own ? e - s : 0u;
    uint32_t pl = excl_scan16(len, lane);
    // guards for memory safety only: keep the pieces inside the tile
    len = pl >= g.cnt ? 0u : min(len, g.cnt - pl);
    pl = min(pl, g.cnt);
    const uint32_t sb = excl_scan16((len + 3u) & ~3u, lane);
    if (own) {
        m.start[lane] = s;
        m.plen[lane] = pl;
        m.sbeg[lane] = sb;
    }
    const uint32_t tot_pl = (uint32_t)__shfl((int)(pl + len), (int)(g.Kg - 1), 64);
    const uint32_t tot_sb = (uint32_t)__shfl((int)(sb + ((len + 3u) & ~3u)), (int)(g.Kg - 1), 64);
    if (lane == 0) {
        m.plen[g.Kg] = tot_pl;
        m.sbeg[g.Kg] = tot_sb;
    }
    lds_wave_sync();
    // chunk table: largest k < Kg with plen[k] <= 64*c
    for (uint32_t c = (uint32_t)lane; c * 64u < tot_pl; c += 64u) {
        uint32_t lo = 0, hi = g.Kg;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (m.plen[mid] <= c * 64u) lo = mid;
            else hi = mid;
        }
        m.cseg[c] = lo;
    }
}

}  // namespace

template <int EM, int W, int PF>
__global__ __launch_bounds__(W * 64) void k_merge_keys(Phase ph, Bufs b, RoundArgs ra,
                                                       const uint32_t* __restrict__ table, uint32_t flip) {
    constexpr uint32_t NT = W * 64;
    const uint64_t L = ra.L;
    const uint32_t K = ra.K, Tout = ra.Tout;
    const uint64_t tiles = ph.tiles;
    extern __shared__ __align__(16) uint32_t smem[];
    const uint32_t cap = Tout + 4u * K;
    uint32_t* bufA = smem;
    uint32_t* bufB = smem + cap;
    uint32_t* scr = smem + 2 * cap;
    uint32_t* mbase = scr + W * Xpose<EM>::WORDS;     // two piece tables of kMetaWords
    auto meta = [&](int which) {
        uint32_t* mb = mbase + kMetaWords * (uint32_t)which;
        return Meta{mb, mb + 17, mb + 34, mb + 51};
    };

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wave-uniform
    const uint32_t tid = threadIdx.x;
    const uint64_t G = gridDim.x;
    uint32_t* wscr = scr + (uint32_t)wave * Xpose<EM>::WORDS;

    uint64_t t = blockIdx.x;
    if (t >= tiles) return;

    // registers of the prefetch stage
    uint32_t pf_val[PF];
    uint32_t pf_dst[PF];
    uint32_t nx_s = 0, nx_e = 0;   // wave 0: split indices of the tile after next

    auto issue_loads = [&](uint64_t tt, const Meta& m) {
        const TileGeo g = tile_geo(ph, b, tt, ra);
        const uint32_t* src = g.src;
#pragma unroll
        for (int r = 0; r < PF; ++r) {
            const uint32_t j = (uint32_t)r * NT + tid;
            pf_dst[r] = 0xFFFFFFFFu;
            if (j < m.plen[g.Kg]) {
                uint32_t lo = m.cseg[j >> 6];        // largest k with plen[k] <= j
                while (lo + 1u < g.Kg && m.plen[lo + 1u] <= j) ++lo;
                const uint32_t off = j - m.plen[lo];
                pf_val[r] = src[g.gb + (uint64_t)lo * L + m.start[lo] + off];
                pf_dst[r] = m.sbeg[lo] + off;
            }
        }
    };
    auto store_loads = [&](uint32_t* X) {
#pragma unroll
        for (int r = 0; r < PF; ++r)
            if (pf_dst[r] != 0xFFFFFFFFu) X[pf_dst[r]] = pf_val[r];
    };

    // prologue: piece table and keys of the first tile, split of the second
    {
        const TileGeo g0 = tile_geo(ph, b, t, ra);
        if (wave == 0) {
            uint32_t s, e;
            load_split(table, t, g0, L, K, lane, s, e);
            build_meta(meta(0), s, e, g0, lane);
            if (t + G < tiles) load_split(table, t + G, tile_geo(ph, b, t + G, ra), L, K, lane, nx_s, nx_e);
        }
        lds_barrier();
        issue_loads(t, meta(0));
        store_loads(bufA);
        lds_barrier();
    }

    int cur = 0;
    for (;;) {
        const TileGeo g = tile_geo(ph, b, t, ra);
        uint32_t* dst = g.dst;
        const uint32_t flip_out = g.final_pass ? flip : 0u;
        const Meta mc = meta(cur);
        const Meta mn = meta(cur ^ 1);
        const uint64_t tn = t + G;
        const bool has_next = tn < tiles;

        // wave 0: piece table of the next tile, split indices of the one after
        if (wave == 0 && has_next) {
            const TileGeo gn = tile_geo(ph, b, tn, ra);
            build_meta(mn, nx_s, nx_e, gn, lane);
            if (tn + G < tiles)
                load_split(table, tn + G, tile_geo(ph, b, tn + G, ra), L, K, lane, nx_s, nx_e);
        }

        uint32_t* X = bufA;
        uint32_t* Y = bufB;
        const uint64_t obase = g.gb + g.obeg;
        bool issued = false;
        if (g.Kg == 1) {
            lds_barrier();
            if (has_next) {
                issue_loads(tn, mn);
                issued = true;
            }
            for (uint32_t j = tid; j < g.cnt; j += NT) dst[obase + j] = X[j] ^ flip_out;
        } else {
            const bool vec = ((uintptr_t)(dst + obase) & 15u) == 0;
            for (uint32_t lvl = 0; (1u << lvl) < g.Kg; ++lvl) {
                const bool last = (2u << lvl) >= g.Kg;
                if (last) {
                    GlobalSinkKeys out{dst + obase, flip_out, g.cnt, vec};
                    merge_level_keys<EM>(X, mc.sbeg, mc.plen, g.Kg, lvl, out, wscr, wave, W, lane);
                } else {
                    LdsSinkKeys out{Y};
                    merge_level_keys<EM>(X, mc.sbeg, mc.plen, g.Kg, lvl, out, wscr, wave, W, lane);
                }
                lds_barrier();
                // the next tile's piece table is visible now; its loads overlap
                // the remaining levels
                if (!issued && has_next) {
                    issue_loads(tn, mn);
                    issued = true;
                }
                uint32_t* tmp = X; X = Y; Y = tmp;
            }
        }
        if (!has_next) break;
        lds_barrier();        // every wave is done reading this tile's LDS
        store_loads(bufA);
        lds_barrier();
        t = tn;
        cur ^= 1;
    }
}

static hipError_t allow_lds(const void* f, size_t bytes) {
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int EM, int W>
static hipError_t launch_variant(const Phase& ph, const Bufs& b, const RoundArgs& ra, const uint32_t* table,
                                 uint32_t flip, unsigned grid, hipStream_t s) {
    constexpr int PF = (int)((kToutKeys + W * 64 - 1) / (W * 64));
    const size_t lds = (2u * (ra.Tout + 4u * ra.K) + W * Xpose<EM>::WORDS + 2u * kMetaWords) * sizeof(uint32_t);
    hipError_t e = allow_lds((const void*)k_merge_keys<EM, W, PF>, lds);
    if (e != hipSuccess) return e;
    // persistent grid: as many workgroups as fit in the LDS of `grid` CUs
    int dev = 0, lds_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
        lds_cu <= 0)
        lds_cu = 160 * 1024;
    const uint64_t per_cu = (uint64_t)lds_cu / lds > 0 ? (uint64_t)lds_cu / lds : 1;
    const uint64_t want = (uint64_t)grid * per_cu;
    const unsigned blocks = (unsigned)(want < ph.tiles ? want : ph.tiles);
    hipLaunchKernelGGL((k_merge_keys<EM, W, PF>), dim3(blocks), dim3(W * 64), lds, s, ph, b, ra, table, flip);
    return hipGetLastError();
}

hipError_t launch_merge_keys(const Phase& ph, const Bufs& b, const RoundArgs& ra, const uint32_t* table,
                             uint32_t flip, unsigned grid, int variant, hipStream_t s) {
    if (ra.Tout > kToutKeys || ra.K > kMaxFanout || ra.Tout % 4 || ra.L % 4) return hipErrorInvalidValue;
    if (ph.tiles == 0) return hipSuccess;
    if (variant == 1) return launch_variant<8, 16>(ph, b, ra, table, flip, grid, s);
    if (variant == 2) return launch_variant<8, 8>(ph, b, ra, table, flip, grid, s);
    return launch_variant<16, 8>(ph, b, ra, table, flip, grid, s);
}

}  // namespace mms
