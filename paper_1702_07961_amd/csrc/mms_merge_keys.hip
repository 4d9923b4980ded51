// Keys-only K-way merge round (§4.2, §7) as a persistent kernel.
//
// Each workgroup walks the output tiles t = blockIdx.x, blockIdx.x + G, ...
// of a round.  A tile's input is the K pieces of its group's runs bounded by
// the split indices of its first and last output (§4.1).  The pieces are
// placed at 4-aligned offsets of LDS buffer X and merged pairwise, level by
// level, with the conflict-free block step of merge_pair_range_keys (log2 K
// levels: X->Y->X->...); the last level stores straight to memory.
//
// Memory latency is hidden by a three-stage pipeline: as tile t starts, the
// keys of tile t+G are loaded into registers in 16-byte chunks (each thread
// holds a few chunks with their LDS destinations) and land in the LDS buffer
// that tile t's last level does not read.  The piece table of a tile is
// built in two steps one tile apart, by three waves besides their share of
// the merge: wave 0 lays out the pieces of tile t+3G from split-table rows
// the memory unit copied into LDS one tile earlier, then waves 1 and 2
// derive the chunk table and the per-level wave plan of tile t+2G from its
// layout.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mms_device.h"
#include "mms_internal.h"
#include "mms_tile_plan.h"

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
    // flags as full words: the struct is copied across loop iterations and
    // must stay in registers
    uint32_t first;       // first tile of its group
    uint32_t last;        // last tile of its group
    uint32_t final_pass;  // last pass of the segment
};

// lL = log2(L) (run lengths are T times a power of two)
__device__ __forceinline__ TileGeo tile_geo(const Phase& ph, const Bufs& b, uint64_t t, const RoundArgs& ra,
                                            int lL) {
    const TileRef tr = tile_ref(ph, b, t);
    TileGeo g;
    // a tile index is below 2^23 (n < 2^32, Tout >= 1024, plus one per
    // group) and the quotient below 2^22 unless tpg = 1, where the estimate
    // is exact; a divisor above the index gives 0, so it may be clamped
    const uint32_t grp = udiv_small(tr.local, (uint32_t)min<uint64_t>(ra.tpg, (1u << 23)));
    const uint64_t i = tr.local - (uint64_t)grp * ra.tpg;
    const uint64_t span = (uint64_t)ra.K * ra.L;
    const uint64_t gb = (uint64_t)grp * span;
    g.src = tr.src_k;
    g.dst = tr.dst_k;
    g.gb = gb;
    g.glen = min(span, tr.n - gb);
    g.Kg = (uint32_t)((g.glen + ra.L - 1) >> lL);
    g.obeg = i * (uint64_t)ra.Tout;
    g.cnt = (uint32_t)min<uint64_t>(ra.Tout, g.glen - g.obeg);
    g.first = i == 0 ? 1u : 0u;
    g.last = g.obeg + ra.Tout >= g.glen ? 1u : 0u;
    g.final_pass = tr.final_pass ? 1u : 0u;
    return g;
}

// Split indices of tile t for run `lane` (lanes < Kg): start s, end e.
// The table rows t and t+1 are read with scalar loads (the table was written
// by an earlier launch), so the wave does not wait on its own outstanding
// vector memory traffic, which includes the previous tile's stores.
typedef const __attribute__((address_space(4))) uint32_t* ScalarU32;

__device__ __forceinline__ void load_split(const uint32_t* __restrict__ table, uint64_t t, const TileGeo& g,
                                           uint64_t L, uint32_t K, int lane, uint32_t& s, uint32_t& e) {
    const ScalarU32 tc = (ScalarU32)table;
    const uint64_t r0 = t * K, r1 = r0 + K;
    s = 0;
    e = 0;
#pragma unroll
    for (uint32_t k = 0; k < kMaxFanout; ++k) {
        if (k < g.Kg) {
            const uint32_t nk = (uint32_t)min(L, g.glen - (uint64_t)k * L);
            uint32_t sk = g.first ? 0u : tc[r0 + k];
            uint32_t ek = g.last ? nk : tc[r1 + k];
            // guards for memory safety only; exact splits satisfy s <= e <= nk
            sk = min(sk, nk);
            ek = min(max(ek, sk), nk);
            s = (uint32_t)lane == k ? sk : s;
            e = (uint32_t)lane == k ? ek : e;
        }
    }
}

// Split indices of a tile for run `lane` (lanes < Kg) from its two table
// rows held in LDS (row t at rows[0..K), row t+1 at rows[K..2K)), with the
// same guards as load_split.
__device__ __forceinline__ void split_from_rows(const uint32_t* rows, const TileGeo& g, uint64_t L, uint32_t K,
                                                int lane, uint32_t& s, uint32_t& e) {
    s = 0;
    e = 0;
    if ((uint32_t)lane < g.Kg) {
        const uint32_t k = (uint32_t)lane;
        // every run but the group's last holds L keys (wave-uniform values)
        const uint32_t nk = k + 1u < g.Kg ? (uint32_t)L : (uint32_t)(g.glen - (uint64_t)(g.Kg - 1u) * L);
        const uint32_t sk = g.first ? 0u : min(rows[k], nk);
        s = sk;
        e = g.last ? nk : min(max(rows[K + k], sk), nk);
    }
}

// Rows t and t+1 of the split table (2K consecutive words; the table has a
// row past the last tile) copied into LDS by the memory unit, one word per
// lane, without passing through registers.  The copy is issued in inline
// assembly (saving and restoring M0, which holds its LDS address) so that the
// compiler does not track it: after a tracked copy into LDS the compiler
// makes the next LDS read of every wave wait for all of the wave's
// outstanding memory operations, since it cannot tell that the read does not
// touch the copy's target, and here that read comes on every tile while the
// previous tile's stores are still in flight.  The caller waits for the copy
// itself: wave 0, the only wave that issues it, drains its memory counter on
// every path between the copy and the next read of the rows.
__device__ __forceinline__ void fetch_rows_async(const uint32_t* __restrict__ table, uint64_t t, uint32_t K,
                                                 uint32_t* rows, int lane) {
    // the rows' address as a wave-uniform base plus a per-lane offset
    const uint64_t base = (uint64_t)(uintptr_t)(table + t * K);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)base);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(base >> 32));
    const uint64_t row = ((uint64_t)hi << 32) | lo;
    const uint32_t lds = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(uintptr_t)rows);
    if ((uint32_t)lane < 2u * K) {
        uint32_t saved;
        asm volatile(
            "s_mov_b32 %0, m0\n\t"
            "s_mov_b32 m0, %2\n\t"
            "s_nop 0\n\t"
            "global_load_lds_dword %1, %3\n\t"
            "s_nop 0\n\t"
            "s_mov_b32 m0, %0"
            : "=&s"(saved)
            : "v"(4u * (uint32_t)lane), "s"(lds), "s"(row)
            : "memory");
    }
}

// words of one piece table (with its chunk table)
constexpr uint32_t kMetaWords = 3u * 17u + kPlanWords + ((kToutKeys + 4u * kMaxFanout) / 64u + 1u + 3u) / 4u;

// Chunk table from the piece layout: largest k < Kg with sbeg[k] <= 64*c.
__device__ __forceinline__ void build_chunks(const Meta& m, uint32_t Kg, int lane) {
    const uint32_t tot_sb = m.sbeg[Kg];
    for (uint32_t c = (uint32_t)lane; c * 64u < tot_sb; c += 64u) {
        uint32_t lo = 0, hi = Kg;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (m.sbeg[mid] <= c * 64u) lo = mid;
            else hi = mid;
        }
        m.cseg[c] = (uint8_t)lo;
    }
}

// The whole piece table by one wave (the pipeline's prologue).
template <int W>
__device__ __forceinline__ void build_meta(const Meta& m, uint32_t s, uint32_t e, const TileGeo& g, uint64_t L,
                                          int lane) {
    build_pieces(m, s, e, g.Kg, g.cnt, L, lane);
    lds_wave_sync();
    build_chunks(m, g.Kg, lane);
    build_plan<W>(m, g.Kg, lane);
}

}  // namespace

// MINW: waves per SIMD the register allocation must allow (HIP's second
// launch bound); 4 with 8-wave workgroups lets two workgroups share a CU.
template <int EM, int W, int PC, int MINW>
__global__ __launch_bounds__(W * 64, MINW) void k_merge_keys(Phase ph, Bufs b, RoundArgs ra,
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
    // the block merge reads up to 64*EM words past a buffer's last run
    static_assert(W * Xpose<EM>::WORDS >= 64u * EM, "LDS after bufB is shorter than a merge block");
    static_assert(W >= 3, "waves 0, 1 and 2 build the piece tables");
    uint32_t* mbase = scr + W * Xpose<EM>::WORDS;     // four piece tables of kMetaWords
    auto meta = [&](int which) {
        uint32_t* mb = mbase + kMetaWords * (uint32_t)which;
        return Meta{mb, mb + 17, mb + 34, mb + 51, reinterpret_cast<uint8_t*>(mb + 51 + kPlanWords)};
    };

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wave-uniform
    const uint32_t tid = threadIdx.x;
    const uint64_t G = gridDim.x;
    uint32_t* wscr = scr + (uint32_t)wave * Xpose<EM>::WORDS;

    uint64_t t = blockIdx.x;
    if (t >= tiles) return;
    const int lL = __builtin_ctzll(L);

    // registers of the prefetch stage: chunks of 4 LDS slots per thread
    u32x4a4 pf_val[PC];
    uint32_t pf_dst[PC];
    // wave 0: split-table rows of tile t+3G (at loop start), copied in by the
    // memory unit one tile ahead
    uint32_t* rows = mbase + 4u * kMetaWords;

    // Chunk P (a multiple of 4 in LDS slot coordinates) lies in piece k with
    // sbeg[k] <= P < sbeg[k] + len_k rounded up to 4, so off = P - sbeg[k] <
    // len_k: its first key exists.  Every chunk is one 16-byte load (global
    // addresses are only 4-byte aligned) of the four keys from its first one
    // on; keys past the piece's end land in padding slots that no merge step
    // reads.  A chunk that would read past the group's last key is read d
    // keys earlier instead and shifted back by d as it is stored (groups of
    // two or more runs hold more than one base tile; a lone run is not loaded
    // at all, its tile is copied from memory).  One load form for every chunk
    // keeps all of a thread's loads in flight together.
    auto issue_loads = [&](const TileGeo& g, const Meta& m) {
        if (g.Kg < 2) {
#pragma unroll
            for (int r = 0; r < PC; ++r) pf_dst[r] = 0xFFFFFFFFu;
            return;
        }
        const uint32_t slots = m.sbeg[g.Kg];
        const uint32_t glen = (uint32_t)g.glen;
        const uint32_t Kg = g.Kg;
        cgu32* gsrc = gptr(g.src) + g.gb;
        // Each chunk's piece in three rounds of LDS reads, the reads of all
        // of a thread's chunks issued together in each round: the chunk
        // table gives the piece holding slot 64*floor(P/64), the next two
        // piece starts move it on by up to two pieces (further only past a
        // piece shorter than 64 slots, in a loop that seldom runs), and the
        // piece's source offset gives the chunk's position in the group.
        // Every lane loads (a lane past the tile's last chunk reads chunk 0
        // again and discards it), so no load sits under a branch.
        uint32_t P[PC], k[PC];
        bool used[PC], more[PC];
#pragma unroll
        for (int r = 0; r < PC; ++r) {
            const uint32_t P0 = 4u * ((uint32_t)r * NT + tid);
            used[r] = P0 < slots;
            P[r] = used[r] ? P0 : 0u;
            k[r] = m.cseg[P[r] >> 6];
        }
#pragma unroll
        for (int r = 0; r < PC; ++r) {
            const uint32_t k0 = k[r];
            const uint32_t s1 = m.sbeg[k0 + 1u], s2 = m.sbeg[min(k0 + 2u, kMaxFanout)];
            const bool a1 = k0 + 1u < Kg && s1 <= P[r];
            const bool a2 = k0 + 2u < Kg && s2 <= P[r];   // implies a1: piece starts ascend
            k[r] = k0 + (uint32_t)a1 + (uint32_t)a2;
            more[r] = a2;
        }
#pragma unroll
        for (int r = 0; r < PC; ++r)
            if (more[r])
                while (k[r] + 1u < Kg && m.sbeg[k[r] + 1u] <= P[r]) ++k[r];
#pragma unroll
        for (int r = 0; r < PC; ++r) {
            const uint32_t q = m.src0[k[r]] + P[r];                    // inside the group
            const uint32_t d = q + 4u > glen ? q + 4u - glen : 0u;     // 0..3
            pf_val[r] = *reinterpret_cast<cgu32x4a4*>(gsrc + (q - d));
            pf_dst[r] = used[r] ? (P[r] | (d << 30)) : 0xFFFFFFFFu;
        }
    };
    auto store_loads = [&](uint32_t* X) {
#pragma unroll
        for (int r = 0; r < PC; ++r) {
            // every lane's load is waited for here, not only the stored
            // ones: otherwise the compiler cannot tell, where the next
            // tile's loads reuse these registers, that no load into them is
            // outstanding, and waits there for all of the wave's memory
            // operations (the previous tile's stores included)
            u32x4a4 v = pf_val[r];
            asm volatile("" ::"v"(v.x), "v"(v.y), "v"(v.z), "v"(v.w));
            if (pf_dst[r] != 0xFFFFFFFFu) {
                const uint32_t d = pf_dst[r] >> 30;
                if (d) {   // key j of the chunk is component j + d
                    v.x = d == 1u ? v.y : d == 2u ? v.z : v.w;
                    v.y = d == 1u ? v.z : v.w;
                    v.z = v.w;
                }
                *reinterpret_cast<u32x4*>(X + (pf_dst[r] & 0x3FFFFFFFu)) = v;
            }
        }
    };

    // Pipeline: while tile t is merged, the keys of tile t+G are in flight
    // (issued as tile t starts), waves 1 and 2 finish the piece table of tile
    // t+2G and wave 0 lays out the pieces of tile t+3G from split indices it
    // loaded one tile earlier.  Four piece tables rotate (tiles t .. t+3G);
    // every step reads what an earlier tile's barriers published.
    // Prologue: whole piece tables of the first two tiles, the layout of the
    // third, the split indices of the fourth, and the first tile's keys.
    // Tile geometries are recomputed where they are used (a few scalar
    // instructions each) rather than carried across iterations.
    auto nxt = [](int i) { return (i + 1) & 3; };
    {
        const TileGeo g = tile_geo(ph, b, t, ra, lL);
        if (wave == 0) {
            uint32_t s, e;
            load_split(table, t, g, L, K, lane, s, e);
            build_meta<W>(meta(0), s, e, g, L, lane);
            if (t + G < tiles) {
                const TileGeo g1 = tile_geo(ph, b, t + G, ra, lL);
                load_split(table, t + G, g1, L, K, lane, s, e);
                build_meta<W>(meta(1), s, e, g1, L, lane);
                if (t + 2 * G < tiles) {
                    const TileGeo gp = tile_geo(ph, b, t + 2 * G, ra, lL);
                    load_split(table, t + 2 * G, gp, L, K, lane, s, e);
                    build_pieces(meta(2), s, e, gp.Kg, gp.cnt, L, lane);
                    if (t + 3 * G < tiles) fetch_rows_async(table, t + 3 * G, K, rows, lane);
                }
            }
        }
        lds_barrier();
        issue_loads(g, meta(0));
        if (wave == 0) vm_drain();   // the rows copy is older than these loads
        store_loads(bufA);
        lds_barrier();
    }

    int cur = 0;
    uint32_t* in = bufA;      // LDS buffer holding the current tile's pieces
    uint32_t* other = bufB;
    for (;;) {
        const TileGeo g = tile_geo(ph, b, t, ra, lL);
        uint32_t* dst = g.dst;
        const uint32_t flip_out = g.final_pass ? flip : 0u;
        const Meta mc = meta(cur);
        const Meta mn = meta(nxt(cur));
        const uint64_t tn = t + G, t2 = t + 2 * G;
        const bool has_next = tn < tiles, has2 = t2 < tiles;

        // wave 0: piece layout of tile t+3G from its split-table rows (copied
        // into LDS one tile ago), then the copy of tile t+4G's rows; it is
        // complete once wave 0 drains its memory counter before storing the
        // next tile's keys below
        const uint64_t t3 = t2 + G;
        // the waves that build piece tables reach level 0's barrier last:
        // they issue first until it
        if (wave < 3) __builtin_amdgcn_s_setprio(2);
        if (wave == 0 && has2 && t3 < tiles) {
            const TileGeo g3 = tile_geo(ph, b, t3, ra, lL);
            uint32_t s3, e3;
            split_from_rows(rows, g3, L, K, lane, s3, e3);
            build_pieces(meta(nxt(nxt(nxt(cur)))), s3, e3, g3.Kg, g3.cnt, L, lane);
            if (t3 + G < tiles) fetch_rows_async(table, t3 + G, K, rows, lane);
        }
        // waves 1 and 2: chunk table and wave plan of tile t+2G
        if (has2 && (wave == 1 || wave == 2)) {
            const Meta m2 = meta(nxt(nxt(cur)));
            const uint32_t kg2 = tile_geo(ph, b, t2, ra, lL).Kg;
            if (wave == 1) build_chunks(m2, kg2, lane);
            else build_plan<W>(m2, kg2, lane);
        }
        // the next tile's keys go in flight now and land during the last level
        if (has_next) {
            issue_loads(tile_geo(ph, b, tn, ra, lL), mn);
        } else {
#pragma unroll
            for (int r = 0; r < PC; ++r) pf_dst[r] = 0xFFFFFFFFu;
        }

        uint32_t* X = in;
        uint32_t* Y = other;
        const uint64_t obase = g.gb + g.obeg;
        const int pe = plan_entry<W>(wave);   // balanced over the SIMDs
        uint32_t nlev = 0;
        while ((1u << nlev) < g.Kg) ++nlev;
        // Every tile stores the next tile's keys exactly once, on code every
        // path back to the loop head passes through (no flag or branch decides
        // it), into the buffer this tile's last step does not read: the
        // compiler then knows that the prefetch registers are free at the
        // loop head and issues the next tile's loads without waiting for this
        // tile's stores.  Wave 0 first drains its memory counter: the split-
        // table rows it copied into LDS at the top of this tile are read at
        // the top of the next.
        const bool vec = ((uintptr_t)(dst + obase) & 15u) == 0;
        for (uint32_t lvl = 0; lvl + 1u < nlev; ++lvl) {
            LdsSinkKeys out{Y};
            merge_level_planned<EM>(X, mc.sbeg, mc.plen, mc.plan, g.Kg, lvl, out, wscr, pe, lane);
            lds_barrier();
            if (lvl == 0) __builtin_amdgcn_s_setprio(0);
            uint32_t* tmp = X; X = Y; Y = tmp;
        }
        // the last step reads X (or nothing) and stores to memory; Y is free
        if (wave == 0) vm_drain();
        store_loads(Y);
        if (g.Kg == 1) {   // a lone run: its tile is already in order
            for (uint32_t j = tid; j < g.cnt; j += NT) gptr(dst)[obase + j] = gptr(g.src)[obase + j] ^ flip_out;
        } else {
            GlobalSinkKeys out{dst + obase, flip_out, g.cnt, vec};
            merge_level_planned<EM>(X, mc.sbeg, mc.plen, mc.plan, g.Kg, nlev - 1u, out, wscr, pe, lane);
        }
        lds_barrier();   // publishes the next tile's keys
        __builtin_amdgcn_s_setprio(0);
        if (!has_next) break;
        // the next tile's keys are in Y; X is the buffer this tile read last
        in = Y;
        other = X;
        t = tn;
        cur = nxt(cur);
    }
}

// Largest merge tile for which two 8-wave workgroups of 64x8-key blocks fit
// in one compute unit's 160 KiB of LDS.
constexpr uint32_t kTout2PerCU = 7424;

static hipError_t allow_lds(const void* f, size_t bytes) {
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// TMAX: the largest merge tile the shape accepts (it sizes the prefetch
// registers: chunks of 4 slots per thread for TMAX keys plus up to 3 padding
// slots per piece).
template <int EM, int W, int MINW, uint32_t TMAX>
static hipError_t launch_variant(const Phase& ph, const Bufs& b, const RoundArgs& ra, const uint32_t* table,
                                 uint32_t flip, unsigned grid, hipStream_t s) {
    constexpr int PC = (int)((TMAX + 4u * kMaxFanout + 4u * W * 64u - 1u) / (4u * W * 64u));
    if (ra.Tout > TMAX) return hipErrorInvalidValue;
    const size_t lds =
        (2u * (ra.Tout + 4u * ra.K) + W * Xpose<EM>::WORDS + 4u * kMetaWords + 2u * kMaxFanout) * sizeof(uint32_t);
    hipError_t e = allow_lds((const void*)k_merge_keys<EM, W, PC, MINW>, lds);
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
    hipLaunchKernelGGL((k_merge_keys<EM, W, PC, MINW>), dim3(blocks), dim3(W * 64), lds, s, ph, b, ra, table, flip);
    return hipGetLastError();
}

hipError_t launch_merge_keys(const Phase& ph, const Bufs& b, const RoundArgs& ra, const uint32_t* table,
                             uint32_t flip, unsigned grid, int variant, hipStream_t s) {
    if (ra.Tout > kToutKeys || ra.K > kMaxFanout || ra.Tout % 4 || ra.L % 4) return hipErrorInvalidValue;
    if (ph.tiles == 0) return hipSuccess;
    if (variant == 4) return launch_merge_heap(ph, b, ra, table, flip, s);
    if (variant == 1) return launch_variant<8, 16, 1, kToutKeys>(ph, b, ra, table, flip, grid, s);
    // shape 3 is shape 2 with registers capped for two workgroups per compute
    // unit, which only merge tiles up to kTout2PerCU leave room for in LDS;
    // a larger tile runs as shape 2
    if (variant == 3 && ra.Tout <= kTout2PerCU)
        return launch_variant<8, 8, 4, kTout2PerCU>(ph, b, ra, table, flip, grid, s);
    if (variant == 2 || variant == 3) return launch_variant<8, 8, 1, kToutKeys>(ph, b, ra, table, flip, grid, s);
    return launch_variant<16, 8, 1, kToutKeys>(ph, b, ra, table, flip, grid, s);
}

}  // namespace mms
