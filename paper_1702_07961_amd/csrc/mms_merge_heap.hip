// Keys-only K-way merge with a minBlockHeap per wave (§4.2), the paper's own
// merge structure, with wave64 nodes, offered as merge shape 4 beside the
// LDS merge tree of mms_merge_keys.hip.
//
// Every wave merges one output tile (its partition, §4.1) of its group's K
// runs on its own.  Its heap has K leaves, one per run, and K - 1 internal
// nodes, each a sorted block of B = 64 keys in LDS (one key per lane).  The
// heap property holds between a node and its children (a node's last key is
// at most its children's first keys), so the root holds the 64 smallest keys
// not yet written.  The root is written to memory and refilled by
// fillEmptyNode: the children u and w are merged by a bitonic half-cleaner
// (u ascending against w descending, read from LDS at consecutive reversed
// addresses), the 64 smaller keys fill the empty node, the 64 larger fill
// the child whose last key is the larger (its largest key does not change,
// so the property holds below it), and the other child is now empty: the
// descent continues there down to a leaf, which is refilled from its run.
// Exhausted runs read as the sentinel 0xFFFFFFFF (keys only: a sentinel that
// stands in for an equal real key leaves the written values unchanged).
//
// Pipelining (§7 names it as future work): every leaf keeps a look-ahead
// block in LDS, so a refill is an LDS copy, and the global load of the block
// after it is issued then and lands in the look-ahead slot at the start of
// the next descent, after the root has been written: its latency overlaps
// that write and the descent's merges.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mms_device.h"
#include "mms_internal.h"

namespace mms {

namespace {

constexpr int kHeapWaves = 4;   // waves (independent heaps) per workgroup
// LDS words per wave: 2K-1 nodes and K look-ahead blocks of 64 keys, then the
// next read position and the end of each run's piece
constexpr uint32_t heap_wave_words(uint32_t K) { return (3u * K - 1u) * 64u + 2u * K; }

// sort a bitonic sequence held one key per lane (lane distances 32 .. 1)
__device__ __forceinline__ uint32_t bitonic_lanes(uint32_t x, int lane) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t o = shfl_xor_u32(x, d);
        x = med3_u32(x, o, (lane & d) ? ~0u : 0u);
    }
    return x;
}

}  // namespace

__global__ __launch_bounds__(kHeapWaves * 64) void k_merge_heap(Phase ph, Bufs b, RoundArgs ra,
                                                                const uint32_t* __restrict__ table, uint32_t flip) {
    extern __shared__ __align__(16) uint32_t smem[];
    const uint32_t K = ra.K;
    const uint64_t L = ra.L;
    const int lane = threadIdx.x & 63;
    const uint32_t ul = (uint32_t)lane;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint64_t t = (uint64_t)blockIdx.x * kHeapWaves + (uint64_t)wave;
    if (t >= ph.tiles) return;   // waves are independent: no workgroup barrier below

    const TileRef tr = tile_ref(ph, b, t);
    const uint32_t grp = tr.local / (uint32_t)ra.tpg;
    const uint64_t i = tr.local - (uint64_t)grp * ra.tpg;
    const uint64_t span = (uint64_t)K * L;
    const uint64_t gb = (uint64_t)grp * span;
    const uint64_t glen = min(span, tr.n - gb);
    const uint32_t Kg = (uint32_t)((glen + L - 1) / L);
    const uint64_t obeg = i * (uint64_t)ra.Tout;
    const uint32_t cnt = (uint32_t)min<uint64_t>(ra.Tout, glen - obeg);
    const bool last_tile = obeg + ra.Tout >= glen;
    const uint32_t flip_out = tr.final_pass ? flip : 0u;
    cgu32* src = gptr(tr.src_k) + gb;
    gu32* out = gptr(tr.dst_k) + gb + obeg;

    uint32_t* node = smem + (uint32_t)wave * heap_wave_words(K);   // node v at node + 64 v
    uint32_t* look = node + (2u * K - 1u) * 64u;                    // leaf k's look-ahead
    uint32_t* cur = look + K * 64u;                                 // next position to read, per run
    uint32_t* endp = cur + K;                                       // end of the run's piece

    if (Kg == 1) {   // a lone run: the tile is already in order
        for (uint32_t j = ul; j < cnt; j += 64u) out[j] = src[obeg + j] ^ flip_out;
        return;
    }
    // the piece of run k: [s_k, e_k) from the split indices of the tile's
    // first and last outputs (the clamps only guard memory safety)
    if (ul < K) {
        uint32_t s = 0, e = 0;
        if (ul < Kg) {
            const uint32_t nk = (uint32_t)min<uint64_t>(L, glen - (uint64_t)ul * L);
            s = i == 0 ? 0u : min(table[t * K + ul], nk);
            e = last_tile ? nk : min(max(table[(t + 1) * K + ul], s), nk);
        }
        cur[ul] = s;
        endp[ul] = e;
    }
    lds_wave_sync();
    // lane's key of the block of run k starting at piece position pos
    auto fetch = [&](uint32_t k, uint32_t pos, uint32_t e) -> uint32_t {
        const uint32_t p = pos + ul;
        return p < e ? src[(uint64_t)k * L + p] : kSentKey;
    };
    // leaves and their look-ahead blocks: every load in flight at once
    {
        uint32_t lv[2 * kMaxFanout];
#pragma unroll
        for (uint32_t k = 0; k < kMaxFanout; ++k) {
            if (k < K) {
                const uint32_t s = cur[k], e = endp[k];
                lv[2 * k] = fetch(k, s, e);
                lv[2 * k + 1] = fetch(k, s + 64u, e);
            }
        }
#pragma unroll
        for (uint32_t k = 0; k < kMaxFanout; ++k) {
            if (k < K) {
                node[(K - 1u + k) * 64u + ul] = lv[2 * k];
                look[k * 64u + ul] = lv[2 * k + 1];
                if (lane == 0) cur[k] += 128u;
            }
        }
    }
    lds_wave_sync();

    uint32_t pf = 0;             // the load in flight for look-ahead slot pend
    uint32_t pend = 0xFFFFFFFFu;
    // fill empty node v, descending to a leaf
    auto fill = [&](uint32_t v) {
        if (pend != 0xFFFFFFFFu) {   // park the last load (it has had a root write and a descent)
            look[pend * 64u + ul] = pf;
            pend = 0xFFFFFFFFu;
        }
        while (v < K - 1u) {
            const uint32_t c1 = 2u * v + 1u, c2 = c1 + 1u;
            const uint32_t a = node[c1 * 64u + ul];
            const uint32_t bw = node[c2 * 64u + 63u - ul];    // w reversed
            const uint32_t ua = (uint32_t)__builtin_amdgcn_readlane((int)a, 63);   // u's last key
            const uint32_t wb = (uint32_t)__builtin_amdgcn_readlane((int)bw, 0);   // w's last key
            const uint32_t lo = bitonic_lanes(min(a, bw), lane);
            const uint32_t hi = bitonic_lanes(max(a, bw), lane);
            node[v * 64u + ul] = lo;
            // the child with the larger last key keeps the larger half; the
            // other one is now empty
            const uint32_t keep = ua > wb ? c1 : c2;
            node[keep * 64u + ul] = hi;
            v = ua > wb ? c2 : c1;
        }
        // v is a leaf: take its look-ahead block, start loading the next one
        const uint32_t k = v - (K - 1u);
        node[v * 64u + ul] = look[k * 64u + ul];
        const uint32_t pos = cur[k];
        pf = fetch(k, pos, endp[k]);
        pend = k;
        if (lane == 0) cur[k] = pos + 64u;
        lds_wave_sync();
    };
    // build bottom-up
    for (uint32_t v = K - 1u; v-- > 0;) fill(v);
    // write the root, refill it
    const uint32_t blocks = (cnt + 63u) / 64u;
    for (uint32_t r = 0; r < blocks; ++r) {
        const uint32_t o = r * 64u + ul;
        const uint32_t key = node[ul];
        if (o < cnt) out[o] = key ^ flip_out;
        if (r + 1u < blocks) fill(0u);
    }
}

hipError_t launch_merge_heap(const Phase& ph, const Bufs& b, const RoundArgs& ra, const uint32_t* table,
                             uint32_t flip, hipStream_t s) {
    if (ph.tiles == 0) return hipSuccess;
    if (ra.K < 2 || ra.K > kMaxFanout || (ra.K & (ra.K - 1))) return hipErrorInvalidValue;
    const size_t lds = (size_t)kHeapWaves * heap_wave_words(ra.K) * sizeof(uint32_t);
    hipError_t e = hipFuncSetAttribute((const void*)k_merge_heap, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const uint64_t blocks = (ph.tiles + kHeapWaves - 1) / kHeapWaves;
    hipLaunchKernelGGL(k_merge_heap, dim3((unsigned)blocks), dim3(kHeapWaves * 64), lds, s, ph, b, ra, table, flip);
    return hipGetLastError();
}

}  // namespace mms
