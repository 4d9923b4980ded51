// Internal interface between the host runtime (plan, C ABI) and the kernel
// launchers.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mms {

// Compile-time kernel shapes.  The base case sorts a tile of 64*E*W elements
// per workgroup (E per lane, W waves); a merge workgroup produces an output
// tile of Tout elements with W3 waves, 64*EM elements per merge block.
// Base-case shapes, E x W (tile): 0: 8 x 4, 1: 4 x 8, 2: 16 x 2 (2048),
// 3: 8 x 8, 5: 16 x 4 (4096), 4: 8 x 16, 6: 16 x 8 (8192).  Key-value sorts
// use shapes 0 and 3.  kT1 is the smallest tile.
constexpr int kBaseShapes = 7;
constexpr int kShapeE[kBaseShapes] = {8, 4, 16, 8, 8, 16, 16};
constexpr int kShapeW[kBaseShapes] = {4, 8, 2, 8, 16, 4, 8};
constexpr int base_e(int shape) { return kShapeE[shape]; }
constexpr int base_w(int shape) { return kShapeW[shape]; }
constexpr uint32_t base_tile(int shape) { return 64u * (uint32_t)base_e(shape) * (uint32_t)base_w(shape); }
constexpr uint32_t kT1 = 2048;
static_assert(base_tile(0) == kT1 && base_tile(1) == kT1 && base_tile(2) == kT1, "the smallest tile");
constexpr int kW3 = 8;      // waves of the key-value merge
constexpr uint32_t kToutKeys = 8192;   // largest keys-only merge tile
constexpr uint32_t kToutPairs = 3840;   // two key-value merge workgroups per compute unit
constexpr uint32_t kMaxFanout = 16;

// The buffers of one segment: its input, its output and its ping-pong
// workspace (values null for keys-only sorts).  The plain sort is a single
// segment described by the kernel's Bufs argument; a batch gives every
// segment its own pointers, so segments need not share arrays.
struct SegDesc {
    const uint32_t* in_k;
    const uint32_t* in_v;
    uint32_t* out_k;
    uint32_t* out_v;
    uint32_t* ws_k;
    uint32_t* ws_v;
    uint64_t n;        // segment length (< 2^32)
    uint64_t pad;
};
static_assert(sizeof(SegDesc) == 64, "SegDesc is one 64-byte record");

// One tile of a phase (base case or merge round) of a batch.
struct TileTask {
    uint32_t seg;     // index into the batch's SegDesc table
    uint32_t info;    // bits 0..27 tile index inside the segment's phase,
                      // bit 30: the pass writes the output (else the workspace),
                      // bit 31: last pass of the segment (undo the int32 flip)
};
constexpr uint32_t kTaskTileMask = 0x0FFFFFFFu;
constexpr uint32_t kTaskDstOut = 1u << 30;
constexpr uint32_t kTaskFinal = 1u << 31;

// The buffers of a plain (single-segment) sort.
struct Bufs {
    const uint32_t* in_k;
    const uint32_t* in_v;
    uint32_t* out_k;
    uint32_t* out_v;
    uint32_t* ws_k;
    uint32_t* ws_v;
};

// A phase: either an explicit task list over a SegDesc table, or one segment
// [0, n) in Bufs whose tiles all share dst_out / final.
struct Phase {
    const TileTask* tasks;
    const SegDesc* segs;
    uint64_t n;
    uint32_t dst_out;
    uint32_t final_pass;
    uint64_t tiles;
};

// Device view of tile t of a phase: its segment's buffers already resolved
// to the one this pass reads (src) and the one it writes (dst).
struct TileRef {
    const uint32_t* in_k;   // segment input (base case)
    const uint32_t* in_v;
    const uint32_t* src_k;  // buffer a merge round reads
    const uint32_t* src_v;
    uint32_t* dst_k;        // buffer the pass writes
    uint32_t* dst_v;
    uint64_t n;             // segment length
    uint32_t local;         // tile index inside the segment's phase
    bool final_pass;
};
__device__ __forceinline__ TileRef tile_ref(const Phase& ph, const Bufs& b, uint64_t t) {
    TileRef r;
    bool dst_out;
    if (!ph.tasks) {
        r.in_k = b.in_k;
        r.in_v = b.in_v;
        dst_out = ph.dst_out != 0;
        r.src_k = dst_out ? b.ws_k : b.out_k;
        r.src_v = dst_out ? b.ws_v : b.out_v;
        r.dst_k = dst_out ? b.out_k : b.ws_k;
        r.dst_v = dst_out ? b.out_v : b.ws_v;
        r.n = ph.n;
        r.local = (uint32_t)t;
        r.final_pass = ph.final_pass != 0;
        return r;
    }
    // the task list and the descriptors are uniform and read-only during a
    // launch: scalar loads, which a wave's waits for its vector loads do not
    // hold up
    typedef const __attribute__((address_space(4))) TileTask ScalarTask;
    typedef const __attribute__((address_space(4))) SegDesc ScalarSeg;
    ScalarTask* tk = (ScalarTask*)ph.tasks + t;
    const uint32_t info = tk->info;
    ScalarSeg* sd = (ScalarSeg*)ph.segs + tk->seg;
    dst_out = (info & kTaskDstOut) != 0;
    r.in_k = sd->in_k;
    r.in_v = sd->in_v;
    r.src_k = dst_out ? sd->ws_k : sd->out_k;
    r.src_v = dst_out ? sd->ws_v : sd->out_v;
    r.dst_k = dst_out ? sd->out_k : sd->ws_k;
    r.dst_v = dst_out ? sd->out_v : sd->ws_v;
    r.n = sd->n;
    r.local = info & kTaskTileMask;
    r.final_pass = (info & kTaskFinal) != 0;
    return r;
}

// Geometry of one merge round inside one segment: groups of K runs of length
// L over n elements, each group cut into output tiles of Tout.
struct RoundGeom {
    uint64_t n, L;
    uint32_t K, Tout;
    uint64_t groups;           // ceil(n / (K*L))
    uint64_t tiles_per_group;  // ceil(K*L / Tout) for full groups
    uint64_t tiles;            // total tiles of the round
};
RoundGeom round_geom(uint64_t n, uint64_t L, uint32_t K, uint32_t Tout);

// Merge-round parameters shared by every segment of a batch.
struct RoundArgs {
    uint64_t L;
    uint32_t K;
    uint32_t Tout;
    uint64_t tpg;          // tiles per full group
};

hipError_t launch_tile_sort(bool pairs, const Phase& ph, const Bufs& b, uint32_t flip, int base_shape, hipStream_t s);

hipError_t launch_corank_tiles(const Phase& ph, const Bufs& b, const RoundArgs& ra, uint32_t* table,
                               hipStream_t s);

hipError_t launch_corank_queries(const uint32_t* keys, uint64_t n, uint64_t L, uint32_t K,
                                 const uint64_t* group, const uint64_t* rank, uint64_t nq,
                                 uint32_t* split, uint32_t flip, hipStream_t s);

// Key-value merge round (one workgroup per tile).
hipError_t launch_merge_pairs(const Phase& ph, const Bufs& b, const RoundArgs& ra, const uint32_t* table,
                              uint32_t flip, hipStream_t s);

// Keys-only merge round, persistent: `grid` compute units' worth of
// workgroups walk the phase's tiles.  variant 0: 64x16-key blocks, 8 waves;
// 1: 64x8-key blocks, 16 waves; 2: 64x8, 8 waves; 3: 64x8, 8 waves, two
// workgroups per compute unit (registers capped for it; the merge tile must
// be small enough for two workgroups' LDS); 4: the minBlockHeap merge.
hipError_t launch_merge_keys(const Phase& ph, const Bufs& b, const RoundArgs& ra, const uint32_t* table,
                             uint32_t flip, unsigned grid, int variant, hipStream_t s);

// Keys-only merge round with a minBlockHeap of 64-key nodes per wave (merge
// shape 4): one wave per output tile.
hipError_t launch_merge_heap(const Phase& ph, const Bufs& b, const RoundArgs& ra, const uint32_t* table,
                             uint32_t flip, hipStream_t s);

hipError_t launch_copy(const uint32_t* in, uint32_t* out, uint64_t n, hipStream_t s);

// ---- 64-bit keys (and 64-bit values): plain sorts only ----------------------
// Base tiles: kT64Keys keys (8 per lane x 8 waves) or kT64Pairs pairs (8 x
// 4); merge output tiles kTout64Keys / kTout64Pairs (two workgroups' LDS per
// compute unit).
constexpr uint32_t kT64Keys = 4096;
constexpr uint32_t kT64Pairs = 2048;
constexpr uint32_t kTout64Keys = 3840;
constexpr uint32_t kTout64Pairs = 2048;

struct Bufs64 {
    const uint64_t* in_k;
    const uint64_t* in_v;
    uint64_t* out_k;
    uint64_t* out_v;
    uint64_t* ws_k;
    uint64_t* ws_v;
};
// one pass of a plain 64-bit sort over [0, n)
struct Phase64 {
    uint64_t n;
    uint32_t dst_out;     // this pass writes the output (else the workspace)
    uint32_t final_pass;  // last pass: undo the signed-key mapping
    uint64_t tiles;
};

// ---- the merge-path baseline (pairwise, per-thread serial merges) ----------
constexpr int kMergePathThreads = 256;
constexpr int kMergePathItems = 15;     // outputs per thread (odd: strided LDS reads spread over banks)
constexpr uint32_t kMergePathTile = (uint32_t)kMergePathThreads * kMergePathItems;

hipError_t launch_mp_blocksort(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t flip_in, uint32_t flip_out,
                               hipStream_t s);
hipError_t launch_mp_partition(const uint32_t* src, uint64_t n, uint64_t L, uint32_t* split, hipStream_t s);
hipError_t launch_mp_merge(const uint32_t* src, uint32_t* dst, uint64_t n, uint64_t L, const uint32_t* split,
                           uint32_t flip_out, hipStream_t s);

hipError_t launch_tile_sort64(bool pairs, const Phase64& ph, const Bufs64& b, uint64_t flip, hipStream_t s);
hipError_t launch_corank_tiles64(const Phase64& ph, const Bufs64& b, const RoundArgs& ra, uint32_t* table,
                                 hipStream_t s);
hipError_t launch_merge64(bool pairs, const Phase64& ph, const Bufs64& b, const RoundArgs& ra, const uint32_t* table,
                          uint64_t flip, hipStream_t s);

}  // namespace mms
