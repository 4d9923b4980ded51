// Internal interface between the host runtime (plan, C ABI) and the kernel
// launchers.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mms {

// Compile-time kernel shapes.  The base case sorts T1 = 64*E1*W1 elements
// per workgroup; a merge workgroup produces an output tile of Tout elements
// with W3 waves, 64*EM elements per merge block.
constexpr int kE1 = 8;
constexpr int kW1 = 4;
constexpr uint32_t kT1 = 64u * kE1 * kW1;
constexpr int kEM = 8;      // merge block of the key-value path
constexpr int kEM1 = 8;     // merge block of the keys-only base case
constexpr int kW3 = 8;      // waves of the key-value merge
constexpr uint32_t kToutKeys = 8192;   // largest keys-only merge tile
constexpr uint32_t kToutPairs = 4096;
constexpr uint32_t kMaxFanout = 16;

// One tile of a phase (base case or merge round).  A batch of segments is a
// list of such tiles; the plain sort is the one-segment case and needs no
// list.  Within a segment every position is relative to `base`.
struct TileTask {
    uint64_t base;    // first element of the segment in the arrays
    uint32_t n;       // segment length
    uint32_t info;    // bits 0..27 tile index inside the segment's phase,
                      // bit 30: the pass writes the output (else the workspace),
                      // bit 31: last pass of the segment (undo the int32 flip)
};
constexpr uint32_t kTaskTileMask = 0x0FFFFFFFu;
constexpr uint32_t kTaskDstOut = 1u << 30;
constexpr uint32_t kTaskFinal = 1u << 31;

// A phase: either an explicit task list, or one segment [0, n) whose tiles
// all share dst_out / final.
struct Phase {
    const TileTask* tasks;
    uint64_t n;
    uint32_t dst_out;
    uint32_t final_pass;
    uint64_t tiles;
};

// Device view of tile t of a phase.
struct TileRef {
    uint64_t base;     // segment start
    uint64_t n;        // segment length
    uint32_t local;    // tile index inside the segment's phase
    bool dst_out;
    bool final_pass;
};
__device__ __forceinline__ TileRef tile_ref(const Phase& ph, uint64_t t) {
    if (!ph.tasks) return {0, ph.n, (uint32_t)t, ph.dst_out != 0, ph.final_pass != 0};
    const TileTask tk = ph.tasks[t];
    return {tk.base, tk.n, tk.info & kTaskTileMask, (tk.info & kTaskDstOut) != 0, (tk.info & kTaskFinal) != 0};
}

// The two ping-pong buffers of a sort (output and workspace) plus its input.
struct Bufs {
    const uint32_t* in_k;
    const uint32_t* in_v;
    uint32_t* out_k;
    uint32_t* out_v;
    uint32_t* ws_k;
    uint32_t* ws_v;
};

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

hipError_t launch_tile_sort(bool pairs, const Phase& ph, const Bufs& b, uint32_t flip, hipStream_t s);

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
// 1: 64x8-key blocks, 16 waves; 2: 64x8, 8 waves.
hipError_t launch_merge_keys(const Phase& ph, const Bufs& b, const RoundArgs& ra, const uint32_t* table,
                             uint32_t flip, unsigned grid, int variant, hipStream_t s);

hipError_t launch_copy(const uint32_t* in, uint32_t* out, uint64_t n, hipStream_t s);

}  // namespace mms
