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
constexpr int kEM3 = 16;    // merge block of the keys-only merge rounds
constexpr int kW3 = 8;
constexpr uint32_t kToutKeys = 8192;
constexpr uint32_t kToutPairs = 4096;
constexpr uint32_t kMaxFanout = 16;

// Geometry of one merge round: groups of K runs of length L over n elements,
// each group cut into output tiles of Tout.
struct RoundGeom {
    uint64_t n, L;
    uint32_t K, Tout;
    uint64_t groups;           // ceil(n / (K*L))
    uint64_t tiles_per_group;  // ceil(K*L / Tout) for full groups
    uint64_t tiles;            // total tiles of the round
};
RoundGeom round_geom(uint64_t n, uint64_t L, uint32_t K, uint32_t Tout);

hipError_t launch_tile_sort(bool pairs, const uint32_t* in_k, const uint32_t* in_v, uint32_t* out_k,
                            uint32_t* out_v, uint64_t n, uint32_t flip_in, uint32_t flip_out,
                            hipStream_t s);

hipError_t launch_corank_tiles(const uint32_t* src, const RoundGeom& g, uint32_t* table, hipStream_t s);

hipError_t launch_corank_queries(const uint32_t* keys, uint64_t n, uint64_t L, uint32_t K,
                                 const uint64_t* group, const uint64_t* rank, uint64_t nq,
                                 uint32_t* split, uint32_t flip, hipStream_t s);

hipError_t launch_merge(bool pairs, const uint32_t* src_k, const uint32_t* src_v, uint32_t* dst_k,
                        uint32_t* dst_v, const RoundGeom& g, const uint32_t* table, uint32_t flip_out,
                        hipStream_t s);

size_t merge_lds_bytes(bool pairs, uint32_t Tout, uint32_t K);

// Keys-only merge round, persistent: `grid` workgroups walk the round's
// tiles.  variant 0: 64x16-key blocks, 8 waves; variant 1: 64x8-key blocks,
// 16 waves.
hipError_t launch_merge_keys(const uint32_t* src, uint32_t* dst, const RoundGeom& g, const uint32_t* table,
                             uint32_t flip_out, unsigned grid, int variant, hipStream_t s);

hipError_t launch_copy(const uint32_t* in, uint32_t* out, uint64_t n, hipStream_t s);

}  // namespace mms
