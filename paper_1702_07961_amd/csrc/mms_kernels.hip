// gfx950 kernels of the multiway mergesort and their launchers.
//
//   tile_sort   base case (§4.3): sort tiles of T1 elements on chip
//   corank      partition (§4.1): split indices of K sorted runs at a rank
//   copy        streaming copy, the bandwidth probe
//
// The K-way merges of a round (§4.2, §7) are in mms_merge_keys.hip (keys
// only) and mms_merge_pairs.hip (key-value).
//
// Every sorting kernel works on a Phase: a list of tiles, each inside one
// segment (the plain sort is one segment).  Positions are segment-relative;
// a tile's task says whether its pass writes the output or the workspace.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mms_corank.h"
#include "mms_device.h"
#include "mms_device_kt.h"
#include "mms_internal.h"

namespace mms {

// ===========================================================================
// Keys-only base case: the W sorted wave chunks are merged by bitonic merges
// across waves instead of LDS block merges.  At level lvl (runs of 2^lvl
// chunks) the first stage compares every key with its mirror in the paired
// run (wave w ^ (2^(lvl+1) - 1), lane 63 - l, register E - 1 - e), the next
// stages compare at wave distances 2^(lvl-1) .. 1, each through LDS, and the
// remaining stages (lane distances 32 .. 1, then register distances) run in
// the wave as in its own sort.  Exchanges alternate between two LDS buffers,
// so one barrier separates them.  A lane's E keys sit in LDS as E/4 16-byte
// chunks whose order is permuted with the lane so that both 128-bit access
// groupings of gfx950 are conflict-free: reads serve 16 lanes per cycle over
// 64 banks, writes 8 lanes per cycle over 32 banks.  With a lane stride of
// 8 words, lanes 4 apart (writes) and 8 apart (reads) would share banks, and
// chunk c ^ (bit 2 ^ bit 3 of the lane) separates both; with 16 words, lanes
// 2, 4, 6 apart (writes) and 4, 8, 12 apart (reads) would, and the 2-bit
// permutation (bit 1 ^ bit 3, bit 2) separates both.
// ===========================================================================
template <int E>
__device__ __forceinline__ uint32_t chunk_word(uint32_t lane, uint32_t c) {
    constexpr uint32_t Q = E / 4;
    if constexpr (Q == 1) {
        return lane * 4u;
    } else if constexpr (Q == 2) {
        return lane * 8u + 4u * (c ^ (((lane >> 2) ^ (lane >> 3)) & 1u));
    } else {
        const uint32_t f = (((lane >> 1) ^ (lane >> 3)) & 1u) | (((lane >> 2) & 1u) << 1);
        return lane * 16u + 4u * (c ^ f);
    }
}

template <int E, int W>
__global__ __launch_bounds__(W * 64) void k_tile_sort_keys(Phase ph, Bufs b, uint32_t flip) {
    constexpr uint32_t CH = 64u * E;
    constexpr uint32_t T = CH * W;
    constexpr uint32_t Q = E / 4;
    static_assert(E % 4 == 0 && E <= 16, "E/4 chunks of four keys, at most four");
    extern __shared__ __align__(16) uint32_t smem[];   // two exchange buffers of T words

    const int lane = threadIdx.x & 63;
    const uint32_t ul = (uint32_t)lane;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wave-uniform
    const TileRef tr = tile_ref(ph, b, blockIdx.x);
    const uint64_t base = (uint64_t)tr.local * T;
    const uint32_t cnt = (uint32_t)min<uint64_t>(T, tr.n - base);
    const uint32_t* in_k = tr.in_k + base;
    uint32_t* out_k = tr.dst_k + base;
    const uint32_t flip_out = tr.final_pass ? flip : 0u;

    // The wave sorts whatever it holds, so each lane loads four consecutive
    // keys per 16-byte load (chunk c: positions c*256 + 4*lane ..), which
    // covers the wave's CH keys in E/4 loads; the loads need only 4-byte
    // alignment (a batch's segments start anywhere).
    Elem<false> r[E];
#pragma unroll
    for (uint32_t c = 0; c < Q; ++c) {
        const uint32_t j = (uint32_t)wave * CH + c * 256u + 4u * ul;
        if (j + 4u <= cnt) {
            const u32x4a4 v = *reinterpret_cast<cgu32x4a4*>(gptr(in_k) + j);
            r[4 * c] = {v[0] ^ flip};
            r[4 * c + 1] = {v[1] ^ flip};
            r[4 * c + 2] = {v[2] ^ flip};
            r[4 * c + 3] = {v[3] ^ flip};
        } else {
#pragma unroll
            for (uint32_t q = 0; q < 4u; ++q)
                r[4 * c + q] = j + q < cnt ? Elem<false>{gptr(in_k)[j + q] ^ flip} : Elem<false>::sentinel();
        }
    }
    wave_sort_blocked<E>(r, lane);

    uint32_t buf = 0;
    // keep the minimum (keep = 0) or the maximum (~0) of each key and the
    // partner wave's key at the same (mirror: mirrored) position
    auto exchange = [&](int pw, bool mirror, uint32_t keep) {
        uint32_t* X = smem + buf * T;
        buf ^= 1u;
        uint32_t* mine = X + (uint32_t)wave * CH;
#pragma unroll
        for (uint32_t c = 0; c < Q; ++c)
            *reinterpret_cast<uint4*>(mine + chunk_word<E>(ul, c)) =
                make_uint4(r[4 * c].k, r[4 * c + 1].k, r[4 * c + 2].k, r[4 * c + 3].k);
        lds_barrier();
        const uint32_t* theirs = X + (uint32_t)pw * CH;
#pragma unroll
        for (uint32_t c = 0; c < Q; ++c) {
            uint32_t o[4];
            if (mirror) {
                const uint4 v = *reinterpret_cast<const uint4*>(theirs + chunk_word<E>(63u - ul, Q - 1u - c));
                o[0] = v.w; o[1] = v.z; o[2] = v.y; o[3] = v.x;
            } else {
                const uint4 v = *reinterpret_cast<const uint4*>(theirs + chunk_word<E>(ul, c));
                o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) r[4 * c + j].k = med3_u32(r[4 * c + j].k, o[j], keep);
        }
    };
#pragma unroll
    for (int lvl = 0; (1 << lvl) < W; ++lvl) {
        const int gw = 1 << lvl;
        exchange(wave ^ (2 * gw - 1), true, (wave & gw) ? ~0u : 0u);
#pragma unroll
        for (int dw = gw >> 1; dw >= 1; dw >>= 1) exchange(wave ^ dw, false, (wave & dw) ? ~0u : 0u);
        wave_merge_tail<E>(r, lane);
    }

    // wave w, lane l holds tile positions w*CH + l*E .. + E-1
    const bool vec = ((uintptr_t)out_k & 15u) == 0;
    gu32* g = gptr(out_k);
#pragma unroll
    for (uint32_t c = 0; c < Q; ++c) {
        const uint32_t pos = (uint32_t)wave * CH + ul * (uint32_t)E + 4u * c;
        if (vec && pos + 4u <= cnt) {
            *reinterpret_cast<gu32x4*>(g + pos) = u32x4{r[4 * c].k ^ flip_out, r[4 * c + 1].k ^ flip_out,
                                                        r[4 * c + 2].k ^ flip_out, r[4 * c + 3].k ^ flip_out};
        } else {
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j)
                if (pos + j < cnt) g[pos + j] = r[4 * c + j].k ^ flip_out;
        }
    }
}

// ===========================================================================
// Key-value base case, same scheme as the keys-only one.  Elements are
// (key, tag) words (mms_device_kt.h) with tag = tile position, so their order
// is the stable order and is unique; the values are staged in LDS as loaded
// and gathered by tag when the sorted tile is stored.  Exchanges move the
// words' high and low halves as two arrays in the conflict-free chunk layout.
// LDS: values (T words), then two exchange buffers of 2T words.
// ===========================================================================
template <int E, int W>
__global__ __launch_bounds__(W * 64) void k_tile_sort_pairs(Phase ph, Bufs b, uint32_t flip) {
    constexpr uint32_t CH = 64u * E;
    constexpr uint32_t T = CH * W;
    constexpr uint32_t Q = E / 4;
    static_assert(E % 4 == 0 && E <= 16, "E/4 chunks of four elements, at most four");
    extern __shared__ __align__(16) uint32_t smem[];
    uint32_t* V = smem;

    const int lane = threadIdx.x & 63;
    const uint32_t ul = (uint32_t)lane;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wave-uniform
    const TileRef tr = tile_ref(ph, b, blockIdx.x);
    const uint64_t base = (uint64_t)tr.local * T;
    const uint32_t cnt = (uint32_t)min<uint64_t>(T, tr.n - base);
    const uint32_t* in_k = tr.in_k + base;
    const uint32_t* in_v = tr.in_v + base;
    uint32_t* out_k = tr.dst_k + base;
    uint32_t* out_v = tr.dst_v + base;
    const uint32_t flip_out = tr.final_pass ? flip : 0u;

    // as in the keys-only base case, four consecutive pairs per 16-byte load
    // (each tagged with its own tile position); values staged in LDS alike
    ElemKT r[E];
#pragma unroll
    for (uint32_t c = 0; c < Q; ++c) {
        const uint32_t j = (uint32_t)wave * CH + c * 256u + 4u * ul;
        if (j + 4u <= cnt) {
            const u32x4a4 k = *reinterpret_cast<cgu32x4a4*>(gptr(in_k) + j);
            const u32x4a4 v = *reinterpret_cast<cgu32x4a4*>(gptr(in_v) + j);
#pragma unroll
            for (uint32_t q = 0; q < 4u; ++q) r[4 * c + q] = ElemKT{kt_pack(k[q] ^ flip, j + q)};
            *reinterpret_cast<uint4*>(V + j) = make_uint4(v[0], v[1], v[2], v[3]);
        } else {
#pragma unroll
            for (uint32_t q = 0; q < 4u; ++q) {
                if (j + q < cnt) {
                    r[4 * c + q] = ElemKT{kt_pack(gptr(in_k)[j + q] ^ flip, j + q)};
                    V[j + q] = gptr(in_v)[j + q];
                } else {
                    r[4 * c + q] = ElemKT::sentinel();
                }
            }
        }
    }
    wave_sort_blocked<E>(r, lane);

    uint32_t buf = 0;
    auto exchange = [&](int pw, bool mirror, bool want_first) {
        uint32_t* Xh = smem + T + buf * 2u * T;
        uint32_t* Xl = Xh + T;
        buf ^= 1u;
        const uint32_t me = (uint32_t)wave * CH;
#pragma unroll
        for (uint32_t c = 0; c < Q; ++c) {
            const uint32_t w = me + chunk_word<E>(ul, c);
            *reinterpret_cast<uint4*>(Xh + w) = make_uint4(kt_hi(r[4 * c].d), kt_hi(r[4 * c + 1].d),
                                                           kt_hi(r[4 * c + 2].d), kt_hi(r[4 * c + 3].d));
            *reinterpret_cast<uint4*>(Xl + w) = make_uint4(kt_lo(r[4 * c].d), kt_lo(r[4 * c + 1].d),
                                                           kt_lo(r[4 * c + 2].d), kt_lo(r[4 * c + 3].d));
        }
        lds_barrier();
        const uint32_t them = (uint32_t)pw * CH;
#pragma unroll
        for (uint32_t c = 0; c < Q; ++c) {
            uint32_t oh[4], ol[4];
            if (mirror) {
                const uint32_t w = them + chunk_word<E>(63u - ul, Q - 1u - c);
                const uint4 vh = *reinterpret_cast<const uint4*>(Xh + w);
                const uint4 vl = *reinterpret_cast<const uint4*>(Xl + w);
                oh[0] = vh.w; oh[1] = vh.z; oh[2] = vh.y; oh[3] = vh.x;
                ol[0] = vl.w; ol[1] = vl.z; ol[2] = vl.y; ol[3] = vl.x;
            } else {
                const uint32_t w = them + chunk_word<E>(ul, c);
                const uint4 vh = *reinterpret_cast<const uint4*>(Xh + w);
                const uint4 vl = *reinterpret_cast<const uint4*>(Xl + w);
                oh[0] = vh.x; oh[1] = vh.y; oh[2] = vh.z; oh[3] = vh.w;
                ol[0] = vl.x; ol[1] = vl.y; ol[2] = vl.z; ol[3] = vl.w;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) r[4 * c + j] = pick(r[4 * c + j], ElemKT{kt_join(oh[j], ol[j])}, want_first);
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

    // wave w, lane l holds tile positions w*CH + l*E .. + E-1; values by tag
    const bool vec = (((uintptr_t)out_k | (uintptr_t)out_v) & 15u) == 0;
    gu32* gk = gptr(out_k);
    gu32* gv = gptr(out_v);
#pragma unroll
    for (uint32_t c = 0; c < Q; ++c) {
        const uint32_t pos = (uint32_t)wave * CH + ul * (uint32_t)E + 4u * c;
        const ElemKT* q = r + 4 * c;
        if (vec && pos + 4u <= cnt) {
            *reinterpret_cast<gu32x4*>(gk + pos) = u32x4{kt_key(q[0].d) ^ flip_out, kt_key(q[1].d) ^ flip_out,
                                                         kt_key(q[2].d) ^ flip_out, kt_key(q[3].d) ^ flip_out};
            *reinterpret_cast<gu32x4*>(gv + pos) =
                u32x4{V[kt_tag(q[0].d)], V[kt_tag(q[1].d)], V[kt_tag(q[2].d)], V[kt_tag(q[3].d)]};
        } else {
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) {
                if (pos + j < cnt) {
                    gk[pos + j] = kt_key(q[j].d) ^ flip_out;
                    gv[pos + j] = V[kt_tag(q[j].d)];
                }
            }
        }
    }
}

// One wave per tile of a merge round: the split at the tile's first output.
// The round reads the buffer its tasks do not write.
__global__ __launch_bounds__(256) void k_corank_tiles(Phase ph, Bufs b, RoundArgs ra, uint32_t* __restrict__ table) {
    __shared__ CorankLds sh[4];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint64_t t = (uint64_t)blockIdx.x * 4u + (uint64_t)wave;
    if (t >= ph.tiles) return;
    const TileRef tr = tile_ref(ph, b, t);
    const uint32_t grp = tr.local / (uint32_t)ra.tpg;
    const uint64_t i = tr.local - (uint64_t)grp * ra.tpg;
    const uint64_t span = (uint64_t)ra.K * ra.L;
    const uint64_t gb = (uint64_t)grp * span;
    const uint64_t glen = min(span, tr.n - gb);
    const uint32_t Kg = (uint32_t)((glen + ra.L - 1) / ra.L);
    uint32_t c = 0;
    if (i > 0) c = corank_wave(tr.src_k, gb, glen, ra.L, Kg, (uint32_t)(i * ra.Tout), 0u, lane, &sh[wave]);
    if ((uint32_t)lane < ra.K) table[t * ra.K + (uint64_t)lane] = c;
}

__global__ __launch_bounds__(256) void k_corank_queries(const uint32_t* __restrict__ keys, uint64_t n,
                                                        uint64_t L, uint32_t K, const uint64_t* __restrict__ qg,
                                                        const uint64_t* __restrict__ qr, uint64_t nq,
                                                        uint32_t* __restrict__ split, uint32_t flip) {
    __shared__ CorankLds sh[4];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint64_t q = (uint64_t)blockIdx.x * 4u + (uint64_t)wave;
    if (q >= nq) return;
    const uint64_t g = qg[q];
    const uint64_t r = qr[q];
    const uint64_t groups = (n + (uint64_t)K * L - 1) / ((uint64_t)K * L);
    bool ok = g < groups;
    const uint64_t gb = g * (uint64_t)K * L;
    const uint64_t glen = ok ? min((uint64_t)K * L, n - gb) : 0;
    ok = ok && r <= glen;
    if (!ok) {
        if ((uint32_t)lane < K) split[q * K + (uint64_t)lane] = 0xFFFFFFFFu;
        return;
    }
    const uint32_t Kg = (uint32_t)((glen + L - 1) / L);
    const uint32_t c = corank_wave(keys, gb, glen, L, Kg, (uint32_t)r, flip, lane, &sh[wave]);
    if ((uint32_t)lane < K) split[q * K + (uint64_t)lane] = c;
}

// ===========================================================================
// Streaming copy: each lane moves kCopyUnroll 16-byte chunks per trip, all
// loads in flight before the stores, with non-temporal loads and stores (the
// data is touched once).  Chunk u of a trip is 256 chunks after chunk u-1, so
// every load instruction of a workgroup covers 4 KB of consecutive bytes.
// ===========================================================================
constexpr int kCopyUnroll = 8;
__global__ __launch_bounds__(256) void k_copy_vec4(const u32x4* __restrict__ in, u32x4* __restrict__ out,
                                                   uint64_t n4) {
    constexpr uint64_t BD = 256;
    const uint64_t stride = (uint64_t)gridDim.x * BD * kCopyUnroll;
    uint64_t i = (uint64_t)blockIdx.x * BD * kCopyUnroll + threadIdx.x;
    for (; i + (kCopyUnroll - 1) * BD < n4; i += stride) {
        u32x4 v[kCopyUnroll];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) v[u] = __builtin_nontemporal_load(in + i + u * BD);
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) __builtin_nontemporal_store(v[u], out + i + u * BD);
    }
    // the one partial trip of this workgroup (later trips are past the end)
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u)
        if (i + u * BD < n4) out[i + u * BD] = in[i + u * BD];
}
__global__ __launch_bounds__(256) void k_copy_u32(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                  uint64_t beg, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = beg + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = in[i];
}

// ===========================================================================
// Launchers
// ===========================================================================
RoundGeom round_geom(uint64_t n, uint64_t L, uint32_t K, uint32_t Tout) {
    RoundGeom g{};
    g.n = n;
    g.L = L;
    g.K = K;
    g.Tout = Tout;
    const uint64_t span = (uint64_t)K * L;
    g.tiles_per_group = (span + Tout - 1) / Tout;
    if (n == 0) return g;
    g.groups = (n + span - 1) / span;
    const uint64_t last = n - (g.groups - 1) * span;
    g.tiles = (g.groups - 1) * g.tiles_per_group + (last + Tout - 1) / Tout;
    return g;
}

static hipError_t allow_lds(const void* f, size_t bytes) {
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int E, int W>
static hipError_t launch_tile_sort_keys(const Phase& ph, const Bufs& b, uint32_t flip, hipStream_t s) {
    const size_t lds = 2u * 64u * E * W * sizeof(uint32_t);
    hipError_t e = allow_lds((const void*)k_tile_sort_keys<E, W>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_tile_sort_keys<E, W>), dim3((unsigned)ph.tiles), dim3(W * 64), lds, s, ph, b, flip);
    return hipGetLastError();
}

template <int E, int W>
static hipError_t launch_tile_sort_pairs(const Phase& ph, const Bufs& b, uint32_t flip, hipStream_t s) {
    const size_t lds = 5u * 64u * E * W * sizeof(uint32_t);
    hipError_t e = allow_lds((const void*)k_tile_sort_pairs<E, W>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_tile_sort_pairs<E, W>), dim3((unsigned)ph.tiles), dim3(W * 64), lds, s, ph, b, flip);
    return hipGetLastError();
}

hipError_t launch_tile_sort(bool pairs, const Phase& ph, const Bufs& b, uint32_t flip, int base_shape,
                            hipStream_t s) {
    if (ph.tiles == 0) return hipSuccess;
    if (!pairs) {
        if (base_shape == 1) return launch_tile_sort_keys<base_e(1), base_w(1)>(ph, b, flip, s);
        if (base_shape == 2) return launch_tile_sort_keys<base_e(2), base_w(2)>(ph, b, flip, s);
        if (base_shape == 3) return launch_tile_sort_keys<base_e(3), base_w(3)>(ph, b, flip, s);
        if (base_shape == 4) return launch_tile_sort_keys<base_e(4), base_w(4)>(ph, b, flip, s);
        if (base_shape == 5) return launch_tile_sort_keys<base_e(5), base_w(5)>(ph, b, flip, s);
        if (base_shape == 6) return launch_tile_sort_keys<base_e(6), base_w(6)>(ph, b, flip, s);
        return launch_tile_sort_keys<base_e(0), base_w(0)>(ph, b, flip, s);
    }
    if (base_shape == 3) return launch_tile_sort_pairs<base_e(3), base_w(3)>(ph, b, flip, s);
    if (base_shape == 4) return launch_tile_sort_pairs<base_e(4), base_w(4)>(ph, b, flip, s);
    return launch_tile_sort_pairs<base_e(0), base_w(0)>(ph, b, flip, s);
}

hipError_t launch_corank_tiles(const Phase& ph, const Bufs& b, const RoundArgs& ra, uint32_t* table, hipStream_t s) {
    if (ph.tiles == 0) return hipSuccess;
    const uint64_t blocks = (ph.tiles + 3) / 4;
    hipLaunchKernelGGL(k_corank_tiles, dim3((unsigned)blocks), dim3(256), 0, s, ph, b, ra, table);
    return hipGetLastError();
}

hipError_t launch_corank_queries(const uint32_t* keys, uint64_t n, uint64_t L, uint32_t K, const uint64_t* group,
                                 const uint64_t* rank, uint64_t nq, uint32_t* split, uint32_t flip, hipStream_t s) {
    const uint64_t blocks = (nq + 3) / 4;
    hipLaunchKernelGGL(k_corank_queries, dim3((unsigned)blocks), dim3(256), 0, s, keys, n, L, K, group, rank, nq,
                       split, flip);
    return hipGetLastError();
}

hipError_t launch_copy(const uint32_t* in, uint32_t* out, uint64_t n, hipStream_t s) {
    // 16384 workgroups: measured fastest of 1024..32768 on 400 MB (6.3 TB/s)
    const unsigned blocks = 16384u;
    uint64_t done = 0;
    if ((((uintptr_t)in | (uintptr_t)out) & 15u) == 0) {
        const uint64_t n4 = n / 4;
        if (n4) {
            hipLaunchKernelGGL(k_copy_vec4, dim3(blocks), dim3(256), 0, s, (const u32x4*)in, (u32x4*)out, n4);
        }
        done = n4 * 4;
    }
    if (done < n) hipLaunchKernelGGL(k_copy_u32, dim3(done ? 1u : blocks), dim3(256), 0, s, in, out, done, n);
    return hipGetLastError();
}

}  // namespace mms
