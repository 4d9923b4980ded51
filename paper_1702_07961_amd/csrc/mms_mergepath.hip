// A pairwise merge-path mergesort with per-thread serial merges in LDS: the
// kind of GPU mergesort the paper measures its method against (§1, §3, §6.4:
// a two-way merge where every thread finds its starting point on the merge
// path by binary search and then merges its share of outputs one element at
// a time).  It is built here as a baseline, to show on gfx950 what the paper
// shows on its GPUs: the LDS addresses of a serial merge depend on the data,
// so the input decides how many bank conflicts it takes, while the multiway
// merge's block steps (mms_device.h) touch addresses that do not.
//
//   block sort  each workgroup sorts a tile of NT*VT keys: every thread sorts
//               its VT keys in registers, then log2(NT) levels of pairwise
//               merges through LDS, each thread merging VT outputs serially
//   partition   the merge-path split of every output tile of a pass, by
//               binary search in global memory
//   merge pass  each workgroup merges one output tile of two runs: the
//               pieces are loaded into LDS and each thread merges VT outputs
//               serially from its own merge-path split
//
// Keys are 32-bit (uint32, or int32 with the sign bit flipped on the way in
// and out); the sort is keys-only, so ties need no order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mms_device.h"
#include "mms_internal.h"

namespace mms {

namespace {

constexpr int kMpNT = kMergePathThreads;
constexpr int kMpVT = kMergePathItems;
constexpr uint32_t kMpTile = kMergePathTile;

// Number of A elements among the first `diag` outputs of merge(A, B), A
// first on ties: the smallest p with A[p] > B[diag - 1 - p].
__device__ __forceinline__ uint32_t lds_merge_path(const uint32_t* A, uint32_t la, const uint32_t* B, uint32_t lb,
                                                   uint32_t diag) {
    uint32_t lo = diag > lb ? diag - lb : 0u;
    uint32_t hi = min(diag, la);
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (A[mid] <= B[diag - 1u - mid]) lo = mid + 1u;
        else hi = mid;
    }
    return lo;
}

// Serial merge of VT outputs starting at (a, b): one LDS read per output, at
// the position of whichever run the output came from.  Positions past a run
// read as exhausted (B past its end is never taken; A past its end neither).
template <int VT>
__device__ __forceinline__ void serial_merge(const uint32_t* X, uint32_t aBase, uint32_t la, uint32_t bBase,
                                             uint32_t lb, uint32_t a, uint32_t b, uint32_t (&r)[VT]) {
    uint32_t ka = X[a < la ? aBase + a : 0u];
    uint32_t kb = X[b < lb ? bBase + b : 0u];
#pragma unroll
    for (int i = 0; i < VT; ++i) {
        const bool take_a = b >= lb || (a < la && ka <= kb);
        r[i] = take_a ? ka : kb;
        a += take_a ? 1u : 0u;
        b += take_a ? 0u : 1u;
        const bool ok = take_a ? a < la : b < lb;
        const uint32_t nk = X[ok ? (take_a ? aBase + a : bBase + b) : 0u];
        ka = take_a ? nk : ka;
        kb = take_a ? kb : nk;
    }
}

// odd-even transposition sort of VT registers
template <int VT>
__device__ __forceinline__ void thread_sort(uint32_t (&r)[VT]) {
#pragma unroll
    for (int pass = 0; pass < VT; ++pass) {
#pragma unroll
        for (int i = pass & 1; i + 1 < VT; i += 2) {
            const uint32_t x = r[i], y = r[i + 1];
            r[i] = min(x, y);
            r[i + 1] = max(x, y);
        }
    }
}

}  // namespace

// ===========================================================================
// Block sort
// ===========================================================================
__global__ __launch_bounds__(kMpNT) void k_mp_blocksort(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                        uint64_t n, uint32_t flip_in, uint32_t flip_out) {
    __shared__ uint32_t X[kMpTile];
    const uint32_t tid = threadIdx.x;
    const uint64_t base = (uint64_t)blockIdx.x * kMpTile;
    const uint32_t cnt = (uint32_t)min<uint64_t>(kMpTile, n - base);
#pragma unroll
    for (int j = 0; j < kMpVT; ++j) {
        const uint32_t p = (uint32_t)j * kMpNT + tid;
        X[p] = p < cnt ? gptr(in)[base + p] ^ flip_in : 0xFFFFFFFFu;
    }
    __syncthreads();
    uint32_t r[kMpVT];
#pragma unroll
    for (int j = 0; j < kMpVT; ++j) r[j] = X[tid * kMpVT + j];
    thread_sort<kMpVT>(r);
    for (uint32_t w = 1; w < (uint32_t)kMpNT; w <<= 1) {   // runs of w threads' outputs
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kMpVT; ++j) X[tid * kMpVT + j] = r[j];
        __syncthreads();
        const uint32_t R = w * kMpVT;
        const uint32_t first = tid & ~(2u * w - 1u);          // first thread of the pair
        const uint32_t aBase = first * kMpVT, bBase = aBase + R;
        const uint32_t diag = (tid - first) * kMpVT;
        const uint32_t p = lds_merge_path(X + aBase, R, X + bBase, R, diag);
        serial_merge<kMpVT>(X, aBase, R, bBase, R, p, diag - p, r);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kMpVT; ++j) X[tid * kMpVT + j] = r[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kMpVT; ++j) {
        const uint32_t p = (uint32_t)j * kMpNT + tid;
        if (p < cnt) gptr(out)[base + p] = X[p] ^ flip_out;
    }
}

// ===========================================================================
// Partition of a merge pass: runs of length L merged in pairs, output tiles
// of kMpTile; split[t] = A elements before tile t's first output.
// ===========================================================================
__global__ __launch_bounds__(256) void k_mp_partition(const uint32_t* __restrict__ src, uint64_t n, uint64_t L,
                                                      uint64_t tpg, uint64_t tiles, uint32_t* __restrict__ split) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= tiles) return;
    const uint64_t g = t / tpg, i = t - g * tpg;
    const uint64_t gb = g * 2 * L;
    const uint64_t glen = min(2 * L, n - gb);
    const uint64_t la = min(L, glen), lb = glen - la;
    const uint64_t diag = i * kMpTile;
    cgu32* A = gptr(src) + gb;
    cgu32* B = A + la;
    uint64_t lo = diag > lb ? diag - lb : 0, hi = min(diag, la);
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (A[mid] <= B[diag - 1 - mid]) lo = mid + 1;
        else hi = mid;
    }
    split[t] = (uint32_t)lo;
}

// ===========================================================================
// Merge pass: one workgroup per output tile
// ===========================================================================
__global__ __launch_bounds__(kMpNT) void k_mp_merge(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                                                    uint64_t n, uint64_t L, uint64_t tpg,
                                                    const uint32_t* __restrict__ split, uint32_t flip_out) {
    __shared__ uint32_t X[kMpTile];
    const uint32_t tid = threadIdx.x;
    const uint64_t t = blockIdx.x;
    const uint64_t g = t / tpg, i = t - g * tpg;
    const uint64_t gb = g * 2 * L;
    const uint64_t glen = min(2 * L, n - gb);
    const uint32_t la_all = (uint32_t)min(L, glen);
    const uint64_t d0 = i * kMpTile;
    const uint32_t cnt = (uint32_t)min<uint64_t>(kMpTile, glen - d0);
    const bool last = d0 + kMpTile >= glen;
    // the clamps only guard memory safety (exact splits satisfy them): A
    // pieces stay inside A, and B pieces inside B, b0 + nb = d1 - a1 <= lb
    const uint64_t lb_all = glen - la_all, d1 = d0 + cnt;
    const uint32_t a0 = i == 0 ? 0u
                               : (uint32_t)min<uint64_t>(max<uint64_t>(split[t], d0 > lb_all ? d0 - lb_all : 0),
                                                         min<uint64_t>(d0, la_all));
    const uint32_t a1 = last ? la_all
                             : (uint32_t)min<uint64_t>(max<uint64_t>(max<uint64_t>(split[t + 1], a0),
                                                                     d1 > lb_all ? d1 - lb_all : 0),
                                                       min<uint64_t>(d1, la_all));
    const uint32_t na = min(a1 - a0, cnt);
    const uint32_t nb = cnt - na;
    const uint64_t b0 = d0 - a0;
    cgu32* A = gptr(src) + gb;
    cgu32* B = A + la_all;
#pragma unroll
    for (int j = 0; j < kMpVT; ++j) {
        const uint32_t p = (uint32_t)j * kMpNT + tid;
        if (p < na) X[p] = A[a0 + p];
        else if (p < cnt) X[p] = B[b0 + (p - na)];
    }
    __syncthreads();
    const uint32_t diag = min(tid * (uint32_t)kMpVT, cnt);
    const uint32_t p = lds_merge_path(X, na, X + na, nb, diag);
    uint32_t r[kMpVT];
    serial_merge<kMpVT>(X, 0u, na, na, nb, p, diag - p, r);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kMpVT; ++j)
        if (tid * kMpVT + j < cnt) X[tid * kMpVT + j] = r[j];
    __syncthreads();
    gu32* O = gptr(dst) + gb + d0;
#pragma unroll
    for (int j = 0; j < kMpVT; ++j) {
        const uint32_t q = (uint32_t)j * kMpNT + tid;
        if (q < cnt) O[q] = X[q] ^ flip_out;
    }
}

// ===========================================================================
// Launchers
// ===========================================================================
hipError_t launch_mp_blocksort(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t flip_in, uint32_t flip_out,
                               hipStream_t s) {
    const uint64_t tiles = (n + kMpTile - 1) / kMpTile;
    if (tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mp_blocksort, dim3((unsigned)tiles), dim3(kMpNT), 0, s, in, out, n, flip_in, flip_out);
    return hipGetLastError();
}

hipError_t launch_mp_partition(const uint32_t* src, uint64_t n, uint64_t L, uint32_t* split, hipStream_t s) {
    const RoundGeom g = round_geom(n, L, 2, kMpTile);
    if (g.tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mp_partition, dim3((unsigned)((g.tiles + 255) / 256)), dim3(256), 0, s, src, n, L,
                       g.tiles_per_group, g.tiles, split);
    return hipGetLastError();
}

hipError_t launch_mp_merge(const uint32_t* src, uint32_t* dst, uint64_t n, uint64_t L, const uint32_t* split,
                           uint32_t flip_out, hipStream_t s) {
    const RoundGeom g = round_geom(n, L, 2, kMpTile);
    if (g.tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mp_merge, dim3((unsigned)g.tiles), dim3(kMpNT), 0, s, src, dst, n, L, g.tiles_per_group,
                       split, flip_out);
    return hipGetLastError();
}

}  // namespace mms
