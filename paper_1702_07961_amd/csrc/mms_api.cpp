// Host runtime of libmms: plan, workspace layout, argument checks, the round
// loop, and the C ABI declared in include/mms.h.  Kernels are launched only
// through the launchers of mms_kernels.hip.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "mms.h"
#include "mms_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(MMS_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// ---- per-kernel timing (mms_timing_*) --------------------------------------
struct TimingRec {
    int kind;
    hipEvent_t a, b;
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<TimingRec> g_recs;
std::vector<hipEvent_t> g_pool;
uint64_t g_launch[MMS_KERNEL_KINDS];
double g_ms[MMS_KERNEL_KINDS];

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets one kernel launch with events on its stream when timing is on.
class Timed {
  public:
    Timed(int kind, hipStream_t s) : kind_(kind), s_(s) {
        std::lock_guard<std::mutex> g(g_tmu);
        if (!g_timing) return;
        a_ = take_event();
        b_ = take_event();
        if (a_ && b_) hipEventRecord(a_, s_);
    }
    ~Timed() {
        if (!a_ || !b_) return;
        hipEventRecord(b_, s_);
        std::lock_guard<std::mutex> g(g_tmu);
        g_recs.push_back({kind_, a_, b_});
    }

  private:
    int kind_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

// One resident workgroup per compute unit for the persistent merge kernel.
unsigned persistent_grid() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
    return (unsigned)cus;
}

// Merge kernel shape; MMS_MERGE_VARIANT=1 selects 16 waves with 512-key blocks.
int merge_variant() {
    static const int v = [] {
        const char* s = getenv("MMS_MERGE_VARIANT");
        return s ? atoi(s) : 0;
    }();
    return v;
}

// Output tile of the keys-only merge; MMS_TOUT overrides (multiple of 256,
// at most the compiled maximum).
uint32_t keys_merge_tile() {
    static const uint32_t v = [] {
        const char* s = getenv("MMS_TOUT");
        uint32_t t = s ? (uint32_t)atoi(s) : mms::kToutKeys;
        if (t < 1024 || t > mms::kToutKeys || t % 256) t = mms::kToutKeys;
        return t;
    }();
    return v;
}

constexpr uint64_t kAlign = 256;
uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Plan {
    uint64_t n;
    bool pairs;
    uint32_t T;
    uint32_t K;
    uint32_t Tout;
    uint32_t rounds;
    uint64_t max_tiles;      // largest tile count over the merge rounds
    uint64_t off_vals;       // workspace offsets (bytes)
    uint64_t off_table;
    uint64_t ws_bytes;
};

// §6.2: ceil(log_K(ceil(n / T))) merge rounds after the base case.
Plan make_plan(uint64_t n, uint32_t flags) {
    Plan p{};
    p.n = n;
    p.pairs = (flags & MMS_PAIRS) != 0;
    p.T = mms::kT1;
    p.K = mms::kMaxFanout;
    p.Tout = p.pairs ? mms::kToutPairs : keys_merge_tile();
    p.rounds = 0;
    p.max_tiles = 0;
    for (uint64_t L = p.T; L < n; L *= p.K) {
        mms::RoundGeom g = mms::round_geom(n, L, p.K, p.Tout);
        if (g.tiles > p.max_tiles) p.max_tiles = g.tiles;
        ++p.rounds;
    }
    const uint64_t kbytes = align_up(n * 4);
    p.off_vals = kbytes;
    p.off_table = p.off_vals + (p.pairs ? align_up(n * 4) : 0);
    p.ws_bytes = p.rounds ? p.off_table + align_up((p.max_tiles + 1) * p.K * 4) : 0;
    return p;
}

bool overlaps(const void* a, uint64_t abytes, const void* b, uint64_t bbytes) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bbytes && y < x + abytes;
}

// a and b either coincide exactly or are disjoint
bool same_or_disjoint(const void* a, const void* b, uint64_t bytes) {
    return a == b || !overlaps(a, bytes, b, bytes);
}

int sort_impl(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, uint64_t n, void* ws,
              size_t ws_bytes, uint32_t flags, void* stream) {
    const bool pairs = vin != nullptr;
    if (flags & ~(MMS_KEY_I32 | MMS_PAIRS)) return fail(MMS_EINVAL, "unknown flags 0x%x", flags);
    if (n == 0) return MMS_OK;
    if (n >= (1ull << 32)) return fail(MMS_EINVAL, "n = %llu exceeds 2^32-1", (unsigned long long)n);
    if (!kin || !kout || (pairs && !vout)) return fail(MMS_EINVAL, "null data pointer");
    const uint64_t bytes = n * 4;
    if (!same_or_disjoint(kin, kout, bytes)) return fail(MMS_EINVAL, "keys in/out partially overlap");
    if (pairs) {
        if (!same_or_disjoint(vin, vout, bytes)) return fail(MMS_EINVAL, "values in/out partially overlap");
        if (overlaps(kout, bytes, vout, bytes) || overlaps(kin, bytes, vin, bytes) ||
            overlaps(kout, bytes, vin, bytes) || overlaps(kin, bytes, vout, bytes))
            return fail(MMS_EINVAL, "key and value buffers overlap");
    }
    const Plan p = make_plan(n, flags | (pairs ? MMS_PAIRS : 0u));
    if (p.rounds) {
        if (!ws) return fail(MMS_EINVAL, "workspace required (%llu bytes)", (unsigned long long)p.ws_bytes);
        if (ws_bytes < p.ws_bytes)
            return fail(MMS_EINVAL, "workspace too small: %zu < %llu", ws_bytes, (unsigned long long)p.ws_bytes);
        if ((uintptr_t)ws % kAlign) return fail(MMS_EINVAL, "workspace not 256-byte aligned");
        if (overlaps(ws, p.ws_bytes, kin, bytes) || overlaps(ws, p.ws_bytes, kout, bytes) ||
            (pairs && (overlaps(ws, p.ws_bytes, vin, bytes) || overlaps(ws, p.ws_bytes, vout, bytes))))
            return fail(MMS_EINVAL, "workspace overlaps data");
    }
    hipStream_t s = (hipStream_t)stream;
    const uint32_t flip = (flags & MMS_KEY_I32) ? 0x80000000u : 0u;
    uint8_t* wsb = (uint8_t*)ws;
    uint32_t* ws_k = (uint32_t*)wsb;
    uint32_t* ws_v = pairs ? (uint32_t*)(wsb + p.off_vals) : nullptr;
    uint32_t* table = p.rounds ? (uint32_t*)(wsb + p.off_table) : nullptr;

    // pass i writes buffer B_i; B_R must be the output, so B_i is the output
    // when R - i is even and the workspace otherwise
    auto buf_k = [&](uint32_t i) { return ((p.rounds - i) % 2 == 0) ? kout : ws_k; };
    auto buf_v = [&](uint32_t i) { return ((p.rounds - i) % 2 == 0) ? vout : ws_v; };

    hipError_t e;
    {
        Timed tm(MMS_KERNEL_TILE_SORT, s);
        e = mms::launch_tile_sort(pairs, kin, vin, buf_k(0), pairs ? buf_v(0) : nullptr, n, flip,
                                  p.rounds == 0 ? flip : 0u, s);
    }
    if (e != hipSuccess) return hip_fail(e, "tile sort launch");
    uint64_t L = p.T;
    for (uint32_t r = 0; r < p.rounds; ++r, L *= p.K) {
        const mms::RoundGeom g = mms::round_geom(n, L, p.K, p.Tout);
        {
            Timed tm(MMS_KERNEL_PARTITION, s);
            e = mms::launch_corank_tiles(buf_k(r), g, table, s);
        }
        if (e != hipSuccess) return hip_fail(e, "partition launch");
        {
            Timed tm(MMS_KERNEL_MERGE, s);
            if (pairs)
                e = mms::launch_merge(true, buf_k(r), buf_v(r), buf_k(r + 1), buf_v(r + 1), g, table,
                                      r + 1 == p.rounds ? flip : 0u, s);
            else
                e = mms::launch_merge_keys(buf_k(r), buf_k(r + 1), g, table, r + 1 == p.rounds ? flip : 0u,
                                           persistent_grid(), merge_variant(), s);
        }
        if (e != hipSuccess) return hip_fail(e, "merge launch");
    }
    return MMS_OK;
}

}  // namespace

extern "C" {

const char* mms_last_error(void) { return g_err.c_str(); }

int mms_version(void) { return 100; }

int mms_plan(uint64_t n, uint32_t flags, mms_plan_t* out) {
    if (!out) return fail(MMS_EINVAL, "null plan pointer");
    if (flags & ~(MMS_KEY_I32 | MMS_PAIRS)) return fail(MMS_EINVAL, "unknown flags 0x%x", flags);
    if (n >= (1ull << 32)) return fail(MMS_EINVAL, "n = %llu exceeds 2^32-1", (unsigned long long)n);
    const Plan p = make_plan(n, flags);
    out->n = n;
    out->flags = flags;
    out->tile = p.T;
    out->lanes_per_tile = mms::kW1 * 64;
    out->fanout = p.K;
    out->merge_tile = p.Tout;
    out->rounds = n ? p.rounds : 0;
    out->passes = n ? 1 + p.rounds : 0;
    out->workspace_bytes = p.ws_bytes;
    return MMS_OK;
}

size_t mms_workspace_bytes(uint64_t n, uint32_t flags) {
    if (n == 0 || n >= (1ull << 32)) return 0;
    return (size_t)make_plan(n, flags).ws_bytes;
}

int mms_sort_u32(const uint32_t* d_in, uint32_t* d_out, uint64_t n, void* d_ws, size_t ws_bytes, uint32_t flags,
                 void* stream) {
    if (flags & MMS_PAIRS) return fail(MMS_EINVAL, "MMS_PAIRS is for workspace sizing; use mms_sort_pairs_u32");
    return sort_impl(d_in, nullptr, d_out, nullptr, n, d_ws, ws_bytes, flags, stream);
}

int mms_sort_pairs_u32(const uint32_t* d_kin, const uint32_t* d_vin, uint32_t* d_kout, uint32_t* d_vout,
                       uint64_t n, void* d_ws, size_t ws_bytes, uint32_t flags, void* stream) {
    if (n && !d_vin) return fail(MMS_EINVAL, "null value pointer");
    return sort_impl(d_kin, d_vin, d_kout, d_vout, n, d_ws, ws_bytes, flags & ~MMS_PAIRS, stream);
}

int mms_partition_u32(const uint32_t* d_keys, uint64_t n, uint64_t run_len, uint32_t K, const uint64_t* d_group,
                      const uint64_t* d_rank, uint64_t nqueries, uint32_t* d_split, uint32_t flags, void* stream) {
    if (flags & ~(MMS_KEY_I32 | MMS_PAIRS)) return fail(MMS_EINVAL, "unknown flags 0x%x", flags);
    if (K < 1 || K > mms::kMaxFanout) return fail(MMS_EINVAL, "K = %u outside [1, %u]", K, mms::kMaxFanout);
    if (run_len == 0) return fail(MMS_EINVAL, "run_len must be positive");
    if (n >= (1ull << 32)) return fail(MMS_EINVAL, "n = %llu exceeds 2^32-1", (unsigned long long)n);
    if (nqueries == 0) return MMS_OK;
    if (!d_keys && n) return fail(MMS_EINVAL, "null keys");
    if (!d_group || !d_rank || !d_split) return fail(MMS_EINVAL, "null query or output pointer");
    const uint32_t flip = (flags & MMS_KEY_I32) ? 0x80000000u : 0u;
    hipError_t e;
    {
        Timed tm(MMS_KERNEL_PARTITION, (hipStream_t)stream);
        e = mms::launch_corank_queries(d_keys, n, run_len, K, d_group, d_rank, nqueries, d_split, flip,
                                       (hipStream_t)stream);
    }
    if (e != hipSuccess) return hip_fail(e, "partition launch");
    return MMS_OK;
}

int mms_copy_u32(const uint32_t* d_in, uint32_t* d_out, uint64_t n, void* stream) {
    if (n == 0) return MMS_OK;
    if (!d_in || !d_out) return fail(MMS_EINVAL, "null pointer");
    if (overlaps(d_in, n * 4, d_out, n * 4)) return fail(MMS_EINVAL, "copy buffers overlap");
    hipError_t e;
    {
        Timed tm(MMS_KERNEL_COPY, (hipStream_t)stream);
        e = mms::launch_copy(d_in, d_out, n, (hipStream_t)stream);
    }
    if (e != hipSuccess) return hip_fail(e, "copy launch");
    return MMS_OK;
}

int mms_timing_enable(int on) {
    std::lock_guard<std::mutex> g(g_tmu);
    g_timing = on != 0;
    return MMS_OK;
}

int mms_timing_reset(void) {
    std::lock_guard<std::mutex> g(g_tmu);
    for (auto& r : g_recs) {
        hipEventSynchronize(r.b);
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
    for (int k = 0; k < MMS_KERNEL_KINDS; ++k) {
        g_launch[k] = 0;
        g_ms[k] = 0.0;
    }
    return MMS_OK;
}

int mms_timing_read(mms_timing_t* out) {
    if (!out) return fail(MMS_EINVAL, "null timing pointer");
    std::lock_guard<std::mutex> g(g_tmu);
    for (auto& r : g_recs) {
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return hip_fail(e, "timing event");
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return hip_fail(e, "timing event");
        g_launch[r.kind] += 1;
        g_ms[r.kind] += ms;
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
    for (int k = 0; k < MMS_KERNEL_KINDS; ++k) {
        out->launches[k] = g_launch[k];
        out->total_ms[k] = g_ms[k];
    }
    return MMS_OK;
}

}  // extern "C"
