// Host runtime of libmms: plans, workspace layout, argument checks, the
// phase loop (base case, then partition + merge per round), the segmented
// batch with its hipGraph cache, the tuning table, and the C ABI declared in
// include/mms.h.  Kernels are launched only through the launchers of
// mms_kernels.hip and mms_merge_keys.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "mms.h"
#include "mms_host.h"
#include "mms_internal.h"

namespace mms {
namespace host {

namespace {
thread_local std::string g_err;
}

const char* last_error() { return g_err.c_str(); }

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) { return fail(MMS_EHIP, "%s: %s", what, hipGetErrorString(e)); }

// ---- per-kernel timing (mms_timing_*) --------------------------------------
namespace {
struct TimingRec {
    int kind;
    hipEvent_t a, b;
};
std::mutex g_tmu;
bool g_timing = false;
uint32_t g_kinds = (1u << MMS_KERNEL_KINDS) - 1u;   // kinds that are timed
std::vector<TimingRec> g_recs;
std::vector<hipEvent_t> g_pool;
uint64_t g_launch[MMS_KERNEL_KINDS];
double g_ms[MMS_KERNEL_KINDS];
thread_local bool g_capturing = false;   // launches are being captured into a graph

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
}  // namespace

void set_capturing(bool on) { g_capturing = on; }

Timed::Timed(int kind, hipStream_t s) : kind_(kind), s_(s) {
    if (g_capturing) return;
    std::lock_guard<std::mutex> g(g_tmu);
    if (!g_timing || !((g_kinds >> kind) & 1u)) return;
    a_ = take_event();
    b_ = take_event();
    if (a_ && b_) (void)hipEventRecord(a_, s_);
}

Timed::~Timed() {
    if (!a_ || !b_) return;
    (void)hipEventRecord(b_, s_);
    std::lock_guard<std::mutex> g(g_tmu);
    g_recs.push_back({kind_, a_, b_});
}

// ---- tuning ------------------------------------------------------------------
// Ordered by max_log2_n; a sort of n uses the first entry with
// ceil(log2 n) <= max_log2_n (the last entry otherwise).
namespace {
std::mutex g_tune_mu;
std::vector<mms_tuning_t> g_tuning;
}  // namespace

uint32_t ceil_log2(uint64_t n) {
    uint32_t l = 0;
    while ((1ull << l) < n) ++l;
    return l;
}

Tune env_default() {
    Tune t{mms::kMaxFanout, mms::kToutKeys, 0, 0};
    if (const char* s = getenv("MMS_TOUT")) t.Tout = (uint32_t)atoi(s);
    if (const char* s = getenv("MMS_MERGE_VARIANT")) t.variant = atoi(s);
    if (const char* s = getenv("MMS_BASE_SHAPE")) t.base = atoi(s);
    if (const char* s = getenv("MMS_FANOUT")) t.K = (uint32_t)atoi(s);
    return t;
}

bool valid_tune(uint32_t K, uint32_t Tout, int variant, int base) {
    return K >= 2 && K <= mms::kMaxFanout && (K & (K - 1)) == 0 && Tout >= 1024 && Tout <= mms::kToutKeys &&
           Tout % 256 == 0 && variant >= 0 && variant <= 4 && base >= 0 && base < mms::kBaseShapes;
}

// Entries of one kind (keys-only or key-value) ordered by max_log2_n; a sort
// takes the first with ceil(log2 n) <= max_log2_n, else the last.  Key-value
// sorts use the keys-only entries when the table has none of their own.
Tune tune_for(uint64_t n, bool pairs) {
    Tune t = env_default();
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        const uint32_t want = pairs ? MMS_PAIRS : 0u;
        bool any = false;
        for (const auto& x : g_tuning) any = any || (x.flags & MMS_PAIRS) == want;
        const uint32_t kind = any ? want : 0u;
        const uint32_t l = ceil_log2(n);
        const mms_tuning_t* e = nullptr;
        for (const auto& x : g_tuning) {
            if ((x.flags & MMS_PAIRS) != kind) continue;
            e = &x;
            if (l <= x.max_log2_n) break;
        }
        if (e) t = Tune{e->fanout, e->merge_tile, (int)e->variant, (int)e->base};
    }
    if (!valid_tune(t.K, t.Tout, t.variant, t.base)) t = Tune{mms::kMaxFanout, mms::kToutKeys, 0, 0};
    if (pairs) {
        t.Tout = mms::kToutPairs;
        // key-value base cases: 8 per lane x 4 or 8 waves (8 x 16 sorts pairs
        // slower than 8 x 8: its LDS holds one workgroup per CU)
        if (t.base == 4) t.base = 3;
        else if (mms::base_e(t.base) != 8) t.base = 0;
    }
    return t;
}

// A batch of ns segments holding `total` elements has the parallel work of a
// sort of `total` elements, so it takes that size's launch parameters; its
// base tile stays within the mean segment (a larger tile would mostly sort
// sentinels), else the 2048-key shape.
Tune tune_for_batch(uint64_t total, uint64_t ns, bool pairs) {
    Tune t = tune_for(std::max<uint64_t>(total, 1), pairs);
    const uint64_t mean = ns ? total / ns : total;
    if (mms::base_tile(t.base) > std::max<uint64_t>(mms::kT1, mean)) t.base = 0;
    return t;
}

// One resident workgroup per compute unit for the persistent merge kernel.
unsigned persistent_grid() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
    return (unsigned)cus;
}

// ---- the phase loop ----------------------------------------------------------
namespace {
struct PhaseList {
    Phase base;                    // base-case pass
    std::vector<Phase> rounds;     // merge rounds
};

int run_phases(bool pairs, const PhaseList& pl, const Bufs& b, uint32_t* table, const Tune& tune, uint32_t flip,
               hipStream_t s) {
    hipError_t e;
    {
        Timed tm(MMS_KERNEL_TILE_SORT, s);
        e = launch_tile_sort(pairs, pl.base, b, flip, tune.base, s);
    }
    if (e != hipSuccess) return hip_fail(e, "tile sort launch");
    uint64_t L = base_tile(tune.base);
    for (size_t r = 0; r < pl.rounds.size(); ++r, L *= tune.K) {
        const Phase& ph = pl.rounds[r];
        if (ph.tiles == 0) continue;
        const RoundArgs ra{L, tune.K, tune.Tout, (L * tune.K + tune.Tout - 1) / tune.Tout};
        {
            Timed tm(MMS_KERNEL_PARTITION, s);
            e = launch_corank_tiles(ph, b, ra, table, s);
        }
        if (e != hipSuccess) return hip_fail(e, "partition launch");
        {
            Timed tm(MMS_KERNEL_MERGE, s);
            if (pairs) e = launch_merge_pairs(ph, b, ra, table, flip, s);
            else e = launch_merge_keys(ph, b, ra, table, flip, persistent_grid(), tune.variant, s);
        }
        if (e != hipSuccess) return hip_fail(e, "merge launch");
    }
    return MMS_OK;
}
}  // namespace

// ---- batches -------------------------------------------------------------------
void build_batch_tasks(const uint64_t* seg_n, uint64_t ns, bool pairs, const Tune& tune, BatchTasks& bt) {
    bt.pairs = pairs;
    bt.tune = tune;
    bt.phases.assign(1, {});
    bt.max_round_tiles = 0;
    bt.ntasks = 0;
    const uint32_t T = base_tile(tune.base), K = tune.K;
    for (uint64_t s = 0; s < ns; ++s) {
        const uint64_t n = seg_n[s];
        if (n == 0) continue;
        const uint32_t R = rounds_for(n, T, K);
        if (bt.phases.size() < (size_t)R + 1) bt.phases.resize(R + 1);
        const uint32_t base_info = ((R % 2 == 0) ? kTaskDstOut : 0u) | (R == 0 ? kTaskFinal : 0u);
        for (uint64_t t = 0; t * T < n; ++t) bt.phases[0].push_back({(uint32_t)s, (uint32_t)t | base_info});
        uint64_t L = T;
        for (uint32_t r = 0; r < R; ++r, L *= K) {
            const RoundGeom g = round_geom(n, L, K, tune.Tout);
            const uint32_t info = (((R - r - 1) % 2 == 0) ? kTaskDstOut : 0u) | (r + 1 == R ? kTaskFinal : 0u);
            for (uint64_t t = 0; t < g.tiles; ++t) bt.phases[1 + r].push_back({(uint32_t)s, (uint32_t)t | info});
        }
    }
    for (size_t r = 0; r < bt.phases.size(); ++r) {
        bt.ntasks += bt.phases[r].size();
        if (r) bt.max_round_tiles = std::max<uint64_t>(bt.max_round_tiles, bt.phases[r].size());
    }
}

// A segment of n elements has at most n/T + 1 base tiles; round r has at
// most n/Tout + n/(T*K) + 1 tiles (one per Tout outputs plus one per group,
// groups <= n/(K*L) + 1 with L >= T); it has at most rounds_for(n, T, K)
// rounds.  Every base-case shape's tile is at least kT1, so the bounds taken
// at T = kT1 hold for all of them.
uint64_t batch_tasks_bound(uint64_t total, uint64_t ns, uint64_t maxn, uint32_t K, uint32_t Tout) {
    const uint64_t round = total / Tout + total / ((uint64_t)kT1 * K) + ns + 1;
    return total / kT1 + ns + 1 + (uint64_t)rounds_for(maxn, kT1, K) * round;
}

uint64_t batch_table_bound(uint64_t total, uint64_t ns, uint32_t Tout) {
    // groups are at least 2T long, so per-round tiles <= total/Tout + total/(2T) + ns + 1
    const uint64_t round = total / Tout + total / (2ull * kT1) + ns + 1;
    return align_up((round + 1) * kMaxFanout * 4);
}

void tuning_floor(uint32_t& K, uint32_t& Tout) {
    const Tune d = tune_for(1ull << 20, false);
    K = d.K;
    Tout = std::min<uint32_t>(d.Tout, kToutPairs);
    std::lock_guard<std::mutex> g(g_tune_mu);
    for (const auto& x : g_tuning) {
        if (!valid_tune(x.fanout, x.merge_tile, (int)x.variant, (int)x.base)) continue;
        K = std::min(K, x.fanout);
        if (!(x.flags & MMS_PAIRS)) Tout = std::min(Tout, x.merge_tile);   // key-value merges use kToutPairs
    }
}

void add_segment_tiles(uint64_t n, const Tune& tune, std::vector<uint64_t>& per_phase) {
    if (n == 0) return;
    const uint32_t T = base_tile(tune.base);
    const uint32_t R = rounds_for(n, T, tune.K);
    if (per_phase.size() < (size_t)R + 1) per_phase.resize(R + 1, 0);
    per_phase[0] += (n + T - 1) / T;
    uint64_t L = T;
    for (uint32_t r = 0; r < R; ++r, L *= tune.K) per_phase[1 + r] += round_geom(n, L, tune.K, tune.Tout).tiles;
}

int run_batch(const BatchTasks& bt, const SegDesc* d_segs, const TileTask* d_tasks, uint32_t* table, uint32_t flip,
              hipStream_t s) {
    PhaseList pl;
    size_t at = 0;
    for (size_t i = 0; i < bt.phases.size(); ++i) {
        const Phase ph{d_tasks + at, d_segs, 0, 0, 0, bt.phases[i].size()};
        if (i == 0) pl.base = ph;
        else pl.rounds.push_back(ph);
        at += bt.phases[i].size();
    }
    return run_phases(bt.pairs, pl, Bufs{}, table, bt.tune, flip, s);
}

int run_plain(bool pairs, const Phase& base, const std::vector<Phase>& rounds, const Bufs& b, uint32_t* table,
              const Tune& tune, uint32_t flip, hipStream_t s) {
    PhaseList pl{base, rounds};
    return run_phases(pairs, pl, b, table, tune, flip, s);
}

}  // namespace host
}  // namespace mms

using namespace mms::host;

namespace {

// ---- plain sort plan ---------------------------------------------------------
struct Plan {
    uint64_t n;
    bool pairs;
    uint32_t T;
    Tune tune;
    uint32_t rounds;
    uint64_t max_tiles;      // largest tile count over the merge rounds
    uint64_t off_vals;       // workspace offsets (bytes)
    uint64_t off_table;
    uint64_t ws_bytes;
};

Plan make_plan(uint64_t n, uint32_t flags) {
    Plan p{};
    p.n = n;
    p.pairs = (flags & MMS_PAIRS) != 0;
    p.tune = tune_for(n, p.pairs);
    p.T = mms::base_tile(p.tune.base);
    p.rounds = rounds_for(n, p.T, p.tune.K);
    p.max_tiles = 0;
    uint64_t L = p.T;
    for (uint32_t r = 0; r < p.rounds; ++r, L *= p.tune.K) {
        const mms::RoundGeom g = mms::round_geom(n, L, p.tune.K, p.tune.Tout);
        p.max_tiles = std::max<uint64_t>(p.max_tiles, g.tiles);
    }
    p.off_vals = align_up(n * 4);
    p.off_table = p.off_vals + (p.pairs ? align_up(n * 4) : 0);
    p.ws_bytes = p.rounds ? p.off_table + align_up((p.max_tiles + 1) * p.tune.K * 4) : 0;
    return p;
}

bool overlaps(const void* a, uint64_t abytes, const void* b, uint64_t bbytes) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bbytes && y < x + abytes;
}

// a and b either coincide exactly or are disjoint
bool same_or_disjoint(const void* a, const void* b, uint64_t bytes) { return a == b || !overlaps(a, bytes, b, bytes); }

// esize: bytes per key (and per value)
int check_buffers(const void* kin, const void* vin, void* kout, void* vout, uint64_t n, void* ws, uint64_t ws_need,
                  size_t ws_bytes, uint64_t esize = 4) {
    const bool pairs = vin != nullptr;
    if (!kin || !kout || (pairs && !vout)) return fail(MMS_EINVAL, "null data pointer");
    const uint64_t bytes = n * esize;
    if (!same_or_disjoint(kin, kout, bytes)) return fail(MMS_EINVAL, "keys in/out partially overlap");
    if (pairs) {
        if (!same_or_disjoint(vin, vout, bytes)) return fail(MMS_EINVAL, "values in/out partially overlap");
        if (overlaps(kout, bytes, vout, bytes) || overlaps(kin, bytes, vin, bytes) ||
            overlaps(kout, bytes, vin, bytes) || overlaps(kin, bytes, vout, bytes))
            return fail(MMS_EINVAL, "key and value buffers overlap");
    }
    if (ws_need) {
        if (!ws) return fail(MMS_EINVAL, "workspace required (%llu bytes)", (unsigned long long)ws_need);
        if (ws_bytes < ws_need)
            return fail(MMS_EINVAL, "workspace too small: %zu < %llu", ws_bytes, (unsigned long long)ws_need);
        if ((uintptr_t)ws % kAlign) return fail(MMS_EINVAL, "workspace not 256-byte aligned");
        if (overlaps(ws, ws_need, kin, bytes) || overlaps(ws, ws_need, kout, bytes) ||
            (pairs && (overlaps(ws, ws_need, vin, bytes) || overlaps(ws, ws_need, vout, bytes))))
            return fail(MMS_EINVAL, "workspace overlaps data");
    }
    return MMS_OK;
}

int sort_impl(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, uint64_t n, void* ws,
              size_t ws_bytes, uint32_t flags, void* stream) {
    const bool pairs = vin != nullptr;
    if (flags & ~(MMS_KEY_I32 | MMS_PAIRS)) return fail(MMS_EINVAL, "unknown flags 0x%x", flags);
    if (n == 0) return MMS_OK;
    if (n >= (1ull << 32)) return fail(MMS_EINVAL, "n = %llu exceeds 2^32-1", (unsigned long long)n);
    const Plan p = make_plan(n, flags | (pairs ? MMS_PAIRS : 0u));
    int rc = check_buffers(kin, vin, kout, vout, n, ws, p.ws_bytes, ws_bytes);
    if (rc) return rc;
    uint8_t* wsb = (uint8_t*)ws;
    mms::Bufs b{kin, vin, kout, vout, (uint32_t*)wsb, pairs ? (uint32_t*)(wsb + p.off_vals) : nullptr};
    uint32_t* table = p.rounds ? (uint32_t*)(wsb + p.off_table) : nullptr;
    // pass i writes the output when R - i is even, so pass R lands there
    const mms::Phase base{nullptr, nullptr, n, (p.rounds % 2 == 0) ? 1u : 0u, p.rounds == 0 ? 1u : 0u,
                          (n + p.T - 1) / p.T};
    std::vector<mms::Phase> rounds;
    uint64_t L = p.T;
    for (uint32_t r = 0; r < p.rounds; ++r, L *= p.tune.K) {
        const mms::RoundGeom g = mms::round_geom(n, L, p.tune.K, p.tune.Tout);
        rounds.push_back(mms::Phase{nullptr, nullptr, n, ((p.rounds - r - 1) % 2 == 0) ? 1u : 0u,
                                    r + 1 == p.rounds ? 1u : 0u, g.tiles});
    }
    return run_plain(pairs, base, rounds, b, table, p.tune, (flags & MMS_KEY_I32) ? 0x80000000u : 0u,
                     (hipStream_t)stream);
}

// ---- 64-bit keys (§6.3 also sorts 8-byte integers) ----------------------------
// Base tiles of kT64Keys keys or kT64Pairs pairs, merge tiles of
// kTout64Keys / kTout64Pairs, fan-out 16 (MMS64_FANOUT overrides it for
// experiments: 2, 4, 8 or 16).
uint32_t fanout64() {
    const char* e = getenv("MMS64_FANOUT");
    const uint32_t v = e ? (uint32_t)atoi(e) : 16u;
    return (v >= 2 && v <= mms::kMaxFanout && (v & (v - 1)) == 0) ? v : 16u;
}

struct Plan64 {
    uint64_t n;
    bool pairs;
    uint32_t T, K, Tout, rounds;
    uint64_t max_tiles, off_vals, off_table, ws_bytes;
};

Plan64 make_plan64(uint64_t n, bool pairs) {
    Plan64 p{};
    p.n = n;
    p.pairs = pairs;
    p.T = pairs ? mms::kT64Pairs : mms::kT64Keys;
    p.K = fanout64();
    p.Tout = pairs ? mms::kTout64Pairs : mms::kTout64Keys;
    p.rounds = rounds_for(n, p.T, p.K);
    uint64_t L = p.T;
    for (uint32_t r = 0; r < p.rounds; ++r, L *= p.K)
        p.max_tiles = std::max<uint64_t>(p.max_tiles, mms::round_geom(n, L, p.K, p.Tout).tiles);
    p.off_vals = align_up(n * 8);
    p.off_table = p.off_vals + (pairs ? align_up(n * 8) : 0);
    p.ws_bytes = p.rounds ? p.off_table + align_up((p.max_tiles + 1) * p.K * 4) : 0;
    return p;
}

int sort64_impl(const uint64_t* kin, const uint64_t* vin, uint64_t* kout, uint64_t* vout, uint64_t n, void* ws,
                size_t ws_bytes, uint32_t flags, hipStream_t s) {
    const bool pairs = vin != nullptr;
    if (flags & ~MMS_KEY_I64) return fail(MMS_EINVAL, "unknown flags 0x%x for a 64-bit sort", flags);
    if (n == 0) return MMS_OK;
    if (n >= (1ull << 32)) return fail(MMS_EINVAL, "n = %llu exceeds 2^32-1", (unsigned long long)n);
    const Plan64 p = make_plan64(n, pairs);
    int rc = check_buffers(kin, vin, kout, vout, n, ws, p.ws_bytes, ws_bytes, 8);
    if (rc) return rc;
    uint8_t* wsb = (uint8_t*)ws;
    const mms::Bufs64 b{kin, vin, kout, vout, (uint64_t*)wsb, pairs ? (uint64_t*)(wsb + p.off_vals) : nullptr};
    uint32_t* table = p.rounds ? (uint32_t*)(wsb + p.off_table) : nullptr;
    const uint64_t flip = (flags & MMS_KEY_I64) ? 0x8000000000000000ull : 0ull;
    hipError_t e;
    {
        // pass i writes the output when R - i is even, so pass R lands there
        const mms::Phase64 base{n, (p.rounds % 2 == 0) ? 1u : 0u, p.rounds == 0 ? 1u : 0u, (n + p.T - 1) / p.T};
        Timed tm(MMS_KERNEL_TILE_SORT, s);
        e = mms::launch_tile_sort64(pairs, base, b, flip, s);
    }
    if (e != hipSuccess) return hip_fail(e, "tile sort launch");
    uint64_t L = p.T;
    for (uint32_t r = 0; r < p.rounds; ++r, L *= p.K) {
        const mms::RoundGeom g = mms::round_geom(n, L, p.K, p.Tout);
        const mms::Phase64 ph{n, ((p.rounds - r - 1) % 2 == 0) ? 1u : 0u, r + 1 == p.rounds ? 1u : 0u, g.tiles};
        const mms::RoundArgs ra{L, p.K, p.Tout, (L * p.K + p.Tout - 1) / p.Tout};
        {
            Timed tm(MMS_KERNEL_PARTITION, s);
            e = mms::launch_corank_tiles64(ph, b, ra, table, s);
        }
        if (e != hipSuccess) return hip_fail(e, "partition launch");
        {
            Timed tm(MMS_KERNEL_MERGE, s);
            e = mms::launch_merge64(pairs, ph, b, ra, table, flip, s);
        }
        if (e != hipSuccess) return hip_fail(e, "merge launch");
    }
    return MMS_OK;
}

// ---- merge-path baseline -----------------------------------------------------------
// A block sort of kMergePathTile-key tiles, then ceil(log2(tiles)) pairwise
// merge passes, each a partition launch and a merge launch; buffers
// ping-pong between the output and the workspace, which also holds the
// split table.
struct PlanMP {
    uint32_t rounds;
    uint64_t max_tiles, off_table, ws_bytes;
};

PlanMP make_plan_mp(uint64_t n) {
    PlanMP p{};
    p.rounds = rounds_for(n, mms::kMergePathTile, 2);
    uint64_t L = mms::kMergePathTile;
    for (uint32_t r = 0; r < p.rounds; ++r, L *= 2)
        p.max_tiles = std::max<uint64_t>(p.max_tiles, mms::round_geom(n, L, 2, mms::kMergePathTile).tiles);
    p.off_table = align_up(n * 4);
    p.ws_bytes = p.rounds ? p.off_table + align_up((p.max_tiles + 1) * 4) : 0;
    return p;
}

int mergepath_impl(const uint32_t* in, uint32_t* out, uint64_t n, void* ws, size_t ws_bytes, uint32_t flags,
                   hipStream_t s) {
    if (flags & ~MMS_KEY_I32) return fail(MMS_EINVAL, "unknown flags 0x%x for the merge-path sort", flags);
    if (n == 0) return MMS_OK;
    if (n >= (1ull << 32)) return fail(MMS_EINVAL, "n = %llu exceeds 2^32-1", (unsigned long long)n);
    const PlanMP p = make_plan_mp(n);
    int rc = check_buffers(in, nullptr, out, nullptr, n, ws, p.ws_bytes, ws_bytes);
    if (rc) return rc;
    uint32_t* wk = (uint32_t*)ws;
    uint32_t* split = p.rounds ? (uint32_t*)((uint8_t*)ws + p.off_table) : nullptr;
    const uint32_t flip = (flags & MMS_KEY_I32) ? 0x80000000u : 0u;
    // pass i writes the output when R - i is even, so pass R lands there
    auto buf = [&](uint32_t pass) { return ((p.rounds - pass) % 2 == 0) ? out : wk; };
    hipError_t e;
    {
        Timed tm(MMS_KERNEL_TILE_SORT, s);
        e = mms::launch_mp_blocksort(in, buf(0), n, flip, p.rounds == 0 ? flip : 0u, s);
    }
    if (e != hipSuccess) return hip_fail(e, "block sort launch");
    uint64_t L = mms::kMergePathTile;
    for (uint32_t r = 0; r < p.rounds; ++r, L *= 2) {
        const uint32_t* src = buf(r);
        uint32_t* dst = buf(r + 1);
        {
            Timed tm(MMS_KERNEL_PARTITION, s);
            e = mms::launch_mp_partition(src, n, L, split, s);
        }
        if (e != hipSuccess) return hip_fail(e, "partition launch");
        {
            Timed tm(MMS_KERNEL_MERGE, s);
            e = mms::launch_mp_merge(src, dst, n, L, split, r + 1 == p.rounds ? flip : 0u, s);
        }
        if (e != hipSuccess) return hip_fail(e, "merge launch");
    }
    return MMS_OK;
}

// ---- segmented batch -----------------------------------------------------------
// Every segment is sorted as its own plain sort; each phase's tiles of all
// segments form one task list, so the batch runs one launch per kernel and
// phase.  The workspace mirrors the arrays: segment s uses
// ws[h_offsets[s] .. h_offsets[s+1]) for keys (and the values region likewise),
// followed by the partition table and the batch metadata (the SegDesc table,
// then the task lists phase after phase).
struct SegPlan {
    bool pairs;
    uint64_t total;                    // h_offsets[num_segs]
    std::vector<uint64_t> seg_off;     // non-empty segments
    std::vector<uint64_t> seg_n;
    BatchTasks bt;
    uint64_t off_vals, off_table, off_meta, seg_bytes, meta_bytes, ws_bytes;
};

int make_seg_plan(const uint64_t* off, uint64_t ns, uint32_t flags, SegPlan& sp) {
    sp.pairs = (flags & MMS_PAIRS) != 0;
    sp.total = off[ns];
    uint64_t maxn = 0;
    sp.seg_off.clear();
    sp.seg_n.clear();
    for (uint64_t s = 0; s < ns; ++s) {
        if (off[s + 1] < off[s]) return fail(MMS_EINVAL, "offsets decrease at segment %llu", (unsigned long long)s);
        const uint64_t n = off[s + 1] - off[s];
        maxn = std::max<uint64_t>(maxn, n);
        if (n) {
            sp.seg_off.push_back(off[s]);
            sp.seg_n.push_back(n);
        }
    }
    if (maxn >= (1ull << 32)) return fail(MMS_EINVAL, "a segment holds 2^32 or more elements");
    build_batch_tasks(sp.seg_n.data(), sp.seg_n.size(), sp.pairs, tune_for_batch(sp.total, sp.seg_n.size(), sp.pairs),
                      sp.bt);
    sp.off_vals = align_up(sp.total * 4);
    sp.off_table = sp.off_vals + (sp.pairs ? align_up(sp.total * 4) : 0);
    sp.off_meta = sp.off_table + sp.bt.table_bytes();
    sp.seg_bytes = align_up(sp.seg_n.size() * sizeof(mms::SegDesc));
    sp.meta_bytes = align_up(sp.seg_bytes + sp.bt.ntasks * sizeof(mms::TileTask));
    sp.ws_bytes = sp.off_meta + sp.meta_bytes;
    return MMS_OK;
}

// A captured batch, keyed by offsets, pointers and tuning: the host image of
// its metadata in pinned host memory the library owns (uploaded into the
// caller's workspace by an asynchronous copy on the caller's stream before
// every launch), and the instantiated graph of all kernel launches.  The
// event is recorded after each launch, so an entry is torn down only after
// the last work that reads its image or runs its graph has finished.
struct SegEntry {
    std::string key;
    SegPlan plan;
    void* h_meta = nullptr;
    hipEvent_t last_use = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
};

std::mutex g_seg_mu;
std::list<SegEntry> g_seg_cache;   // most recent first
constexpr size_t kSegCacheMax = 8;

void drop_entry(SegEntry& e) {
    if (e.last_use) {
        (void)hipEventSynchronize(e.last_use);
        (void)hipEventDestroy(e.last_use);
    }
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.graph) (void)hipGraphDestroy(e.graph);
    if (e.h_meta) (void)hipHostFree(e.h_meta);
    e.last_use = nullptr;
    e.exec = nullptr;
    e.graph = nullptr;
    e.h_meta = nullptr;
}

std::string seg_key(const uint64_t* off, uint64_t ns, uint32_t flags, const void* const* ptrs, int nptr,
                    const Tune& t) {
    std::string k;
    auto put = [&](const void* p, size_t n) { k.append((const char*)p, n); };
    put(&ns, sizeof ns);
    put(&flags, sizeof flags);
    put(&t, sizeof t);
    for (int i = 0; i < nptr; ++i) put(&ptrs[i], sizeof(void*));
    put(off, (ns + 1) * sizeof(uint64_t));
    return k;
}

bool seg_graph_enabled() {
    static const bool on = [] {
        const char* s = getenv("MMS_NO_GRAPH");
        return !(s && atoi(s) != 0);
    }();
    return on;
}

int segmented_impl(const uint32_t* kin, uint32_t* kout, const uint32_t* vin, uint32_t* vout, const uint64_t* off,
                   uint64_t ns, void* ws, size_t ws_bytes, uint32_t flags, hipStream_t s) {
    const bool pairs = vin != nullptr;
    if (flags & ~(MMS_KEY_I32 | MMS_PAIRS)) return fail(MMS_EINVAL, "unknown flags 0x%x", flags);
    if (ns == 0) return MMS_OK;
    if (!off) return fail(MMS_EINVAL, "null offsets");
    SegPlan sp;
    int rc = make_seg_plan(off, ns, flags | (pairs ? MMS_PAIRS : 0u), sp);
    if (rc) return rc;
    if (sp.seg_n.empty()) return MMS_OK;
    rc = check_buffers(kin, vin, kout, vout, sp.total, ws, sp.ws_bytes, ws_bytes);
    if (rc) return rc;

    const void* ptrs[5] = {kin, kout, vin, vout, ws};
    const std::string key = seg_key(off, ns, flags | (pairs ? MMS_PAIRS : 0u), ptrs, 5, sp.bt.tune);
    std::lock_guard<std::mutex> lock(g_seg_mu);
    auto it = std::find_if(g_seg_cache.begin(), g_seg_cache.end(), [&](const SegEntry& e) { return e.key == key; });
    if (it == g_seg_cache.end()) {
        SegEntry e;
        e.key = key;
        e.plan = std::move(sp);
        const SegPlan& p = e.plan;
        uint8_t* wsb = (uint8_t*)ws;
        uint32_t* ws_k = (uint32_t*)wsb;
        uint32_t* ws_v = pairs ? (uint32_t*)(wsb + p.off_vals) : nullptr;
        // host image of the metadata: SegDesc table, then the tasks
        hipError_t he = hipHostMalloc(&e.h_meta, p.meta_bytes, hipHostMallocDefault);
        if (he != hipSuccess) {
            e.h_meta = nullptr;
            return fail(MMS_ENOMEM, "pinned staging of the batch metadata: %s", hipGetErrorString(he));
        }
        he = hipEventCreateWithFlags(&e.last_use, hipEventDisableTiming);
        if (he != hipSuccess) {
            e.last_use = nullptr;
            drop_entry(e);
            return hip_fail(he, "batch event");
        }
        uint8_t* img = (uint8_t*)e.h_meta;
        memset(img, 0, p.meta_bytes);
        mms::SegDesc* sd = (mms::SegDesc*)img;
        for (size_t i = 0; i < p.seg_n.size(); ++i) {
            const uint64_t o = p.seg_off[i];
            sd[i] = mms::SegDesc{kin + o, pairs ? vin + o : nullptr, kout + o, pairs ? vout + o : nullptr,
                                 ws_k + o, pairs ? ws_v + o : nullptr, p.seg_n[i], 0};
        }
        size_t at = p.seg_bytes;
        for (auto& v : p.bt.phases) {
            if (!v.empty()) memcpy(img + at, v.data(), v.size() * sizeof(mms::TileTask));
            at += v.size() * sizeof(mms::TileTask);
        }
        g_seg_cache.push_front(std::move(e));
        while (g_seg_cache.size() > kSegCacheMax) {
            drop_entry(g_seg_cache.back());
            g_seg_cache.pop_back();
        }
        it = g_seg_cache.begin();
    } else if (it != g_seg_cache.begin()) {
        g_seg_cache.splice(g_seg_cache.begin(), g_seg_cache, it);
        it = g_seg_cache.begin();
    }
    SegEntry& e = *it;
    const SegPlan& p = e.plan;
    uint8_t* d_meta = (uint8_t*)ws + p.off_meta;
    const mms::SegDesc* d_segs = (const mms::SegDesc*)d_meta;
    const mms::TileTask* d_tasks = (const mms::TileTask*)(d_meta + p.seg_bytes);
    uint32_t* table = (uint32_t*)((uint8_t*)ws + p.off_table);
    const uint32_t flip = (flags & MMS_KEY_I32) ? 0x80000000u : 0u;
    // the metadata goes into the caller's workspace on the caller's stream,
    // ahead of the launches that read it (every call: the caller may have
    // used the workspace for something else in between)
    hipError_t ue = hipMemcpyAsync(d_meta, e.h_meta, p.meta_bytes, hipMemcpyHostToDevice, s);
    if (ue != hipSuccess) return hip_fail(ue, "batch metadata upload");
    if (!seg_graph_enabled()) {
        rc = run_batch(p.bt, d_segs, d_tasks, table, flip, s);
        const hipError_t ee = hipEventRecord(e.last_use, s);
        if (rc) return rc;
        return ee == hipSuccess ? MMS_OK : hip_fail(ee, "batch event");
    }

    if (!e.exec) {
        hipStream_t cap = nullptr;
        hipError_t he = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
        if (he != hipSuccess) return hip_fail(he, "capture stream");
        he = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (he != hipSuccess) {
            (void)hipStreamDestroy(cap);
            return hip_fail(he, "begin capture");
        }
        set_capturing(true);
        rc = run_batch(p.bt, d_segs, d_tasks, table, flip, cap);
        set_capturing(false);
        hipGraph_t graph = nullptr;
        he = hipStreamEndCapture(cap, &graph);
        (void)hipStreamDestroy(cap);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (he != hipSuccess) return hip_fail(he, "end capture");
        he = hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0);
        if (he != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return hip_fail(he, "graph instantiate");
        }
        e.graph = graph;
    }
    hipError_t he;
    {
        Timed tm(MMS_KERNEL_SEGMENTED, s);
        he = hipGraphLaunch(e.exec, s);
    }
    if (he != hipSuccess) return hip_fail(he, "graph launch");
    he = hipEventRecord(e.last_use, s);
    if (he != hipSuccess) return hip_fail(he, "batch event");
    return MMS_OK;
}

}  // namespace

extern "C" {

const char* mms_last_error(void) { return last_error(); }

int mms_version(void) { return 200; }

int mms_plan(uint64_t n, uint32_t flags, mms_plan_t* out) {
    if (!out) return fail(MMS_EINVAL, "null plan pointer");
    if (flags & ~(MMS_KEY_I32 | MMS_PAIRS | MMS_KEY_I64 | MMS_KEYS64 | MMS_MERGEPATH))
        return fail(MMS_EINVAL, "unknown flags 0x%x", flags);
    if (n >= (1ull << 32)) return fail(MMS_EINVAL, "n = %llu exceeds 2^32-1", (unsigned long long)n);
    if (flags & MMS_MERGEPATH) {
        if (flags & (MMS_PAIRS | MMS_KEYS64 | MMS_KEY_I64))
            return fail(MMS_EINVAL, "the merge-path sort takes 32-bit keys only");
        const PlanMP p = make_plan_mp(n);
        out->n = n;
        out->flags = flags;
        out->tile = mms::kMergePathTile;
        out->lanes_per_tile = mms::kMergePathThreads;
        out->fanout = 2;
        out->merge_tile = mms::kMergePathTile;
        out->rounds = n ? p.rounds : 0;
        out->passes = n ? 1 + p.rounds : 0;
        out->workspace_bytes = p.ws_bytes;
        return MMS_OK;
    }
    if (flags & MMS_KEYS64) {
        const Plan64 p = make_plan64(n, (flags & MMS_PAIRS) != 0);
        out->n = n;
        out->flags = flags;
        out->tile = p.T;
        out->lanes_per_tile = (p.pairs ? 4 : 8) * 64;
        out->fanout = p.K;
        out->merge_tile = p.Tout;
        out->rounds = n ? p.rounds : 0;
        out->passes = n ? 1 + p.rounds : 0;
        out->workspace_bytes = p.ws_bytes;
        return MMS_OK;
    }
    const Plan p = make_plan(n, flags);
    out->n = n;
    out->flags = flags;
    out->tile = p.T;
    out->lanes_per_tile = mms::base_w(p.tune.base) * 64;
    out->fanout = p.tune.K;
    out->merge_tile = p.tune.Tout;
    out->rounds = n ? p.rounds : 0;
    out->passes = n ? 1 + p.rounds : 0;
    out->workspace_bytes = p.ws_bytes;
    return MMS_OK;
}

size_t mms_workspace_bytes(uint64_t n, uint32_t flags) {
    if (n == 0 || n >= (1ull << 32)) return 0;
    if (flags & MMS_MERGEPATH) return (size_t)make_plan_mp(n).ws_bytes;
    if (flags & MMS_KEYS64) return (size_t)make_plan64(n, (flags & MMS_PAIRS) != 0).ws_bytes;
    return (size_t)make_plan(n, flags).ws_bytes;
}

int mms_sort_mergepath_u32(const uint32_t* d_in, uint32_t* d_out, uint64_t n, void* d_ws, size_t ws_bytes,
                           uint32_t flags, void* stream) {
    return mergepath_impl(d_in, d_out, n, d_ws, ws_bytes, flags, (hipStream_t)stream);
}

int mms_sort_u64(const uint64_t* d_in, uint64_t* d_out, uint64_t n, void* d_ws, size_t ws_bytes, uint32_t flags,
                 void* stream) {
    return sort64_impl(d_in, nullptr, d_out, nullptr, n, d_ws, ws_bytes, flags, (hipStream_t)stream);
}

int mms_sort_pairs_u64(const uint64_t* d_kin, const uint64_t* d_vin, uint64_t* d_kout, uint64_t* d_vout,
                       uint64_t n, void* d_ws, size_t ws_bytes, uint32_t flags, void* stream) {
    if (n && !d_vin) return fail(MMS_EINVAL, "null value pointer");
    return sort64_impl(d_kin, d_vin, d_kout, d_vout, n, d_ws, ws_bytes, flags, (hipStream_t)stream);
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

size_t mms_segmented_workspace_bytes(const uint64_t* h_offsets, uint64_t num_segs, uint32_t flags) {
    if (!h_offsets || num_segs == 0) return 0;
    SegPlan sp;
    if (make_seg_plan(h_offsets, num_segs, flags, sp)) return 0;
    return sp.seg_n.empty() ? 0 : (size_t)sp.ws_bytes;
}

int mms_segmented_sort(const uint32_t* d_kin, uint32_t* d_kout, const uint32_t* d_vin, uint32_t* d_vout,
                       const uint64_t* h_offsets, uint64_t num_segs, void* d_ws, size_t ws_bytes, uint32_t flags,
                       void* stream) {
    if ((d_vin == nullptr) != (d_vout == nullptr)) return fail(MMS_EINVAL, "values need both input and output");
    return segmented_impl(d_kin, d_kout, d_vin, d_vout, h_offsets, num_segs, d_ws, ws_bytes, flags & ~MMS_PAIRS,
                          (hipStream_t)stream);
}

int mms_set_tuning(const mms_tuning_t* entries, uint32_t count) {
    if (count && !entries) return fail(MMS_EINVAL, "null tuning table");
    std::vector<mms_tuning_t> v(entries, entries + count);
    for (const auto& x : v) {
        if (!valid_tune(x.fanout, x.merge_tile, (int)x.variant, (int)x.base))
            return fail(MMS_EINVAL, "invalid tuning entry (fanout %u, merge_tile %u, variant %u, base %u)",
                        x.fanout, x.merge_tile, x.variant, x.base);
        if (x.flags & ~MMS_PAIRS) return fail(MMS_EINVAL, "tuning entry flags 0x%x", x.flags);
    }
    std::stable_sort(v.begin(), v.end(), [](const mms_tuning_t& a, const mms_tuning_t& b) {
        return a.max_log2_n < b.max_log2_n;
    });
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tuning = std::move(v);
    return MMS_OK;
}

int mms_get_tuning(uint64_t n, uint32_t flags, mms_tuning_t* out) {
    if (!out) return fail(MMS_EINVAL, "null tuning pointer");
    const Tune t = tune_for(n ? n : 1, (flags & MMS_PAIRS) != 0);
    out->max_log2_n = ceil_log2(n ? n : 1);
    out->fanout = t.K;
    out->merge_tile = t.Tout;
    out->variant = (uint32_t)t.variant;
    out->base = (uint32_t)t.base;
    out->flags = flags & MMS_PAIRS;
    return MMS_OK;
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

int mms_timing_kinds(uint32_t mask) {
    const uint32_t all = (1u << MMS_KERNEL_KINDS) - 1u;
    if (!(mask & all) || (mask & ~all)) return fail(MMS_EINVAL, "timing kinds mask 0x%x selects no known kind", mask);
    std::lock_guard<std::mutex> g(g_tmu);
    g_kinds = mask;
    return MMS_OK;
}

int mms_timing_reset(void) {
    std::lock_guard<std::mutex> g(g_tmu);
    for (auto& r : g_recs) {
        (void)hipEventSynchronize(r.b);
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
