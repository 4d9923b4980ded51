// Host-side pieces shared by the C ABI (mms_api.cpp) and the serving loop
// (mms_server.cpp): error reporting, per-kernel timing, tuning lookup, and
// the batch builder + phase loop that enqueue a sort of many segments.
// Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "mms.h"
#include "mms_internal.h"

namespace mms {
namespace host {

// Set the calling thread's mms_last_error() message and return `code`.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_fail(hipError_t e, const char* what);
const char* last_error();

// Brackets one kernel launch (or graph launch) with events on its stream
// while mms_timing is enabled.
class Timed {
  public:
    Timed(int kind, hipStream_t s);
    ~Timed();
    Timed(const Timed&) = delete;
    Timed& operator=(const Timed&) = delete;

  private:
    int kind_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

// Launches made on this thread are being captured into a graph (no timing).
void set_capturing(bool on);

struct Tune {
    uint32_t K;      // merge fan-out
    uint32_t Tout;   // merge output tile
    int variant;     // keys-only merge kernel shape
    int base;        // keys-only base-case shape (elements per lane x waves)
};
Tune tune_for(uint64_t n, bool pairs);
Tune tune_for_batch(uint64_t total, uint64_t ns, bool pairs);
uint32_t ceil_log2(uint64_t n);

constexpr uint64_t kAlign = 256;
inline uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// §6.2: ceil(log_K(ceil(n / T))) merge rounds after the base case.
inline uint32_t rounds_for(uint64_t n, uint32_t T, uint32_t K) {
    uint32_t r = 0;
    for (uint64_t L = T; L < n; L *= K) ++r;
    return r;
}

// Workgroups of the persistent merge kernel (one per compute unit).
unsigned persistent_grid();

// The tile tasks of a batch of non-empty segments: phases[0] is the base
// case, phases[1 + r] merge round r.  Every segment is planned exactly as a
// plain sort of its own length with the batch's tuning; segment s with R_s
// rounds writes the output in pass i when R_s - i is even, so its last pass
// lands there.
struct BatchTasks {
    bool pairs = false;
    Tune tune{};
    std::vector<std::vector<TileTask>> phases;
    uint64_t max_round_tiles = 0;
    uint64_t ntasks = 0;
    uint64_t table_bytes() const {
        return phases.size() > 1 ? align_up((max_round_tiles + 1) * tune.K * 4) : 0;
    }
};
void build_batch_tasks(const uint64_t* seg_n, uint64_t ns, bool pairs, const Tune& tune, BatchTasks& bt);

// Smallest fan-out and merge tile any sort can currently be planned with
// (over the tuning table, the default, and the key-value tile).
void tuning_floor(uint32_t& K, uint32_t& Tout);

// Upper bounds on the task count and partition-table bytes of a batch of at
// most `ns` segments, `total` elements and segments of at most `maxn`
// elements, planned with fan-out >= K and merge tile >= Tout.
uint64_t batch_tasks_bound(uint64_t total, uint64_t ns, uint64_t maxn, uint32_t K, uint32_t Tout);
uint64_t batch_table_bound(uint64_t total, uint64_t ns, uint32_t Tout);

// Tiles of each phase of the plain sort of n elements under `tune`
// (entry 0: base case, entry 1 + r: round r), added to `per_phase`.
void add_segment_tiles(uint64_t n, const Tune& tune, std::vector<uint64_t>& per_phase);

// Enqueue every phase of a batch on stream s.  d_segs holds its SegDesc
// table and d_tasks its task lists phase after phase (device memory);
// table is the partition table of table_bytes().
int run_batch(const BatchTasks& bt, const SegDesc* d_segs, const TileTask* d_tasks, uint32_t* table, uint32_t flip,
              hipStream_t s);

}  // namespace host
}  // namespace mms
