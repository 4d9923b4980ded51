// Serving loop of libmms: admission by arena budget, continuous batching of
// the admitted requests into batched sorts on several streams, completion
// threads, and the C ABI mms_server_* / mms_submit / mms_poll / mms_wait /
// mms_release declared in include/mms.h.
//
// Life of a request:
//   submit   -> queued (FIFO)            [client thread]
//   admit    -> result + workspace ranges allocated in the arena   [scheduler]
//   launch   -> joins the next batch of its kind; the batch's SegDesc table
//               and task lists are staged in a metadata slot and the batch
//               runs the segmented sort's phases on one of the streams
//   complete -> its stream's completion thread sees the batch event, stamps
//               the request, returns the workspace and the slot
//   release  -> the result range returns to the arena (at once, or after the
//               caller's stream has passed the release point)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mms.h"
#include "mms_host.h"
#include "mms_internal.h"

using namespace mms::host;

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over byte ranges (multiples of 256) of the arena's
// data region; free ranges ordered by offset and merged with their
// neighbours when returned.  Any part of an allocation may be returned on
// its own.
class RangeAlloc {
  public:
    void init(uint64_t off, uint64_t size) {
        free_.clear();
        if (size) free_[off] = size;
        total_ = size;
        used_ = 0;
    }
    bool alloc(uint64_t bytes, uint64_t& off) {
        if (bytes == 0) {
            off = 0;
            return true;
        }
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const uint64_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        if (bytes == 0) return;
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                off = prev->first;
                bytes += prev->second;
                free_.erase(prev);
            }
        }
        next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            free_.erase(next);
        }
        free_[off] = bytes;
    }
    uint64_t used() const { return used_; }
    uint64_t total() const { return total_; }

  private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t total_ = 0, used_ = 0;
};

enum class St { Queued, Admitted, Running, Done, Failed };

struct Req {
    mms_request r{};
    St st = St::Queued;
    int status = MMS_PENDING;
    std::string err;
    uint64_t res_off = 0, res_bytes = 0;   // result: keys, then values
    uint64_t ws_off = 0, ws_bytes = 0;     // workspace: keys, then values
    uint64_t half = 0;                     // bytes of the keys part of each range
    hipEvent_t ready = nullptr;            // input ready (recorded at submit)
    double t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
    uint64_t batch = 0;
    uint32_t batch_reqs = 0;
    uint32_t stream = 0;
};

struct Batch {
    uint64_t id = 0;
    Tune tune{};
    std::vector<uint64_t> tickets;
    int slot = -1;
    int stream = 0;
    hipEvent_t done = nullptr;
    int status = MMS_OK;
    std::string err;
};

struct Deferred {
    hipEvent_t ev;
    uint64_t off, bytes;
};

struct Slot {
    uint64_t dev_off = 0;        // byte offset in the arena
    void* host = nullptr;        // pinned staging for the metadata upload
    size_t host_bytes = 0;
};

}  // namespace

struct mms_server {
    mms_server_cfg cfg{};
    bool dry = false;
    int device = 0;
    uint8_t* arena = nullptr;
    std::vector<hipStream_t> streams;
    bool own_streams = false;
    uint64_t slot_bytes = 0;
    std::vector<Slot> slots;
    std::vector<int> free_slots;
    Clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv_sched;              // progress may be possible
    std::condition_variable cv_done;               // a request finished
    std::vector<std::condition_variable> cv_comp;  // per stream: a batch was enqueued
    uint64_t gen = 0;
    bool stopping = false;
    bool stop_completion = false;

    RangeAlloc alloc;
    std::unordered_map<uint64_t, Req> reqs;
    std::deque<uint64_t> queue;       // waiting for admission
    std::deque<uint64_t> admitted;    // admitted, not yet in a batch
    std::vector<std::deque<Batch>> inflight;
    std::vector<Deferred> deferred;
    std::vector<hipEvent_t> event_pool;
    uint64_t next_ticket = 1;
    uint64_t next_batch = 1;
    uint64_t live_admitted = 0;       // admitted and not released
    uint32_t rr = 0;
    mms_server_stats stats{};

    std::thread scheduler;
    std::vector<std::thread> completers;

    double now_us() const {
        return std::chrono::duration<double, std::micro>(Clock::now() - t0).count();
    }
};

namespace {

uint64_t elem_bytes(uint64_t n) { return align_up(n * 4); }

bool is_pairs(const mms_request& r) { return (r.flags & MMS_PAIRS) != 0; }

// Footprint of a request: result, and workspace when it needs merge rounds.
void footprint(const mms_request& r, uint64_t& half, uint64_t& res, uint64_t& ws) {
    half = elem_bytes(r.n);
    res = half * (is_pairs(r) ? 2 : 1);
    ws = r.n > mms::kT1 ? res : 0;
}

hipEvent_t take_event(mms_server* s) {
    if (!s->event_pool.empty()) {
        hipEvent_t e = s->event_pool.back();
        s->event_pool.pop_back();
        return e;
    }
    // Blocking sync: a completion thread sleeps in hipEventSynchronize rather
    // than spinning on a core the submitting threads need.
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming | hipEventBlockingSync) != hipSuccess) return nullptr;
    return e;
}

void give_event(mms_server* s, hipEvent_t e) {
    if (e) s->event_pool.push_back(e);
}

void bump(mms_server* s) {
    ++s->gen;
    s->cv_sched.notify_one();
}

// Return deferred result ranges whose release point the caller's stream has
// passed.  Caller holds the lock.
void reap_deferred(mms_server* s) {
    for (size_t i = 0; i < s->deferred.size();) {
        Deferred& d = s->deferred[i];
        if (hipEventQuery(d.ev) == hipSuccess) {
            s->alloc.release(d.off, d.bytes);
            give_event(s, d.ev);
            d = s->deferred.back();
            s->deferred.pop_back();
        } else {
            ++i;
        }
    }
}

// FIFO admission: the head of the queue is admitted when its ranges fit and
// the request limit allows; nothing behind it overtakes it.
void admit(mms_server* s) {
    while (!s->queue.empty() && s->live_admitted < s->cfg.max_requests) {
        Req& q = s->reqs[s->queue.front()];
        uint64_t half, res, ws, ro = 0, wo = 0;
        footprint(q.r, half, res, ws);
        if (!s->alloc.alloc(res, ro)) break;
        if (!s->alloc.alloc(ws, wo)) {
            s->alloc.release(ro, res);
            break;
        }
        q.res_off = ro;
        q.res_bytes = res;
        q.ws_off = wo;
        q.ws_bytes = ws;
        q.half = half;
        q.st = St::Admitted;
        q.t_admit = s->now_us();
        s->admitted.push_back(s->queue.front());
        s->queue.pop_front();
        ++s->live_admitted;
        ++s->stats.admitted;
        s->stats.peak_used_bytes = std::max(s->stats.peak_used_bytes, s->alloc.used());
    }
}

int pick_stream(mms_server* s) {
    const int S = (int)s->streams.size();
    int best = -1;
    for (int k = 0; k < S; ++k) {
        const int i = (int)((s->rr + k) % S);
        if (s->inflight[i].size() >= s->cfg.max_inflight) continue;
        if (best < 0 || s->inflight[i].size() < s->inflight[best].size()) best = i;
    }
    if (best >= 0) s->rr = (uint32_t)(best + 1);
    return best;
}

// Device bytes of a batch's metadata: SegDesc table, task lists, partition
// table.
uint64_t meta_bytes(uint64_t segs, uint64_t ntasks, uint64_t max_round_tiles, uint32_t K, bool rounds) {
    return align_up(align_up(segs * sizeof(mms::SegDesc)) + ntasks * sizeof(mms::TileTask)) +
           (rounds ? align_up((max_round_tiles + 1) * K * 4) : 0);
}

// Size class of a request: sizes within one class differ by less than a
// factor of 16, so a batch's requests finish at about the same time and a
// small request never waits for a large one's sort.
uint32_t size_class(uint64_t n) { return ceil_log2(n) / 4u; }

// The next batch: the oldest admitted request and, in admission order, every
// later one of the same kind and size class within the batch limits and the
// metadata slot (the others form later batches, which the other streams run
// at the same time).  The batch is planned with the tuning of the
// candidates' total (capped by the batch limits), as a segmented sort of them
// would be.
Batch form_batch(mms_server* s, int stream, int slot) {
    Batch b;
    b.id = s->next_batch++;
    b.stream = stream;
    b.slot = slot;
    const Req& head = s->reqs[s->admitted.front()];
    const uint32_t kind = head.r.flags;
    const uint32_t cls = size_class(head.r.n);
    uint64_t cand_keys = 0, cand_n = 0;
    for (uint64_t t : s->admitted) {
        const Req& q = s->reqs[t];
        if (q.r.flags != kind || size_class(q.r.n) != cls || cand_n >= s->cfg.max_batch_requests) continue;
        if (cand_n && cand_keys + q.r.n > s->cfg.max_batch_keys) continue;
        cand_keys += q.r.n;
        ++cand_n;
    }
    b.tune = tune_for_batch(cand_keys, cand_n, (kind & MMS_PAIRS) != 0);
    uint64_t keys = 0, ntasks = 0;
    std::vector<uint64_t> phases, mine;
    std::deque<uint64_t> rest;
    for (uint64_t t : s->admitted) {
        Req& q = s->reqs[t];
        bool take = q.r.flags == kind && size_class(q.r.n) == cls && b.tickets.size() < s->cfg.max_batch_requests &&
                    keys + q.r.n <= s->cfg.max_batch_keys;
        if (take) {
            mine.assign(phases.size(), 0);
            add_segment_tiles(q.r.n, b.tune, mine);
            std::vector<uint64_t> sum(std::max(phases.size(), mine.size()), 0);
            uint64_t add = 0, maxr = 0;
            for (size_t p = 0; p < sum.size(); ++p) {
                const uint64_t a = p < phases.size() ? phases[p] : 0, m = p < mine.size() ? mine[p] : 0;
                sum[p] = a + m;
                add += m;
                if (p) maxr = std::max(maxr, sum[p]);
            }
            if (meta_bytes(b.tickets.size() + 1, ntasks + add, maxr, b.tune.K, sum.size() > 1) <= s->slot_bytes) {
                phases.swap(sum);
                ntasks += add;
            } else {
                take = false;
                if (b.tickets.empty() && t == s->admitted.front()) {
                    // cannot run even alone (the tuning changed after creation)
                    s->alloc.release(q.ws_off, q.ws_bytes);
                    q.ws_bytes = 0;
                    q.st = St::Failed;
                    q.status = MMS_EINVAL;
                    q.err = "request needs more batch metadata than a slot holds under the current tuning";
                    q.t_done = s->now_us();
                    ++s->stats.completed;
                    s->cv_done.notify_all();
                    continue;
                }
            }
        }
        if (take) {
            b.tickets.push_back(t);
            keys += q.r.n;
        } else {
            rest.push_back(t);
        }
    }
    s->admitted.swap(rest);
    const double t = s->now_us();
    for (uint64_t tk : b.tickets) {
        Req& q = s->reqs[tk];
        q.st = St::Running;
        q.t_launch = t;
        q.batch = b.id;
        q.batch_reqs = (uint32_t)b.tickets.size();
        q.stream = (uint32_t)stream;
    }
    ++s->stats.batches;
    s->stats.max_batch_seen = std::max<uint64_t>(s->stats.max_batch_seen, b.tickets.size());
    return b;
}

// Enqueue a batch on its stream (no lock held; the requests it names are
// Running, so no other thread changes their fields).
void enqueue_batch(mms_server* s, Batch& b, std::vector<Req*>& rq) {
    if (s->dry) return;
    (void)hipSetDevice(s->device);
    hipStream_t st = s->streams[b.stream];
    const bool pairs = is_pairs(rq[0]->r);
    const uint32_t flip = (rq[0]->r.flags & MMS_KEY_I32) ? 0x80000000u : 0u;
    auto hip_err = [&](hipError_t e, const char* what) {
        hip_fail(e, what);
        b.status = MMS_EHIP;
        b.err = last_error();
    };
    for (Req* q : rq) {
        if (q->ready) {
            hipError_t e = hipStreamWaitEvent(st, q->ready, 0);
            if (e != hipSuccess) {
                hip_err(e, "wait for request input");
                break;
            }
        }
    }
    if (b.status == MMS_OK) {
        std::vector<uint64_t> seg_n(rq.size());
        for (size_t i = 0; i < rq.size(); ++i) seg_n[i] = rq[i]->r.n;
        BatchTasks bt;
        build_batch_tasks(seg_n.data(), seg_n.size(), pairs, b.tune, bt);
        const uint64_t seg_bytes = align_up(rq.size() * sizeof(mms::SegDesc));
        const uint64_t img_bytes = align_up(seg_bytes + bt.ntasks * sizeof(mms::TileTask));
        if (img_bytes + bt.table_bytes() > s->slot_bytes) {   // excluded when the batch was formed
            b.status = MMS_EINVAL;
            b.err = "batch metadata exceeds its slot";
        } else {
            Slot& sl = s->slots[b.slot];
            if (sl.host_bytes < img_bytes) {
                if (sl.host) (void)hipHostFree(sl.host);
                sl.host = nullptr;
                sl.host_bytes = 0;
                hipError_t e = hipHostMalloc(&sl.host, img_bytes, hipHostMallocDefault);
                if (e != hipSuccess) {
                    sl.host = nullptr;
                    hip_err(e, "pinned staging allocation");
                } else {
                    sl.host_bytes = img_bytes;
                }
            }
            if (b.status == MMS_OK) {
                uint8_t* img = (uint8_t*)sl.host;
                mms::SegDesc* sd = (mms::SegDesc*)img;
                for (size_t i = 0; i < rq.size(); ++i) {
                    const Req& q = *rq[i];
                    uint32_t* res = (uint32_t*)(s->arena + q.res_off);
                    uint32_t* ws = (uint32_t*)(s->arena + q.ws_off);
                    sd[i] = mms::SegDesc{q.r.d_keys, pairs ? q.r.d_vals : nullptr, res,
                                         pairs ? (uint32_t*)((uint8_t*)res + q.half) : nullptr,
                                         q.ws_bytes ? ws : nullptr,
                                         (pairs && q.ws_bytes) ? (uint32_t*)((uint8_t*)ws + q.half) : nullptr,
                                         q.r.n, 0};
                }
                uint64_t at = seg_bytes;
                for (auto& v : bt.phases) {
                    if (!v.empty()) memcpy(img + at, v.data(), v.size() * sizeof(mms::TileTask));
                    at += v.size() * sizeof(mms::TileTask);
                }
                uint8_t* dev = s->arena + sl.dev_off;
                hipError_t e = hipMemcpyAsync(dev, img, img_bytes, hipMemcpyHostToDevice, st);
                if (e != hipSuccess) {
                    hip_err(e, "metadata upload");
                } else {
                    const int rc = run_batch(bt, (const mms::SegDesc*)dev, (const mms::TileTask*)(dev + seg_bytes),
                                             (uint32_t*)(dev + img_bytes), flip, st);
                    if (rc) {
                        b.status = rc;
                        b.err = last_error();
                    }
                }
            }
        }
    }
    // the event also covers a partly enqueued batch, so its ranges are
    // returned only after whatever was launched has finished
    hipError_t e = hipEventRecord(b.done, st);
    if (e != hipSuccess) {
        if (b.status == MMS_OK) hip_err(e, "batch event");
        (void)hipStreamSynchronize(st);
        (void)hipEventDestroy(b.done);
        b.done = nullptr;
    }
}

// Mark a batch complete.  Caller holds the lock.
void finish_batch(mms_server* s, Batch& b, double t_done) {
    for (uint64_t tk : b.tickets) {
        Req& q = s->reqs[tk];
        s->alloc.release(q.ws_off, q.ws_bytes);
        q.ws_bytes = 0;
        give_event(s, q.ready);
        q.ready = nullptr;
        q.t_done = t_done;
        if (b.status == MMS_OK) {
            q.st = St::Done;
            q.status = MMS_OK;
        } else {
            q.st = St::Failed;
            q.status = b.status;
            q.err = b.err;
        }
        ++s->stats.completed;
    }
    give_event(s, b.done);
    b.done = nullptr;
    s->free_slots.push_back(b.slot);
    bump(s);
    s->cv_done.notify_all();
}

void scheduler_main(mms_server* s) {
    if (!s->dry) (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        const uint64_t seen = s->gen;
        if (!s->deferred.empty()) reap_deferred(s);
        if (!s->stopping) admit(s);
        bool launched = false;
        while (!s->stopping && !s->admitted.empty() && !s->free_slots.empty()) {
            const int stream = pick_stream(s);
            if (stream < 0) break;
            const int slot = s->free_slots.back();
            s->free_slots.pop_back();
            Batch b = form_batch(s, stream, slot);
            if (b.tickets.empty()) {
                s->free_slots.push_back(slot);
                --s->stats.batches;
                continue;
            }
            if (!s->dry) {
                b.done = take_event(s);
                if (!b.done) {
                    b.status = MMS_EHIP;
                    b.err = "event creation failed";
                }
            }
            std::vector<Req*> rq;
            for (uint64_t t : b.tickets) rq.push_back(&s->reqs[t]);   // stable: unordered_map nodes
            if (b.status == MMS_OK) {
                lk.unlock();
                enqueue_batch(s, b, rq);
                lk.lock();
            }
            if (s->dry || !b.done) {
                finish_batch(s, b, s->now_us());
            } else {
                s->inflight[b.stream].push_back(std::move(b));
                s->cv_comp[stream].notify_one();
            }
            launched = true;
        }
        // batches in flight are drained by the completion threads
        if (s->stopping) break;
        if (launched) continue;
        if (s->gen != seen) continue;
        if (!s->deferred.empty()) s->cv_sched.wait_for(lk, std::chrono::microseconds(200));
        else s->cv_sched.wait(lk, [&] { return s->gen != seen; });
    }
}

void completer_main(mms_server* s, int i) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_comp[i].wait(lk, [&] { return !s->inflight[i].empty() || s->stop_completion; });
        if (s->inflight[i].empty()) break;
        hipEvent_t ev = s->inflight[i].front().done;
        lk.unlock();
        hipError_t e = hipEventSynchronize(ev);
        const double t = s->now_us();
        lk.lock();
        Batch b = std::move(s->inflight[i].front());
        s->inflight[i].pop_front();
        if (e != hipSuccess && b.status == MMS_OK) {
            b.status = MMS_EHIP;
            b.err = std::string("batch execution: ") + hipGetErrorString(e);
        }
        finish_batch(s, b, t);
    }
}

void fill_result(const mms_server* s, const Req& q, mms_result* out) {
    if (!out) return;
    memset(out, 0, sizeof *out);
    out->status = q.status;
    out->flags = q.r.flags;
    out->n = q.r.n;
    if (q.st == St::Done) {
        out->d_keys = (uint32_t*)(s->arena + q.res_off);
        out->d_vals = is_pairs(q.r) ? (uint32_t*)(s->arena + q.res_off + q.half) : nullptr;
    }
    out->t_submit_us = q.t_submit;
    out->t_admit_us = q.t_admit;
    out->t_launch_us = q.t_launch;
    out->t_done_us = q.t_done;
    out->batch = q.batch;
    out->batch_requests = q.batch_reqs;
    out->stream_index = q.stream;
}

int poll_locked(mms_server* s, uint64_t ticket, mms_result* out) {
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(MMS_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    const Req& q = it->second;
    fill_result(s, q, out);
    if (q.st == St::Done) return MMS_OK;
    if (q.st == St::Failed) return fail(q.status, "%s", q.err.c_str());
    return MMS_PENDING;
}

void destroy_resources(mms_server* s) {
    if (!s->dry) {
        (void)hipSetDevice(s->device);
        for (auto& d : s->deferred) {
            (void)hipEventSynchronize(d.ev);
            (void)hipEventDestroy(d.ev);
        }
        for (auto& kv : s->reqs)
            if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
        for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
        for (auto& sl : s->slots)
            if (sl.host) (void)hipHostFree(sl.host);
        if (s->own_streams)
            for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    }
    delete s;
}

}  // namespace

extern "C" {

int mms_server_create(const mms_server_cfg* cfg_in, mms_server** out) {
    if (!cfg_in || !out) return fail(MMS_EINVAL, "null argument");
    *out = nullptr;
    mms_server_cfg cfg = *cfg_in;
    if (cfg.flags & ~MMS_SERVER_DRY_RUN) return fail(MMS_EINVAL, "unknown server flags 0x%x", cfg.flags);
    if (!cfg.d_arena) return fail(MMS_EINVAL, "null arena");
    if ((uintptr_t)cfg.d_arena % kAlign) return fail(MMS_EINVAL, "arena not 256-byte aligned");
    if (cfg.num_streams > MMS_SERVER_MAX_STREAMS) return fail(MMS_EINVAL, "more than %d streams", MMS_SERVER_MAX_STREAMS);
    if (cfg.max_inflight == 0) cfg.max_inflight = 2;
    if (cfg.max_requests == 0) cfg.max_requests = 65536;
    if (cfg.max_batch_requests == 0) cfg.max_batch_requests = 1024;
    if (cfg.max_batch_keys == 0) cfg.max_batch_keys = 1ull << 28;
    if (cfg.max_inflight > 16) return fail(MMS_EINVAL, "max_inflight above 16");
    if (cfg.max_batch_requests > (1u << 20)) return fail(MMS_EINVAL, "max_batch_requests above 2^20");
    if (cfg.max_batch_keys > (1ull << 36)) return fail(MMS_EINVAL, "max_batch_keys above 2^36");

    mms_server* s = new mms_server();
    s->dry = (cfg.flags & MMS_SERVER_DRY_RUN) != 0;
    s->arena = (uint8_t*)cfg.d_arena;
    s->t0 = Clock::now();
    const int S = cfg.num_streams ? (int)cfg.num_streams : 2;
    if (!s->dry) {
        hipError_t e = hipGetDevice(&s->device);
        if (e != hipSuccess) {
            delete s;
            return hip_fail(e, "current device");
        }
        if (cfg.num_streams) {
            for (int i = 0; i < S; ++i) s->streams.push_back((hipStream_t)cfg.streams[i]);
        } else {
            s->own_streams = true;
            for (int i = 0; i < S; ++i) {
                hipStream_t st = nullptr;
                e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
                if (e != hipSuccess) {
                    destroy_resources(s);
                    return hip_fail(e, "stream creation");
                }
                s->streams.push_back(st);
            }
        }
    } else {
        s->streams.assign(S, nullptr);
    }
    // metadata slots at the start of the arena, sized for the largest batch
    const uint64_t nslots = (uint64_t)S * cfg.max_inflight;
    uint32_t Kmin, Tmin;
    tuning_floor(Kmin, Tmin);
    const uint64_t nb = cfg.max_batch_keys, rb = cfg.max_batch_requests;
    s->slot_bytes = align_up(rb * sizeof(mms::SegDesc)) +
                    align_up(batch_tasks_bound(nb, rb, std::min<uint64_t>(nb, 0xFFFFFFFFull), Kmin, Tmin) *
                             sizeof(mms::TileTask)) +
                    batch_table_bound(nb, rb, Tmin);
    const uint64_t meta = nslots * s->slot_bytes;
    if (meta >= cfg.arena_bytes) {
        const unsigned long long need = meta;
        destroy_resources(s);
        return fail(MMS_EINVAL, "arena of %llu bytes holds no data after %llu bytes of batch metadata",
                    (unsigned long long)cfg.arena_bytes, need);
    }
    for (uint64_t i = 0; i < nslots; ++i) {
        Slot sl;
        sl.dev_off = i * s->slot_bytes;
        s->slots.push_back(sl);
        s->free_slots.push_back((int)(nslots - 1 - i));
    }
    const uint64_t data = (cfg.arena_bytes - meta) / kAlign * kAlign;
    s->alloc.init(meta, data);
    s->cfg = cfg;
    s->cfg.num_streams = (uint32_t)S;
    s->stats.data_budget_bytes = data;
    s->stats.meta_bytes = meta;
    s->inflight.resize(S);
    s->cv_comp = std::vector<std::condition_variable>(S);
    s->scheduler = std::thread(scheduler_main, s);
    if (!s->dry)
        for (int i = 0; i < S; ++i) s->completers.emplace_back(completer_main, s, i);
    *out = s;
    return MMS_OK;
}

int mms_submit(mms_server* s, const mms_request* r, uint64_t* ticket) {
    if (!s || !r || !ticket) return fail(MMS_EINVAL, "null argument");
    *ticket = 0;
    if (r->flags & ~(MMS_PAIRS | MMS_KEY_I32)) return fail(MMS_EINVAL, "unknown request flags 0x%x", r->flags);
    if (r->n == 0) return fail(MMS_EINVAL, "empty request");
    if (r->n >= (1ull << 32)) return fail(MMS_EINVAL, "n = %llu exceeds 2^32-1", (unsigned long long)r->n);
    if (!r->d_keys || (is_pairs(*r) && !r->d_vals)) return fail(MMS_EINVAL, "null input pointer");
    if (!is_pairs(*r) && r->d_vals) return fail(MMS_EINVAL, "values given without MMS_PAIRS");
    uint64_t half, res, ws;
    footprint(*r, half, res, ws);
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->stopping) return fail(MMS_ESHUTDOWN, "server is shutting down");
    if (r->n > s->cfg.max_batch_keys) {
        ++s->stats.rejected;
        return fail(MMS_EINVAL, "n = %llu exceeds max_batch_keys %llu", (unsigned long long)r->n,
                    (unsigned long long)s->cfg.max_batch_keys);
    }
    if (res + ws > s->alloc.total()) {
        ++s->stats.rejected;
        return fail(MMS_ENOMEM, "request needs %llu bytes, the data budget is %llu",
                    (unsigned long long)(res + ws), (unsigned long long)s->alloc.total());
    }
    Req q;
    q.r = *r;
    q.t_submit = s->now_us();
    if (!s->dry && r->stream) {
        q.ready = take_event(s);
        if (!q.ready) return fail(MMS_EHIP, "event creation failed");
        hipError_t e = hipEventRecord(q.ready, (hipStream_t)r->stream);
        if (e != hipSuccess) {
            give_event(s, q.ready);
            return hip_fail(e, "record input event");
        }
    }
    const uint64_t t = s->next_ticket++;
    s->reqs.emplace(t, std::move(q));
    s->queue.push_back(t);
    ++s->stats.submitted;
    bump(s);
    *ticket = t;
    return MMS_OK;
}

int mms_poll(mms_server* s, uint64_t ticket, mms_result* out) {
    if (!s) return fail(MMS_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    return poll_locked(s, ticket, out);
}

int mms_wait(mms_server* s, uint64_t ticket, int64_t timeout_ms, mms_result* out) {
    if (!s) return fail(MMS_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto final_or_gone = [&] {
        auto it = s->reqs.find(ticket);
        return it == s->reqs.end() || it->second.st == St::Done || it->second.st == St::Failed;
    };
    if (timeout_ms < 0) s->cv_done.wait(lk, final_or_gone);
    else s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), final_or_gone);
    return poll_locked(s, ticket, out);
}

int mms_release(mms_server* s, uint64_t ticket, void* stream) {
    if (!s) return fail(MMS_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(MMS_ENOENT, "unknown or released ticket %llu", (unsigned long long)ticket);
    Req& q = it->second;
    if (q.st != St::Done && q.st != St::Failed)
        return fail(MMS_EINVAL, "ticket %llu is still pending", (unsigned long long)ticket);
    if (q.res_bytes) {
        hipEvent_t ev = nullptr;
        if (!s->dry && stream) {
            ev = take_event(s);
            if (ev && hipEventRecord(ev, (hipStream_t)stream) != hipSuccess) {
                give_event(s, ev);
                ev = nullptr;
                (void)hipStreamSynchronize((hipStream_t)stream);
            }
        }
        if (ev) s->deferred.push_back({ev, q.res_off, q.res_bytes});
        else s->alloc.release(q.res_off, q.res_bytes);
    }
    s->reqs.erase(it);
    --s->live_admitted;
    ++s->stats.released;
    bump(s);
    return MMS_OK;
}

int mms_server_get_stats(mms_server* s, mms_server_stats* out) {
    if (!s || !out) return fail(MMS_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->queued = s->queue.size();
    uint64_t running = s->admitted.size();
    for (auto& q : s->inflight)
        for (auto& b : q) running += b.tickets.size();
    out->running = running;
    out->used_bytes = s->alloc.used();
    return MMS_OK;
}

int mms_server_destroy(mms_server* s) {
    if (!s) return fail(MMS_EINVAL, "null server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        for (uint64_t t : s->queue) {
            Req& q = s->reqs[t];
            q.st = St::Failed;
            q.status = MMS_ESHUTDOWN;
            q.err = "server shut down before admission";
        }
        s->queue.clear();
        for (uint64_t t : s->admitted) {
            Req& q = s->reqs[t];
            s->alloc.release(q.res_off, q.res_bytes);
            s->alloc.release(q.ws_off, q.ws_bytes);
            q.res_bytes = q.ws_bytes = 0;
            q.st = St::Failed;
            q.status = MMS_ESHUTDOWN;
            q.err = "server shut down before launch";
        }
        s->admitted.clear();
        bump(s);
        s->cv_done.notify_all();
    }
    s->cv_sched.notify_all();
    if (s->scheduler.joinable()) s->scheduler.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop_completion = true;
        for (auto& c : s->cv_comp) c.notify_all();
    }
    for (auto& t : s->completers) t.join();
    destroy_resources(s);
    return MMS_OK;
}

}  // extern "C"
