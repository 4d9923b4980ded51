/*
 * mms.h — C ABI of libmms, a multiway mergesort of 32-bit keys and stable
 * key-value pairs on an AMD Instinct MI355X (gfx950).
 *
 * Method: Casanova, Iacono, Karsin, Sitchinava, Weichert, "An Efficient
 * Multiway Mergesort for GPU Architectures" (arXiv 1702.07961).  A sort is a
 * base-case pass that sorts tiles of T keys on chip (§4.3), followed by
 * ceil(log_K(ceil(n/T))) merge rounds (§6.2); each round splits every group
 * of K sorted runs into independent output tiles at exact split indices
 * (§4.1, parallel partitioning) and merges each tile's K pieces through LDS
 * (§4.2, I/O-efficient merging; §7 names this partition-then-merge variant).
 *
 * Conventions shared by every call:
 *   - Return value: an MMS_* status.  A negative status leaves a message in
 *     the calling thread's mms_last_error().  No C++ exception crosses the ABI.
 *   - Device pointers ("d_") are HIP device allocations owned by the caller;
 *     the library never frees caller memory.  Host pointers ("h_") are read
 *     during the call only.
 *   - Asynchrony: work is enqueued on the caller's stream (a hipStream_t
 *     passed as void*, NULL = the null stream).  The call returns after
 *     enqueueing; buffers must stay valid until that work completes.  Errors
 *     detected while enqueueing are returned; a fault inside a kernel
 *     surfaces as MMS_EHIP at the next synchronising call.
 *   - Sizes: n counts elements.  n == 0 is a no-op returning MMS_OK.
 *     n >= 2^32 returns MMS_EINVAL (positions are 32-bit on the device).
 */
#ifndef MMS_H
#define MMS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MMS_OK 0
#define MMS_PENDING 1
#define MMS_EINVAL (-1)
#define MMS_ENOMEM (-2)
#define MMS_EHIP (-3)
#define MMS_ENOENT (-4)
#define MMS_ESHUTDOWN (-5)

/* flags */
#define MMS_PAIRS 0x1u    /* workspace sizing: key-value pairs                */
#define MMS_KEY_I32 0x2u  /* keys are int32 (signed order) instead of uint32  */
#define MMS_KEY_I64 0x4u  /* 64-bit keys are int64 (signed order)             */
#define MMS_KEYS64 0x8u   /* plan / workspace sizing: 64-bit keys (and values) */
#define MMS_MERGEPATH 0x10u /* plan / workspace sizing: the merge-path baseline */

/* Message for the last failing call on this thread ("" if none). */
const char* mms_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int mms_version(void);

/*
 * Sort plan (host only, no device work): the tile and fan-out parameters the
 * sort of n elements will use and the number of global-memory passes, which
 * is 1 (base case) + rounds, rounds = ceil(log_K(ceil(n / tile))) (§6.2).
 */
typedef struct {
    uint64_t n;
    uint32_t flags;
    uint32_t tile;          /* base-case tile size T in elements            */
    uint32_t lanes_per_tile;/* threads of one base-case workgroup            */
    uint32_t fanout;        /* merge fan-out K                              */
    uint32_t merge_tile;    /* output tile of one merge workgroup           */
    uint32_t rounds;        /* merge rounds                                  */
    uint32_t passes;        /* 1 + rounds                                   */
    uint64_t workspace_bytes;
} mms_plan_t;

int mms_plan(uint64_t n, uint32_t flags, mms_plan_t* out);

/* Bytes of device workspace the sort of n elements needs (flags: MMS_PAIRS). */
size_t mms_workspace_bytes(uint64_t n, uint32_t flags);

/*
 * Sort n keys ascending (§4: the problem statement; the result is the sorted
 * multiset).  d_in and d_out hold n uint32 (int32 with MMS_KEY_I32); they
 * may be the same buffer, but must not partially overlap.  d_ws is a device
 * buffer of at least mms_workspace_bytes(n, flags) bytes, 256-byte aligned,
 * not overlapping d_in or d_out.  Errors: MMS_EINVAL (bad pointer, size,
 * flags, overlap or workspace), MMS_EHIP (launch failure).
 */
int mms_sort_u32(const uint32_t* d_in, uint32_t* d_out, uint64_t n,
                 void* d_ws, size_t ws_bytes, uint32_t flags, void* stream);

/*
 * Stable sort of n (key, value) pairs by key: equal keys keep their input
 * order, so the output is unique (the order of (key, input index) pairs).
 * Same rules as mms_sort_u32; workspace from
 * mms_workspace_bytes(n, flags | MMS_PAIRS).  d_kin may equal d_kout and
 * d_vin may equal d_vout.
 */
int mms_sort_pairs_u32(const uint32_t* d_kin, const uint32_t* d_vin,
                       uint32_t* d_kout, uint32_t* d_vout, uint64_t n,
                       void* d_ws, size_t ws_bytes, uint32_t flags, void* stream);

/*
 * 64-bit keys (§6.3 also sorts 8-byte integers): the same method on 64-bit
 * keys, and stable pairs of 64-bit keys and 64-bit values.
 *
 * mms_sort_u64 sorts n keys ascending: uint64 order, or int64 order with
 * MMS_KEY_I64.  mms_sort_pairs_u64 sorts n (key, value) pairs stably by key
 * (equal keys keep their input order, so the result is unique).  d_in /
 * d_out (d_kin / d_kout, d_vin / d_vout) hold n 8-byte elements and may be
 * the same buffer, but must not partially overlap; keys and values must not
 * overlap each other.  d_ws holds at least
 * mms_workspace_bytes(n, MMS_KEYS64 [| MMS_PAIRS]) bytes, 256-byte aligned,
 * disjoint from the data; mms_plan with MMS_KEYS64 reports the tile, fan-out
 * and passes.  Asynchronous on `stream` like every sort.  Errors:
 * MMS_EINVAL (pointers, overlap, workspace, flags other than MMS_KEY_I64,
 * n >= 2^32), MMS_EHIP (launch failure).
 */
int mms_sort_u64(const uint64_t* d_in, uint64_t* d_out, uint64_t n,
                 void* d_ws, size_t ws_bytes, uint32_t flags, void* stream);
int mms_sort_pairs_u64(const uint64_t* d_kin, const uint64_t* d_vin,
                       uint64_t* d_kout, uint64_t* d_vout, uint64_t n,
                       void* d_ws, size_t ws_bytes, uint32_t flags, void* stream);

/*
 * Baseline for comparison, not the paper's method: a pairwise merge-path
 * mergesort of the kind the paper measures against (§1 and §6.4: two-way
 * merges in which every thread finds its start on the merge path by binary
 * search and merges its outputs one at a time from shared memory, at
 * addresses that depend on the keys, so bank conflicts depend on the input).
 * Tiles of 3840 keys (256 threads x 15) are sorted in a workgroup by
 * per-thread sorts and eight levels of such merges; then ceil(log2(tiles))
 * merge passes follow, each a partition launch and a merge launch.  Keys
 * only, ascending: uint32, or int32 with MMS_KEY_I32.  Same buffer rules as
 * mms_sort_u32; d_ws holds mms_workspace_bytes(n, MMS_MERGEPATH) bytes.
 * Errors: MMS_EINVAL, MMS_EHIP.
 */
int mms_sort_mergepath_u32(const uint32_t* d_in, uint32_t* d_out, uint64_t n,
                           void* d_ws, size_t ws_bytes, uint32_t flags, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that forbid allocation): mms_sort_u32 without a
 * workspace argument.  The workspace is a fixed array of
 * MMS_NOALLOC_SCRATCH_BYTES bytes of device memory inside the library, one
 * copy on each GPU it runs on, held until the process ends; the call itself
 * allocates nothing (its first call on a device looks up that device's copy).
 * Sorts n keys ascending exactly as mms_sort_u32 does (uint32, or int32 with
 * MMS_KEY_I32), on `stream`, with the same buffer rules.  Every call on one
 * GPU shares that GPU's array, so calls whose work may overlap on one GPU
 * (other streams, other threads) race; serialise them.  Errors: MMS_EINVAL
 * (flags, pointers, overlap, n >= 2^32, or n whose workspace,
 * mms_workspace_bytes(n, flags), exceeds MMS_NOALLOC_SCRATCH_BYTES: about
 * 1.6e7 keys), MMS_EHIP (launch failure).
 */
#define MMS_NOALLOC_SCRATCH_BYTES (64ull << 20)
int mms_sort_u32_noalloc(const uint32_t* d_in, uint32_t* d_out, uint64_t n, uint32_t flags, void* stream);

/*
 * §4.1 parallel partitioning on its own: split indices of groups of K sorted
 * runs at given ranks.  The n elements of d_keys form groups of K runs laid
 * out back to back: run k of group g starts at g*K*run_len + k*run_len and
 * has min(run_len, remaining) elements (so only the last group may be short
 * or hold fewer than K runs).  For each query q < nqueries, with group
 * d_group[q] and rank d_rank[q] (0 <= rank <= size of that group),
 * d_split[q*K + k] receives the number of elements of run k among the first
 * `rank` elements of the group's merged order, where equal keys are ordered
 * by (run index, position); entries for runs the group lacks are 0.  Runs
 * must be sorted in the key order that flags select.  d_group, d_rank
 * (uint64) and d_split (uint32, nqueries*K) are device buffers.
 * Errors: MMS_EINVAL for K outside [1, 16], run_len == 0 or n >= 2^32.
 * A query whose group or rank is out of range yields an all-0xFFFFFFFF row.
 */
int mms_partition_u32(const uint32_t* d_keys, uint64_t n, uint64_t run_len, uint32_t K,
                      const uint64_t* d_group, const uint64_t* d_rank, uint64_t nqueries,
                      uint32_t* d_split, uint32_t flags, void* stream);

/*
 * Streaming copy of n uint32 (d_in -> d_out), the bandwidth probe the
 * sort's passes are compared with.  Buffers must not overlap.
 */
int mms_copy_u32(const uint32_t* d_in, uint32_t* d_out, uint64_t n, void* stream);

/*
 * Batched (segmented) sort: every segment s = [h_offsets[s], h_offsets[s+1])
 * of the arrays is sorted on its own, exactly as mms_sort_u32 (keys only,
 * d_vin == d_vout == NULL) or mms_sort_pairs_u32 (stable) would sort it.
 * h_offsets is a host array of num_segs + 1 non-decreasing element offsets;
 * elements outside [h_offsets[0], h_offsets[num_segs]) are untouched, and
 * empty segments are allowed.  Each segment must hold fewer than 2^32
 * elements.  Buffers follow mms_sort_u32's aliasing rules over the whole
 * range; d_ws holds mms_segmented_workspace_bytes(...) bytes.
 *
 * All segments advance together: one launch per kernel and phase covers
 * every segment's tiles (the base case, then per round the partition and
 * the merge).  The first call with a given (offsets, pointers, flags,
 * tuning) captures those launches into a hipGraph, and later calls with the
 * same signature replay it with a single graph launch on `stream`.
 *
 * Memory: all device memory is the caller's.  The workspace holds the
 * ping-pong buffers, the partition table and the batch metadata (a 64-byte
 * descriptor per non-empty segment and 8 bytes per tile task).  The library
 * keeps, per captured signature (up to 8, least recently used evicted), a
 * host image of that metadata in pinned host memory, and every call copies
 * it into the workspace with an asynchronous copy on `stream` ahead of the
 * launches, so the workspace may be used for anything else between calls.
 * An evicted signature is torn down only after its last launch completes.
 * Errors: MMS_EINVAL (offsets decreasing, buffers, workspace), MMS_ENOMEM
 * (pinned staging of the metadata), MMS_EHIP (capture, copy or launch).
 */
size_t mms_segmented_workspace_bytes(const uint64_t* h_offsets, uint64_t num_segs, uint32_t flags);
int mms_segmented_sort(const uint32_t* d_kin, uint32_t* d_kout, const uint32_t* d_vin, uint32_t* d_vout,
                       const uint64_t* h_offsets, uint64_t num_segs, void* d_ws, size_t ws_bytes,
                       uint32_t flags, void* stream);

/*
 * Tuning table (written by the autotuner; §6.2 tunes K and the number of
 * workers per platform).  Entries are of one of two kinds, flags 0 for
 * keys-only sorts and MMS_PAIRS for key-value sorts; a kind with no entries
 * uses the keys-only ones.  A sort of n elements uses the first entry of its
 * kind with ceil(log2 n) <= max_log2_n, else the last one; a batched sort of
 * num_segs segments holding n elements in all uses the entry for n, with its
 * base tile capped at max(2048, n / num_segs) (shape 0 otherwise).
 *   fanout      merge fan-out K (power of two, 2..16)
 *   merge_tile  keys-only merge output tile (multiple of 256, 1024..8192;
 *               key-value merges use 4096 whatever the entry says)
 *   variant     keys-only merge kernel shape (0: 64x16-key blocks, 8 waves;
 *               1: 64x8-key blocks, 16 waves; 2: 64x8-key blocks, 8 waves;
 *               3: as 2 with two workgroups per compute unit, for merge tiles
 *               up to 7168; 4: the minBlockHeap of §4.2, one heap of
 *               64-key nodes per wave and one merge tile per wave)
 *   base        base-case shape, keys per lane x waves (§4.3's base case
 *               sorts one tile per workgroup): 0: 8 x 4, 1: 4 x 8, 2: 16 x 2,
 *               all 2048-key tiles; 3: 8 x 8 and 5: 16 x 4, 4096-key tiles;
 *               4: 8 x 16 and 6: 16 x 8, 8192-key tiles.  Key-value sorts
 *               use shape 3 for shape 4, shapes 0 and 3 as given, else 0.
 *   flags       0 or MMS_PAIRS, the kind
 * count == 0 restores the built-in default (K = 16, 8192, variant 0, base 0,
 * overridable by MMS_FANOUT / MMS_TOUT / MMS_MERGE_VARIANT /
 * MMS_BASE_SHAPE).  Workspace sizes depend on the table: query
 * mms_workspace_bytes after changing it.  mms_get_tuning reports the
 * parameters a sort of n elements of the kind `flags` selects.
 * Process-wide, thread-safe.
 */
typedef struct {
    uint32_t max_log2_n;
    uint32_t fanout;
    uint32_t merge_tile;
    uint32_t variant;
    uint32_t base;
    uint32_t flags;
} mms_tuning_t;

int mms_set_tuning(const mms_tuning_t* entries, uint32_t count);
int mms_get_tuning(uint64_t n, uint32_t flags, mms_tuning_t* out);

/*
 * Serving loop: a server owns a device arena (caller memory, e.g. a torch
 * tensor), admits sort requests first-come first-served while the arena has
 * room for them, and coalesces the admitted requests of one kind into
 * batched sorts (the segmented sort's kernels, one launch per phase over all
 * requests of the batch) on two or more streams, so that requests arriving
 * while earlier ones run join the next batch and their work overlaps on the
 * device.  Each result is the request sorted exactly as mms_sort_u32 /
 * mms_sort_pairs_u32 would sort it alone (§4's problem statement; stable for
 * pairs), and stays in the arena until mms_release.
 *
 * Memory: at creation the server reserves metadata slots (per-batch task
 * lists and partition tables) at the start of the arena; the rest is the
 * data budget.  A request of n elements needs 4n bytes for its result (8n
 * for pairs) plus as much again of workspace while it runs (none when n fits
 * one base-case tile), each rounded up to 256 bytes.  It is admitted when
 * every earlier request has been admitted and both ranges fit; the workspace
 * returns to the budget when its batch completes, the result on release.  A
 * request that could never fit the data budget is refused at submission
 * (MMS_ENOMEM).  The server calls no device allocator.
 *
 * Threads: a scheduler thread admits and launches; one completion thread per
 * stream waits for the batches of its stream in order and stamps their
 * requests.  Every call below is thread-safe except mms_server_destroy,
 * which must not overlap any other call on the same server.
 */
#define MMS_SERVER_MAX_STREAMS 8
#define MMS_SERVER_DRY_RUN 0x1u  /* run admission and completion with no device
                                    work: results are not computed, the arena is
                                    never dereferenced (scheduler tests) */

typedef struct {
    void* d_arena;              /* device buffer, 256-byte aligned, caller-owned  */
    uint64_t arena_bytes;
    void* streams[MMS_SERVER_MAX_STREAMS]; /* caller streams (hipStream_t); unused: NULL */
    uint32_t num_streams;       /* 0: the server creates 2 non-blocking streams   */
    uint32_t max_inflight;      /* batches enqueued and not complete, per stream (0: 2) */
    uint32_t max_requests;      /* requests admitted and not released (0: 65536) */
    uint32_t max_batch_requests;/* requests per batch (0: 1024)                  */
    uint64_t max_batch_keys;    /* elements per batch, also the largest request (0: 2^28) */
    uint32_t flags;             /* MMS_SERVER_DRY_RUN                             */
    uint32_t reserved;
} mms_server_cfg;

typedef struct mms_server mms_server;

typedef struct {
    uint32_t flags;             /* MMS_PAIRS (values present), MMS_KEY_I32        */
    uint32_t reserved;
    uint64_t n;                 /* elements, 1 <= n <= max_batch_keys            */
    const uint32_t* d_keys;     /* device input, caller-owned, unchanged          */
    const uint32_t* d_vals;     /* device input values (MMS_PAIRS), else NULL     */
    void* stream;               /* the input is read after the work enqueued on this
                                   stream before mms_submit (NULL: the caller has
                                   already synchronised it)                      */
} mms_request;

typedef struct {
    int32_t status;             /* MMS_OK, MMS_PENDING or a negative status       */
    uint32_t flags;
    uint64_t n;
    uint32_t* d_keys;           /* sorted keys inside the arena                   */
    uint32_t* d_vals;           /* permuted values (pairs), else NULL             */
    double t_submit_us;         /* host steady clock, µs since server creation    */
    double t_admit_us;
    double t_launch_us;
    double t_done_us;           /* stamped by the completion thread               */
    uint64_t batch;             /* sequence number of the batch it ran in         */
    uint32_t batch_requests;    /* requests in that batch                         */
    uint32_t stream_index;
} mms_result;

typedef struct {
    uint64_t submitted, admitted, completed, released, rejected, batches;
    uint64_t queued;            /* waiting for admission                          */
    uint64_t running;           /* admitted, not complete                         */
    uint64_t data_budget_bytes; /* arena bytes available to requests              */
    uint64_t used_bytes;        /* of which in use (results + workspaces)         */
    uint64_t peak_used_bytes;
    uint64_t meta_bytes;        /* arena bytes reserved for batch metadata        */
    uint64_t max_batch_seen;    /* largest batch so far (requests)                */
} mms_server_stats;

/* Create a server.  Errors: MMS_EINVAL (arena, limits, streams), MMS_EHIP. */
int mms_server_create(const mms_server_cfg* cfg, mms_server** out);

/* Queue a request and return its ticket (> 0).  Errors: MMS_EINVAL (flags,
 * n = 0, n > max_batch_keys, null pointers), MMS_ENOMEM (larger than the data
 * budget), MMS_ESHUTDOWN (the server is being destroyed). */
int mms_submit(mms_server* s, const mms_request* r, uint64_t* ticket);

/* State of a ticket: MMS_PENDING while queued or running, MMS_OK with the
 * result filled in when done, the request's error status if it failed,
 * MMS_ENOENT for an unknown or released ticket. */
int mms_poll(mms_server* s, uint64_t ticket, mms_result* out);

/* mms_poll that blocks until the ticket is done or timeout_ms passes
 * (negative: no limit); MMS_PENDING on timeout. */
int mms_wait(mms_server* s, uint64_t ticket, int64_t timeout_ms, mms_result* out);

/* Return a finished request's arena space.  With a non-NULL stream the space
 * is reused only after the work enqueued on that stream so far (readers of
 * the result) completes.  Errors: MMS_ENOENT (unknown or already released),
 * MMS_EINVAL (still pending). */
int mms_release(mms_server* s, uint64_t ticket, void* stream);

int mms_server_get_stats(mms_server* s, mms_server_stats* out);

/* Stop admitting (queued requests fail with MMS_ESHUTDOWN), wait for the
 * batches in flight, join the threads and free the server.  Arena contents
 * are left as they are. */
int mms_server_destroy(mms_server* s);

/*
 * Per-kernel timing, for measurement harnesses.  While enabled, every kernel
 * of a selected kind the library launches is bracketed by two hipEvents
 * recorded on the stream it is launched on, and mms_timing_read() waits for
 * those events and returns, per kernel kind, the number of launches and
 * their summed durations since the last reset.  Each timed launch costs two
 * event records (a few microseconds of stream time).  mms_timing_kinds()
 * selects the kinds (bit k for kind k; all kinds until it is called; a mask
 * with no known kind is rejected with MMS_EINVAL).  The state is
 * process-wide; calls are thread-safe.
 */
typedef enum {
    MMS_KERNEL_TILE_SORT = 0,  /* base case (§4.3)          */
    MMS_KERNEL_PARTITION = 1,  /* split indices (§4.1)      */
    MMS_KERNEL_MERGE = 2,      /* K-way merge (§4.2)        */
    MMS_KERNEL_COPY = 3,       /* bandwidth probe           */
    MMS_KERNEL_SEGMENTED = 4,  /* one batched graph launch  */
    MMS_KERNEL_KINDS = 5
} mms_kernel_kind;

typedef struct {
    uint64_t launches[MMS_KERNEL_KINDS];
    double total_ms[MMS_KERNEL_KINDS];
} mms_timing_t;

int mms_timing_enable(int on);
int mms_timing_kinds(uint32_t mask);
int mms_timing_reset(void);
int mms_timing_read(mms_timing_t* out);

#ifdef __cplusplus
}
#endif

#endif /* MMS_H */
