/*
 * libpss -- Parallel Space Saving for the k-majority problem on one MI355X.
 *
 * The method is that of Cafaro, Pulimeno, Epicoco and Aloisio, "Parallel
 * Space Saving on Multi and Many-Core Processors" (arXiv 1606.04669):
 *   - the input array A of n items is cut into C contiguous blocks
 *     (Section 3, block distribution; Algorithm 1, bounds of the sub-array);
 *   - each block is summarised by sequential Space Saving with k counters
 *     (Section 3, second paragraph);
 *   - the block summaries are merged by COMBINE with Prune(k) (Algorithm 2)
 *     in a reduction (Algorithm 1, ParallelReduction);
 *   - the result is pruned to the items above the k-majority threshold
 *     (Algorithm 1, Pruned; Section 3: f >= floor(n/k) + 1).
 *
 * Conventions fixed by this library (the paper leaves them open):
 *   - items are uint32; every value, 0 and 0xFFFFFFFF included, is an item;
 *   - eviction takes the counter with the minimum count and, among those, the
 *     smallest item id; the new item gets count m+1 and error m;
 *   - a summary with fewer than k used counters has minimum m = 0;
 *   - COMBINE adds errors like counts; Prune(k) keeps the first k entries in
 *     the order (count descending, error ascending, item ascending), which is
 *     also the order of every result this library returns;
 *   - the reduction is a fixed binary tree over block index: at each level
 *     summaries 2j and 2j+1 are combined and an odd last one is promoted;
 *   - block c covers [floor(c*n/C), floor((c+1)*n/C)); C changes results and
 *     is reported back so that a CPU replay can reproduce them;
 *   - an item is reported iff count * k > N, where N is the stream length the
 *     summary covers.
 *
 * Memory: pointers named d_* are device pointers (HIP device memory, e.g. a
 * torch tensor's data_ptr()), owned by the caller and required to stay valid
 * until the work queued on `stream` has finished.  Pointers named h_* are
 * host pointers owned by the caller.  Contexts and summaries own their device
 * memory.  `stream` is a hipStream_t (NULL = the null stream).
 *
 * Errors: every int-returning function returns PSS_OK (0) or a negative
 * PSS_E* code and never throws.  A failed call leaves summaries unchanged.
 * Updates and merges are all or nothing also when the failure is found on
 * the device after the call has returned (a block whose internal invariant
 * check fails): the summary's entries and its N stay as they were, and the
 * next pss_query on it returns PSS_EDEVICE once (later queries see the
 * unchanged summary).
 * Handles are not thread-safe: serialise calls on one summary or context.
 * A context's workspace (block summaries, scratch) is shared by the calls
 * made with it: queue them on one stream, or synchronise between calls made
 * on different streams.
 */
#ifndef PSS_H
#define PSS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One reported entry (24 bytes, host memory). */
typedef struct {
    uint32_t item;     /* the item id */
    uint32_t reserved; /* always 0 */
    uint64_t count;    /* estimated frequency f^ (>= true frequency) */
    uint64_t error;    /* error bound e: count - error <= true frequency */
} pss_entry;

typedef struct pss_ctx pss_ctx;         /* one HIP device, workspace, tuning */
typedef struct pss_summary pss_summary; /* one device-resident summary of k counters */

enum {
    PSS_OK = 0,
    PSS_EINVAL = -1,  /* null handle/pointer, k < 2, kind unknown, k mismatch */
    PSS_ERANGE = -2,  /* size outside what the call supports (e.g. k > n in pss_run) */
    PSS_ENOMEM = -3,  /* device or host allocation failed */
    PSS_EBUSY = -4,   /* resource limit reached; retry later */
    PSS_ETRUNC = -5,  /* h_out too small: *n_out holds the required count */
    PSS_EDEVICE = -6  /* a HIP runtime call or kernel launch failed */
};

enum {
    PSS_Q_MAJORITY = 0, /* entries with count * k > N, canonical order */
    PSS_Q_TOPK = 1      /* the first `cap` entries in canonical order */
};

/* Largest k this library accepts (2^20; 0 for a null ctx).  Above
 * pss_max_lds_k() a block's state (hash, counters, minimum-level list) lives
 * in a device-memory slab instead of LDS; results are the same either way. */
uint32_t pss_max_k(const pss_ctx* ctx);

/* Largest k whose block state fits one workgroup's LDS on this context's
 * device (0 for a null ctx). */
uint32_t pss_max_lds_k(const pss_ctx* ctx);

/* Create a context on HIP device `device`.  *out receives the handle.
 * Returns PSS_EINVAL (bad device / null out), PSS_EDEVICE or PSS_ENOMEM. */
int pss_ctx_create(int device, pss_ctx** out);

/* Release a context and its workspace.  Summaries created from it must be
 * destroyed first.  NULL is accepted. */
void pss_ctx_destroy(pss_ctx* ctx);

/* Limit the device memory the context's workspaces (block summaries, block
 * scratch, COMBINE and report scratch) may hold in all to `bytes` (0 = no
 * limit).  A call that would grow them beyond it returns PSS_ENOMEM before
 * queueing any work, so summaries are left unchanged.  Workspace already
 * held is kept.  Returns PSS_EINVAL for a null ctx. */
int pss_ctx_set_budget(pss_ctx* ctx, uint64_t bytes);

/* Chunk count the library picks for n items and k counters when a call is
 * given chunks = 0 (a deterministic function of n, k and the device). */
uint32_t pss_plan_chunks(const pss_ctx* ctx, uint64_t n, uint32_t k);

/* Autotuner for the chunk count C (Algorithm 1's number of blocks), the one
 * parameter that changes results: times the block summaries and the
 * reduction tree over d_items[0, n) with k counters for C in {P/4, P/2, P,
 * 2P}, P = pss_plan_chunks(n, k) (with block state in device memory, none
 * beyond the planner's 16-GiB state budget; one warm-up and the best of two
 * timed runs each), and returns the fastest in *best_chunks (its time in *best_ms, may
 * be NULL).  Pass the result as `chunks` to pss_update / pss_run and record
 * it: a CPU replay with the same C reproduces the results.  Every call
 * times afresh (the best C depends on the data).  Blocks until done; uses the
 * context's workspace.  PSS_ERANGE for n = 0, n >= 2^32 - 128 or k > pss_max_k(). */
int pss_tune_chunks(pss_ctx* ctx, const uint32_t* d_items, uint64_t n, uint32_t k, void* stream,
                    uint32_t* best_chunks, double* best_ms);

/* Create an empty summary with k counters (2 <= k <= pss_max_k()).
 * Empty means N = 0 and no monitored items: the identity of COMBINE. */
int pss_create(pss_ctx* ctx, uint32_t k, pss_summary** out);

/* Release a summary (after the work queued on it has finished).  NULL is
 * accepted. */
void pss_destroy(pss_summary* s);

/* Append n items (device array d_items, n < 2^32 - 128) to summary s:
 *   B = fixed-tree COMBINE of the Space Saving summaries of C blocks of
 *       d_items (Algorithm 1 up to the reduction), then S <- COMBINE(S, B)
 *       and N <- N + n.
 * chunks = C (0: pss_plan_chunks).  *chunks_used (may be NULL) receives C.
 * Asynchronous on `stream`.  n = 0 is a no-op. */
int pss_update(pss_summary* s, const uint32_t* d_items, uint64_t n, uint32_t chunks, void* stream,
               uint32_t* chunks_used);

/* dst <- COMBINE(dst, src) (Algorithm 2), N(dst) <- N(dst) + N(src).
 * Both summaries must have the same k (else PSS_EINVAL).  Asynchronous.
 * N lives on the device with the summary: a merge queued after an update
 * sees the N that update produced. */
int pss_merge(pss_summary* dst, const pss_summary* src, void* stream);

/* Query a summary; blocks until the result is on the host.
 * kind PSS_Q_MAJORITY: the entries with count * k > N (Algorithm 1, Pruned);
 *      if more than cap qualify, returns PSS_ETRUNC with *n_out = required.
 * kind PSS_Q_TOPK: the first min(cap, size) entries.
 * Entries are in canonical order.  *stream_len (may be NULL) receives N.
 * Returns PSS_EDEVICE (once) when an earlier update or merge on s found a
 * failed block and was not applied; s and N are then as before that call. */
int pss_query(const pss_summary* s, int kind, pss_entry* h_out, uint32_t cap, uint32_t* n_out,
              uint64_t* stream_len, void* stream);

/* ParallelSpaceSaving(A, n, C, k) (Algorithm 1) in one call: the k-majority
 * candidates of the device array d_items[0, n), written to h_out (cap
 * entries) in canonical order, *n_out = number reported.  Requires
 * 2 <= k <= n < 2^32 - 128 (PSS_ERANGE otherwise).  chunks = 0 picks C; *chunks_used (may
 * be NULL) receives it.  Blocks until the result is on the host. */
int pss_run(pss_ctx* ctx, const uint32_t* d_items, uint64_t n, uint32_t k, uint32_t chunks,
            pss_entry* h_out, uint32_t cap, uint32_t* n_out, uint32_t* chunks_used, void* stream);

/* Inspection of the first step: runs the block summaries of d_items[0, n)
 * for C = chunks blocks (same kernel launch as pss_update) and copies the
 * summaries of the nsel blocks listed in h_sel to the host: block h_sel[i]
 * goes to h_out[i*k ...] (unordered entries), its size to h_sizes[i] and its
 * minimum (0 when not full) to h_mins[i].  PSS_ERANGE for n >= 2^32 - 128.
 * Blocks until done. */
int pss_block_summaries(pss_ctx* ctx, const uint32_t* d_items, uint64_t n, uint32_t k, uint32_t chunks,
                        const uint32_t* h_sel, uint32_t nsel, pss_entry* h_out, uint32_t* h_sizes,
                        uint64_t* h_mins, void* stream);

/* pss_run without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the same computation and result as pss_run with the
 * same C, on the calling thread's current HIP device, asynchronous on
 * `stream`, with the result left in device memory:
 *   d_out  -- device array of cap pss_entry (caller-owned): the first
 *             min(q, cap) reported entries in canonical order;
 *   d_nout -- device uint32 (caller-owned): q, the number of entries with
 *             count * k > n, or 0xFFFFFFFF when a block failed an internal
 *             check (then d_out is not written);
 *   *chunks_used (host, may be NULL) -- C.
 * Its workspace is one fixed device array per GPU (pss_noalloc_scratch_bytes,
 * 128 MiB), taken at the first call on each device and held until the
 * process ends; no call allocates anything.  Every call on a GPU shares that
 * GPU's array: calls that overlap on one GPU (other streams, other threads)
 * race and must be serialised by the caller.
 * Limits (PSS_ERANGE otherwise): 2 <= k <= n < 2^32 - 128; k within the LDS
 * limit (pss_max_lds_k); the C blocks' summaries and error scratch,
 * C * (12 k + 8) + 4 C * ceil32(slots(k)) bytes with about 1.7 k + 64 hash
 * slots, within the array (e.g. k = 2000: C <= 3,500).  chunks = 0 picks
 * pss_plan_chunks' count, lowered to fit.  PSS_EINVAL for null pointers. */
int pss_run_noalloc(const uint32_t* d_items, uint64_t n, uint32_t k, uint32_t chunks, pss_entry* d_out,
                    uint32_t cap, uint32_t* d_nout, uint32_t* chunks_used, void* stream);

/* Size in bytes of pss_run_noalloc's per-device workspace array. */
uint64_t pss_noalloc_scratch_bytes(void);

/* Measurement helper: the read bandwidth (GB/s, 10^9 bytes/s) a plain
 * streaming kernel reaches over the device buffer d_buf[0, bytes) (16-byte
 * aligned), the best of `reps` timed launches after a warm-up; the
 * reference the block kernel's read roofline is compared against next to
 * the published peak.  Reads only; uses the context's report buffer as a
 * (never written) sink.  Blocks until done. */
int pss_read_bandwidth(pss_ctx* ctx, const void* d_buf, uint64_t bytes, uint32_t reps, void* stream, double* gbps);

/* Test hook for the all-or-nothing contract above: queue on `stream` a fold
 * into s of a block summary that carries the failure mark a block kernel
 * writes when one of its internal checks fails, as if an update of n items
 * had produced it.  s and its N must stay as they were, and the next
 * pss_query on s must return PSS_EDEVICE.  Uses the context's workspace. */
int pss_test_fold_failed_block(pss_summary* s, uint64_t n, void* stream);

/* ---- Frequent (Misra-Gries) in the same pipeline ----
 *
 * Section 2 of the paper names Frequent as the counter-based summary whose
 * parallel merge the authors built before Space Saving.  For the k-majority
 * problem it keeps k - 1 counters: a monitored item adds 1; an unmonitored
 * one takes a free counter with count 1, else every counter loses 1 (those
 * at 0 are freed) and the item is dropped; D counts these decrement steps,
 * so f - D <= count <= f and D * k <= n.  Summaries merge by adding the
 * counts of the union and, beyond k - 1 items, subtracting the k-th largest
 * count c from all and keeping the positive ones (D = D1 + D2 + c).  The
 * parallel form is Algorithm 1 with this merge: the same blocks for the same
 * C, the same fixed tree; results depend only on n, k and C.  Entries carry
 * error 0 (D bounds every entry). */

/* Largest k of the Frequent path on this context's device (its block state,
 * merges and report in LDS); 0 for a null ctx. */
uint32_t pss_frequent_max_k(const pss_ctx* ctx);

/* Chunk count pss_frequent_run picks for n items and k counters when given
 * chunks = 0: pss_plan_chunks' rule applied to the Frequent block kernel,
 * whose per-block LDS footprint differs (a deterministic function of n, k
 * and the device; 1 for a null ctx). */
uint32_t pss_frequent_plan_chunks(const pss_ctx* ctx, uint64_t n, uint32_t k);

/* Parallel Frequent over the device array d_items[0, n), k - 1 counters per
 * block, C = chunks blocks (0: pss_frequent_plan_chunks).  kind PSS_Q_MAJORITY: the
 * entries with (count + D) * k > n (every true k-majority item is among
 * them), PSS_ETRUNC with *n_out = required when more than cap; kind
 * PSS_Q_TOPK: the first min(cap, size) entries of the merged summary.  Order:
 * count descending, item ascending.  *h_decrements (may be NULL) receives
 * the merged summary's D, *chunks_used (may be NULL) C.  Requires
 * 2 <= k <= n < 2^32 - 128 and k <= pss_frequent_max_k() (else PSS_ERANGE).
 * Blocks until the result is on the host; uses the context's workspace.
 * With pss_timing_enable, its phases count as block summaries (0), tree
 * (1) and report (3) in pss_phase_times. */
int pss_frequent_run(pss_ctx* ctx, const uint32_t* d_items, uint64_t n, uint32_t k, uint32_t chunks, int kind,
                     pss_entry* h_out, uint32_t cap, uint32_t* n_out, uint64_t* h_decrements, uint32_t* chunks_used,
                     void* stream);

/* Frequent block summaries (before the tree) of the nsel blocks listed in
 * h_sel: entries of block h_sel[i] to h_out + i*k (any order, error 0), its
 * size (<= k - 1) to h_sizes[i], its D to h_decrements[i].  Blocks until
 * done. */
int pss_frequent_block_summaries(pss_ctx* ctx, const uint32_t* d_items, uint64_t n, uint32_t k, uint32_t chunks,
                                 const uint32_t* h_sel, uint32_t nsel, pss_entry* h_out, uint32_t* h_sizes,
                                 uint64_t* h_decrements, void* stream);

/* ---- Batched form: many independent streams in one graph launch ----
 *
 * Stream s is the device array h_items[s][0, h_lens[s]) with k = h_ks[s]
 * counters; its result is exactly that of pss_run on it with
 * C = h_chunks[s] (Algorithm 1 with Algorithm 2 as the reduction): the batch
 * changes scheduling only.  Requires 2 <= k_s <= n_s, n_s < 2^32 - 128 and
 * k_s <= pss_batch_max_k() (PSS_ERANGE otherwise). */
typedef struct pss_batch pss_batch;

typedef struct {
    uint32_t nstreams, nblocks, nlevels, nclasses;
    uint64_t target_len;      /* tuned block length (items) */
    uint32_t slots_x16;       /* tuned hash slots per counter x16 (0 = per-k default) */
    uint32_t waves_per_group; /* tuned waves per workgroup of the block kernels */
    uint32_t tune_candidates; /* configurations the autotuner timed */
    double tune_ms;           /* time spent tuning */
    uint64_t report_entries;  /* sum of k_s: size of h_out in pss_batch_run */
} pss_batch_info_t;

/* Largest k a batched stream may have on this context (block state and a
 * COMBINE both in LDS). */
uint32_t pss_batch_max_k(const pss_ctx* ctx);

/* Plan a batch.  h_items (host array of nstreams device pointers, each to be
 * kept valid for the life of the batch), h_lens, h_ks: the streams.
 * h_chunks[s]: C_s, or 0 to let the autotuner choose it; on success every
 * entry holds the C_s used (record them to reproduce results).  tune != 0
 * also tunes the result-neutral knobs when every C_s is given.  The
 * autotuner times candidate configurations (block length, hash load factor,
 * waves per workgroup) on a sample of the streams; the chosen launch
 * sequence is captured into a HIP graph. */
int pss_batch_create(pss_ctx* ctx, uint32_t nstreams, const uint32_t* const* h_items, const uint64_t* h_lens,
                     const uint32_t* h_ks, uint32_t* h_chunks, int tune, pss_batch** out);

/* Run a batch (graph replay, or eager launches when eager != 0) on `stream`
 * and wait for it.  Stream s's reported entries (count * k_s > n_s, canonical
 * order) go to h_out[o_s ...] with o_s = k_0 + ... + k_{s-1}; their number
 * to h_counts[s].  h_out holds report_entries entries. */
int pss_batch_run(pss_batch* b, int eager, pss_entry* h_out, uint32_t* h_counts, void* stream);

/* The plan's shape and tuning. */
int pss_batch_info(const pss_batch* b, pss_batch_info_t* info);

/* Release a batch (waits for the device).  NULL is accepted. */
void pss_batch_destroy(pss_batch* b);

/* create + run + destroy in one call (no tuning of given C_s). */
int pss_run_batched(pss_ctx* ctx, uint32_t nstreams, const uint32_t* const* h_items, const uint64_t* h_lens,
                    const uint32_t* h_ks, uint32_t* h_chunks, pss_entry* h_out, uint32_t* h_counts, void* stream);

/* ---- Served form: a pool of device-resident summaries and a request loop ----
 *
 * Summary sid (k = h_ks[sid] counters, starting empty) lives in device
 * memory for the life of the server.  An append of n items is exactly
 * pss_update on that summary (B = fixed-tree COMBINE of the Space Saving
 * summaries of the C blocks of the items, then S <- COMBINE(S, B),
 * N <- N + n); a query is pss_query.  Requests on one summary take effect in
 * submission order.  A server thread batches pending requests into launches
 * (continuous batching: requests that arrive while launches run are admitted
 * into the next launch as slots and memory free up), several launches in
 * flight at once; device memory for staged items and launch workspace is
 * bounded by opts.hbm_budget. */
typedef struct pss_server pss_server;

typedef struct {
    uint64_t hbm_budget;   /* device bytes for staged items + launch workspace (0: 64 GiB), split over slots */
    uint32_t slots;        /* launches in flight (0: 2; at most 8) */
    uint32_t max_requests; /* requests per launch (0: 4096) */
    uint64_t block_len;    /* target block length for appends with chunks = 0 (0: 16384) */
    uint64_t stage_bytes;  /* pinned host staging per slot, allocated at creation; a launch's
                              items fit it unless one append alone is larger (0: 256 MiB) */
} pss_server_opts;

typedef struct {
    int status;            /* PSS_OK or the error the request ended with */
    uint32_t n_out;        /* entries reported (majority: before truncation to cap) */
    uint64_t stream_len;   /* N of the summary after this append / at this query */
    uint32_t chunks_used;  /* C of an append (record it to reproduce results) */
    uint32_t launch;       /* the launch that ran the request (0: none needed) */
    double latency_ms;     /* submission to completion */
    double queue_ms;       /* submission to admission into a launch */
} pss_server_result;

typedef struct {
    uint64_t launches, requests, items_appended;
    uint32_t max_launch_requests, pending;
    int status;            /* PSS_OK, or the error that stopped the server */
    double stage_ms;       /* host time copying append items into pinned staging */
    double gpu_ms;         /* device time of the launches (copies included; launches overlap) */
} pss_server_stats_t;

/* Largest k a served summary may have on this context. */
uint32_t pss_server_max_k(const pss_ctx* ctx);

/* Start a server with nsummaries empty summaries (k = h_ks[i]; 2 <= k <=
 * pss_server_max_k(), else PSS_EINVAL / PSS_ERANGE).  opts may be NULL. */
int pss_server_create(pss_ctx* ctx, uint32_t nsummaries, const uint32_t* h_ks, const pss_server_opts* opts,
                      pss_server** out);

/* Finish every submitted request, stop the thread, release the pool. */
void pss_server_destroy(pss_server* srv);

/* Submit an append of h_items[0, n) (host memory, caller-owned, valid until
 * the ticket completes) to summary sid with C = chunks blocks (0: chosen from
 * opts.block_len, reported by pss_server_wait).  Returns at once with
 * *ticket.  PSS_ERANGE if n >= 2^32 - 128 or the append can never fit the budget. */
int pss_server_append(pss_server* srv, uint32_t sid, const uint32_t* h_items, uint64_t n, uint32_t chunks,
                      uint64_t* ticket);

/* Submit a query of summary sid (kind as pss_query; cap bounds a top query).
 * Returns at once with *ticket. */
int pss_server_query(pss_server* srv, uint32_t sid, int kind, uint32_t cap, uint64_t* ticket);

/* Wait for a ticket (each ticket once): fills *res and, for a query, up to
 * cap entries of h_out (canonical order).  Returns the request's status, or
 * PSS_ETRUNC for a majority query with more than cap entries, or PSS_EINVAL
 * for an unknown ticket. */
int pss_server_wait(pss_server* srv, uint64_t ticket, pss_entry* h_out, uint32_t cap, pss_server_result* res);

/* Counters of the server since it started. */
int pss_server_stats(pss_server* srv, pss_server_stats_t* st);

/* Phase timing.  While enabled, pss_update, pss_run and pss_query record HIP
 * events on the call's stream around each phase: 0 = block summaries
 * (chunk_summary kernel), 1 = COMBINE tree, 2 = fold into the summary,
 * 3 = report (extract kernel and copy to the host).  pss_phase_times waits
 * for the recorded events, writes the accumulated milliseconds (ms[4]) and
 * launch counts (launches[4]) since the last reset, and resets them when
 * reset != 0.  Returns PSS_EINVAL for a null ctx. */
int pss_timing_enable(pss_ctx* ctx, int enable);
int pss_phase_times(pss_ctx* ctx, double* ms, uint32_t* launches, int reset);

/* Static description of an error code. */
const char* pss_strerror(int code);

/* Diagnostics for PSS_EDEVICE: the hipError_t of the last failed kernel
 * launch (or launch-side runtime call) that a call made on this host thread
 * turned into PSS_EDEVICE (0 if none; invariant failures that a kernel
 * reports in its output are not recorded), and the HIP name of a hipError_t
 * value (a static string).  The server's own launches run on its thread and
 * report PSS_EDEVICE through their requests. */
int pss_last_device_error(void);
const char* pss_device_error_name(int hip_error);

#ifdef __cplusplus
}
#endif

#endif /* PSS_H */
