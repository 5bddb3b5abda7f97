// Served Parallel Space Saving: a pool of device-resident summaries and a
// request loop with continuous batching.
//
// An append to summary S with items A is S <- COMBINE(S, B), N <- N + |A|,
// where B is the fixed-tree COMBINE of the Space Saving summaries of the
// blocks of A (Algorithm 1 up to the reduction, Algorithm 2 as the operator)
// -- exactly what pss_update does.  A query reports S (count * k > N, or the
// first `cap` entries) in the canonical order.  Requests on one summary take
// effect in submission order.
//
// A server thread admits pending requests into launches: a launch takes, in
// submission order, requests whose summary has no earlier request still
// waiting, at most one per summary, while the launch's staging memory and
// workspace fit its share of the device-memory budget.  A launch copies its
// appends' items to the device in one transfer, runs the block kernels of all
// its appends (one persistent launch per k size class), one tree launch per
// level, one fold launch and one query launch, and copies the query results
// back.  Several launches are in flight at once (one per slot, each on its
// own stream); a launch touching a summary that an in-flight launch also
// touches waits for it on the device.  New requests are admitted as soon as a
// slot frees up, so work that arrives while the GPU is busy joins the next
// launch instead of waiting for the queue to drain.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <string.h>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "pss.h"
#include "pss_ctx.h"
#include "pss_kernels.h"
#include "pss_layout.h"

using namespace pss;

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

constexpr uint32_t kSrvClasses = 7;
// Pending requests a launch may pass over (blocked or too large) before it
// stops looking further down the queue.
constexpr size_t kScanLimit = 65536;

enum ReqType { kAppend = 0, kQuery = 1 };

struct Request {
    uint64_t ticket = 0;
    int type = kAppend;
    uint32_t sid = 0;
    const uint32_t* items = nullptr;  // host, caller-owned until done
    uint64_t n = 0;
    uint32_t chunks = 0;
    int kind = 0;
    uint32_t cap = 0;
    Clock::time_point t_submit, t_launch, t_done;
    // results
    bool done = false;
    int rc = PSS_OK;
    uint64_t stream_len = 0;  // N after the append / at the query
    uint32_t launch = 0;
    std::vector<pss_entry> out;
    uint32_t n_out = 0;
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    hipEvent_t t0 = nullptr, t1 = nullptr;  // device time of the launch
    bool busy = false;
    uint64_t seq = 0;  // launch number running on the slot
    std::vector<Request*> reqs;
    DeviceBuffer dev;        // staged items, block summaries, descriptors, query output
    void* pin = nullptr;     // host staging (items + descriptors), then query output
    size_t pin_bytes = 0;
    // layout of the current launch in `dev` / `pin`
    size_t off_items = 0, off_desc = 0, desc_bytes = 0, off_out = 0, out_bytes = 0;
    uint32_t nquery = 0;
    std::vector<uint32_t> query_index;  // reqs[] index of query j
};

uint32_t class_of(uint32_t k) {
    uint32_t l = sort_lanes_per_k(k);
    if (l < 2) l = 2;
    return log2_pow2(l) - 1;
}

uint32_t append_chunks(uint64_t n, uint32_t k, uint64_t block_len) {
    uint64_t c = (n + block_len / 2) / block_len;
    uint64_t cap = n / (16ull * k);
    if (c > cap) c = cap;
    if (c < 1) c = 1;
    if (c > kMaxChunks) c = kMaxChunks;
    return (uint32_t)c;
}

int grow_pinned(void** p, size_t* bytes, size_t need) {
    if (need <= *bytes) return PSS_OK;
    size_t nb = std::max(need, *bytes * 2);
    void* q = nullptr;
    if (hipHostMalloc(&q, nb, hipHostMallocDefault) != hipSuccess) return PSS_ENOMEM;
    if (*p) (void)hipHostFree(*p);
    *p = q;
    *bytes = nb;
    return PSS_OK;
}

}  // namespace

struct pss_server {
    pss_ctx* ctx = nullptr;
    uint32_t nsum = 0;
    std::vector<uint32_t> ks;
    std::vector<uint64_t> s_off;   // pool entry offset of each summary
    std::vector<uint64_t> n_host;  // N of each summary, in submission order
    uint32_t kmax = 0;
    pss_server_opts opts{};
    size_t slot_budget = 0;        // device bytes one launch may use

    DeviceBuffer pool_mem;
    WideSummary pool{};

    std::vector<Slot> slots;
    std::vector<int> last_slot;        // slot of the last launch touching each summary (-1: none)
    std::vector<uint64_t> last_seq;    // that launch's number

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> pending;
    std::unordered_map<uint64_t, Request*> live;
    uint64_t next_ticket = 1;
    bool stop = false;
    int fatal = PSS_OK;
    std::thread worker;

    // statistics
    uint64_t launches = 0, requests = 0, appended = 0;
    uint32_t max_launch_requests = 0;
    double stage_ms = 0.0, gpu_ms = 0.0;
};

namespace {

// Device bytes a launch needs for an append of n items with k counters and
// C blocks: the staged items, the block summaries and their error scratch.
size_t append_bytes(uint64_t n, uint32_t k, uint32_t C) {
    return align_up(n * 4, 16) + (size_t)C * k * 12 + (size_t)C * 8 + (size_t)C * sizeof(BatchBlock) +
           (size_t)C * sizeof(BatchNode) + sizeof(ServeFold) + (size_t)C * 4 * ChunkLayout::make(k, false).err_stride;
}

// Copies every append's items into the pinned staging buffer; large launches
// split the bytes over several threads (one core does not reach the host's
// memory bandwidth).
void stage_items(const Slot& sl, char* hp, const std::vector<uint64_t>& item_off, uint64_t total_bytes) {
    struct Piece {
        char* dst;
        const char* src;
        size_t bytes;
    };
    std::vector<Piece> pieces;
    for (uint32_t r = 0; r < sl.reqs.size(); ++r) {
        const Request* q = sl.reqs[r];
        if (q->type == kAppend && q->n) pieces.push_back({hp + item_off[r] * 4, (const char*)q->items, q->n * 4});
    }
    const size_t kParallelBytes = 16u << 20;
    unsigned nt = std::thread::hardware_concurrency();
    nt = std::max(1u, std::min(nt, 16u));
    if (total_bytes < kParallelBytes || nt == 1) {
        for (const Piece& p : pieces) memcpy(p.dst, p.src, p.bytes);
        return;
    }
    // thread t copies bytes [t * share, (t + 1) * share) of the concatenation
    const uint64_t share = (total_bytes + nt - 1) / nt;
    auto work = [&](unsigned t) {
        uint64_t lo = t * share, hi = std::min<uint64_t>(total_bytes, lo + share), pos = 0;
        for (const Piece& p : pieces) {
            const uint64_t a = std::max(lo, pos), b = std::min(hi, pos + p.bytes);
            if (a < b) memcpy(p.dst + (a - pos), p.src + (a - pos), b - a);
            pos += p.bytes;
            if (pos >= hi) break;
        }
    };
    std::vector<std::thread> th;
    for (unsigned t = 1; t < nt; ++t) th.emplace_back(work, t);
    work(0);
    for (std::thread& x : th) x.join();
}

size_t query_bytes(uint32_t cap) { return (size_t)cap * sizeof(DevEntry) + 4 + sizeof(ServeQuery); }

// Builds and enqueues one launch on slot `si` from the requests in sl.reqs.
int run_launch(pss_server* srv, uint32_t si) {
    Slot& sl = srv->slots[si];
    // appends: blocks, grouped by size class, longest first inside a class
    struct HB {
        BatchBlock d;
        uint32_t cls, req, c;
    };
    std::vector<HB> hb;
    std::vector<uint64_t> item_off(sl.reqs.size(), 0);
    uint64_t items_total = 0;
    uint32_t nappend = 0;
    sl.query_index.clear();
    for (uint32_t r = 0; r < sl.reqs.size(); ++r) {
        Request* q = sl.reqs[r];
        if (q->type != kAppend) {
            sl.query_index.push_back(r);
            continue;
        }
        ++nappend;
        item_off[r] = items_total;
        items_total += align_up(q->n, 4);  // 16-B aligned streams
        const uint32_t k = srv->ks[q->sid];
        for (uint32_t c = 0; c < q->chunks; ++c) {
            HB h;
            h.d.items = nullptr;  // set once the staging address is known
            h.d.n = q->n;
            h.d.begin = (uint64_t)c * q->n / q->chunks;  // Algorithm 1's block bounds
            h.d.end = (uint64_t)(c + 1) * q->n / q->chunks;
            h.d.out = 0;
            h.d.eoff = 0;
            h.d.k = k;
            h.d.slots_x16 = ChunkLayout::default_slots_x16(k, hash_choices(k, false));
            h.cls = class_of(k);
            h.req = r;
            h.c = c;
            hb.push_back(h);
        }
    }
    std::sort(hb.begin(), hb.end(), [](const HB& x, const HB& y) {
        if (x.cls != y.cls) return x.cls < y.cls;
        const uint64_t lx = x.d.end - x.d.begin, ly = y.d.end - y.d.begin;
        if (lx != ly) return lx > ly;
        if (x.req != y.req) return x.req < y.req;
        return x.c < y.c;
    });
    const uint32_t nb = (uint32_t)hb.size();
    std::vector<uint64_t> first_blk(sl.reqs.size(), 0);
    {
        uint64_t acc = 0;
        for (uint32_t r = 0; r < sl.reqs.size(); ++r) {
            first_blk[r] = acc;
            if (sl.reqs[r]->type == kAppend) acc += sl.reqs[r]->chunks;
        }
    }
    std::vector<uint32_t> where(nb);
    uint64_t entries = 0, ewords = 0;
    for (uint32_t i = 0; i < nb; ++i) {
        hb[i].d.out = entries;
        entries += hb[i].d.k;
        hb[i].d.eoff = ewords;
        ewords += ChunkLayout::make(hb[i].d.k, false, hb[i].d.slots_x16).err_stride;
        where[first_blk[hb[i].req] + hb[i].c] = i;
    }
    // tree levels over every append, then the folds
    std::vector<BatchNode> nodes;
    std::vector<uint32_t> lvl_first, lvl_count, lvl_kmax;
    uint32_t cmax = 0;
    for (Request* q : sl.reqs)
        if (q->type == kAppend) cmax = std::max(cmax, q->chunks);
    for (uint32_t step = 1; step < cmax; step <<= 1) {
        const uint32_t f0 = (uint32_t)nodes.size();
        uint32_t km = 0;
        for (uint32_t r = 0; r < sl.reqs.size(); ++r) {
            Request* q = sl.reqs[r];
            if (q->type != kAppend) continue;
            for (uint64_t a = 0; a + step < q->chunks; a += 2ull * step) {
                BatchNode nd;
                const uint32_t ia = where[first_blk[r] + a], ib = where[first_blk[r] + a + step];
                nd.a_off = hb[ia].d.out;
                nd.b_off = hb[ib].d.out;
                nd.a = ia;
                nd.b = ib;
                nd.k = srv->ks[q->sid];
                nd.pad = 0;
                nodes.push_back(nd);
                km = std::max(km, nd.k);
            }
        }
        lvl_first.push_back(f0);
        lvl_count.push_back((uint32_t)nodes.size() - f0);
        lvl_kmax.push_back(km);
    }
    std::vector<ServeFold> folds;
    uint32_t fold_kmax = 0;
    for (uint32_t r = 0; r < sl.reqs.size(); ++r) {
        Request* q = sl.reqs[r];
        if (q->type != kAppend) continue;
        ServeFold f;
        const uint32_t root = where[first_blk[r]];
        f.s_off = srv->s_off[q->sid];
        f.root_off = hb[root].d.out;
        f.sid = q->sid;
        f.root = root;
        f.k = srv->ks[q->sid];
        f.pad = 0;
        folds.push_back(f);
        fold_kmax = std::max(fold_kmax, f.k);
    }
    std::vector<ServeQuery> queries;
    uint64_t out_entries = 0;
    uint32_t query_kmax = 0;
    for (uint32_t r : sl.query_index) {
        Request* q = sl.reqs[r];
        ServeQuery d;
        d.s_off = srv->s_off[q->sid];
        d.n = q->stream_len;
        d.out_off = out_entries;
        d.sid = q->sid;
        d.k = srv->ks[q->sid];
        d.kind = (uint32_t)q->kind;
        d.cap = q->cap;
        out_entries += q->cap;
        queries.push_back(d);
        query_kmax = std::max(query_kmax, d.k);
    }
    sl.nquery = (uint32_t)queries.size();

    // device layout: items | block summaries (item, cnt, err, size, min) |
    // descriptors (blocks, nodes, folds, queries, queues) | query output
    // (entries, counts) | error scratch of the blocks
    const size_t it_b = align_up(items_total * 4, 256);
    const size_t e4 = align_up(entries * 4, 256);
    const size_t h4 = align_up((size_t)nb * 4, 256);
    const size_t bb = align_up((size_t)nb * sizeof(BatchBlock), 256);
    const size_t ndb = align_up(nodes.size() * sizeof(BatchNode), 256);
    const size_t fb = align_up(folds.size() * sizeof(ServeFold), 256);
    const size_t qb = align_up(queries.size() * sizeof(ServeQuery), 256);
    const size_t qq = 256;
    const size_t ob = align_up(out_entries * sizeof(DevEntry), 256);
    // the counts of the queries, then the launch's fold-failure word
    const size_t cb = align_up(((size_t)queries.size() + 1) * 4, 256);
    sl.off_items = 0;
    const size_t off_sum = it_b;
    sl.off_desc = off_sum + 3 * e4 + 2 * h4;
    sl.desc_bytes = bb + ndb + fb + qb;
    const size_t off_queue = sl.off_desc + sl.desc_bytes;
    sl.off_out = off_queue + qq;
    sl.out_bytes = ob + cb;
    const size_t off_errs = sl.off_out + sl.out_bytes;
    const size_t total = off_errs + align_up(ewords * 4, 256);
    int rc = sl.dev.grow(total);
    if (rc != PSS_OK) return rc;
    // host staging: items then descriptors, contiguous as on the device
    const size_t pin_need = std::max(it_b + sl.desc_bytes, sl.out_bytes);
    rc = grow_pinned(&sl.pin, &sl.pin_bytes, pin_need);
    if (rc != PSS_OK) return rc;
    char* dbase = (char*)sl.dev.ptr;
    char* hp = (char*)sl.pin;
    const auto ts = Clock::now();
    stage_items(sl, hp, item_off, items_total * 4);
    const double stage = ms_between(ts, Clock::now());
    for (uint32_t i = 0; i < nb; ++i) hb[i].d.items = (const uint32_t*)(dbase + item_off[hb[i].req] * 4);
    char* hd = hp + it_b;
    for (uint32_t i = 0; i < nb; ++i) memcpy(hd + i * sizeof(BatchBlock), &hb[i].d, sizeof(BatchBlock));
    if (!nodes.empty()) memcpy(hd + bb, nodes.data(), nodes.size() * sizeof(BatchNode));
    if (!folds.empty()) memcpy(hd + bb + ndb, folds.data(), folds.size() * sizeof(ServeFold));
    if (!queries.empty()) memcpy(hd + bb + ndb + fb, queries.data(), queries.size() * sizeof(ServeQuery));

    hipStream_t st = sl.st;
    if (hipEventRecord(sl.t0, st) != hipSuccess) return PSS_EDEVICE;
    // items and descriptors: two transfers from the pinned staging
    if ((it_b && hipMemcpyAsync(dbase, hp, it_b, hipMemcpyHostToDevice, st) != hipSuccess) ||
        hipMemcpyAsync(dbase + sl.off_desc, hd, sl.desc_bytes, hipMemcpyHostToDevice, st) != hipSuccess)
        return PSS_EDEVICE;
    BlockSummaries sums;
    sums.item = (uint32_t*)(dbase + off_sum);
    sums.cnt = (uint32_t*)(dbase + off_sum + e4);
    sums.err = (uint32_t*)(dbase + off_sum + 2 * e4);
    sums.size = (uint32_t*)(dbase + off_sum + 3 * e4);
    sums.min = (uint32_t*)(dbase + off_sum + 3 * e4 + h4);
    const BatchBlock* d_blocks = (const BatchBlock*)(dbase + sl.off_desc);
    const BatchNode* d_nodes = (const BatchNode*)(dbase + sl.off_desc + bb);
    const ServeFold* d_folds = (const ServeFold*)(dbase + sl.off_desc + bb + ndb);
    const ServeQuery* d_queries = (const ServeQuery*)(dbase + sl.off_desc + bb + ndb + fb);
    uint32_t* d_queue = (uint32_t*)(dbase + off_queue);
    DevEntry* d_out = (DevEntry*)(dbase + sl.off_out);
    uint32_t* d_counts = (uint32_t*)(dbase + sl.off_out + ob);
    uint32_t* d_errs = (uint32_t*)(dbase + off_errs);

    rc = check(launch_zero_words(d_queue, kSrvClasses, st));
    if (rc == PSS_OK) rc = check(launch_zero_words(d_counts + queries.size(), 1, st));
    for (uint32_t i = 0; rc == PSS_OK && i < nb;) {
        const uint32_t cls = hb[i].cls, first = i;
        uint32_t kc = 0;
        while (i < nb && hb[i].cls == cls) kc = std::max(kc, hb[i++].d.k);
        const uint32_t count = i - first;
        const uint32_t stride = align16(ChunkLayout::make(kc, false).lds_bytes);
        uint64_t per_cu = lds_waves(srv->ctx->lds_per_cu, stride);
        per_cu = std::max<uint64_t>(1, std::min<uint64_t>(per_cu, 32));
        const uint32_t grid =
            (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)srv->ctx->cu_count * per_cu, count));
        rc = check(launch_batch_blocks(d_blocks + first, count, d_queue + cls, 2u << cls, stride, 1, grid,
                                       BlockSummaries{sums.item, sums.cnt, sums.err, sums.size + first,
                                                      sums.min + first},
                                       d_errs, st));
    }
    for (size_t l = 0; rc == PSS_OK && l < lvl_first.size(); ++l)
        rc = check(launch_batch_combine(d_nodes + lvl_first[l], lvl_count[l], lvl_kmax[l], sums, st));
    if (rc == PSS_OK)
        rc = check(launch_serve_fold(d_folds, (uint32_t)folds.size(), fold_kmax, srv->pool, sums,
                                     d_counts + queries.size(), st));
    if (rc == PSS_OK)
        rc = check(launch_serve_query(d_queries, (uint32_t)queries.size(), query_kmax, srv->pool, d_out, d_counts, st));
    if (rc == PSS_OK && sl.out_bytes &&
        hipMemcpyAsync(sl.pin, dbase + sl.off_out, sl.out_bytes, hipMemcpyDeviceToHost, st) != hipSuccess)
        rc = PSS_EDEVICE;
    if (rc == PSS_OK && (hipEventRecord(sl.t1, st) != hipSuccess || hipEventRecord(sl.done, st) != hipSuccess))
        rc = PSS_EDEVICE;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stage_ms += stage;
    }
    sl.out_bytes = ob;  // entries part; counts follow at ob
    (void)nappend;
    return rc;
}

// Results of a finished launch into its requests (server lock held).
void finish_launch(pss_server* srv, Slot& sl, int rc) {
    float gms = 0.f;
    if (rc == PSS_OK && hipEventElapsedTime(&gms, sl.t0, sl.t1) == hipSuccess) srv->gpu_ms += gms;
    const auto now = Clock::now();
    const char* base = (const char*)sl.pin;
    const uint32_t* counts = (const uint32_t*)(base + sl.out_bytes);
    // a fold met a failed block: the summaries were left as they were, and the
    // launch (and the server, as after any device failure) fails
    if (rc == PSS_OK && counts[sl.query_index.size()] != 0) {
        rc = PSS_EDEVICE;
        srv->fatal = PSS_EDEVICE;
    }
    uint64_t off = 0;
    for (uint32_t j = 0; j < sl.query_index.size(); ++j) {
        Request* q = sl.reqs[sl.query_index[j]];
        if (rc == PSS_OK) {
            const uint32_t c = counts[j];
            if (c > srv->ks[q->sid]) {
                q->rc = PSS_EDEVICE;  // a kernel reported a failed invariant
            } else {
                q->n_out = c;
                const uint32_t w = std::min(c, q->cap);
                q->out.resize(w);
                if (w) memcpy(q->out.data(), base + off * sizeof(DevEntry), (size_t)w * sizeof(pss_entry));
            }
        }
        off += q->cap;
    }
    for (Request* q : sl.reqs) {
        if (rc != PSS_OK) q->rc = rc;
        q->t_done = now;
        q->done = true;
    }
    sl.reqs.clear();
    sl.busy = false;
}

void server_loop(pss_server* srv) {
    DeviceGuard g(srv->ctx->device);
    std::unique_lock<std::mutex> lk(srv->mu);
    for (;;) {
        // completions
        bool any_busy = false;
        for (Slot& sl : srv->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipSuccess) {
                finish_launch(srv, sl, PSS_OK);
                srv->cv_done.notify_all();
            } else if (q != hipErrorNotReady) {
                finish_launch(srv, sl, PSS_EDEVICE);
                srv->fatal = PSS_EDEVICE;
                srv->cv_done.notify_all();
            } else {
                any_busy = true;
            }
        }
        if (srv->fatal != PSS_OK && !srv->pending.empty()) {
            // a launch failed: fail what is still waiting instead of running it
            for (Request* q : srv->pending) {
                q->rc = srv->fatal;
                q->t_done = Clock::now();
                q->done = true;
            }
            srv->pending.clear();
            srv->cv_done.notify_all();
        }
        if (srv->stop && srv->pending.empty() && !any_busy) break;
        // admit: the first free slot takes what is pending
        int free_slot = -1;
        for (uint32_t i = 0; i < srv->slots.size(); ++i)
            if (!srv->slots[i].busy) {
                free_slot = (int)i;
                break;
            }
        if (free_slot >= 0 && !srv->pending.empty() && srv->fatal == PSS_OK) {
            Slot& sl = srv->slots[free_slot];
            const uint64_t seq = ++srv->launches;
            std::unordered_set<uint32_t> blocked;
            size_t used = 0, staged = 0;
            std::deque<Request*> rest;
            std::vector<int> wait_slots;
            while (!srv->pending.empty() && sl.reqs.size() < srv->opts.max_requests && rest.size() < kScanLimit) {
                Request* q = srv->pending.front();
                srv->pending.pop_front();
                size_t need = q->type == kAppend ? append_bytes(q->n, srv->ks[q->sid], q->chunks) : query_bytes(q->cap);
                const size_t qitems = q->type == kAppend ? q->n * 4 : 0;
                if (blocked.count(q->sid) ||
                    (!sl.reqs.empty() && (used + need > srv->slot_budget ||
                                          staged + qitems > (size_t)srv->opts.stage_bytes))) {
                    blocked.insert(q->sid);  // later requests on it keep their order
                    rest.push_back(q);
                    continue;
                }
                used += need;
                staged += qitems;
                blocked.insert(q->sid);  // at most one request per summary per launch
                q->launch = (uint32_t)seq;
                q->t_launch = Clock::now();
                const int ls = srv->last_slot[q->sid];
                if (ls >= 0 && ls != free_slot && srv->slots[ls].busy && srv->slots[ls].seq == srv->last_seq[q->sid])
                    wait_slots.push_back(ls);
                srv->last_slot[q->sid] = free_slot;
                srv->last_seq[q->sid] = seq;
                sl.reqs.push_back(q);
            }
            while (!rest.empty()) {  // unadmitted requests go back in order, ahead of newer ones
                srv->pending.push_front(rest.back());
                rest.pop_back();
            }
            sl.busy = true;
            sl.seq = seq;
            srv->requests += sl.reqs.size();
            srv->max_launch_requests = std::max<uint32_t>(srv->max_launch_requests, (uint32_t)sl.reqs.size());
            for (Request* q : sl.reqs)
                if (q->type == kAppend) srv->appended += q->n;
            std::sort(wait_slots.begin(), wait_slots.end());
            wait_slots.erase(std::unique(wait_slots.begin(), wait_slots.end()), wait_slots.end());
            lk.unlock();
            int rc = PSS_OK;
            for (int ws : wait_slots)
                if (hipStreamWaitEvent(sl.st, srv->slots[ws].done, 0) != hipSuccess) rc = PSS_EDEVICE;
            if (rc == PSS_OK) rc = run_launch(srv, (uint32_t)free_slot);
            lk.lock();
            if (rc != PSS_OK) {
                finish_launch(srv, sl, rc);
                srv->fatal = rc;
                srv->cv_done.notify_all();
            }
            continue;
        }
        if (any_busy)
            srv->cv_work.wait_for(lk, std::chrono::microseconds(20));
        else
            srv->cv_work.wait(lk, [&] { return srv->stop || !srv->pending.empty(); });
    }
}

int submit(pss_server* srv, Request* q, uint64_t* ticket) {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return PSS_EINVAL;
    if (srv->fatal != PSS_OK) return srv->fatal;
    q->ticket = srv->next_ticket++;
    q->t_submit = Clock::now();
    if (q->type == kAppend) {
        srv->n_host[q->sid] += q->n;
        q->stream_len = srv->n_host[q->sid];
    } else {
        q->stream_len = srv->n_host[q->sid];
    }
    srv->live[q->ticket] = q;
    if (q->type == kAppend && q->n == 0) {  // nothing to run: complete at once
        q->t_launch = q->t_done = q->t_submit;
        q->done = true;
    } else {
        srv->pending.push_back(q);
        srv->cv_work.notify_one();
    }
    *ticket = q->ticket;
    return PSS_OK;
}

}  // namespace

extern "C" {

uint32_t pss_server_max_k(const pss_ctx* ctx) {
    if (!ctx) return 0;
    const uint32_t kb = pss_batch_max_k(ctx);
    uint32_t lo = 2, hi = kb;
    if (hi < lo || combine_lds_bytes(lo, true) > ctx->lds_max) return 0;
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo + 1) / 2;
        if (combine_lds_bytes(mid, true) <= ctx->lds_max) lo = mid; else hi = mid - 1;
    }
    return lo;
}

int pss_server_create(pss_ctx* ctx, uint32_t nsummaries, const uint32_t* h_ks, const pss_server_opts* opts,
                      pss_server** out) {
    if (!ctx || !out || nsummaries == 0 || !h_ks) return PSS_EINVAL;
    *out = nullptr;
    const uint32_t kcap = pss_server_max_k(ctx);
    for (uint32_t s = 0; s < nsummaries; ++s) {
        if (h_ks[s] < 2) return PSS_EINVAL;
        if (h_ks[s] > kcap) return PSS_ERANGE;
    }
    DeviceGuard g(ctx->device);
    pss_server* srv = new (std::nothrow) pss_server();
    if (!srv) return PSS_ENOMEM;
    srv->ctx = ctx;
    int rc = PSS_OK;
    try {
        srv->opts.hbm_budget = opts && opts->hbm_budget ? opts->hbm_budget : (64ull << 30);
        srv->opts.slots = opts && opts->slots ? std::min<uint32_t>(opts->slots, 8) : 2;
        srv->opts.max_requests = opts && opts->max_requests ? opts->max_requests : 4096;
        srv->opts.block_len = opts && opts->block_len ? opts->block_len : (1ull << 14);
        srv->opts.stage_bytes = opts && opts->stage_bytes ? opts->stage_bytes : (256ull << 20);
        srv->slot_budget = (size_t)(srv->opts.hbm_budget / srv->opts.slots);
        srv->nsum = nsummaries;
        srv->ks.assign(h_ks, h_ks + nsummaries);
        srv->s_off.resize(nsummaries);
        srv->n_host.assign(nsummaries, 0);
        srv->last_slot.assign(nsummaries, -1);
        srv->last_seq.assign(nsummaries, 0);
        uint64_t o = 0;
        for (uint32_t s = 0; s < nsummaries; ++s) {
            srv->s_off[s] = o;
            o += srv->ks[s];
            srv->kmax = std::max(srv->kmax, srv->ks[s]);
        }
        // pool: item (u32), cnt, err (u64) at the summaries' offsets; size, min per summary
        const size_t e4 = align_up(o * 4, 256), e8 = align_up(o * 8, 256);
        const size_t h4 = align_up((size_t)nsummaries * 4, 256), h8 = align_up((size_t)nsummaries * 8, 256);
        rc = srv->pool_mem.grow(e4 + 2 * e8 + h4 + h8);
        if (rc == PSS_OK) {
            char* p = (char*)srv->pool_mem.ptr;
            srv->pool.item = (uint32_t*)p;
            srv->pool.cnt = (uint64_t*)(p + e4);
            srv->pool.err = (uint64_t*)(p + e4 + e8);
            srv->pool.size = (uint32_t*)(p + e4 + 2 * e8);
            srv->pool.min = (uint64_t*)(p + e4 + 2 * e8 + h4);
            // every summary starts empty (the identity of COMBINE)
            if (hipMemset(srv->pool.size, 0, h4) != hipSuccess || hipMemset(srv->pool.min, 0, h8) != hipSuccess ||
                hipDeviceSynchronize() != hipSuccess)
                rc = PSS_EDEVICE;
        }
        srv->slots.resize(srv->opts.slots);
        for (Slot& sl : srv->slots) {
            if (rc != PSS_OK) break;
            // default priority streams
            if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
                hipEventCreate(&sl.t0) != hipSuccess || hipEventCreate(&sl.t1) != hipSuccess)
                rc = PSS_EDEVICE;
        }
        // staging for a launch's items, allocated up front: pinned host memory
        // and device memory for the items plus their block summaries
        for (Slot& sl : srv->slots) {
            if (rc != PSS_OK) break;
            rc = grow_pinned(&sl.pin, &sl.pin_bytes, (size_t)srv->opts.stage_bytes);
            if (rc == PSS_OK)
                rc = sl.dev.grow(std::min<size_t>(srv->slot_budget, 2 * (size_t)srv->opts.stage_bytes));
        }
        if (rc == PSS_OK) srv->worker = std::thread(server_loop, srv);
    } catch (...) {
        rc = PSS_ENOMEM;
    }
    if (rc != PSS_OK) {
        for (Slot& sl : srv->slots) {
            if (sl.st) (void)hipStreamDestroy(sl.st);
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.t0) (void)hipEventDestroy(sl.t0);
            if (sl.t1) (void)hipEventDestroy(sl.t1);
        }
        srv->pool_mem.release();
        delete srv;
        return rc;
    }
    *out = srv;
    return PSS_OK;
}

void pss_server_destroy(pss_server* srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv_work.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
    DeviceGuard g(srv->ctx->device);
    (void)hipDeviceSynchronize();
    for (Slot& sl : srv->slots) {
        sl.dev.release();
        if (sl.pin) (void)hipHostFree(sl.pin);
        if (sl.st) (void)hipStreamDestroy(sl.st);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.t0) (void)hipEventDestroy(sl.t0);
        if (sl.t1) (void)hipEventDestroy(sl.t1);
    }
    for (auto& kv : srv->live) delete kv.second;  // every submitted request not yet waited for
    srv->pool_mem.release();
    delete srv;
}

int pss_server_append(pss_server* srv, uint32_t sid, const uint32_t* h_items, uint64_t n, uint32_t chunks,
                      uint64_t* ticket) {
    if (!srv || !ticket || sid >= srv->nsum || (n > 0 && !h_items)) return PSS_EINVAL;
    if (n >= kStreamBound || chunks > kMaxChunks) return PSS_ERANGE;
    const uint32_t k = srv->ks[sid];
    const uint32_t C = n == 0 ? 0 : (chunks ? chunks : append_chunks(n, k, srv->opts.block_len));
    if (n && append_bytes(n, k, C) > srv->slot_budget) return PSS_ERANGE;  // can never be admitted
    Request* q = new (std::nothrow) Request();
    if (!q) return PSS_ENOMEM;
    q->type = kAppend;
    q->sid = sid;
    q->items = h_items;
    q->n = n;
    q->chunks = C;
    int rc = submit(srv, q, ticket);
    if (rc != PSS_OK) delete q;
    return rc;
}

int pss_server_query(pss_server* srv, uint32_t sid, int kind, uint32_t cap, uint64_t* ticket) {
    if (!srv || !ticket || sid >= srv->nsum) return PSS_EINVAL;
    if (kind != PSS_Q_MAJORITY && kind != PSS_Q_TOPK) return PSS_EINVAL;
    Request* q = new (std::nothrow) Request();
    if (!q) return PSS_ENOMEM;
    q->type = kQuery;
    q->sid = sid;
    q->kind = kind;
    // the device writes at most cap entries: every reported one for a majority
    // query (fewer than k), the first min(cap, k) for a top query
    q->cap = kind == PSS_Q_MAJORITY ? srv->ks[sid] : std::min(cap, srv->ks[sid]);
    int rc = submit(srv, q, ticket);
    if (rc != PSS_OK) delete q;
    return rc;
}

int pss_server_wait(pss_server* srv, uint64_t ticket, pss_entry* h_out, uint32_t cap, pss_server_result* res) {
    if (!srv || !res) return PSS_EINVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->live.find(ticket);
    if (it == srv->live.end()) return PSS_EINVAL;
    Request* q = it->second;
    srv->cv_done.wait(lk, [&] { return q->done; });
    srv->live.erase(it);
    lk.unlock();
    res->status = q->rc;
    res->n_out = q->n_out;
    res->stream_len = q->stream_len;
    res->chunks_used = q->type == kAppend ? q->chunks : 0;
    res->launch = q->launch;
    res->latency_ms = ms_between(q->t_submit, q->t_done);
    res->queue_ms = ms_between(q->t_submit, q->t_launch);
    int rc = q->rc;
    if (rc == PSS_OK && q->type == kQuery) {
        const uint32_t w = std::min<uint32_t>((uint32_t)q->out.size(), cap);
        if (w && !h_out) rc = PSS_EINVAL;
        else if (w) memcpy(h_out, q->out.data(), (size_t)w * sizeof(pss_entry));
        if (rc == PSS_OK && q->kind == PSS_Q_MAJORITY && q->n_out > cap) rc = PSS_ETRUNC;
        if (q->kind == PSS_Q_TOPK) res->n_out = std::min(q->n_out, cap);
    }
    delete q;
    return rc;
}

int pss_server_stats(pss_server* srv, pss_server_stats_t* st) {
    if (!srv || !st) return PSS_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    st->launches = srv->launches;
    st->requests = srv->requests;
    st->items_appended = srv->appended;
    st->max_launch_requests = srv->max_launch_requests;
    st->pending = (uint32_t)srv->pending.size();
    st->status = srv->fatal;
    st->stage_ms = srv->stage_ms;
    st->gpu_ms = srv->gpu_ms;
    return PSS_OK;
}

}  // extern "C"
