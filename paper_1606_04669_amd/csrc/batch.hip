// Batched Parallel Space Saving: many independent streams, each with its own
// k and block count, run as one captured HIP graph.  Per stream the result is
// exactly Algorithm 1 with Algorithm 2 as the reduction (the same blocks, the
// same fixed tree, the same report as pss_run with the same C); the batch only
// changes how the work is scheduled:
//
//  * blocks of every stream are grouped by size class (the register sort
//    width of their k) and each class is one persistent launch whose waves
//    take blocks, longest first, from a queue; the classes run concurrently;
//  * each tree level of every stream is one launch over all streams' pairs;
//  * one launch reports every stream.
//
// The autotuner picks the target block length (hence each stream's C, which
// it records), the hash load factor and the waves per workgroup by timing
// candidates on a sample of the batch's own streams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <string.h>
#include <vector>

#include "pss.h"
#include "pss_ctx.h"
#include "pss_kernels.h"
#include "pss_layout.h"

using namespace pss;

namespace {

constexpr uint32_t kMaxClasses = 7;  // sort_lanes_per_k in {2, 4, ..., 64} (1 folds into 2)

struct Tuning {
    uint64_t target_len = 1u << 16;
    uint32_t slots_x16 = 0;  // 0: the per-k default
    uint32_t waves = 1;
};

struct ClassLaunch {
    uint32_t sort_lanes = 0;
    uint32_t first = 0, count = 0;  // block indices [first, first + count)
    uint32_t lds_stride = 0;
    uint32_t waves = 1;
    uint32_t grid = 0;
    uint64_t items = 0;  // items of the class's blocks
};

struct Level {
    uint32_t first = 0, count = 0, kmax = 0;
};

uint32_t class_lanes(uint32_t k) {
    uint32_t l = sort_lanes_per_k(k);
    return l < 2 ? 2 : l;
}

uint32_t class_index(uint32_t lanes) { return log2_pow2(lanes) - 1; }

// The block count a tuning gives a stream: blocks of about target_len items,
// never shorter than 16 k items (the tree moves about C k entries), at least 1.
uint32_t tuned_chunks(uint64_t n, uint32_t k, uint64_t target_len) {
    uint64_t c = (n + target_len / 2) / target_len;
    uint64_t cap = n / (16ull * k);
    if (c > cap) c = cap;
    if (c < 1) c = 1;
    if (c > kMaxChunks) c = kMaxChunks;
    return (uint32_t)c;
}

}  // namespace

struct pss_batch {
    pss_ctx* ctx = nullptr;
    uint32_t nstreams = 0;
    std::vector<const uint32_t*> items;
    std::vector<uint64_t> lens;
    std::vector<uint32_t> ks, chunks;
    std::vector<uint64_t> out_off;  // report offset of each stream (sum of earlier k)
    uint64_t out_entries = 0;
    Tuning tune;
    double tune_ms = 0.0;
    uint32_t tune_candidates = 0;

    uint32_t nblocks = 0;
    uint32_t nrep = 0;
    uint64_t entries = 0;
    uint32_t kmax = 0;
    std::vector<ClassLaunch> classes;
    std::vector<Level> levels;

    DeviceBuffer mem;                 // block summaries, descriptors, queues, report
    BlockSummaries sums{};
    BatchBlock* d_blocks = nullptr;
    BatchNode* d_nodes = nullptr;
    BatchReport* d_reps = nullptr;
    uint32_t* d_queues = nullptr;
    DevEntry* d_out = nullptr;
    uint32_t* d_counts = nullptr;
    uint32_t* d_errs = nullptr;  // error scratch of the blocks
    void* pinned = nullptr;
    size_t pinned_bytes = 0;

    hipStream_t side[kMaxClasses] = {};
    hipStream_t own = nullptr;  // tuning runs
    hipEvent_t fork = nullptr;
    hipEvent_t join[kMaxClasses] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void free_plan_device(pss_batch* b) {
    b->mem.release();
    if (b->pinned) (void)hipHostFree(b->pinned);
    b->pinned = nullptr;
    b->pinned_bytes = 0;
}

void destroy_graph(pss_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Lays out blocks, tree levels and reports for the streams listed in `sel`
// under tuning t (chunks[s] fixed where nonzero, else from t), uploads the
// descriptors and sizes the workspace.
int build_plan(pss_batch* b, const std::vector<uint32_t>& sel, const Tuning& t, std::vector<uint32_t>& chunks) {
    pss_ctx* ctx = b->ctx;
    struct HostBlock {
        BatchBlock d;
        uint32_t cls;
        uint32_t stream, c;
    };
    std::vector<HostBlock> hb;
    b->kmax = 0;
    for (uint32_t s : sel) {
        const uint32_t k = b->ks[s];
        const uint64_t n = b->lens[s];
        if (chunks[s] == 0) chunks[s] = tuned_chunks(n, k, t.target_len);
        const uint32_t C = chunks[s];
        b->kmax = std::max(b->kmax, k);
        for (uint32_t c = 0; c < C; ++c) {
            HostBlock h;
            h.d.items = b->items[s];
            h.d.n = n;
            h.d.begin = (uint64_t)c * n / C;  // Algorithm 1's block bounds
            h.d.end = (uint64_t)(c + 1) * n / C;
            h.d.out = 0;
            h.d.eoff = 0;
            h.d.k = k;
            h.d.slots_x16 = t.slots_x16 ? t.slots_x16 : ChunkLayout::default_slots_x16(k, hash_choices(k, false));
            h.cls = class_index(class_lanes(k));
            h.stream = s;
            h.c = c;
            hb.push_back(h);
        }
    }
    // class-contiguous, longest blocks first inside a class (ties by stream, block)
    std::sort(hb.begin(), hb.end(), [](const HostBlock& x, const HostBlock& y) {
        if (x.cls != y.cls) return x.cls < y.cls;
        const uint64_t lx = x.d.end - x.d.begin, ly = y.d.end - y.d.begin;
        if (lx != ly) return lx > ly;
        if (x.stream != y.stream) return x.stream < y.stream;
        return x.c < y.c;
    });
    b->nblocks = (uint32_t)hb.size();
    // stream s, block c -> block index
    std::vector<uint64_t> first_of(b->nstreams, 0);
    {
        uint64_t acc = 0;
        for (uint32_t s : sel) {
            first_of[s] = acc;
            acc += chunks[s];
        }
    }
    std::vector<uint32_t> where(hb.size());
    uint64_t off = 0, eoff = 0;
    for (uint32_t i = 0; i < b->nblocks; ++i) {
        hb[i].d.out = off;
        off += hb[i].d.k;
        hb[i].d.eoff = eoff;
        eoff += ChunkLayout::make(hb[i].d.k, false, hb[i].d.slots_x16).err_stride;
        where[first_of[hb[i].stream] + hb[i].c] = i;
    }
    b->entries = off;

    b->classes.clear();
    for (uint32_t i = 0; i < b->nblocks;) {
        ClassLaunch cl;
        cl.first = i;
        const uint32_t cls = hb[i].cls;
        uint32_t kc = 0, slots = 0;
        while (i < b->nblocks && hb[i].cls == cls) {
            kc = std::max(kc, hb[i].d.k);
            slots = std::max(slots, hb[i].d.slots_x16);
            cl.items += hb[i].d.end - hb[i].d.begin;
            ++i;
        }
        cl.count = i - cl.first;
        cl.sort_lanes = 2u << cls;
        // every block's layout fits the stride: footprint grows with k and load factor
        cl.lds_stride = align16(ChunkLayout::make(kc, false, slots).lds_bytes);
        uint32_t w = t.waves;
        const uint32_t wmax = cl.sort_lanes <= 8 ? 4 : cl.sort_lanes <= 16 ? 2 : 1;
        if (w > wmax) w = wmax;
        while (w > 1 && (size_t)w * cl.lds_stride > ctx->lds_max) w >>= 1;
        if ((size_t)cl.lds_stride > ctx->lds_max) return PSS_ERANGE;
        cl.waves = w;
        uint64_t per_cu = lds_waves(ctx->lds_per_cu, w * cl.lds_stride);
        per_cu = std::max<uint64_t>(1, std::min<uint64_t>(per_cu, 32 / w));
        const uint64_t resident = (uint64_t)std::max(1, ctx->cu_count) * per_cu;
        const uint64_t need = (cl.count + w - 1) / w;
        cl.grid = (uint32_t)std::max<uint64_t>(1, std::min(resident, need));
        b->classes.push_back(cl);
    }

    // tree levels over every stream (Algorithm 1's reduction, fixed shape)
    std::vector<BatchNode> nodes;
    b->levels.clear();
    uint32_t cmax = 0;
    for (uint32_t s : sel) cmax = std::max(cmax, chunks[s]);
    for (uint32_t step = 1; step < cmax; step <<= 1) {
        Level lv;
        lv.first = (uint32_t)nodes.size();
        for (uint32_t s : sel) {
            const uint32_t C = chunks[s];
            for (uint64_t a = 0; a + step < C; a += 2ull * step) {
                BatchNode nd;
                const uint32_t ia = where[first_of[s] + a], ib = where[first_of[s] + a + step];
                nd.a_off = hb[ia].d.out;
                nd.b_off = hb[ib].d.out;
                nd.a = ia;
                nd.b = ib;
                nd.k = b->ks[s];
                nd.pad = 0;
                nodes.push_back(nd);
                lv.kmax = std::max(lv.kmax, nd.k);
            }
        }
        lv.count = (uint32_t)nodes.size() - lv.first;
        b->levels.push_back(lv);
    }
    std::vector<BatchReport> reps;
    for (uint32_t s : sel) {
        BatchReport r;
        const uint32_t root = where[first_of[s]];
        r.root_off = hb[root].d.out;
        r.root = root;
        r.k = b->ks[s];
        r.n = b->lens[s];
        r.out_off = b->out_off[s];
        reps.push_back(r);
    }

    // one allocation: summaries (item, cnt, err), headers, descriptors, queues, report
    const size_t e4 = align_up(b->entries * 4, 256);
    const size_t h4 = align_up((size_t)b->nblocks * 4, 256);
    const size_t bb = align_up(hb.size() * sizeof(BatchBlock), 256);
    const size_t nb = align_up(std::max<size_t>(1, nodes.size()) * sizeof(BatchNode), 256);
    const size_t rb = align_up(reps.size() * sizeof(BatchReport), 256);
    const size_t qb = 256;
    const size_t ob = align_up(b->out_entries * sizeof(DevEntry), 256);
    const size_t cb = align_up((size_t)b->nstreams * 4, 256);
    const size_t eb = align_up(eoff * 4, 256);  // error scratch of the blocks
    const size_t total = 3 * e4 + 2 * h4 + bb + nb + rb + qb + ob + cb + eb;
    int rc = b->mem.grow(total);
    if (rc != PSS_OK) return rc;
    char* p = (char*)b->mem.ptr;
    b->sums.item = (uint32_t*)p; p += e4;
    b->sums.cnt = (uint32_t*)p; p += e4;
    b->sums.err = (uint32_t*)p; p += e4;
    b->sums.size = (uint32_t*)p; p += h4;
    b->sums.min = (uint32_t*)p; p += h4;
    b->d_blocks = (BatchBlock*)p; p += bb;
    b->d_nodes = (BatchNode*)p; p += nb;
    b->d_reps = (BatchReport*)p; p += rb;
    b->d_queues = (uint32_t*)p; p += qb;
    b->d_out = (DevEntry*)p; p += ob;
    b->d_counts = (uint32_t*)p; p += cb;
    b->d_errs = (uint32_t*)p;
    std::vector<BatchBlock> db(hb.size());
    for (size_t i = 0; i < hb.size(); ++i) db[i] = hb[i].d;
    if (hipMemcpy(b->d_blocks, db.data(), db.size() * sizeof(BatchBlock), hipMemcpyHostToDevice) != hipSuccess ||
        (nodes.size() &&
         hipMemcpy(b->d_nodes, nodes.data(), nodes.size() * sizeof(BatchNode), hipMemcpyHostToDevice) != hipSuccess) ||
        hipMemcpy(b->d_reps, reps.data(), reps.size() * sizeof(BatchReport), hipMemcpyHostToDevice) != hipSuccess)
        return PSS_EDEVICE;
    b->nrep = (uint32_t)reps.size();
    return PSS_OK;
}

// The launch sequence on `st`: zero the queues, the class launches forked
// onto side streams (they run concurrently), the tree levels, the report.
int enqueue(pss_batch* b, hipStream_t st) {
    int rc = check(launch_zero_words(b->d_queues, kMaxClasses, st));
    if (rc != PSS_OK) return rc;
    if (hipEventRecord(b->fork, st) != hipSuccess) return PSS_EDEVICE;
    // the class with the most work first: the classes share the device's few
    // hardware queues, and the last one to start finishes the batch.  Work is
    // estimated as items x (1 + log2 of the sort class): larger k costs more
    // per item.
    uint32_t order[kMaxClasses];
    const size_t nc = b->classes.size();
    auto work = [&](size_t i) {
        const ClassLaunch& c = b->classes[i];
        return (double)c.items * (1.0 + (double)log2_pow2(c.sort_lanes));
    };
    for (size_t i = 0; i < nc; ++i) order[i] = (uint32_t)i;
    std::sort(order, order + nc, [&](uint32_t a, uint32_t c) { return work(a) > work(c); });
    for (size_t oi = 0; oi < nc; ++oi) {
        const size_t i = order[oi];
        const ClassLaunch& cl = b->classes[i];
        hipStream_t ss = b->side[i];
        if (hipStreamWaitEvent(ss, b->fork, 0) != hipSuccess) return PSS_EDEVICE;
        rc = check(launch_batch_blocks(b->d_blocks + cl.first, cl.count, b->d_queues + i, cl.sort_lanes, cl.lds_stride,
                                       cl.waves, cl.grid,
                                       BlockSummaries{b->sums.item, b->sums.cnt, b->sums.err, b->sums.size + cl.first,
                                                      b->sums.min + cl.first},
                                       b->d_errs, ss));
        if (rc != PSS_OK) return rc;
        if (hipEventRecord(b->join[i], ss) != hipSuccess || hipStreamWaitEvent(st, b->join[i], 0) != hipSuccess)
            return PSS_EDEVICE;
    }
    for (const Level& lv : b->levels) {
        rc = check(launch_batch_combine(b->d_nodes + lv.first, lv.count, lv.kmax, b->sums, st));
        if (rc != PSS_OK) return rc;
    }
    return check(launch_batch_extract(b->d_reps, b->nrep, b->kmax, b->sums, b->d_out, b->d_counts, st));
}

int make_streams(pss_batch* b) {
    if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking) != hipSuccess)
        return PSS_EDEVICE;
    for (uint32_t i = 0; i < kMaxClasses; ++i) {
        // default priority (no priority streams)
        if (hipStreamCreateWithFlags(&b->side[i], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming) != hipSuccess)
            return PSS_EDEVICE;
    }
    return PSS_OK;
}

void destroy_batch(pss_batch* b) {
    if (!b) return;
    DeviceGuard g(b->ctx->device);
    (void)hipDeviceSynchronize();
    destroy_graph(b);
    free_plan_device(b);
    for (uint32_t i = 0; i < kMaxClasses; ++i) {
        if (b->side[i]) (void)hipStreamDestroy(b->side[i]);
        if (b->join[i]) (void)hipEventDestroy(b->join[i]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->own) (void)hipStreamDestroy(b->own);
    delete b;
}

// Milliseconds of one eager run of the plan (after one untimed run).
int time_plan(pss_batch* b, hipStream_t st, float* ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return PSS_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return PSS_EDEVICE;
    }
    int rc = enqueue(b, st);
    if (rc == PSS_OK && hipEventRecord(e0, st) != hipSuccess) rc = PSS_EDEVICE;
    if (rc == PSS_OK) rc = enqueue(b, st);
    if (rc == PSS_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(ms, e0, e1) != hipSuccess))
        rc = PSS_EDEVICE;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

// Coordinate search over (target block length, hash load factor, waves per
// workgroup), each candidate timed on a sample of the batch's streams (every
// 8th stream, all of them for small batches).  Results never depend on the
// last two; the first fixes each untuned stream's C.
int autotune(pss_batch* b, hipStream_t st, bool tune_len) {
    std::vector<uint32_t> sample;
    const uint32_t stride = b->nstreams >= 64 ? 8 : 1;
    for (uint32_t s = 0; s < b->nstreams; s += stride) sample.push_back(s);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    (void)hipEventRecord(t0, st);
    auto trial = [&](const Tuning& t, float* ms) -> int {
        std::vector<uint32_t> ch = b->chunks;  // user-fixed counts stay, the rest follow t
        int rc = build_plan(b, sample, t, ch);
        if (rc != PSS_OK) return rc;
        ++b->tune_candidates;
        return time_plan(b, st, ms);
    };
    Tuning best = b->tune;
    float best_ms = 0.f;
    int rc = trial(best, &best_ms);
    if (rc != PSS_OK) return rc;
    auto consider = [&](Tuning t) -> int {
        float ms = 0.f;
        int r = trial(t, &ms);
        if (r == PSS_ERANGE) return PSS_OK;  // does not fit: skip the candidate
        if (r != PSS_OK) return r;
        if (ms < best_ms) {
            best_ms = ms;
            best = t;
        }
        return PSS_OK;
    };
    if (tune_len) {
        const Tuning base = best;
        for (uint64_t len : {1ull << 14, 1ull << 15, 1ull << 17, 1ull << 18}) {
            Tuning t = base;
            t.target_len = len;
            if ((rc = consider(t)) != PSS_OK) return rc;
        }
    }
    {
        const Tuning base = best;
        for (uint32_t sl : {32u, 48u, 64u}) {
            Tuning t = base;
            t.slots_x16 = sl;
            if ((rc = consider(t)) != PSS_OK) return rc;
        }
    }
    {
        const Tuning base = best;
        for (uint32_t w : {2u, 4u}) {
            Tuning t = base;
            t.waves = w;
            if ((rc = consider(t)) != PSS_OK) return rc;
        }
    }
    b->tune = best;
    float ms = 0.f;
    (void)hipEventRecord(t1, st);
    if (hipEventSynchronize(t1) == hipSuccess && hipEventElapsedTime(&ms, t0, t1) == hipSuccess) b->tune_ms = ms;
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    return PSS_OK;
}

}  // namespace

extern "C" {

uint32_t pss_batch_max_k(const pss_ctx* ctx) {
    if (!ctx) return 0;
    // block state and a COMBINE of two k-summaries both in LDS
    uint32_t lo = 2, hi = kMaxK;
    auto fits = [&](uint32_t k) {
        return !chunk_layout(k, ctx->lds_max).global_state && combine_lds_bytes(k, false) <= ctx->lds_max &&
               extract_lds_bytes(k) <= ctx->lds_max;
    };
    if (!fits(lo)) return 0;
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo + 1) / 2;
        if (fits(mid)) lo = mid; else hi = mid - 1;
    }
    return lo;
}

int pss_batch_create(pss_ctx* ctx, uint32_t nstreams, const uint32_t* const* h_items, const uint64_t* h_lens,
                     const uint32_t* h_ks, uint32_t* h_chunks, int tune, pss_batch** out) {
    if (!ctx || !out || nstreams == 0 || !h_items || !h_lens || !h_ks || !h_chunks) return PSS_EINVAL;
    *out = nullptr;
    const uint32_t kcap = pss_batch_max_k(ctx);
    bool any_auto = false;
    for (uint32_t s = 0; s < nstreams; ++s) {
        if (!h_items[s] || h_ks[s] < 2) return PSS_EINVAL;
        if ((uint64_t)h_ks[s] > h_lens[s] || h_lens[s] >= kStreamBound || h_ks[s] > kcap) return PSS_ERANGE;
        if (h_chunks[s] > kMaxChunks) return PSS_ERANGE;
        if (h_chunks[s] == 0) any_auto = true;
    }
    DeviceGuard g(ctx->device);
    pss_batch* b = new (std::nothrow) pss_batch();
    if (!b) return PSS_ENOMEM;
    b->ctx = ctx;
    int rc = PSS_OK;
    try {
        b->nstreams = nstreams;
        b->items.assign(h_items, h_items + nstreams);
        b->lens.assign(h_lens, h_lens + nstreams);
        b->ks.assign(h_ks, h_ks + nstreams);
        b->chunks.assign(h_chunks, h_chunks + nstreams);
        b->out_off.resize(nstreams);
        uint64_t o = 0;
        for (uint32_t s = 0; s < nstreams; ++s) {
            b->out_off[s] = o;
            o += b->ks[s];
        }
        b->out_entries = o;
        rc = make_streams(b);
        if (rc == PSS_OK && (tune || any_auto)) rc = autotune(b, b->own, any_auto);
        std::vector<uint32_t> all(nstreams);
        for (uint32_t s = 0; s < nstreams; ++s) all[s] = s;
        if (rc == PSS_OK) rc = build_plan(b, all, b->tune, b->chunks);
        // capture the launch sequence once; replays reuse it
        if (rc == PSS_OK) {
            hipStream_t cs = nullptr;
            if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) rc = PSS_EDEVICE;
            if (rc == PSS_OK && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
                rc = PSS_EDEVICE;
            if (rc == PSS_OK) {
                int erc = enqueue(b, cs);
                hipError_t ec = hipStreamEndCapture(cs, &b->graph);
                if (erc != PSS_OK) rc = erc;
                else if (ec != hipSuccess) rc = PSS_EDEVICE;
            }
            if (rc == PSS_OK && hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
                rc = PSS_EDEVICE;
            if (cs) (void)hipStreamDestroy(cs);
        }
        if (rc == PSS_OK) {
            b->pinned_bytes = align_up(b->out_entries * sizeof(DevEntry), 256) + align_up((size_t)nstreams * 4, 256);
            if (hipHostMalloc(&b->pinned, b->pinned_bytes, hipHostMallocDefault) != hipSuccess) {
                b->pinned = nullptr;
                rc = PSS_ENOMEM;
            }
        }
    } catch (const std::bad_alloc&) {
        rc = PSS_ENOMEM;
    }
    if (rc != PSS_OK) {
        destroy_batch(b);
        return rc;
    }
    for (uint32_t s = 0; s < nstreams; ++s) h_chunks[s] = b->chunks[s];
    *out = b;
    return PSS_OK;
}

void pss_batch_destroy(pss_batch* b) { destroy_batch(b); }

int pss_batch_run(pss_batch* b, int eager, pss_entry* h_out, uint32_t* h_counts, void* stream) {
    if (!b || !h_out || !h_counts) return PSS_EINVAL;
    DeviceGuard g(b->ctx->device);
    hipStream_t st = (hipStream_t)stream;
    int rc = PSS_OK;
    if (eager) {
        rc = enqueue(b, st);
    } else if (hipGraphLaunch(b->exec, st) != hipSuccess) {
        rc = PSS_EDEVICE;
    }
    if (rc != PSS_OK) return rc;
    const size_t eb = align_up(b->out_entries * sizeof(DevEntry), 256);
    if (hipMemcpyAsync(b->pinned, b->d_out, b->out_entries * sizeof(DevEntry), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipMemcpyAsync((char*)b->pinned + eb, b->d_counts, (size_t)b->nstreams * 4, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return PSS_EDEVICE;
    const uint32_t* cnt = (const uint32_t*)((const char*)b->pinned + eb);
    for (uint32_t s = 0; s < b->nstreams; ++s)
        if (cnt[s] > b->ks[s]) return PSS_EDEVICE;  // a kernel reported a failed invariant
    for (uint32_t s = 0; s < b->nstreams; ++s) {
        h_counts[s] = cnt[s];
        memcpy(h_out + b->out_off[s], (const char*)b->pinned + b->out_off[s] * sizeof(DevEntry),
               (size_t)cnt[s] * sizeof(pss_entry));
    }
    return PSS_OK;
}

int pss_batch_info(const pss_batch* b, pss_batch_info_t* info) {
    if (!b || !info) return PSS_EINVAL;
    info->nstreams = b->nstreams;
    info->nblocks = b->nblocks;
    info->nlevels = (uint32_t)b->levels.size();
    info->nclasses = (uint32_t)b->classes.size();
    info->target_len = b->tune.target_len;
    info->slots_x16 = b->tune.slots_x16;
    info->waves_per_group = b->tune.waves;
    info->tune_candidates = b->tune_candidates;
    info->tune_ms = b->tune_ms;
    info->report_entries = b->out_entries;
    return PSS_OK;
}

int pss_run_batched(pss_ctx* ctx, uint32_t nstreams, const uint32_t* const* h_items, const uint64_t* h_lens,
                    const uint32_t* h_ks, uint32_t* h_chunks, pss_entry* h_out, uint32_t* h_counts, void* stream) {
    if (!h_out || !h_counts) return PSS_EINVAL;
    pss_batch* b = nullptr;
    int rc = pss_batch_create(ctx, nstreams, h_items, h_lens, h_ks, h_chunks, 0, &b);
    if (rc != PSS_OK) return rc;
    rc = pss_batch_run(b, 0, h_out, h_counts, stream);
    pss_batch_destroy(b);
    return rc;
}

}  // extern "C"
