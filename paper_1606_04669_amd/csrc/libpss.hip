// C-ABI of libpss: contexts, device-resident summaries, and the launch
// sequence of the parallel algorithm (Algorithm 1): block summaries, the fixed
// COMBINE tree, the fold into the live summary, and the report.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <vector>
#include <mutex>
#include <new>
#include <string.h>

#include "pss.h"
#include "pss_ctx.h"
#include "pss_kernels.h"
#include "pss_layout.h"

using namespace pss;

namespace {

// Device memory the HBM-resident block states of one update may take; the
// planner lowers C below this.
constexpr size_t kStateBudget = 16ull << 30;
// Rounds of resident waves the planner aims for: more blocks even out the
// tail of the block launch, fewer keep the reduction tree small.
#ifndef PSS_PLAN_ROUNDS
#define PSS_PLAN_ROUNDS 4
#endif
constexpr uint64_t kPlanRounds = PSS_PLAN_ROUNDS;

}  // namespace

namespace pss {
thread_local int t_last_device_error = 0;

namespace {
// Blocks for n items and k counters when per_cu block waves fit a CU at once:
// `rounds` times the resident waves of the chip, while keeping blocks long
// next to k (the reduction tree moves ~C*k entries).
uint64_t plan_for_residency(int cu_count, uint64_t per_cu, uint64_t n, uint32_t k, uint64_t rounds) {
    per_cu = std::min<uint64_t>(std::max<uint64_t>(per_cu, 1), 32);  // 32 waves per CU at most
    const uint64_t want = (uint64_t)std::max(cu_count, 1) * per_cu * rounds;
    uint64_t cap_len = n / (16ull * k);
    if (cap_len < 1) cap_len = 1;
    return std::min(want, cap_len);
}
}  // namespace

uint32_t plan_chunks(int cu_count, size_t lds_per_cu, size_t lds_max, uint64_t n, uint32_t k) {
    if (n == 0 || k < 2) return 1;
    if (k > kMaxK) k = kMaxK;
    const ChunkLayout L = chunk_layout(k, lds_max);
    const uint64_t per_cu = lds_waves(lds_per_cu, L.lds_bytes);
    // many resident waves (small k): twice the rounds, the tree stays cheap.
    // The LDS classes with few resident waves (k > 1024) run one round: their
    // blocks are alike in length and finish together, and their tree is the
    // costly one.
    const uint64_t rounds = per_cu >= 8 ? 2 * kPlanRounds : L.global_state ? kPlanRounds : 1;
    uint64_t c = plan_for_residency(cu_count, per_cu, n, k, rounds);
    if (L.global_state) c = std::min<uint64_t>(c, kStateBudget / (L.state_bytes + 4ull * L.err_stride));
    c = std::min<uint64_t>(c, kMaxChunks);
    return (uint32_t)std::max<uint64_t>(c, 1);
}

uint32_t plan_frequent_chunks(int cu_count, size_t lds_per_cu, uint64_t n, uint32_t k) {
    if (n == 0 || k < 2) return 1;
    if (k > kMaxK) k = kMaxK;
    const uint64_t per_cu = lds_waves(lds_per_cu, FreqLayout::make(k).lds_bytes);
    // the Frequent block's decrement passes make its block lengths uneven:
    // several rounds even them out
    const uint64_t c = plan_for_residency(cu_count, per_cu, n, k, per_cu >= 8 ? 2 * kPlanRounds : kPlanRounds);
    return (uint32_t)std::max<uint64_t>(std::min<uint64_t>(c, kMaxChunks), 1);
}
}  // namespace pss

namespace {
// Concurrent COMBINE workgroups (one scratch slab each) when a COMBINE's
// arrays do not fit LDS.
constexpr uint32_t kCombineSlabsPerCu = 2;

}  // namespace

struct pss_summary {
    pss_ctx* ctx = nullptr;
    uint32_t k = 0;
    void* mem = nullptr;
    WideSummary view{};  // entries, header, and on the device the stream length N and the fault word
};

namespace {

BlockSummaries carve_blocks(void* base, uint32_t chunks, uint32_t k) {
    BlockSummaries v;
    size_t per = (size_t)chunks * k * sizeof(uint32_t);
    char* p = (char*)base;
    v.item = (uint32_t*)p;
    p += align_up(per, 256);
    v.cnt = (uint32_t*)p;
    p += align_up(per, 256);
    v.err = (uint32_t*)p;
    p += align_up(per, 256);
    v.size = (uint32_t*)p;
    p += align_up((size_t)chunks * 4, 256);
    v.min = (uint32_t*)p;
    return v;
}

size_t blocks_bytes(uint32_t chunks, uint32_t k) {
    size_t per = (size_t)chunks * k * sizeof(uint32_t);
    return 3 * align_up(per, 256) + 2 * align_up((size_t)chunks * 4, 256);
}

size_t summary_bytes(uint32_t k) {
    return align_up((size_t)k * 4, 256) + 2 * align_up((size_t)k * 8, 256) + 256 + 256;
}

// Header block (256 B): size (u32), fault word (u32), N (u64); then min.
WideSummary carve_summary(void* base, uint32_t k) {
    WideSummary v;
    char* p = (char*)base;
    v.item = (uint32_t*)p;
    p += align_up((size_t)k * 4, 256);
    v.cnt = (uint64_t*)p;
    p += align_up((size_t)k * 8, 256);
    v.err = (uint64_t*)p;
    p += align_up((size_t)k * 8, 256);
    v.size = (uint32_t*)p;
    v.fault = (uint32_t*)(p + 4);
    v.total = (uint64_t*)(p + 8);
    p += 256;
    v.min = (uint64_t*)p;
    return v;
}

bool k_fits(const pss_ctx*, uint32_t k) { return k >= 2 && k <= kMaxK; }

size_t ctx_device_bytes(const pss_ctx* ctx) {
    return ctx->blocks.bytes + ctx->gstate.bytes + ctx->cscratch.bytes + ctx->wscratch.bytes + ctx->query.bytes;
}

// Grows one of the context's workspaces within its device-memory budget
// (0 = none): PSS_ENOMEM, before anything is launched, when it would not fit.
int ctx_grow(pss_ctx* ctx, DeviceBuffer& b, size_t need) {
    if (need <= b.bytes) return PSS_OK;
    if (ctx->budget && ctx_device_bytes(ctx) - b.bytes + need > ctx->budget) return PSS_ENOMEM;
    return b.grow(need);
}

// Where the arrays of each kernel live for k counters on this device.
struct KPlan {
    ChunkLayout L;
    bool comb_lds;  // block-tree COMBINE (32-bit counts)
    bool wide_lds;  // fold / merge (64-bit counts)
    bool ext_lds;   // report sort
};

KPlan kplan(const pss_ctx* ctx, uint32_t k) {
    KPlan p;
    p.L = chunk_layout(k, ctx->lds_max);
    p.comb_lds = combine_lds_bytes(k, false) <= ctx->lds_max;
    p.wide_lds = combine_lds_bytes(k, true) <= ctx->lds_max;
    p.ext_lds = extract_lds_bytes(k) <= ctx->lds_max;
    return p;
}

uint32_t combine_slabs(const pss_ctx* ctx) { return (uint32_t)std::max(1, ctx->cu_count) * kCombineSlabsPerCu; }

// Scratch of fold, merge and report (stream-ordered, so one buffer serves all).
int ensure_wscratch(pss_ctx* ctx, const KPlan& p, uint32_t k) {
    size_t need = 0;
    if (!p.wide_lds) need = std::max(need, combine_scratch_bytes(k, true));
    if (!p.ext_lds) need = std::max(need, extract_scratch_bytes(k));
    return need ? ctx_grow(ctx, ctx->wscratch, need) : PSS_OK;
}

hipEvent_t take_event(pss_ctx* ctx) {
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records an event on the stream when timing is on; returns it (or null).
hipEvent_t mark(pss_ctx* ctx, hipStream_t st) {
    if (!ctx->timing) return nullptr;
    hipEvent_t e = take_event(ctx);
    if (e && hipEventRecord(e, st) != hipSuccess) {
        ctx->event_pool.push_back(e);
        return nullptr;
    }
    return e;
}

void close_phase(pss_ctx* ctx, int phase, hipEvent_t a, hipStream_t st) {
    if (!a) return;
    hipEvent_t b = mark(ctx, st);
    if (!b) {
        ctx->event_pool.push_back(a);
        return;
    }
    try {
        ctx->marks.push_back(PhaseMark{phase, a, b});
    } catch (...) {
        ctx->event_pool.push_back(a);
        ctx->event_pool.push_back(b);
    }
}

// block summaries of d_items[0, n) into the context workspace
int run_blocks(pss_ctx* ctx, const KPlan& p, const uint32_t* d_items, uint64_t n, uint32_t chunks, hipStream_t st,
               BlockSummaries* out) {
    const uint32_t k = p.L.k;
    int rc = ctx_grow(ctx, ctx->blocks, blocks_bytes(chunks, k));
    if (rc != PSS_OK) return rc;
    // per-block scratch: the state slabs (state in device memory), then the
    // error arrays
    const size_t gbytes = p.L.global_state ? align_up((size_t)chunks * p.L.state_bytes, 256) : 0;
    rc = ctx_grow(ctx, ctx->gstate, gbytes + (size_t)chunks * p.L.err_stride * 4);
    if (rc != PSS_OK) return rc;
    unsigned char* gs = p.L.global_state ? (unsigned char*)ctx->gstate.ptr : nullptr;
    uint32_t* errs = (uint32_t*)((unsigned char*)ctx->gstate.ptr + gbytes);
    *out = carve_blocks(ctx->blocks.ptr, chunks, k);
    return check(launch_chunk_summary(d_items, n, chunks, p.L, *out, gs, errs, st));
}

int ensure_pinned(pss_ctx* ctx, size_t bytes) {
    if (bytes <= ctx->pinned_bytes) return PSS_OK;
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return PSS_ENOMEM;
    if (ctx->pinned) hipHostFree(ctx->pinned);
    ctx->pinned = p;
    ctx->pinned_bytes = bytes;
    return PSS_OK;
}

}  // namespace

extern "C" {

int pss_timing_enable(pss_ctx* ctx, int enable) {
    if (!ctx) return PSS_EINVAL;
    ctx->timing = enable != 0;
    return PSS_OK;
}

int pss_phase_times(pss_ctx* ctx, double* ms, uint32_t* launches, int reset) {
    if (!ctx) return PSS_EINVAL;
    DeviceGuard g(ctx->device);
    int rc = PSS_OK;
    for (const PhaseMark& pm : ctx->marks) {
        float t = 0.f;
        if (hipEventSynchronize(pm.b) != hipSuccess || hipEventElapsedTime(&t, pm.a, pm.b) != hipSuccess)
            rc = PSS_EDEVICE;
        else {
            ctx->phase_ms[pm.phase] += t;
            ctx->phase_n[pm.phase] += 1;
        }
        ctx->event_pool.push_back(pm.a);
        ctx->event_pool.push_back(pm.b);
    }
    ctx->marks.clear();
    for (int i = 0; i < 4; ++i) {
        if (ms) ms[i] = ctx->phase_ms[i];
        if (launches) launches[i] = ctx->phase_n[i];
        if (reset) {
            ctx->phase_ms[i] = 0;
            ctx->phase_n[i] = 0;
        }
    }
    return rc;
}

int pss_last_device_error(void) { return pss::t_last_device_error; }

int pss_ctx_set_budget(pss_ctx* ctx, uint64_t bytes) {
    if (!ctx) return PSS_EINVAL;
    ctx->budget = (size_t)bytes;
    return PSS_OK;
}

const char* pss_device_error_name(int hip_error) { return hipGetErrorName((hipError_t)hip_error); }

const char* pss_strerror(int code) {
    switch (code) {
    case PSS_OK: return "ok";
    case PSS_EINVAL: return "invalid argument";
    case PSS_ERANGE: return "size out of supported range";
    case PSS_ENOMEM: return "out of memory";
    case PSS_EBUSY: return "resource busy";
    case PSS_ETRUNC: return "output buffer too small";
    case PSS_EDEVICE: return "HIP device error";
    default: return "unknown error";
    }
}

int pss_ctx_create(int device, pss_ctx** out) {
    if (!out) return PSS_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return PSS_EDEVICE;
    if (device < 0 || device >= ndev) return PSS_EINVAL;
    pss_ctx* ctx = new (std::nothrow) pss_ctx();
    if (!ctx) return PSS_ENOMEM;
    ctx->device = device;
    DeviceGuard g(device);
    int cus = 0, lds = 0, ldscu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) {
        delete ctx;
        return PSS_EDEVICE;
    }
    if (hipDeviceGetAttribute(&ldscu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) != hipSuccess)
        ldscu = lds;
    ctx->cu_count = cus;
    ctx->lds_max = (size_t)lds;
    ctx->lds_per_cu = (size_t)(ldscu > 0 ? ldscu : lds);
    *out = ctx;
    return PSS_OK;
}

void pss_ctx_destroy(pss_ctx* ctx) {
    if (!ctx) return;
    DeviceGuard g(ctx->device);
    for (auto& kv : ctx->run_cache) pss_destroy(kv.second);
    pss_phase_times(ctx, nullptr, nullptr, 1);
    for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
    ctx->blocks.release();
    ctx->gstate.release();
    ctx->cscratch.release();
    ctx->wscratch.release();
    ctx->query.release();
    if (ctx->pinned) hipHostFree(ctx->pinned);
    delete ctx;
}

uint32_t pss_max_k(const pss_ctx* ctx) { return ctx ? kMaxK : 0; }

uint32_t pss_max_lds_k(const pss_ctx* ctx) {
    if (!ctx) return 0;
    // the LDS-resident layout grows with k, so the largest fitting k is found by bisection
    uint32_t lo = 2, hi = kMaxK;
    if (chunk_layout(lo, ctx->lds_max).global_state) return 0;
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo + 1) / 2;
        if (!chunk_layout(mid, ctx->lds_max).global_state) lo = mid; else hi = mid - 1;
    }
    return lo;
}

uint32_t pss_plan_chunks(const pss_ctx* ctx, uint64_t n, uint32_t k) {
    if (!ctx) return 1;
    return pss::plan_chunks(ctx->cu_count, ctx->lds_per_cu, ctx->lds_max, n, k);
}

uint32_t pss_frequent_plan_chunks(const pss_ctx* ctx, uint64_t n, uint32_t k) {
    if (!ctx) return 1;
    return pss::plan_frequent_chunks(ctx->cu_count, ctx->lds_per_cu, n, k);
}

int pss_tune_chunks(pss_ctx* ctx, const uint32_t* d_items, uint64_t n, uint32_t k, void* stream,
                    uint32_t* best_chunks, double* best_ms) {
    if (!ctx || !d_items || !best_chunks) return PSS_EINVAL;
    if (k < 2) return PSS_EINVAL;
    if (!k_fits(ctx, k) || n == 0 || n >= kStreamBound) return PSS_ERANGE;
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const KPlan kp = kplan(ctx, k);
    const uint32_t base = pss_plan_chunks(ctx, n, k);
    std::vector<uint32_t> cand;
    // with the block state in device memory, no candidate beyond the planner's state budget
    const uint64_t cap = kp.L.global_state ? kStateBudget / (kp.L.state_bytes + 4ull * kp.L.err_stride) : kMaxChunks;
    for (uint64_t c : {(uint64_t)base / 4, (uint64_t)base / 2, (uint64_t)base, (uint64_t)2 * base}) {
        c = std::max<uint64_t>(1, std::min<uint64_t>({c, (uint64_t)kMaxChunks, cap, n}));
        if (std::find(cand.begin(), cand.end(), (uint32_t)c) == cand.end()) cand.push_back((uint32_t)c);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return PSS_EDEVICE;
    }
    uint32_t best = base;
    float best_t = -1.f;
    int rc = PSS_OK;
    for (uint32_t C : cand) {
        // the block summaries and the tree: the steps whose cost depends on C
        unsigned char* cs = nullptr;
        uint32_t slabs = 0;
        if (!kp.comb_lds && C > 1) {
            slabs = std::min(combine_slabs(ctx), C / 2);
            rc = ctx_grow(ctx, ctx->cscratch, (size_t)slabs * combine_scratch_bytes(k, false));
            if (rc != PSS_OK) break;
            cs = (unsigned char*)ctx->cscratch.ptr;
        }
        float t_min = -1.f;
        for (int rep = 0; rep < 3 && rc == PSS_OK; ++rep) {  // the first is a warm-up
            BlockSummaries b;
            if (hipEventRecord(e0, st) != hipSuccess) rc = PSS_EDEVICE;
            if (rc == PSS_OK) rc = run_blocks(ctx, kp, d_items, n, C, st, &b);
            for (uint32_t step = 1; rc == PSS_OK && step < C; step <<= 1)
                rc = check(launch_combine_level(b, k, C, step, kp.comb_lds, cs, slabs, st));
            float t = 0.f;
            if (rc == PSS_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                 hipEventElapsedTime(&t, e0, e1) != hipSuccess))
                rc = PSS_EDEVICE;
            if (rc == PSS_OK && rep > 0 && (t_min < 0.f || t < t_min)) t_min = t;
        }
        if (rc != PSS_OK) break;
        if (best_t < 0.f || t_min < best_t) {
            best_t = t_min;
            best = C;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != PSS_OK) return rc;
    *best_chunks = best;
    if (best_ms) *best_ms = best_t;
    return PSS_OK;
}

int pss_create(pss_ctx* ctx, uint32_t k, pss_summary** out) {
    if (!ctx || !out) return PSS_EINVAL;
    *out = nullptr;
    if (k < 2) return PSS_EINVAL;
    if (!k_fits(ctx, k)) return PSS_ERANGE;
    DeviceGuard g(ctx->device);
    pss_summary* s = new (std::nothrow) pss_summary();
    if (!s) return PSS_ENOMEM;
    s->ctx = ctx;
    s->k = k;
    if (hipMalloc(&s->mem, summary_bytes(k)) != hipSuccess) {
        delete s;
        return PSS_ENOMEM;
    }
    s->view = carve_summary(s->mem, k);
    if (hipMemset(s->view.size, 0, 256) != hipSuccess || hipMemset(s->view.min, 0, 256) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        hipFree(s->mem);
        delete s;
        return PSS_EDEVICE;
    }
    *out = s;
    return PSS_OK;
}

void pss_destroy(pss_summary* s) {
    if (!s) return;
    DeviceGuard g(s->ctx->device);
    if (s->mem) hipFree(s->mem);
    delete s;
}

int pss_update(pss_summary* s, const uint32_t* d_items, uint64_t n, uint32_t chunks, void* stream,
               uint32_t* chunks_used) {
    if (!s) return PSS_EINVAL;
    pss_ctx* ctx = s->ctx;
    const uint32_t k = s->k;
    if (n == 0) {
        if (chunks_used) *chunks_used = chunks;
        return PSS_OK;
    }
    if (!d_items) return PSS_EINVAL;
    if (n >= kStreamBound) return PSS_ERANGE;
    const uint32_t C = chunks ? chunks : pss_plan_chunks(ctx, n, k);
    if (C > kMaxChunks) return PSS_ERANGE;
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const KPlan kp = kplan(ctx, k);
    int rc = ensure_wscratch(ctx, kp, k);
    if (rc != PSS_OK) return rc;
    unsigned char* cs = nullptr;
    uint32_t slabs = 0;
    if (!kp.comb_lds && C > 1) {
        slabs = std::min(combine_slabs(ctx), C / 2);
        rc = ctx_grow(ctx, ctx->cscratch, (size_t)slabs * combine_scratch_bytes(k, false));
        if (rc != PSS_OK) return rc;
        cs = (unsigned char*)ctx->cscratch.ptr;
    }
    BlockSummaries b;
    hipEvent_t t0 = mark(ctx, st);
    rc = run_blocks(ctx, kp, d_items, n, C, st, &b);
    if (rc != PSS_OK) return rc;
    close_phase(ctx, 0, t0, st);
    hipEvent_t t1 = mark(ctx, st);
    for (uint32_t step = 1; step < C; step <<= 1) {
        rc = check(launch_combine_level(b, k, C, step, kp.comb_lds, cs, slabs, st));
        if (rc != PSS_OK) return rc;
    }
    close_phase(ctx, 1, t1, st);
    hipEvent_t t2 = mark(ctx, st);
    rc = check(launch_fold(s->view, b, k, n, kp.wide_lds, (unsigned char*)ctx->wscratch.ptr, st));
    if (rc != PSS_OK) return rc;
    close_phase(ctx, 2, t2, st);
    if (chunks_used) *chunks_used = C;
    return PSS_OK;
}

int pss_merge(pss_summary* dst, const pss_summary* src, void* stream) {
    if (!dst || !src || dst == src) return PSS_EINVAL;
    if (dst->k != src->k || dst->ctx->device != src->ctx->device) return PSS_EINVAL;
    pss_ctx* ctx = dst->ctx;
    DeviceGuard g(ctx->device);
    const KPlan kp = kplan(ctx, dst->k);
    int rc = ensure_wscratch(ctx, kp, dst->k);
    if (rc != PSS_OK) return rc;
    rc = check(launch_merge(dst->view, src->view, dst->k, kp.wide_lds, (unsigned char*)ctx->wscratch.ptr,
                            (hipStream_t)stream));
    return rc;
}

int pss_query(const pss_summary* s, int kind, pss_entry* h_out, uint32_t cap, uint32_t* n_out,
              uint64_t* stream_len, void* stream) {
    if (!s || !n_out || (cap > 0 && !h_out)) return PSS_EINVAL;
    if (kind != PSS_Q_MAJORITY && kind != PSS_Q_TOPK) return PSS_EINVAL;
    pss_ctx* ctx = s->ctx;
    const uint32_t k = s->k;
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const size_t ebytes = (size_t)k * sizeof(DevEntry);
    const size_t qbytes = 256 + ebytes;
    const KPlan kp = kplan(ctx, k);
    int rc = ensure_wscratch(ctx, kp, k);
    if (rc != PSS_OK) return rc;
    rc = ctx_grow(ctx, ctx->query, qbytes);
    if (rc != PSS_OK) return rc;
    rc = ensure_pinned(ctx, qbytes);
    if (rc != PSS_OK) return rc;
    uint32_t* d_count = (uint32_t*)ctx->query.ptr;
    DevEntry* d_ent = (DevEntry*)((char*)ctx->query.ptr + 256);
    const uint32_t dev_cap = kind == PSS_Q_TOPK ? std::min(cap, k) : k;
    hipEvent_t t3 = mark(ctx, st);
    rc = check(launch_extract(s->view, k, kind, dev_cap, d_ent, d_count, kp.ext_lds,
                              (unsigned char*)ctx->wscratch.ptr, st));
    if (rc != PSS_OK) return rc;
    if (hipMemcpyAsync(ctx->pinned, ctx->query.ptr, qbytes, hipMemcpyDeviceToHost, st) != hipSuccess)
        return PSS_EDEVICE;
    close_phase(ctx, 3, t3, st);
    if (hipStreamSynchronize(st) != hipSuccess) return PSS_EDEVICE;
    const uint32_t q = ((const uint32_t*)ctx->pinned)[0];
    const uint32_t fault = ((const uint32_t*)ctx->pinned)[1];
    const uint64_t N = ((const uint64_t*)ctx->pinned)[1];
    if (stream_len) *stream_len = N;
    // an earlier update or merge found a failed block and left the summary as
    // it was: reported once, here
    if (fault) return PSS_EDEVICE;
    if (q > k) return PSS_EDEVICE;  // a kernel reported a failed invariant
    *n_out = q;
    if (kind == PSS_Q_MAJORITY && q > cap) return PSS_ETRUNC;
    const uint32_t w = std::min(q, cap);
    if (w) memcpy(h_out, (const char*)ctx->pinned + 256, (size_t)w * sizeof(pss_entry));
    return PSS_OK;
}

int pss_run(pss_ctx* ctx, const uint32_t* d_items, uint64_t n, uint32_t k, uint32_t chunks, pss_entry* h_out,
            uint32_t cap, uint32_t* n_out, uint32_t* chunks_used, void* stream) {
    if (!ctx || !d_items || !n_out || (cap > 0 && !h_out)) return PSS_EINVAL;
    if (k < 2 || (uint64_t)k > n) return PSS_ERANGE;
    if (!k_fits(ctx, k)) return PSS_ERANGE;
    DeviceGuard g(ctx->device);
    pss_summary* s = nullptr;
    try {
        auto it = ctx->run_cache.find(k);
        if (it == ctx->run_cache.end()) {
            int rc = pss_create(ctx, k, &s);
            if (rc != PSS_OK) return rc;
            ctx->run_cache[k] = s;
        } else {
            s = it->second;
        }
    } catch (const std::bad_alloc&) {
        if (s) pss_destroy(s);
        return PSS_ENOMEM;
    }
    hipStream_t st = (hipStream_t)stream;
    int rc = check(launch_reset(s->view, st));
    if (rc != PSS_OK) return rc;
    rc = pss_update(s, d_items, n, chunks, stream, chunks_used);
    if (rc != PSS_OK) return rc;
    return pss_query(s, PSS_Q_MAJORITY, h_out, cap, n_out, nullptr, stream);
}

// ---- Frequent (Misra-Gries) in the same pipeline ----

namespace {

// Largest k of the Frequent path on this context: block state, merge and
// report all in LDS.
bool frequent_k_fits(const pss_ctx* ctx, uint32_t k) {
    return k >= 2 && k <= kMaxK && FreqLayout::make(k).lds_bytes <= ctx->lds_max &&
           frequent_merge_lds_bytes(k) <= ctx->lds_max && extract_lds_bytes(k) <= ctx->lds_max;
}

int frequent_blocks(pss_ctx* ctx, const uint32_t* d_items, uint64_t n, uint32_t k, uint32_t chunks, hipStream_t st,
                    BlockSummaries* out) {
    int rc = ctx_grow(ctx, ctx->blocks, blocks_bytes(chunks, k));
    if (rc != PSS_OK) return rc;
    *out = carve_blocks(ctx->blocks.ptr, chunks, k);
    return check(launch_frequent_blocks(d_items, n, chunks, FreqLayout::make(k), *out, st));
}

}  // namespace

uint32_t pss_frequent_max_k(const pss_ctx* ctx) {
    if (!ctx) return 0;
    uint32_t lo = 2, hi = kMaxK;
    if (!frequent_k_fits(ctx, lo)) return 0;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo + 1) / 2;
        if (frequent_k_fits(ctx, mid)) lo = mid; else hi = mid - 1;
    }
    return lo;
}

int pss_frequent_run(pss_ctx* ctx, const uint32_t* d_items, uint64_t n, uint32_t k, uint32_t chunks, int kind,
                     pss_entry* h_out, uint32_t cap, uint32_t* n_out, uint64_t* h_decrements, uint32_t* chunks_used,
                     void* stream) {
    if (!ctx || !d_items || !n_out || (cap > 0 && !h_out)) return PSS_EINVAL;
    if (kind != PSS_Q_MAJORITY && kind != PSS_Q_TOPK) return PSS_EINVAL;
    if (k < 2 || (uint64_t)k > n || n >= kStreamBound) return PSS_ERANGE;
    if (!frequent_k_fits(ctx, k)) return PSS_ERANGE;
    const uint32_t C = chunks ? chunks : pss_frequent_plan_chunks(ctx, n, k);
    if (C > kMaxChunks) return PSS_ERANGE;
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const size_t qbytes = 256 + (size_t)k * sizeof(DevEntry);
    int rc = ctx_grow(ctx, ctx->query, qbytes);
    if (rc != PSS_OK) return rc;
    rc = ensure_pinned(ctx, qbytes);
    if (rc != PSS_OK) return rc;
    BlockSummaries b;
    hipEvent_t t0 = mark(ctx, st);
    rc = frequent_blocks(ctx, d_items, n, k, C, st, &b);
    if (rc != PSS_OK) return rc;
    close_phase(ctx, 0, t0, st);
    hipEvent_t t1 = mark(ctx, st);
    for (uint32_t step = 1; rc == PSS_OK && step < C; step <<= 1) rc = check(launch_frequent_level(b, k, C, step, st));
    if (rc != PSS_OK) return rc;
    close_phase(ctx, 1, t1, st);
    uint32_t* d_count = (uint32_t*)ctx->query.ptr;
    DevEntry* d_ent = (DevEntry*)((char*)ctx->query.ptr + 256);
    const uint32_t dev_cap = kind == PSS_Q_TOPK ? std::min(cap, k) : k;
    hipEvent_t t3 = mark(ctx, st);
    rc = check(launch_frequent_report(b, k, n, kind, dev_cap, d_ent, d_count, st));
    if (rc != PSS_OK) return rc;
    if (hipMemcpyAsync(ctx->pinned, ctx->query.ptr, qbytes, hipMemcpyDeviceToHost, st) != hipSuccess)
        return PSS_EDEVICE;
    close_phase(ctx, 3, t3, st);
    if (hipStreamSynchronize(st) != hipSuccess) return PSS_EDEVICE;
    const uint32_t q = ((const uint32_t*)ctx->pinned)[0];
    if (q > k) return PSS_EDEVICE;  // a kernel reported a failed invariant
    if (h_decrements) *h_decrements = ((const uint64_t*)ctx->pinned)[1];
    if (chunks_used) *chunks_used = C;
    *n_out = q;
    if (kind == PSS_Q_MAJORITY && q > cap) return PSS_ETRUNC;
    const uint32_t w = std::min(q, cap);
    if (w) memcpy(h_out, (const char*)ctx->pinned + 256, (size_t)w * sizeof(pss_entry));
    return PSS_OK;
}

int pss_frequent_block_summaries(pss_ctx* ctx, const uint32_t* d_items, uint64_t n, uint32_t k, uint32_t chunks,
                                 const uint32_t* h_sel, uint32_t nsel, pss_entry* h_out, uint32_t* h_sizes,
                                 uint64_t* h_decrements, void* stream) {
    if (!ctx || (n > 0 && !d_items) || chunks == 0 ||
        (nsel > 0 && (!h_sel || !h_out || !h_sizes || !h_decrements)))
        return PSS_EINVAL;
    if (k < 2) return PSS_EINVAL;
    if (!frequent_k_fits(ctx, k) || n >= kStreamBound || chunks > kMaxChunks) return PSS_ERANGE;
    for (uint32_t i = 0; i < nsel; ++i)
        if (h_sel[i] >= chunks) return PSS_EINVAL;
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    BlockSummaries b;
    int rc = frequent_blocks(ctx, d_items, n, k, chunks, st, &b);
    if (rc != PSS_OK) return rc;
    if (hipStreamSynchronize(st) != hipSuccess) return PSS_EDEVICE;
    for (uint32_t i = 0; i < nsel; ++i) {
        const uint32_t c = h_sel[i];
        uint32_t sz = 0, d = 0;
        if (hipMemcpy(&sz, b.size + c, 4, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(&d, b.min + c, 4, hipMemcpyDeviceToHost) != hipSuccess)
            return PSS_EDEVICE;
        if (sz >= k) return PSS_EDEVICE;
        h_sizes[i] = sz;
        h_decrements[i] = d;
        if (sz == 0) continue;
        std::vector<uint32_t> tmp(2 * (size_t)sz);
        const size_t off = (size_t)c * k;
        if (hipMemcpy(tmp.data(), b.item + off, 4 * (size_t)sz, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(tmp.data() + sz, b.cnt + off, 4 * (size_t)sz, hipMemcpyDeviceToHost) != hipSuccess)
            return PSS_EDEVICE;
        pss_entry* o = h_out + (size_t)i * k;
        for (uint32_t e = 0; e < sz; ++e) {
            o[e].item = tmp[e];
            o[e].reserved = 0;
            o[e].count = tmp[sz + e];
            o[e].error = 0;
        }
    }
    return PSS_OK;
}

int pss_test_fold_failed_block(pss_summary* s, uint64_t n, void* stream) {
    if (!s) return PSS_EINVAL;
    pss_ctx* ctx = s->ctx;
    const uint32_t k = s->k;
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const KPlan kp = kplan(ctx, k);
    int rc = ensure_wscratch(ctx, kp, k);
    if (rc != PSS_OK) return rc;
    rc = ctx_grow(ctx, ctx->blocks, blocks_bytes(1, k));
    if (rc != PSS_OK) return rc;
    const BlockSummaries b = carve_blocks(ctx->blocks.ptr, 1, k);
    // the block kernel's failure mark: size 0xFFFFFFFF, minimum 0
    if (hipMemsetAsync(b.size, 0xFF, 4, st) != hipSuccess || hipMemsetAsync(b.min, 0, 4, st) != hipSuccess)
        return PSS_EDEVICE;
    return check(launch_fold(s->view, b, k, n, kp.wide_lds, (unsigned char*)ctx->wscratch.ptr, st));
}

int pss_block_summaries(pss_ctx* ctx, const uint32_t* d_items, uint64_t n, uint32_t k, uint32_t chunks,
                        const uint32_t* h_sel, uint32_t nsel, pss_entry* h_out, uint32_t* h_sizes,
                        uint64_t* h_mins, void* stream) {
    if (!ctx || (n > 0 && !d_items) || chunks == 0 || (nsel > 0 && (!h_sel || !h_out || !h_sizes || !h_mins)))
        return PSS_EINVAL;
    if (k < 2) return PSS_EINVAL;
    if (!k_fits(ctx, k) || n >= kStreamBound || chunks > kMaxChunks) return PSS_ERANGE;
    for (uint32_t i = 0; i < nsel; ++i)
        if (h_sel[i] >= chunks) return PSS_EINVAL;
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    BlockSummaries b;
    int rc = run_blocks(ctx, kplan(ctx, k), d_items, n, chunks, st, &b);
    if (rc != PSS_OK) return rc;
    if (hipStreamSynchronize(st) != hipSuccess) return PSS_EDEVICE;
    for (uint32_t i = 0; i < nsel; ++i) {
        const uint32_t c = h_sel[i];
        uint32_t sz = 0, mn = 0;
        if (hipMemcpy(&sz, b.size + c, 4, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(&mn, b.min + c, 4, hipMemcpyDeviceToHost) != hipSuccess)
            return PSS_EDEVICE;
        if (sz > k) return PSS_EDEVICE;
        h_sizes[i] = sz;
        h_mins[i] = mn;
        if (sz == 0) continue;
        uint32_t* tmp = new (std::nothrow) uint32_t[3 * (size_t)sz];
        if (!tmp) return PSS_ENOMEM;
        const size_t off = (size_t)c * k;
        if (hipMemcpy(tmp, b.item + off, 4 * (size_t)sz, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(tmp + sz, b.cnt + off, 4 * (size_t)sz, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(tmp + 2 * (size_t)sz, b.err + off, 4 * (size_t)sz, hipMemcpyDeviceToHost) != hipSuccess) {
            delete[] tmp;
            return PSS_EDEVICE;
        }
        pss_entry* o = h_out + (size_t)i * k;
        for (uint32_t e = 0; e < sz; ++e) {
            o[e].item = tmp[e];
            o[e].reserved = 0;
            o[e].count = tmp[sz + e];
            o[e].error = tmp[2 * (size_t)sz + e];
        }
        delete[] tmp;
    }
    return PSS_OK;
}

}  // extern "C"
