// One-shot run of the parallel algorithm (Algorithm 1 with Algorithm 2 as
// the reduction operator) that allocates nothing, for callers that cannot
// allocate device memory: code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation.  Its workspace -- the block summaries and
// the blocks' error scratch -- is one file-scope device array; each GPU the
// library runs on holds its own copy until the process ends.  Every call on a
// GPU shares that GPU's copy, so calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pss.h"
#include "pss_ctx.h"
#include "pss_kernels.h"
#include "pss_layout.h"

#ifndef PSS_NOALLOC_SCRATCH_MIB
#define PSS_NOALLOC_SCRATCH_MIB 128
#endif

namespace pss {
namespace {

constexpr size_t kScratchBytes = (size_t)PSS_NOALLOC_SCRATCH_MIB << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Per device: the address of its copy of `scratch` (host code must not use
// the array's name as a device address) and the properties the planner uses.
struct DeviceState {
    bool ready = false;
    int rc = PSS_OK;
    unsigned char* ptr = nullptr;
    int cu_count = 0;
    size_t lds_max = 0, lds_per_cu = 0;
};
constexpr int kMaxDevices = 64;
DeviceState g_dev[kMaxDevices];
std::mutex g_mu;

// Once per device, with that device current.
int device_state(int dev, const DeviceState** out) {
    if (dev < 0 || dev >= kMaxDevices) return PSS_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceState& d = g_dev[dev];
    if (!d.ready) {
        void* p = nullptr;
        int cus = 0, lds = 0, ldscu = 0;
        d.rc = PSS_OK;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
            d.rc = PSS_EDEVICE;
        } else {
            if (hipDeviceGetAttribute(&ldscu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
                ldscu <= 0)
                ldscu = lds;
            d.ptr = (unsigned char*)p;
            d.cu_count = cus;
            d.lds_max = (size_t)lds;
            d.lds_per_cu = (size_t)ldscu;
        }
        d.ready = true;
    }
    *out = &d;
    return d.rc;
}

// Workspace of C blocks of k counters: SoA block summaries, then one error
// scratch array per block.
size_t workspace_bytes(uint32_t chunks, const ChunkLayout& L) {
    const size_t per = (size_t)chunks * L.k * 4;
    return 3 * align_up(per, 256) + 2 * align_up((size_t)chunks * 4, 256) + (size_t)chunks * L.err_stride * 4;
}

}  // namespace
}  // namespace pss

using namespace pss;

extern "C" int pss_run_noalloc(const uint32_t* d_items, uint64_t n, uint32_t k, uint32_t chunks, pss_entry* d_out,
                               uint32_t cap, uint32_t* d_nout, uint32_t* chunks_used, void* stream) {
    if (!d_items || !d_nout || (cap > 0 && !d_out)) return PSS_EINVAL;
    if (k < 2 || (uint64_t)k > n || n >= kStreamBound) return PSS_ERANGE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PSS_EDEVICE;
    const DeviceState* ds = nullptr;
    int rc = device_state(dev, &ds);
    if (rc != PSS_OK) return rc;
    // the block state, a COMBINE and the report must all fit LDS
    const ChunkLayout L = chunk_layout(k, ds->lds_max);
    if (L.global_state || combine_lds_bytes(k, false) > ds->lds_max || extract_lds_bytes(k) > ds->lds_max)
        return PSS_ERANGE;
    uint32_t C = chunks;
    if (C == 0) {
        C = plan_chunks(ds->cu_count, ds->lds_per_cu, ds->lds_max, n, k);
        while (C > 1 && workspace_bytes(C, L) > kScratchBytes) C = (uint32_t)(C - 1 - (C - 1) / 64);
    }
    if (C > kMaxChunks || workspace_bytes(C, L) > kScratchBytes) return PSS_ERANGE;
    unsigned char* p = ds->ptr;
    const size_t per = align_up((size_t)C * k * 4, 256);
    const size_t hdr = align_up((size_t)C * 4, 256);
    BlockSummaries b;
    b.item = (uint32_t*)p;
    b.cnt = (uint32_t*)(p + per);
    b.err = (uint32_t*)(p + 2 * per);
    b.size = (uint32_t*)(p + 3 * per);
    b.min = (uint32_t*)(p + 3 * per + hdr);
    uint32_t* errs = (uint32_t*)(p + 3 * per + 2 * hdr);
    hipStream_t st = (hipStream_t)stream;
    rc = check(launch_chunk_summary(d_items, n, C, L, b, nullptr, errs, st));
    for (uint32_t step = 1; rc == PSS_OK && step < C; step <<= 1)
        rc = check(launch_combine_level(b, k, C, step, true, nullptr, 0, st));
    if (rc == PSS_OK) rc = check(launch_root_extract(b, k, n, cap, (DevEntry*)d_out, d_nout, st));
    if (rc == PSS_OK && chunks_used) *chunks_used = C;
    return rc;
}

extern "C" uint64_t pss_noalloc_scratch_bytes(void) { return kScratchBytes; }
