// Host-side state of a libpss context, shared by the C-ABI translation
// units (plain and batched paths).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <vector>

#include "pss.h"

namespace pss {

constexpr uint32_t kMaxChunks = 1u << 22;
// Largest k: the HBM-resident block state indexes counters and hash slots
// with 32 bits, and the report sorts next_pow2(k) entries in one workgroup.
constexpr uint32_t kMaxK = 1u << 20;

// Device allocation that only grows (hipFree waits for the device).
struct DeviceBuffer {
    void* ptr = nullptr;
    size_t bytes = 0;
    int grow(size_t need) {
        if (need <= bytes) return PSS_OK;
        void* p = nullptr;
        if (hipMalloc(&p, need) != hipSuccess) return PSS_ENOMEM;
        if (ptr) (void)hipFree(ptr);
        ptr = p;
        bytes = need;
        return PSS_OK;
    }
    void release() {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Makes `dev` current for the scope.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Chunk count for n items and k counters on a device with these
// properties (pss_plan_chunks).
uint32_t plan_chunks(int cu_count, size_t lds_per_cu, size_t lds_max, uint64_t n, uint32_t k);
// The same for the Frequent block kernel, from its own LDS footprint
// (pss_frequent_plan_chunks).
uint32_t plan_frequent_chunks(int cu_count, size_t lds_per_cu, uint64_t n, uint32_t k);

// The HIP error behind the last PSS_EDEVICE returned on this thread.
extern thread_local int t_last_device_error;

inline int check(hipError_t e) {
    if (e == hipSuccess) return PSS_OK;
    t_last_device_error = (int)e;
    return PSS_EDEVICE;
}

struct PhaseMark {
    int phase;
    hipEvent_t a, b;
};

}  // namespace pss

struct pss_ctx {
    int device = 0;
    bool timing = false;
    std::vector<hipEvent_t> event_pool;
    std::vector<pss::PhaseMark> marks;
    double phase_ms[4] = {0, 0, 0, 0};
    uint32_t phase_n[4] = {0, 0, 0, 0};
    int cu_count = 0;
    size_t budget = 0;           // device bytes the workspaces below may hold in all (0 = no limit)
    size_t lds_max = 0;          // dynamic LDS per workgroup
    size_t lds_per_cu = 0;
    pss::DeviceBuffer blocks;    // block summaries of one update
    pss::DeviceBuffer gstate;    // per-block scratch: state slabs (when the state does not fit LDS) and error arrays
    pss::DeviceBuffer cscratch;  // COMBINE level slabs when they do not fit LDS
    pss::DeviceBuffer wscratch;  // fold / merge / report arrays when they do not fit LDS
    pss::DeviceBuffer query;     // report buffer
    void* pinned = nullptr;      // host staging for reports
    size_t pinned_bytes = 0;
    std::map<uint32_t, pss_summary*> run_cache;
};
