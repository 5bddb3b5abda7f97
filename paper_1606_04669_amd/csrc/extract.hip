// Report step (Algorithm 1, Pruned): the entries of a summary above the
// k-majority threshold, count * k > N (Section 3: f >= floor(N/k) + 1), or the
// first `cap` entries, in the canonical order (count desc, error asc, item
// asc).  One workgroup sorts the <= k entries in LDS with a bitonic network.
#include "pss_device.h"
#include "pss_layout.h"
#include "pss_kernels.h"

namespace pss {

constexpr uint32_t kExtractThreads = 1024;

__host__ __device__ inline uint32_t extract_cap(uint32_t k) {
    uint32_t P = next_pow2(k);
    return P < 2 ? 2 : P;
}

// Sort arrays (count, error, item) of next_pow2(k) entries, then 16 bytes of
// small shared state, which stays in LDS when the arrays go to scratch.
__host__ __device__ inline uint32_t extract_big_bytes(uint32_t k) { return extract_cap(k) * (8 + 8 + 4); }
constexpr uint32_t kExtractSmallBytes = 16;

uint32_t extract_lds_bytes(uint32_t k) { return extract_big_bytes(k) + kExtractSmallBytes; }
size_t extract_scratch_bytes(uint32_t k) { return extract_big_bytes(k); }

__device__ __forceinline__ bool ext_better(uint64_t ca, uint64_t ea, uint32_t ia, uint64_t cb, uint64_t eb,
                                           uint32_t ib) {
    if (ca != cb) return ca > cb;
    if (ea != eb) return ea < eb;
    return ia < ib;
}

// Canonical sort and report of one summary (entries s_item/s_cnt/s_err,
// `size` of them) by one workgroup.  base: the sort arrays (LDS or a scratch
// slab) for next_pow2(k) entries; small: 16 bytes of LDS.
template <typename CT>
__device__ void extract_body(const uint32_t* s_item, const CT* s_cnt, const CT* s_err, uint32_t size, uint32_t k,
                             uint64_t N, int kind, uint32_t cap, DevEntry* out, uint32_t* out_count,
                             unsigned char* base, uint32_t* small) {
    const uint32_t P0 = extract_cap(k);
    uint64_t* cc = (uint64_t*)base;
    uint64_t* ce = cc + P0;
    uint32_t* ci = (uint32_t*)(ce + P0);
    const uint32_t tid = threadIdx.x;
    if (size > k) {  // the summary carries the failure mark of a block kernel
        if (tid == 0) *out_count = 0xFFFFFFFFu;
        return;
    }
    uint32_t P = next_pow2(size);
    if (P < 2) P = 2;
    for (uint32_t i = tid; i < P; i += kExtractThreads) {
        if (i < size) {
            cc[i] = s_cnt[i];
            ce[i] = s_err[i];
            ci[i] = s_item[i];
        } else {  // padding sorts after every real entry (real counts are >= 1)
            cc[i] = 0;
            ce[i] = ~0ull;
            ci[i] = 0xFFFFFFFFu;
        }
    }
    __syncthreads();
    for (uint32_t w = 2; w <= P; w <<= 1) {
        for (uint32_t stride = w >> 1; stride > 0; stride >>= 1) {
            for (uint32_t t = tid; t < P / 2; t += kExtractThreads) {
                uint32_t i = 2 * t - (t & (stride - 1));
                uint32_t j = i + stride;
                bool up = (i & w) == 0;
                bool jb = ext_better(cc[j], ce[j], ci[j], cc[i], ce[i], ci[i]);
                if (jb == up) {
                    uint64_t tc = cc[i], te = ce[i];
                    uint32_t ti = ci[i];
                    cc[i] = cc[j]; ce[i] = ce[j]; ci[i] = ci[j];
                    cc[j] = tc; ce[j] = te; ci[j] = ti;
                }
            }
            __syncthreads();
        }
    }
    uint32_t q;
    if (kind == 0) {
        // reported prefix: count > floor(N / k)
        const uint64_t thr = N / k;
        if (tid == 0) small[0] = 0;
        __syncthreads();
        for (uint32_t i = tid; i < size; i += kExtractThreads) {
            bool in = cc[i] > thr;
            bool next_out = (i + 1 >= size) || !(cc[i + 1] > thr);
            if (in && next_out) small[0] = i + 1;
        }
        __syncthreads();
        q = small[0];
    } else {
        q = size < cap ? size : cap;
    }
    const uint32_t wn = q < cap ? q : cap;
    for (uint32_t i = tid; i < wn; i += kExtractThreads) {
        DevEntry e;
        e.item = ci[i];
        e.reserved = 0;
        e.count = cc[i];
        e.error = ce[i];
        out[i] = e;
    }
    if (tid == 0) *out_count = q;
}

// G: the sort arrays live in a global scratch slab (k beyond LDS).
// The threshold uses the summary's own N; the report header also carries
// the summary's fault word (cleared once read: it is reported once) and N.
template <bool G>
__global__ __launch_bounds__(kExtractThreads) void extract_kernel(WideSummary s, uint32_t k, int kind, uint32_t cap,
                                                                  DevEntry* out, uint32_t* out_count,
                                                                  unsigned char* scratch) {
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned char* base = G ? scratch : smem;
    uint32_t* small = (uint32_t*)(G ? smem : smem + extract_big_bytes(k));
    const uint64_t N = *s.total;
    const uint32_t fault = *s.fault;
    extract_body<uint64_t>(s.item, s.cnt, s.err, s.size[0], k, N, kind, cap, out, out_count, base, small);
    if (threadIdx.x == 0) {
        out_count[1] = fault;
        *(uint64_t*)(out_count + 2) = N;
        if (fault) *s.fault = 0u;
    }
}

// Majority reports of a batch, one workgroup per stream, straight from the
// root of its tree (32-bit counts).
__global__ __launch_bounds__(kExtractThreads) void batch_extract_kernel(const BatchReport* __restrict__ reps,
                                                                        uint32_t count, uint32_t kmax,
                                                                        BlockSummaries v, DevEntry* out,
                                                                        uint32_t* out_count) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* small = (uint32_t*)(smem + extract_big_bytes(kmax));
    for (uint32_t j = blockIdx.x; j < count; j += gridDim.x) {
        const BatchReport r = reps[j];
        __syncthreads();  // the previous stream is done with LDS
        extract_body<uint32_t>(v.item + r.root_off, v.cnt + r.root_off, v.err + r.root_off, v.size[r.root], r.k, r.n,
                               0, r.k, out + r.out_off, out_count + j, smem, small);
    }
}

hipError_t launch_batch_extract(const BatchReport* reps, uint32_t count, uint32_t kmax, const BlockSummaries& base,
                                DevEntry* out, uint32_t* out_count, hipStream_t stream) {
    (void)hipGetLastError();  // a stale error of an earlier, unrelated call is not this launch's
    if (count == 0) return hipSuccess;
    const uint32_t lds = extract_lds_bytes(kmax);
    hipFuncSetAttribute((const void*)batch_extract_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(batch_extract_kernel, dim3(count), dim3(kExtractThreads), lds, stream, reps, count, kmax, base,
                       out, out_count);
    return hipGetLastError();
}

// Majority report straight from a tree root (block summary 0, 32-bit
// counts) for a stream of N items; arguments by value, nothing to stage.
__global__ __launch_bounds__(kExtractThreads) void root_extract_kernel(BlockSummaries v, uint32_t k, uint64_t N,
                                                                       uint32_t cap, DevEntry* out,
                                                                       uint32_t* out_count) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* small = (uint32_t*)(smem + extract_big_bytes(k));
    extract_body<uint32_t>(v.item, v.cnt, v.err, v.size[0], k, N, 0, cap, out, out_count, smem, small);
}

hipError_t launch_root_extract(const BlockSummaries& v, uint32_t k, uint64_t N, uint32_t cap, DevEntry* out,
                               uint32_t* out_count, hipStream_t stream) {
    (void)hipGetLastError();  // a stale error of an earlier, unrelated call is not this launch's
    const uint32_t lds = extract_lds_bytes(k);
    hipFuncSetAttribute((const void*)root_extract_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(root_extract_kernel, dim3(1), dim3(kExtractThreads), lds, stream, v, k, N, cap, out,
                       out_count);
    return hipGetLastError();
}

// Frequent report from the root: (count + D) * k > N is count > floor(N/k) - D,
// the threshold of a stream of max(0, floor(N/k) - D) * k items; errors are 0,
// so the canonical order is count descending, item ascending.
__global__ __launch_bounds__(kExtractThreads) void frequent_report_kernel(BlockSummaries v, uint32_t k, uint64_t N,
                                                                          int kind, uint32_t cap, DevEntry* out,
                                                                          uint32_t* out_count) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* small = (uint32_t*)(smem + extract_big_bytes(k));
    const uint64_t d = v.min[0];
    const uint64_t q = N / k;
    const uint64_t n_eff = q > d ? (q - d) * k : 0;
    extract_body<uint32_t>(v.item, v.cnt, v.err, v.size[0], k, n_eff, kind, cap, out, out_count, smem, small);
    if (threadIdx.x == 0) *(uint64_t*)(out_count + 2) = d;
}

hipError_t launch_frequent_report(const BlockSummaries& v, uint32_t k, uint64_t N, int kind, uint32_t cap,
                                  DevEntry* out, uint32_t* out_count, hipStream_t stream) {
    (void)hipGetLastError();  // a stale error of an earlier, unrelated call is not this launch's
    const uint32_t lds = extract_lds_bytes(k);
    hipFuncSetAttribute((const void*)frequent_report_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(frequent_report_kernel, dim3(1), dim3(kExtractThreads), lds, stream, v, k, N, kind, cap, out,
                       out_count);
    return hipGetLastError();
}

// Served queries: one workgroup per query on a persistent summary of the
// pool (u64 counts), kind and cap per query.
__global__ __launch_bounds__(kExtractThreads) void serve_query_kernel(const ServeQuery* __restrict__ q,
                                                                      uint32_t count, uint32_t kmax,
                                                                      WideSummary pool, DevEntry* out,
                                                                      uint32_t* out_count) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* small = (uint32_t*)(smem + extract_big_bytes(kmax));
    for (uint32_t j = blockIdx.x; j < count; j += gridDim.x) {
        const ServeQuery d = q[j];
        __syncthreads();  // the previous query is done with LDS
        extract_body<uint64_t>(pool.item + d.s_off, pool.cnt + d.s_off, pool.err + d.s_off, pool.size[d.sid], d.k,
                               d.n, (int)d.kind, d.cap, out + d.out_off, out_count + j, smem, small);
    }
}

hipError_t launch_serve_query(const ServeQuery* q, uint32_t count, uint32_t kmax, const WideSummary& pool,
                              DevEntry* out, uint32_t* out_count, hipStream_t stream) {
    (void)hipGetLastError();  // a stale error of an earlier, unrelated call is not this launch's
    if (count == 0) return hipSuccess;
    const uint32_t lds = extract_lds_bytes(kmax);
    hipFuncSetAttribute((const void*)serve_query_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(serve_query_kernel, dim3(count), dim3(kExtractThreads), lds, stream, q, count, kmax, pool, out,
                       out_count);
    return hipGetLastError();
}

__global__ void zero_words_kernel(uint32_t* p, uint32_t count) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0u;
}

hipError_t launch_zero_words(uint32_t* p, uint32_t count, hipStream_t stream) {
    (void)hipGetLastError();  // a stale error of an earlier, unrelated call is not this launch's
    if (count == 0) return hipSuccess;
    const uint32_t grid = (count + 255) / 256 < 1024 ? (count + 255) / 256 : 1024;
    hipLaunchKernelGGL(zero_words_kernel, dim3(grid), dim3(256), 0, stream, p, count);
    return hipGetLastError();
}

hipError_t launch_extract(const WideSummary& s, uint32_t k, int kind, uint32_t cap, DevEntry* out,
                          uint32_t* out_count, bool in_lds, unsigned char* scratch, hipStream_t stream) {
    (void)hipGetLastError();  // a stale error of an earlier, unrelated call is not this launch's
    if (!s.total || !s.fault) return hipErrorInvalidValue;
    const uint32_t bytes = extract_lds_bytes(k);
    if (in_lds) {
        hipFuncSetAttribute((const void*)extract_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        hipLaunchKernelGGL(extract_kernel<false>, dim3(1), dim3(kExtractThreads), bytes, stream, s, k, kind, cap, out,
                           out_count, (unsigned char*)nullptr);
    } else {
        if (!scratch) return hipErrorInvalidValue;
        hipLaunchKernelGGL(extract_kernel<true>, dim3(1), dim3(kExtractThreads), kExtractSmallBytes, stream, s, k,
                           kind, cap, out, out_count, scratch);
    }
    return hipGetLastError();
}

__global__ void reset_kernel(WideSummary s) {
    if (threadIdx.x == 0) {
        s.size[0] = 0;
        s.min[0] = 0;
        *s.total = 0;
        *s.fault = 0u;
    }
}

hipError_t launch_reset(const WideSummary& s, hipStream_t stream) {
    (void)hipGetLastError();  // a stale error of an earlier, unrelated call is not this launch's
    if (!s.total || !s.fault) return hipErrorInvalidValue;
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, stream, s);
    return hipGetLastError();
}

}  // namespace pss
