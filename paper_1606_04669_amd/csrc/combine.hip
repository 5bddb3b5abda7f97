// COMBINE with Prune(k) (Algorithm 2) and the fixed binary reduction tree
// (Algorithm 1, ParallelReduction).  One workgroup merges one pair.
//
// Candidates of S_C live in LDS: S2's entries are staged first (count and
// error raised by m1, as for items only in S2), then every S1 entry looks its
// item up in a hash of S2: a shared item adds both estimates and retires the
// staged S2 entry; an item only in S1 is raised by m2.  Prune(k) keeps the k
// best candidates in the order (count desc, error asc, item asc): the k-th
// best key is found by a most-significant-digit radix select over the
// composite key U = (~count, error, item), smaller U = better, and every
// candidate with U at most that key is kept.  Items are unique in a summary,
// so U is a total order and the kept set is exactly the first k.
#include "pss_device.h"
#include "pss_layout.h"
#include "pss_kernels.h"

namespace pss {

// Threads of a COMBINE workgroup: 256 where many pairs share the chip, 1024
// (the candidates four times as fast per pair) where few pairs leave CUs idle
// and where the candidate arrays lie in device memory.
constexpr uint32_t kCombineThreads = 256;
constexpr uint32_t kCombineThreadsWide = 1024;
// Tree levels of at most this many pairs run with the wide workgroups.
#ifndef PSS_COMBINE_WIDE_PAIRS
#define PSS_COMBINE_WIDE_PAIRS 512
#endif
constexpr uint32_t kCombineWidePairs = PSS_COMBINE_WIDE_PAIRS;
constexpr uint8_t kAlive = 1, kCand = 2;

// Storage of one COMBINE: the candidate arrays and the S2 hash ("big",
// O(k)) live in LDS when they fit, else in a global slab per node; the
// radix-select histograms (two, used in turn) and the reduction words
// ("small") are always in LDS.
template <typename CO>
struct CombineLds {
    uint32_t cap;   // candidate capacity (2k)
    uint32_t hsize; // S2 hash slots
    uint32_t off_cc, off_ce, off_ci, off_flag, off_hash, big_bytes;
    uint32_t off_hist, off_misc, off_keys, off_red, small_bytes;

    __host__ __device__ static CombineLds make(uint32_t k) {
        CombineLds L;
        L.cap = 2 * k;
        L.hsize = next_pow2(2 * k);
        if (L.hsize < 64) L.hsize = 64;
        uint32_t o = 0;
        L.off_cc = o;   o = align16(o + sizeof(CO) * L.cap);
        L.off_ce = o;   o = align16(o + sizeof(CO) * L.cap);
        L.off_ci = o;   o = align16(o + 4 * L.cap);
        L.off_flag = o; o = align16(o + L.cap);
        L.off_hash = o; o = align16(o + 4 * L.hsize);
        L.big_bytes = o;
        L.off_hist = 0;
        L.off_misc = 2 * 4 * 256;
        L.off_keys = L.off_misc + 64;  // OR and AND of the candidates' key words
        L.off_red = L.off_keys + 64;
        L.small_bytes = L.off_red + 8 * (kCombineThreadsWide / kWave);
        return L;
    }
};

template <typename CO>
__device__ __forceinline__ uint32_t key_digit(CO c, CO e, uint32_t it, uint32_t p) {
    constexpr uint32_t W = sizeof(CO);
    if (p < W) return (uint32_t)((~c) >> (8 * (W - 1 - p))) & 255u;
    if (p < 2 * W) return (uint32_t)(e >> (8 * (2 * W - 1 - p))) & 255u;
    return (it >> (8 * (2 * W + 3 - p))) & 255u;
}

// a strictly better than b in the canonical order
template <typename CO>
__device__ __forceinline__ bool better(CO ca, CO ea, uint32_t ia, CO cb, CO eb, uint32_t ib) {
    if (ca != cb) return ca > cb;
    if (ea != eb) return ea < eb;
    return ia < ib;
}

template <uint32_t NT, typename C1, typename C2, typename CO>
__device__ void combine_node(const uint32_t* i1, const C1* c1, const C1* e1, uint32_t n1, C1 m1_,
                             const uint32_t* i2, const C2* c2, const C2* e2, uint32_t n2, C2 m2_, uint32_t k,
                             uint32_t* io, CO* co, CO* eo, uint32_t* osize, CO* omin, unsigned char* big,
                             unsigned char* small) {
    const CombineLds<CO> L = CombineLds<CO>::make(k);
    CO* cc = (CO*)(big + L.off_cc);
    CO* ce = (CO*)(big + L.off_ce);
    uint32_t* ci = (uint32_t*)(big + L.off_ci);
    uint8_t* flag = (uint8_t*)(big + L.off_flag);
    uint32_t* hash = (uint32_t*)(big + L.off_hash);
    uint32_t* hist = (uint32_t*)(small + L.off_hist);
    uint32_t* misc = (uint32_t*)(small + L.off_misc);
    const uint32_t tid = threadIdx.x;
    const uint32_t hbits = log2_pow2(L.hsize);
    const uint32_t hmask = L.hsize - 1;
    const CO m1 = (CO)m1_, m2 = (CO)m2_;
    if (n1 > k || n2 > k) {
        // an input summary carries the failure mark of a block kernel: pass it on
        if (tid == 0) {
            *osize = 0xFFFFFFFFu;
            *omin = 0;
        }
        return;
    }
    const uint32_t nc = n1 + n2;

    // a thread's first two S1 entries are loaded now, their latency hidden
    // behind staging and hashing S2
    uint32_t px[2];
    C1 pc[2], pe[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const uint32_t i = tid + (uint32_t)r * NT;
        const bool in = i < n1;
        px[r] = in ? i1[i] : 0u;
        pc[r] = in ? c1[i] : (C1)0;
        pe[r] = in ? e1[i] : (C1)0;
    }

    // stage S2 as candidates [n1, n1 + n2): items only in S2 get + m1
    for (uint32_t j = tid; j < n2; j += NT) {
        ci[n1 + j] = i2[j];
        cc[n1 + j] = (CO)c2[j] + m1;
        ce[n1 + j] = (CO)e2[j] + m1;
        flag[n1 + j] = kAlive;
    }
    for (uint32_t h = tid; h < L.hsize; h += NT) hash[h] = 0u;
    __syncthreads();
    for (uint32_t j = tid; j < n2; j += NT) {
        uint32_t h = hash_slot(ci[n1 + j], hbits);
        while (atomicCAS(&hash[h], 0u, j + 1u) != 0u) h = (h + 1) & hmask;
    }
    __syncthreads();
    // S1 entries: Find in S2, add both estimates (and retire S2's), or + m2
    for (uint32_t i = tid, r = 0; i < n1; i += NT, ++r) {
        const uint32_t x = r == 0 ? px[0] : r == 1 ? px[1] : i1[i];
        uint32_t h = hash_slot(x, hbits);
        int32_t found = -1;
        for (;;) {
            uint32_t v = hash[h];
            if (v == 0u) break;
            if (ci[n1 + v - 1] == x) {
                found = (int32_t)(v - 1);
                break;
            }
            h = (h + 1) & hmask;
        }
        CO c = r == 0 ? (CO)pc[0] : r == 1 ? (CO)pc[1] : (CO)c1[i];
        CO e = r == 0 ? (CO)pe[0] : r == 1 ? (CO)pe[1] : (CO)e1[i];
        if (found >= 0) {
            c += cc[n1 + found] - m1;
            e += ce[n1 + found] - m1;
            flag[n1 + found] = 0;
        } else {
            c += m2;
            e += m2;
        }
        ci[i] = x;
        cc[i] = c;
        ce[i] = e;
        flag[i] = kAlive;
    }
    __syncthreads();

    // number of distinct candidates, and the OR and AND of their keys
    // U = (~count, error, item) as six words (a digit on which all agree
    // selects nothing)
    uint32_t* kw = (uint32_t*)(small + L.off_keys);
    uint32_t live = 0;
    uint64_t onc = 0, anc = ~0ull, oe = 0, ae = ~0ull;
    uint32_t oi = 0, ai = ~0u;
    for (uint32_t i = tid; i < nc; i += NT) {
        if (flag[i] & kAlive) {
            const uint64_t nc_ = (uint64_t)(CO)~cc[i], e_ = (uint64_t)ce[i];
            const uint32_t i_ = ci[i];
            live += 1;
            onc |= nc_;
            anc &= nc_;
            oe |= e_;
            ae &= e_;
            oi |= i_;
            ai &= i_;
        }
    }
    if (tid < 4) misc[tid] = 0;
    if (tid < 12) kw[tid] = tid < 6 ? 0u : ~0u;  // OR words at 0..4, AND words at 6..10
    __syncthreads();
    live = wave_sum_u32(live);
    const uint32_t wo[5] = {(uint32_t)onc, (uint32_t)(onc >> 32), (uint32_t)oe, (uint32_t)(oe >> 32), oi};
    const uint32_t wa[5] = {(uint32_t)anc, (uint32_t)(anc >> 32), (uint32_t)ae, (uint32_t)(ae >> 32), ai};
    uint32_t ro[5], ra[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        if (sizeof(CO) == 4 && (j == 1 || j == 3)) {  // high words of 32-bit counts: unused
            ro[j] = 0u;
            ra[j] = ~0u;
            continue;
        }
        ro[j] = wave_or_u32(wo[j]);
        ra[j] = wave_and_u32(wa[j]);
    }
    if (lane_id() == 0) {
        atomicAdd(&misc[0], live);
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            atomicOr(&kw[j], ro[j]);
            atomicAnd(&kw[6 + j], ra[j]);
        }
    }
    __syncthreads();
    const uint32_t ns = misc[0];
    const uint64_t onc_all = ((uint64_t)kw[1] << 32) | kw[0], anc_all = ((uint64_t)kw[7] << 32) | kw[6];
    const uint64_t oe_all = ((uint64_t)kw[3] << 32) | kw[2], ae_all = ((uint64_t)kw[9] << 32) | kw[8];
    const uint32_t oi_all = kw[4], ai_all = kw[10];
    __syncthreads();

    // Prune(k): radix select of the k-th best key when there are more than k.
    // Digits on which all candidates agree are skipped; the select stops
    // once the digit's bin holding the k-th key holds it alone; each pass
    // filters by its digit and counts the next one in the other histogram.
    int32_t star = -1;  // index of the worst kept candidate
    if (ns > k) {
        constexpr uint32_t NB = 2 * sizeof(CO) + 4;
        uint32_t vary = 0;  // digit positions where the candidates' keys differ
        for (uint32_t p = 0; p < NB; ++p)
            vary |= (key_digit<CO>((CO)~onc_all, (CO)oe_all, oi_all, p) !=
                             key_digit<CO>((CO)~anc_all, (CO)ae_all, ai_all, p)
                         ? 1u
                         : 0u)
                    << p;
        // ns > k >= 1 distinct items: their keys differ somewhere
        uint32_t p = (uint32_t)__builtin_ctz(vary | (1u << (NB - 1)));
        uint32_t* hcur = hist;
        uint32_t* hnext = hist + 256;
        static_assert(NT >= 256, "a histogram bin per thread of the first 256");
        if (tid < 256) {
            hcur[tid] = 0u;
            hnext[tid] = 0u;
        }
        for (uint32_t i = tid; i < nc; i += NT) flag[i] = (flag[i] & kAlive) ? (kAlive | kCand) : 0;
        __syncthreads();
        for (uint32_t i = tid; i < nc; i += NT)
            if (flag[i] & kCand) atomicAdd(&hcur[key_digit<CO>(cc[i], ce[i], ci[i], p)], 1u);
        __syncthreads();
        uint32_t rank = k - 1;
        for (;;) {
            if (tid < kWave) {
                // bucket holding the rank-th candidate: 4 bins per lane, then a wave scan
                uint32_t b0 = hcur[4 * tid], b1 = hcur[4 * tid + 1], b2 = hcur[4 * tid + 2], b3 = hcur[4 * tid + 3];
                uint32_t s = b0 + b1 + b2 + b3, incl = s;
                for (int off = 1; off < 64; off <<= 1) {
                    uint32_t t = (uint32_t)__shfl_up((int)incl, off);
                    if ((int)tid >= off) incl += t;
                }
                uint32_t excl = incl - s;
                bool here = excl <= rank && rank < incl;
                if (here) {
                    uint32_t rr = rank - excl, bin = 4 * tid;
                    if (rr >= b0) { rr -= b0; ++bin;
                        if (rr >= b1) { rr -= b1; ++bin;
                            if (rr >= b2) { rr -= b2; ++bin; } } }
                    misc[1] = bin;
                    misc[2] = rr;
                    misc[4] = hcur[bin];
                }
            }
            __syncthreads();
            const uint32_t sel = misc[1];
            rank = misc[2];
            const uint32_t alone = misc[4] == 1u;
            vary &= ~((2u << p) - 1u);  // positions after p
            const bool last = alone || vary == 0u;
            const uint32_t pn = last ? p : (uint32_t)__builtin_ctz(vary);
            if (tid < 256) hcur[tid] = 0u;  // read by the scan only: free for the pass after next
            for (uint32_t i = tid; i < nc; i += NT) {
                if (flag[i] & kCand) {
                    const CO c = cc[i], e = ce[i];
                    const uint32_t it = ci[i];
                    if (key_digit<CO>(c, e, it, p) != sel)
                        flag[i] &= (uint8_t)~kCand;
                    else if (!last)
                        atomicAdd(&hnext[key_digit<CO>(c, e, it, pn)], 1u);
                }
            }
            __syncthreads();
            if (last) break;
            p = pn;
            uint32_t* t = hcur;
            hcur = hnext;
            hnext = t;
        }
        for (uint32_t i = tid; i < nc; i += NT)
            if (flag[i] & kCand) misc[3] = i;
        __syncthreads();
        star = (int32_t)misc[3];
        __syncthreads();
    }

    // keep = alive and not worse than the k-th best; written in candidate order
    CO sc = 0, se = 0;
    uint32_t si = 0;
    if (star >= 0) {
        sc = cc[star];
        se = ce[star];
        si = ci[star];
    }
    // Segments of up to 32 rows of 256 candidates: each wave counts its kept
    // candidates per row into a table, then every thread places its own from
    // the table's running sums (the same in every thread).
    constexpr uint32_t kWaves = NT / kWave;
    constexpr uint32_t kRows = 32;
    static_assert(kRows * kWaves <= 2 * 256, "the count table lies over the histograms");
    uint32_t* rowcnt = hist;
    const uint32_t w = tid / kWave;
    CO local_min = ~(CO)0;
    uint32_t kept = 0;
    for (uint32_t seg = 0; seg < nc; seg += kRows * NT) {
        const uint32_t rows = min(kRows, (nc - seg + NT - 1) / NT);
        uint32_t keepbits = 0;
        for (uint32_t q = 0; q < rows; ++q) {
            const uint32_t i = seg + q * NT + tid;
            bool keep = false;
            if (i < nc && (flag[i] & kAlive)) keep = (star < 0) || !better<CO>(sc, se, si, cc[i], ce[i], ci[i]);
            const uint64_t bm = ballot(keep);
            if (lane_id() == 0) rowcnt[kWaves * q + w] = popc64(bm);
            keepbits |= (keep ? 1u : 0u) << q;
        }
        __syncthreads();
        for (uint32_t q = 0; q < rows; ++q) {
            const bool keep = (keepbits >> q) & 1u;
            const uint64_t bm = ballot(keep);
            uint32_t before = kept;
            for (uint32_t v = 0; v < w; ++v) before += rowcnt[kWaves * q + v];
            if (keep) {
                const uint32_t i = seg + q * NT + tid;
                const uint32_t o = before + mbcnt(bm);
                io[o] = ci[i];
                co[o] = cc[i];
                eo[o] = ce[i];
                local_min = cc[i] < local_min ? cc[i] : local_min;
            }
            for (uint32_t v = 0; v < kWaves; ++v) kept += rowcnt[kWaves * q + v];
        }
        __syncthreads();  // the table is read before the next segment rewrites it
    }
    // minimum of the result: 0 unless all k counters are used
    const CO wmin = sizeof(CO) == 4 ? (CO)wave_min_u32((uint32_t)local_min) : (CO)wave_min_u64((uint64_t)local_min);
    uint64_t* red = (uint64_t*)(small + L.off_red);
    if (lane_id() == 0) red[tid / kWave] = (uint64_t)wmin;
    __syncthreads();
    if (tid == 0) {
        uint64_t mn = red[0];
        for (uint32_t q = 1; q < NT / kWave; ++q) mn = red[q] < mn ? red[q] : mn;
        *osize = kept;
        *omin = (kept == k) ? (CO)mn : (CO)0;
    }
}

// One workgroup per pair of the level, or (global storage) a bounded grid
// whose workgroups each reuse one scratch slab for pairs blockIdx, blockIdx +
// gridDim, ...
template <bool G, uint32_t NT>
__global__ __launch_bounds__(NT) void combine_level_kernel(BlockSummaries v, uint32_t k, uint32_t count,
                                                                        uint32_t step, uint32_t pairs,
                                                                        unsigned char* scratch, uint32_t big_bytes) {
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned char* big = G ? scratch + (uint64_t)blockIdx.x * big_bytes : smem + CombineLds<uint32_t>::make(k).small_bytes;
    for (uint32_t j = blockIdx.x; j < pairs; j += gridDim.x) {
        const uint64_t a = 2ull * step * j;
        const uint64_t b = a + step;
        __syncthreads();  // the previous pair is done with the slab
        combine_node<NT, uint32_t, uint32_t, uint32_t>(v.item + a * k, v.cnt + a * k, v.err + a * k, v.size[a], v.min[a],
                                                   v.item + b * k, v.cnt + b * k, v.err + b * k, v.size[b], v.min[b],
                                                   k, v.item + a * k, v.cnt + a * k, v.err + a * k, &v.size[a],
                                                   &v.min[a], big, smem);
    }
}

// Persistent summaries are updated all or nothing: an input carrying a
// block's failure mark leaves d (entries, header and N) as it was and sets
// d's fault word, which the next report hands to the host.
template <bool G>
__global__ __launch_bounds__(kCombineThreadsWide) void fold_kernel(WideSummary d, BlockSummaries s, uint32_t k,
                                                               uint64_t n, unsigned char* scratch) {
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned char* big = G ? scratch : smem + CombineLds<uint64_t>::make(k).small_bytes;
    const uint32_t n1 = d.size[0], n2 = s.size[0];
    if (n1 > k || n2 > k) {
        if (threadIdx.x == 0) *d.fault = 1u;
        return;
    }
    combine_node<kCombineThreadsWide, uint64_t, uint32_t, uint64_t>(d.item, d.cnt, d.err, n1, d.min[0], s.item, s.cnt,
                                                                    s.err, n2, s.min[0], k, d.item, d.cnt, d.err,
                                                                    d.size, d.min, big, smem);
    if (threadIdx.x == 0) *d.total += n;
}

template <bool G>
__global__ __launch_bounds__(kCombineThreadsWide) void merge_kernel(WideSummary d, WideSummary s, uint32_t k,
                                                                unsigned char* scratch) {
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned char* big = G ? scratch : smem + CombineLds<uint64_t>::make(k).small_bytes;
    const uint32_t n1 = d.size[0], n2 = s.size[0];
    if (n1 > k || n2 > k) {
        if (threadIdx.x == 0) *d.fault = 1u;
        return;
    }
    const uint64_t ns = *s.total;
    combine_node<kCombineThreadsWide, uint64_t, uint64_t, uint64_t>(d.item, d.cnt, d.err, n1, d.min[0], s.item, s.cnt,
                                                                    s.err, n2, s.min[0], k, d.item, d.cnt, d.err,
                                                                    d.size, d.min, big, smem);
    if (threadIdx.x == 0) *d.total += ns;
}

// One tree level of a batch: node j merges two block summaries of one
// stream (any stream, any k up to the launch's bound) into the first.
__global__ __launch_bounds__(kCombineThreads) void batch_combine_kernel(const BatchNode* __restrict__ nodes,
                                                                        uint32_t count, BlockSummaries v) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t small = CombineLds<uint32_t>::make(2).small_bytes;  // independent of k
    for (uint32_t j = blockIdx.x; j < count; j += gridDim.x) {
        const BatchNode nd = nodes[j];
        __syncthreads();  // the previous node is done with LDS
        combine_node<kCombineThreads, uint32_t, uint32_t, uint32_t>(v.item + nd.a_off, v.cnt + nd.a_off, v.err + nd.a_off, v.size[nd.a],
                                                   v.min[nd.a], v.item + nd.b_off, v.cnt + nd.b_off,
                                                   v.err + nd.b_off, v.size[nd.b], v.min[nd.b], nd.k,
                                                   v.item + nd.a_off, v.cnt + nd.a_off, v.err + nd.a_off,
                                                   &v.size[nd.a], &v.min[nd.a], smem + small, smem);
    }
}

hipError_t launch_batch_combine(const BatchNode* nodes, uint32_t count, uint32_t kmax, const BlockSummaries& base,
                                hipStream_t stream) {
    (void)hipGetLastError();  // a stale error of an earlier, unrelated call is not this launch's
    if (count == 0) return hipSuccess;
    const uint32_t lds = combine_lds_bytes(kmax, false);
    hipFuncSetAttribute((const void*)batch_combine_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(batch_combine_kernel, dim3(count), dim3(kCombineThreads), lds, stream, nodes, count, base);
    return hipGetLastError();
}

// Served appends: S_sid <- COMBINE(S_sid, root of the append's tree) for
// every append of a launch (one per summary), u64 counts in the summaries.
// A fold whose tree root carries a block's failure mark leaves its summary
// as it was and sets *failed (the server then fails the launch).
__global__ __launch_bounds__(kCombineThreads) void serve_fold_kernel(const ServeFold* __restrict__ f, uint32_t count,
                                                                     WideSummary pool, BlockSummaries v,
                                                                     uint32_t* failed) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t small = CombineLds<uint64_t>::make(2).small_bytes;  // independent of k
    for (uint32_t j = blockIdx.x; j < count; j += gridDim.x) {
        const ServeFold d = f[j];
        __syncthreads();  // the previous fold is done with LDS
        const uint32_t n1 = pool.size[d.sid], n2 = v.size[d.root];
        if (n1 > d.k || n2 > d.k) {
            if (threadIdx.x == 0) *failed = 1u;
            continue;
        }
        combine_node<kCombineThreads, uint64_t, uint32_t, uint64_t>(pool.item + d.s_off, pool.cnt + d.s_off, pool.err + d.s_off, n1,
                                                   pool.min[d.sid], v.item + d.root_off, v.cnt + d.root_off,
                                                   v.err + d.root_off, n2, v.min[d.root], d.k, pool.item + d.s_off,
                                                   pool.cnt + d.s_off, pool.err + d.s_off, &pool.size[d.sid],
                                                   &pool.min[d.sid], smem + small, smem);
    }
}

hipError_t launch_serve_fold(const ServeFold* f, uint32_t count, uint32_t kmax, const WideSummary& pool,
                             const BlockSummaries& blocks, uint32_t* failed, hipStream_t stream) {
    (void)hipGetLastError();  // a stale error of an earlier, unrelated call is not this launch's
    if (count == 0) return hipSuccess;
    const uint32_t lds = combine_lds_bytes(kmax, true);
    hipFuncSetAttribute((const void*)serve_fold_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(serve_fold_kernel, dim3(count), dim3(kCombineThreads), lds, stream, f, count, pool, blocks,
                       failed);
    return hipGetLastError();
}

uint32_t combine_lds_bytes(uint32_t k, bool wide) {
    return wide ? CombineLds<uint64_t>::make(k).big_bytes + CombineLds<uint64_t>::make(k).small_bytes
                : CombineLds<uint32_t>::make(k).big_bytes + CombineLds<uint32_t>::make(k).small_bytes;
}

size_t combine_scratch_bytes(uint32_t k, bool wide) {
    return wide ? CombineLds<uint64_t>::make(k).big_bytes : CombineLds<uint32_t>::make(k).big_bytes;
}

hipError_t launch_combine_level(const BlockSummaries& v, uint32_t k, uint32_t count, uint32_t step, bool in_lds,
                                unsigned char* scratch, uint32_t slabs, hipStream_t stream) {
    (void)hipGetLastError();  // a stale error of an earlier, unrelated call is not this launch's
    if (step >= count) return hipSuccess;
    // pairs (a, a + step) with a = 2 step j and a + step < count
    const uint32_t pairs = (uint32_t)(((uint64_t)count - step + 2ull * step - 1) / (2ull * step));
    const CombineLds<uint32_t> L = CombineLds<uint32_t>::make(k);
    // levels of few pairs, and every level with the arrays in device memory
    // (bounded grid, large k), take the wide workgroups
    const bool wide = !in_lds || pairs <= kCombineWidePairs;
    if (in_lds) {
        const uint32_t lds = L.big_bytes + L.small_bytes;
        auto launch = [&](auto kern, uint32_t nt) {
            hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            hipLaunchKernelGGL(kern, dim3(pairs), dim3(nt), lds, stream, v, k, count, step, pairs,
                               (unsigned char*)nullptr, 0u);
        };
        if (wide)
            launch(combine_level_kernel<false, kCombineThreadsWide>, kCombineThreadsWide);
        else
            launch(combine_level_kernel<false, kCombineThreads>, kCombineThreads);
    } else {
        if (!scratch || slabs == 0) return hipErrorInvalidValue;
        const uint32_t grid = pairs < slabs ? pairs : slabs;
        if (wide)
            hipLaunchKernelGGL((combine_level_kernel<true, kCombineThreadsWide>), dim3(grid), dim3(kCombineThreadsWide),
                               L.small_bytes, stream, v, k, count, step, pairs, scratch, L.big_bytes);
        else
            hipLaunchKernelGGL((combine_level_kernel<true, kCombineThreads>), dim3(grid), dim3(kCombineThreads),
                               L.small_bytes, stream, v, k, count, step, pairs, scratch, L.big_bytes);
    }
    return hipGetLastError();
}

hipError_t launch_fold(const WideSummary& dst, const BlockSummaries& src, uint32_t k, uint64_t n, bool in_lds,
                       unsigned char* scratch, hipStream_t stream) {
    (void)hipGetLastError();  // a stale error of an earlier, unrelated call is not this launch's
    if (!dst.total || !dst.fault) return hipErrorInvalidValue;
    const CombineLds<uint64_t> L = CombineLds<uint64_t>::make(k);
    if (in_lds) {
        const uint32_t lds = L.big_bytes + L.small_bytes;
        hipFuncSetAttribute((const void*)fold_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(fold_kernel<false>, dim3(1), dim3(kCombineThreadsWide), lds, stream, dst, src, k, n,
                           (unsigned char*)nullptr);
    } else {
        if (!scratch) return hipErrorInvalidValue;
        hipLaunchKernelGGL(fold_kernel<true>, dim3(1), dim3(kCombineThreadsWide), L.small_bytes, stream, dst, src, k, n,
                           scratch);
    }
    return hipGetLastError();
}

hipError_t launch_merge(const WideSummary& dst, const WideSummary& src, uint32_t k, bool in_lds,
                        unsigned char* scratch, hipStream_t stream) {
    (void)hipGetLastError();  // a stale error of an earlier, unrelated call is not this launch's
    if (!dst.total || !dst.fault || !src.total) return hipErrorInvalidValue;
    const CombineLds<uint64_t> L = CombineLds<uint64_t>::make(k);
    if (in_lds) {
        const uint32_t lds = L.big_bytes + L.small_bytes;
        hipFuncSetAttribute((const void*)merge_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(merge_kernel<false>, dim3(1), dim3(kCombineThreadsWide), lds, stream, dst, src, k,
                           (unsigned char*)nullptr);
    } else {
        if (!scratch) return hipErrorInvalidValue;
        hipLaunchKernelGGL(merge_kernel<true>, dim3(1), dim3(kCombineThreadsWide), L.small_bytes, stream, dst, src, k,
                           scratch);
    }
    return hipGetLastError();
}

}  // namespace pss
