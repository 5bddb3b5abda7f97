// Block summaries: sequential Space Saving over each of C contiguous blocks
// of the input (Section 3, second paragraph; Algorithm 1, SpaceSaving on
// [left, right]).  One wave owns one block and keeps its k counters in LDS.
//
// The wave consumes its block in windows of up to 64 consecutive items, one
// item per lane, and reproduces the sequential algorithm exactly:
//
//  * every lane looks its item up in an open-addressed hash (item -> counter)
//    holding the state at window start;
//  * a window without unmonitored items is all hits: increments commute, so
//    the window is applied at once;
//  * otherwise unmonitored items are grouped by value; the first occurrence of
//    each value ("new item") will take a counter, later occurrences add 1;
//  * while counters are free, the j-th new item takes free counter size+j;
//    once all k are used, the j-th new item evicts the j-th victim, where the
//    victims are the counters at the current minimum count m in increasing
//    item id (the sequential rule: minimum count, then smallest id), and is
//    installed with count m+1 and error m;
//  * hits commute with each other; they interact with the evictions only when
//    a hit lands on a counter that is also evicted in the window, and the
//    window can run out of free counters or of counters at level m.  The wave
//    applies the longest prefix of the window free of both and starts the
//    next window at the first item it did not apply.  The first item of a
//    window is always applicable, so every window makes progress.
//
// The counters at the minimum level m are listed once, sorted by item id, when
// the level is first needed.  A listed counter is still a victim candidate
// exactly while its count is m: counts never decrease, an evicted counter is
// re-installed at m+1, and no counter can join level m after it is listed.
//
// The hash maps an item to two 8-slot buckets (64 bytes each, read with four
// 16-byte loads) and keeps its entry in one of their 16 slots; a new item
// takes a free slot of the emptier bucket, or of a 64-slot stash when both
// are full (searched only while it holds entries).  Lookups cost one round
// of four loads whatever the load, and a deleted entry simply becomes empty:
// no probe chains, tombstones or rebuilds.
#include <type_traits>

#include "pss_device.h"
#include "pss_kernels.h"
#include "pss_layout.h"
#include "pss_table.h"

namespace pss {

#ifdef PSS_KERNEL_STATS
// analysis builds only: per-phase cycle and event counts summed over waves
__device__ unsigned long long g_kstats[32];
#define KSTAT_DECL unsigned long long ks_[32] = {0};
#define KSTAT_ADD(i, v) (ks_[(i)] += (unsigned long long)(v))
#define KSTAT_NOW() ((unsigned long long)clock64())
#define KSTAT_FLUSH()                                                        \
    if (lane == 0)                                                           \
        for (int i_ = 0; i_ < 32; ++i_) atomicAdd(&g_kstats[i_], ks_[i_]);
#else
#define KSTAT_DECL
#define KSTAT_ADD(i, v) ((void)0)
#define KSTAT_NOW() 0ull
#define KSTAT_FLUSH()
#endif

// ---------------------------------------------------------------------------
// Sorting the minimum level by item id
// ---------------------------------------------------------------------------

// The item id of the counter in slot s: the key of its table entry.
struct SlotIds {
    const uint64_t* table;
    __device__ __forceinline__ uint32_t operator()(uint32_t s) const { return ((const uint32_t*)table)[2 * s]; }
};

// LDS pointer types of the level sort's arrays (state in LDS).  The sort's
// out-of-line parts take these, so that they address LDS with LDS
// instructions: through a generic pointer a callee would use FLAT ones, and
// each wait for a FLAT load also waits for the wave's global loads and
// stores.
typedef __attribute__((address_space(3))) uint16_t lds_u16;
typedef __attribute__((address_space(3))) uint32_t lds_u32;

// SlotIds of a table in LDS (words: the entries as 32-bit words).
struct LdsIds {
    const lds_u32* words;
    __device__ __forceinline__ uint32_t operator()(uint32_t s) const { return words[2 * s]; }
};

// Count of a slot's entry (the high word under cmask, which drops a packed
// error), or ~0 when the slot holds no counter (empty, or claimed during a
// window).
__device__ __forceinline__ uint32_t slot_count(const uint32_t* words, uint32_t s, uint32_t cmask) {
    const uint32_t c = words[2 * s + 1];
    return live_tag(c) ? (c & cmask) : 0xFFFFFFFFu;
}

// A count word that other lanes have just changed with atomics: from LDS
// with an LDS load, from the HBM-resident state with a volatile load.
template <bool G>
__device__ __forceinline__ uint32_t tag_word(const uint32_t* words, uint32_t i) {
    if constexpr (G)
        return ((const volatile uint32_t*)words)[i];
    else
        return lds_reread(words + i);
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, uint32_t src) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, (int)src);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), (int)src);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, uint32_t lx) {
    uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, (int)lx);
    uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), (int)lx);
    return ((uint64_t)hi << 32) | lo;
}

// Ascending bitonic sort of 64*P keys held in registers; element g lives in
// lane g / P, register g % P.
template <int P>
__device__ __forceinline__ void reg_bitonic_sort(uint64_t (&v)[P], uint32_t lane) {
    constexpr uint32_t N = 64u * P;
    for (uint32_t size = 2; size <= N; size <<= 1) {
        for (uint32_t stride = size >> 1; stride >= (uint32_t)P; stride >>= 1) {
            const uint32_t lx = stride / P;
            const bool lower = (lane & lx) == 0;
#pragma unroll
            for (int j = 0; j < P; ++j) {
                const bool up = ((lane * P + j) & size) == 0;
                const uint64_t o = shfl_xor_u64(v[j], lx);
                const uint64_t mn = v[j] < o ? v[j] : o;
                const uint64_t mx = v[j] < o ? o : v[j];
                v[j] = (lower == up) ? mn : mx;
            }
        }
#pragma unroll
        for (int stride = P / 2; stride > 0; stride >>= 1) {
            if ((uint32_t)stride < size) {
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    if ((j & stride) == 0) {
                        const int j2 = j | stride;
                        const bool up = ((lane * P + j) & size) == 0;
                        const uint64_t a = v[j], b = v[j2];
                        const bool sw = (a > b) == up;
                        v[j] = sw ? b : a;
                        v[j2] = sw ? a : b;
                    }
                }
            }
        }
    }
}

// list[0, len) holds counter indices; reorder them by item id.
template <int P>
__device__ void sort_level_regs(lds_u16* list, const LdsIds ids, uint32_t len, uint32_t lane) {
    uint64_t v[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const uint32_t g = lane * P + j;
        v[j] = ~0ull;
        if (g < len) {
            const uint32_t s = list[g];
            v[j] = ((uint64_t)ids(s) << 32) | s;
        }
    }
    reg_bitonic_sort<P>(v, lane);
    wave_sync();
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const uint32_t g = lane * P + j;
        if (g < len) list[g] = (uint16_t)v[j];
    }
}

template <int P>
__device__ void sort_level_dispatch(lds_u16* list, const LdsIds ids, uint32_t len, uint32_t per_lane,
                                    uint32_t lane) {
    if constexpr (P >= 2) {
        if (per_lane == (uint32_t)P) {
            sort_level_regs<P>(list, ids, len, lane);
            return;
        }
        if constexpr (P > 2) sort_level_dispatch<P / 2>(list, ids, len, per_lane, lane);
    }
}

#ifdef PSS_KERNEL_STATS
#define SORT_T(i) unsigned long long st_##i = clock64();
#define SORT_FLUSH()                                   \
    if (lane == 0) {                                   \
        atomicAdd(&g_kstats[19], st_1 - st_0);         \
        atomicAdd(&g_kstats[20], st_2 - st_1);         \
        atomicAdd(&g_kstats[21], st_3 - st_2);         \
        atomicAdd(&g_kstats[22], st_4 - st_3);         \
        atomicAdd(&g_kstats[23], st_5 - st_4);         \
    }
#else
#define SORT_T(i)
#define SORT_FLUSH()
#endif

// Largest bucket the bucketed sort takes; beyond it (ids that the top digit
// hardly separates) the level is sorted with the register network instead.
constexpr uint32_t kMaxBucket = 48;

// Ascending bitonic sort of Q keys held by one lane.
template <int Q>
__device__ __forceinline__ void lane_sort(uint64_t (&v)[Q]) {
#pragma unroll
    for (int size = 2; size <= Q; size <<= 1) {
#pragma unroll
        for (int stride = size / 2; stride > 0; stride >>= 1) {
#pragma unroll
            for (int j = 0; j < Q; ++j) {
                if ((j & stride) == 0) {
                    const int j2 = j | stride;
                    const bool up = (j & size) == 0;
                    const uint64_t a = v[j], b = v[j2];
                    const bool sw = (a > b) == up;
                    v[j] = sw ? b : a;
                    v[j2] = sw ? a : b;
                }
            }
            __builtin_amdgcn_sched_barrier(0);  // stage by stage: bounded live ranges
        }
    }
}

// A lane's bitonic sequence of Q keys into ascending order.
template <int Q>
__device__ __forceinline__ void lane_merge(uint64_t (&v)[Q]) {
#pragma unroll
    for (int stride = Q / 2; stride > 0; stride >>= 1) {
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            if ((j & stride) == 0) {
                const int j2 = j | stride;
                const uint64_t a = v[j], b = v[j2];
                v[j] = a < b ? a : b;
                v[j2] = a < b ? b : a;
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Bitonic merge of registers [OFF, OFF + W) of a lane (a bitonic sequence)
// into ascending order.
template <int OFF, int W, int Q>
__device__ __forceinline__ void lane_merge_range(uint64_t (&v)[Q]) {
#pragma unroll
    for (int stride = W / 2; stride > 0; stride >>= 1) {
#pragma unroll
        for (int j = OFF; j < OFF + W; ++j) {
            if (((j - OFF) & stride) == 0) {
                const int j2 = j + stride;
                const uint64_t a = v[j], b = v[j2];
                v[j] = a < b ? a : b;
                v[j2] = a < b ? b : a;
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// One pass that sorts lane-sorted runs whose disorder across each lane
// boundary lies within W keys on either side (W <= Q / 2, so a lane's head
// and tail regions are disjoint): every lane merges its last W keys with the
// next lane's first W, keeping the W smallest, and its first W with the
// previous lane's last W, keeping the W largest.  All neighbour keys are
// read before any register changes.
template <int W, int Q>
__device__ __forceinline__ void boundary_merge(uint64_t (&v)[Q], uint32_t lane) {
    static_assert(2 * W <= Q, "head and tail regions must not overlap");
    const bool has_up = lane + 1 < kWave, has_dn = lane > 0;
    const uint32_t up = has_up ? lane + 1 : lane, dn = has_dn ? lane - 1 : lane;
    uint64_t nh[W], pt[W];  // the next lane's head, the previous lane's tail
#pragma unroll
    for (int j = 0; j < W; ++j) {
        nh[j] = shfl_u64(v[j], up);
        pt[j] = shfl_u64(v[Q - W + j], dn);
    }
    // tail: my ascending last W against the next lane's head read in reverse
    // (a bitonic sequence); its lower half holds the W smallest
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const uint64_t a = v[Q - W + j], b = nh[W - 1 - j];
        v[Q - W + j] = has_up && b < a ? b : a;
    }
    // head: the previous lane's tail in reverse against my first W; the upper
    // half holds the W largest
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const uint64_t a = v[j], b = pt[W - 1 - j];
        v[j] = has_dn && b > a ? b : a;
    }
    lane_merge_range<Q - W, W>(v);
    lane_merge_range<0, W>(v);
}

// Lane l takes positions [l Q, (l+1) Q) of list (slots, in an order where
// only entries of one bucket can be out of order; each slot's id is read
// from the table), sorts them in registers by (id, slot), and odd-even merges between
// neighbouring lanes (the lower lane keeping the smaller half) finish the
// order; the wave stops as soon as every lane's last key is at most its
// neighbour's first, after at most 64 rounds (odd-even transposition over 64
// blocks sorts any input).  Before the rounds, when every boundary's disorder
// spans at most Q / 2 keys on each side (a bucket straddling it is short,
// the usual case at Q <= 16), one boundary_merge pass sorts the whole list
// and the rounds find nothing to do.  Out of line: its registers stay apart
// from the caller's.
template <int Q>
__device__ __attribute__((noinline)) void merge_runs(lds_u16* list, const LdsIds ids, uint32_t len, uint32_t lane) {
    uint64_t v[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        const uint32_t g = lane * Q + j;
        const uint32_t s = list[g < len ? g : 0u];
        const uint64_t key = ((uint64_t)ids(s) << 32) | s;
        v[j] = g < len ? key : ~0ull;
    }
    lane_sort<Q>(v);
    const uint32_t up = lane + 1 < kWave ? lane + 1 : lane;
    if constexpr (Q >= 4 && Q <= 32) {
        // disorder at the boundaries: my keys above the next lane's first,
        // my keys below the previous lane's last
        const uint32_t dn = lane > 0 ? lane - 1 : lane;
        const uint64_t next_first = shfl_u64(v[0], up), prev_last = shfl_u64(v[Q - 1], dn);
        uint32_t rt = 0, rh = 0;
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            rt += (lane + 1 < kWave && v[j] > next_first) ? 1u : 0u;
            rh += (lane > 0 && v[j] < prev_last) ? 1u : 0u;
        }
        const uint32_t r = wave_max_u32(rt > rh ? rt : rh);
        // widths up to Q / 2 and 8 (wider ones hold more registers than the
        // kernel can spare at Q = 32); larger disorder goes to the rounds
        if (r > 0u && r <= (uint32_t)Q / 2u) {
            if (r <= 1u)
                boundary_merge<1>(v, lane);
            else if (r <= 2u)
                boundary_merge<2>(v, lane);
            else if constexpr (Q >= 8) {
                if (r <= 4u)
                    boundary_merge<4>(v, lane);
                else if constexpr (Q >= 16) {
                    if (r <= 8u) boundary_merge<8>(v, lane);
                }
            }
        }
    }
    for (uint32_t round = 0; round < kWave; ++round) {
        const uint64_t next_first = shfl_u64(v[0], up);
        if (ballot(lane + 1 < kWave && v[Q - 1] > next_first) == 0) break;
        // pairs (2i + off, 2i + 1 + off): merge, the lower lane keeping the
        // smaller half (its partner's run is read in reverse, which makes the
        // pair's keys a bitonic sequence)
        const uint32_t off = round & 1u;
        const bool lower = ((lane - off) & 1u) == 0u;
        const uint32_t partner = lower ? lane + 1 : lane - 1;
        const bool paired = lane >= off && partner < kWave;
        const uint32_t src = paired ? partner : lane;
        // registers j and Q-1-j pair with the partner's Q-1-j and j: read
        // both before either is replaced
#pragma unroll
        for (int j = 0; j < Q / 2; ++j) {
            const int jj = Q - 1 - j;
            const uint64_t ta = shfl_u64(v[jj], src);
            const uint64_t tb = shfl_u64(v[j], src);
            const uint64_t lo_a = v[j] < ta ? v[j] : ta, hi_a = v[j] < ta ? ta : v[j];
            const uint64_t lo_b = v[jj] < tb ? v[jj] : tb, hi_b = v[jj] < tb ? tb : v[jj];
            v[j] = !paired ? v[j] : (lower ? lo_a : hi_a);
            v[jj] = !paired ? v[jj] : (lower ? lo_b : hi_b);
        }
        lane_merge<Q>(v);
    }
    wave_sync();
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        const uint32_t g = lane * Q + j;
        if (g < len) list[g] = (uint16_t)v[j];
    }
}

// Bucketed sort of list[0, len) by item id for len > 64, 64 * Q >= len: a
// counting sort on 8 bits of the id (the top 8 of the bits where the level's
// ids differ, so bucket order is id order) places every entry in its bucket;
// then merge_runs orders the entries inside each bucket.  Returns false, with
// list as it was, when a bucket is larger than kMaxBucket.  hist lies over
// list (the list is held in registers from the first read to the scatter).
// A lane keeps each of its Q entries as one word, slot | place in
// its bucket << 16 (slots and places are below 2^16 with the state in LDS),
// and their digits four to a word; ids are read from the table when needed,
// and each step takes the entries eight at a time (a scheduling barrier
// between groups bounds the loads and atomics in flight).  Out of line, like
// merge_runs: at large k these registers would otherwise set the kernel's.
template <int Q>
__device__ __attribute__((noinline)) bool sort_level_buckets(lds_u16* list, const LdsIds ids, lds_u32* hist,
                                                             uint32_t len, uint32_t lane) {
    // 8-bit digits; 9 at Q = 32 (levels of over 1024 counters, whose list
    // area holds the 513-word histogram), so buckets stay short enough for
    // merge_runs' boundary pass
    constexpr uint32_t kDB = Q >= 32 ? 9u : 8u;
    constexpr uint32_t kBins = 1u << kDB, kPer = kBins / kWave;
    constexpr int kDpw = (int)(32u / kDB);  // digits per word
    constexpr int kDigitWords = (Q + kDpw - 1) / kDpw;
    constexpr int kGroup = Q < 8 ? Q : 8;
    uint32_t sp[Q], dg[kDigitWords];
    uint32_t orv = 0u, andv = 0xFFFFFFFFu;
    SORT_T(0);
#pragma unroll
    for (int j0 = 0; j0 < Q; j0 += kGroup) {
#pragma unroll
        for (int j = j0; j < j0 + kGroup; ++j) {
            const uint32_t g = lane * Q + j;
            const uint32_t s = list[g < len ? g : 0u];
            const uint32_t id = ids(s);
            sp[j] = s;
            if (g < len) {
                orv |= id;
                andv &= id;
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    SORT_T(1);
    const uint32_t diff = wave_or_u32(orv) ^ wave_and_u32(andv);
    const uint32_t hb = 31u - (uint32_t)__builtin_clz(diff | 1u);
    const uint32_t shift = hb >= kDB - 1u ? hb - (kDB - 1u) : 0u;
    wave_sync();  // the list is read: the histogram may now overwrite it
    for (uint32_t i = lane; i < kBins + 1u; i += kWave) hist[i] = 0u;
    wave_sync();
#pragma unroll
    for (int w = 0; w < kDigitWords; ++w) dg[w] = 0u;
#pragma unroll
    for (int j0 = 0; j0 < Q; j0 += kGroup) {
#pragma unroll
        for (int j = j0; j < j0 + kGroup; ++j) {
            const uint32_t g = lane * Q + j;
            const uint32_t d = (ids(sp[j]) >> shift) & (kBins - 1u);
            dg[j / kDpw] |= d << (kDB * (uint32_t)(j % kDpw));
            const uint32_t pin =
                (g < len) ? __hip_atomic_fetch_add(&hist[d], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT) : 0u;
            sp[j] |= pin << 16;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    wave_sync();
    SORT_T(2);
    uint32_t hc[kPer], hmax = 0u;
#pragma unroll
    for (uint32_t t = 0; t < kPer; ++t) {
        hc[t] = hist[kPer * lane + t];
        hmax = max(hmax, hc[t]);
    }
    if (wave_max_u32(hmax) > kMaxBucket) {
        wave_sync();  // put the list back for the fallback
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            const uint32_t g = lane * Q + j;
            if (g < len) list[g] = (uint16_t)(sp[j] & 0xFFFFu);
        }
        wave_sync();
        return false;
    }
    // exclusive scan of the counts: bucket d starts at hist[d]
    uint32_t sum = 0u;
#pragma unroll
    for (uint32_t t = 0; t < kPer; ++t) sum += hc[t];
    uint32_t incl = sum;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)incl, off);
        if ((int)lane >= off) incl += t;
    }
    uint32_t ex = incl - sum;
    wave_sync();
#pragma unroll
    for (uint32_t t = 0; t < kPer; ++t) {
        hist[kPer * lane + t] = ex;
        ex += hc[t];
    }
    wave_sync();
#pragma unroll
    for (int j0 = 0; j0 < Q; j0 += kGroup) {
#pragma unroll
        for (int j = j0; j < j0 + kGroup; ++j)  // the entry's place in bucket order
            sp[j] = (sp[j] & 0xFFFFu) |
                    ((hist[(dg[j / kDpw] >> (kDB * (uint32_t)(j % kDpw))) & (kBins - 1u)] + (sp[j] >> 16)) << 16);
        __builtin_amdgcn_sched_barrier(0);
    }
    wave_sync();  // the histogram is read: list may now overwrite it
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        const uint32_t g = lane * Q + j;
        if (g < len) list[sp[j] >> 16] = (uint16_t)(sp[j] & 0xFFFFu);
    }
    wave_sync();
    SORT_T(3);
    merge_runs<Q>(list, ids, len, lane);
    SORT_T(4);
    SORT_T(5);
    SORT_FLUSH();
    return true;
}

template <int P>
__device__ bool sort_level_buckets_dispatch(lds_u16* list, const LdsIds ids, lds_u32* hist, uint32_t len,
                                            uint32_t per_lane, uint32_t lane) {
    if constexpr (P >= 2 && P <= 32) {
        if (per_lane == (uint32_t)P) return sort_level_buckets<P>(list, ids, hist, len, lane);
    }
    if constexpr (P > 2)
        return sort_level_buckets_dispatch<P / 2>(list, ids, hist, len, per_lane, lane);
    return false;
}

// Rank sort of list[0, len) by item id, len <= 64: one entry per lane, its
// rank is the number of smaller ids.
template <typename LP, typename ID>
__device__ void sort_level_rank(LP list, const ID& ids, uint32_t len, uint32_t lane) {
    uint32_t s = 0;
    uint32_t key = 0xFFFFFFFFu;
    if (lane < len) {
        s = list[lane];
        key = ids(s);
    }
    uint32_t rank = 0;
    for (uint32_t i = 0; i < len; ++i) {
        const uint32_t ki = __builtin_amdgcn_readlane(key, i);
        rank += ki < key ? 1u : 0u;
    }
    wave_sync();
    if (lane < len) list[rank] = s;
}

// Stable least-significant-digit radix sort of list[0, len) by item id (four
// 8-bit passes), for levels of any size (the state in device memory).
// Within each group of 64 entries the lanes holding the same digit are found
// with eight ballots, so equal digits keep their order.  list2, tkey and
// tkey2 hold len entries each.  Every loop takes kRadixGroups groups of 64
// entries at a time and issues all their loads before using any: each step
// otherwise waits a full device-memory round trip.
constexpr uint32_t kRadixGroups = 8;

template <typename IT, typename ID>
__device__ void sort_level_radix(IT* list, IT* list2, const ID& ids, uint32_t* tkey, uint32_t* tkey2,
                                 uint32_t* hist, uint32_t len, uint32_t lane) {
    constexpr uint32_t U = kRadixGroups;
    for (uint32_t base = 0; base < len; base += U * kWave) {
        uint32_t sl[U], key[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t g = base + u * kWave + lane;
            sl[u] = (uint32_t)list[g < len ? g : 0u];
        }
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) key[u] = ids(sl[u]);
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t g = base + u * kWave + lane;
            if (g < len) tkey[g] = key[u];
        }
    }
    wave_sync();
    IT* src = list;
    IT* dst = list2;
    uint32_t* ks = tkey;
    uint32_t* kd = tkey2;
    for (uint32_t pass = 0; pass < 4; ++pass) {
        const uint32_t sh = 8u * pass;
        for (uint32_t i = lane; i < 256; i += kWave) hist[i] = 0u;
        wave_sync();
        for (uint32_t base = 0; base < len; base += U * kWave) {
            uint32_t key[U];
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t g = base + u * kWave + lane;
                key[u] = ks[g < len ? g : 0u];
            }
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t g = base + u * kWave + lane;
                if (g < len) atomicAdd(&hist[(key[u] >> sh) & 255u], 1u);
            }
        }
        wave_sync();
        const uint32_t h0 = hist[4 * lane], h1 = hist[4 * lane + 1], h2 = hist[4 * lane + 2], h3 = hist[4 * lane + 3];
        const uint32_t sum = h0 + h1 + h2 + h3;
        uint32_t incl = sum;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t t = (uint32_t)__shfl_up((int)incl, off);
            if ((int)lane >= off) incl += t;
        }
        const uint32_t ex = incl - sum;
        wave_sync();
        hist[4 * lane] = ex;
        hist[4 * lane + 1] = ex + h0;
        hist[4 * lane + 2] = ex + h0 + h1;
        hist[4 * lane + 3] = ex + h0 + h1 + h2;
        wave_sync();
        for (uint32_t base = 0; base < len; base += U * kWave) {
            uint32_t key[U];
            IT sv[U];
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t g = base + u * kWave + lane;
                const bool v = g < len;
                key[u] = ks[v ? g : 0u];
                sv[u] = src[v ? g : 0u];
            }
            // the groups in order: each one's places follow the earlier ones'
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t g = base + u * kWave + lane;
                const bool v = g < len;
                const uint32_t d = (key[u] >> sh) & 255u;
                uint64_t same = ballot(v);
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const uint64_t bb = ballot(v && ((d >> b) & 1u));
                    same &= ((d >> b) & 1u) ? bb : ~bb;
                }
                const uint32_t rank = mbcnt(same);
                const uint32_t off = hist[d];
                wave_sync();
                if (v && rank == 0) hist[d] = off + popc64(same);
                if (v) {
                    dst[off + rank] = sv[u];
                    kd[off + rank] = key[u];
                }
                wave_sync();
            }
        }
        IT* t1 = src;
        src = dst;
        dst = t1;
        uint32_t* t2 = ks;
        ks = kd;
        kd = t2;
    }
}

template <int P>
__device__ void sort_level(lds_u16* list, const LdsIds ids, lds_u32* hist, uint32_t len, uint32_t lane) {
    if (len <= 64) {
        sort_level_rank(list, ids, len, lane);
    } else {
        const uint32_t per_lane = next_pow2((len + 63) / 64);
        if (!sort_level_buckets_dispatch<P>(list, ids, hist, len, per_lane, lane)) {
            wave_sync();
            sort_level_dispatch<P>(list, ids, len, per_lane, lane);
        }
    }
    wave_sync();
}

// ---------------------------------------------------------------------------
// Listing a new minimum level (LDS-resident state), out of line
// ---------------------------------------------------------------------------

extern __shared__ __align__(16) unsigned char smem[];

// Finds the minimum count m of the counters and lists the slots at m in id
// order; state at LDS byte offset sbo.  `prev` is the level just
// exhausted: one pass finds the minimum and collects the counters at
// prev + 1, the usual next level, and a second pass collects the true
// minimum level when it differs.  Returns m << 32 | length.
template <int P>
__device__ __forceinline__ uint64_t level_lds_body(uint32_t sbo, const ChunkLayout& L, uint32_t prev,
                                                   uint32_t lane) {
    const uint32_t S = L.slots;
    const uint32_t* words = (const uint32_t*)(smem + sbo + L.off_table);
    lds_u16* list = (lds_u16*)(smem + sbo + L.off_list);
    lds_u32* hist = (lds_u32*)(smem + sbo + L.off_hist);
    const LdsIds ids{(const lds_u32*)(smem + sbo + L.off_table)};
    const uint32_t guess = prev + 1u;
    uint32_t mn = 0xFFFFFFFFu, len = 0;
    for (uint32_t b = 0; b < S; b += 4 * kWave) {
        uint32_t cv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t s = b + j * kWave + lane;
            const uint32_t c = slot_count(words, s < S ? s : 0u, L.count_mask);  // clamped: no branch around the load
            cv[j] = s < S ? c : 0xFFFFFFFFu;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            mn = min(mn, cv[j]);
            const bool take = cv[j] == guess;
            const uint64_t bm = ballot(take);
            if (take) list[len + mbcnt(bm)] = (uint16_t)(b + j * kWave + lane);
            len = uniform(len + popc64(bm));
        }
    }
    const uint32_t m = uniform(wave_min_u32(mn));
    if (m != guess) {
        len = 0;
        for (uint32_t b = 0; b < S; b += 4 * kWave) {
            uint32_t cv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t s = b + j * kWave + lane;
                const uint32_t c = slot_count(words, s < S ? s : 0u, L.count_mask);  // clamped: no branch around the load
            cv[j] = s < S ? c : 0xFFFFFFFFu;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool take = cv[j] == m;
                const uint64_t bm = ballot(take);
                if (take) list[len + mbcnt(bm)] = (uint16_t)(b + j * kWave + lane);
                len = uniform(len + popc64(bm));
            }
        }
    }
    wave_sync();
    sort_level<P>(list, ids, hist, len, lane);
    return ((uint64_t)m << 32) | len;
}

// The same kept out of line, for the large register classes: it runs once
// per level, and inlined its sort registers crowd the window loop into
// scalar-register spills.  (The call saves registers to scratch memory, so
// the small classes, which gain nothing from it, keep it inline.)
template <int P>
__device__ __attribute__((noinline)) uint64_t build_level_lds(uint32_t sbo, ChunkLayout L, uint32_t prev,
                                                             uint32_t lane) {
    return level_lds_body<P>(sbo, L, prev, lane);
}

// The same for state in device memory (slab sb, 32-bit indices; the sort
// histogram in LDS at lds + off_hist): levels of at most 64 entries by rank,
// larger ones by the stable radix sort.  Inline: out of line it saved nothing
// here (this path waits on device memory, not on instruction issue).
__device__ __forceinline__ uint64_t build_level_global(unsigned char* sb, unsigned char* lds,
                                                       const ChunkLayout& L, uint32_t prev, uint32_t lane) {
    const uint32_t S = L.slots;
    const uint32_t* words = (const uint32_t*)(sb + L.off_table);
    uint32_t* list = (uint32_t*)(sb + L.off_list);
    uint32_t* list2 = (uint32_t*)(sb + L.off_list2);
    uint32_t* tkey = (uint32_t*)(sb + L.off_tkey);
    uint32_t* tkey2 = (uint32_t*)(sb + L.off_tkey2);
    uint32_t* hist = (uint32_t*)(lds + L.off_hist);
    const SlotIds ids{(const uint64_t*)(sb + L.off_table)};
    const uint32_t guess = prev + 1u;
    uint32_t mn = 0xFFFFFFFFu, len = 0;
    // 16 slots per lane per step, their loads in flight together
    constexpr int J = 16;
    for (uint32_t b = 0; b < S; b += J * kWave) {
        uint32_t cv[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const uint32_t s = b + j * kWave + lane;
            const uint32_t c = slot_count(words, s < S ? s : 0u, L.count_mask);  // clamped: no branch around the load
            cv[j] = s < S ? c : 0xFFFFFFFFu;
        }
#pragma unroll
        for (int j = 0; j < J; ++j) {
            mn = min(mn, cv[j]);
            const bool take = cv[j] == guess;
            const uint64_t bm = ballot(take);
            if (take) list[len + mbcnt(bm)] = b + j * kWave + lane;
            len = uniform(len + popc64(bm));
        }
    }
    const uint32_t m = uniform(wave_min_u32(mn));
    if (m != guess) {
        len = 0;
        for (uint32_t b = 0; b < S; b += J * kWave) {
            uint32_t cv[J];
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const uint32_t s = b + j * kWave + lane;
                const uint32_t c = slot_count(words, s < S ? s : 0u, L.count_mask);  // clamped: no branch around the load
            cv[j] = s < S ? c : 0xFFFFFFFFu;
            }
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const bool take = cv[j] == m;
                const uint64_t bm = ballot(take);
                if (take) list[len + mbcnt(bm)] = b + j * kWave + lane;
                len = uniform(len + popc64(bm));
            }
        }
    }
    wave_sync();
    if (len <= 64)
        sort_level_rank(list, ids, len, lane);
    else
        sort_level_radix<uint32_t>(list, list2, ids, tkey, tkey2, hist, len, lane);
    wave_sync();
    return ((uint64_t)m << 32) | len;
}

// ---------------------------------------------------------------------------
// The kernel
// ---------------------------------------------------------------------------

// Space Saving over items[begin, end) by one wave (n bounds every load).
// P: registers per lane for the in-register level sort (LDS-resident state);
// G: the state at sb lives in global memory with 32-bit indices (k whose
// state does not fit LDS), else sb is in LDS.  lds holds the input ring and
// the per-window arrays; errs is the block's error scratch (one error of
// L.err_bytes bytes per slot; PK: none, each error rides in its counter's
// count word above kCountBits).  Writes entries [0, size) to o_item/o_cnt/o_err and the header to
// *o_size, *o_min.  Returns kOverflow, with nothing written, when a new
// item found no free slot under the hash functions hk (the caller runs the
// block again with other ones); else kDone.
constexpr uint32_t kDone = 0, kOverflow = 1;
template <int P, bool G, bool PK = false>
__device__ __forceinline__ uint32_t summarize_block(const uint32_t* __restrict__ items, uint64_t n, uint64_t begin,
                                                    uint64_t end, const ChunkLayout& L, int vec_ok, unsigned char* sb,
                                                    unsigned char* lds, uint32_t* __restrict__ errs,
                                                    uint32_t* __restrict__ o_item, uint32_t* __restrict__ o_cnt,
                                                    uint32_t* __restrict__ o_err, uint32_t* __restrict__ o_size,
                                                    uint32_t* __restrict__ o_min, const HashKeys hk) {
    using idx_t = typename std::conditional<G, uint32_t, uint16_t>::type;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t k = L.k;
    const uint32_t T = L.tsize;
    const uint32_t S = L.slots;
    const uint32_t NB = L.nbuckets;
    // the counters: slot s holds key | count << 32
    uint64_t* table = (uint64_t*)(sb + L.off_table);
    uint32_t* words = (uint32_t*)(sb + L.off_table);  // count of slot s: words[2 s + 1]
    const uint4* tbl4 = (const uint4*)(sb + L.off_table);
    idx_t* list = (idx_t*)(sb + L.off_list);
    const SlotIds ids{table};
    uint32_t* ring = (uint32_t*)(lds + L.off_ring);
    const uint4* stash4 = tbl4 + T / 2;
    // the block's error scratch at the layout's width; PK (known at compile
    // time): none, a counter's count word holds its error above the count,
    // and cmask selects the count
    constexpr uint32_t cmask = PK ? kCountMask : 0xFFFFFFFFu;
    const uint32_t ew = L.err_bytes;
    auto err_put = [&](uint32_t s, uint32_t e) {
        if constexpr (!PK) {
            if (ew == 1)
                ((uint8_t*)errs)[s] = (uint8_t)e;
            else if (ew == 2)
                ((uint16_t*)errs)[s] = (uint16_t)e;
            else
                errs[s] = e;
        }
    };
    auto err_get = [&](uint32_t s) -> uint32_t {
        if constexpr (PK) return 0u;
        return ew == 1 ? (uint32_t)((const uint8_t*)errs)[s]
                       : ew == 2 ? (uint32_t)((const uint16_t*)errs)[s] : errs[s];
    };

    // buckets per item: three in the LDS classes above k = 1024 (the layout's
    // table is sized for them), two elsewhere
    constexpr int NCH = (!G && P >= 32) ? 3 : 2;
    if (L.choices != (uint32_t)NCH || PK != (L.err_bytes == 0u)) {  // a layout built for another table shape
        if (lane == 0) {
            *o_size = kBlockFailed;
            *o_min = 0;
        }
        return kDone;
    }
    // the item's third bucket, or none (its mask stays 0)
    auto bucket3 = [&](uint32_t y, uint32_t c1, uint32_t c2) -> uint32_t {
        if constexpr (NCH == 3) return third_bucket(y, NB, c1, c2, hk);
        return 0u;
    };
    const uint32_t ekey = uniform(empty_key_e1<NCH>(NB, hk));  // key of empty slots in the first NCH buckets
    if (ekey == 0u) return kOverflow;  // unusable hash functions: the caller tries others
    for (uint32_t i = lane; i < S; i += kWave) table[i] = empty_entry<NCH>(ekey, i);

    // Wave-uniform state.  Every update goes through uniform() so the compiler
    // keeps it in scalar registers and every loop that contains wave-wide
    // operations (ballot, DPP, readlane, shuffles) has a uniform exit.
    uint32_t size = 0, full = 0, failed = 0;
    uint32_t stash_live = 0;  // counters in the stash
    // minimum level: count m and its listed slots [list_ptr, list_len)
    uint32_t m = 0, list_len = 0, list_ptr = 0;
    uint32_t last_slow = 0;

    // input staging: the ring holds items [rbase, rbase + kRing)
    uint64_t rbase = begin & ~(uint64_t)(kRingHalf - 1);
    {
        Prefetch p0 = fetch_half(items, rbase, n, end, vec_ok, lane);
        Prefetch p1 = fetch_half(items, rbase + kRingHalf, n, end, vec_ok, lane);
        store_half(ring, rbase, p0, lane);
        store_half(ring, rbase + kRingHalf, p1, lane);
    }
    Prefetch pf = fetch_half(items, rbase + kRing, n, end, vec_ok, lane);
    wave_sync();

    KSTAT_DECL
    const unsigned long long t_start = KSTAT_NOW();
    uint64_t pos = begin;
    // each window's items are read from the ring at the end of the window
    // before (the refill at the top never overwrites them)
    uint32_t xn = ring[(uint32_t)(pos + lane) & (kRing - 1)];
    while (pos < end && !failed) {
        KSTAT_ADD(0, 1);
        if (pos >= rbase + kRingHalf) {
            const unsigned long long t0 = KSTAT_NOW();
            store_half(ring, rbase + kRing, pf, lane);  // overwrites the consumed half
            rbase += kRingHalf;
            pf = fetch_half(items, rbase + kRing, n, end, vec_ok, lane);
            wave_sync();
            KSTAT_ADD(9, KSTAT_NOW() - t0);
            KSTAT_ADD(10, 1);
        }
        const unsigned long long tw = KSTAT_NOW();
        // the stash, lane i holding slot T + i: its keys serve this window's
        // lookups
        uint32_t skey = 0;
        bool slive = false;
        if (stash_live) {
            const uint64_t e = table[T + lane];
            skey = (uint32_t)e;
            const uint32_t c = (uint32_t)(e >> 32);
            slive = live_tag(c);
            // move counters back to a bucket with room (deletions free slots
            // all the time).  A counter at the minimum level stays: it may be
            // listed as a victim by slot.
            const bool cand = slive && (!full || (c & cmask) != m);
            if (ballot(cand)) {
                const uint32_t s1 = home_bucket(skey, NB, hk), s2 = alt_bucket(skey, NB, s1, hk);
                const uint32_t s3 = bucket3(skey, s1, s2);
                const Bucket B1 = load_bucket(tbl4, s1), B2 = load_bucket(tbl4, s2);
                const uint32_t e1 = empty_mask(B1), e2 = empty_mask(B2);
                uint32_t e3 = 0u;
                if constexpr (NCH == 3) e3 = empty_mask(load_bucket(tbl4, s3));
                bool moved = false;
                if (cand && (e1 | e2 | e3)) {
                    // the emptiest bucket (the earliest on ties), its first free slot
                    const uint32_t n1 = __builtin_popcount(e1), n2 = __builtin_popcount(e2);
                    const bool first = n1 >= n2;
                    uint32_t fm = first ? e1 : e2, fb = first ? s1 : s2;  // free-slot mask, bucket
                    if (__builtin_popcount(e3) > (first ? n1 : n2)) {
                        fm = e3;
                        fb = s3;
                    }
                    const uint32_t dst = kBucketSlots * fb + (uint32_t)__builtin_ctz(fm);
                    const uint64_t emp = empty_entry<NCH>(ekey, dst);
                    if (atomicCAS((unsigned long long*)&table[dst], (unsigned long long)emp, (unsigned long long)e) ==
                        emp) {
                        err_put(dst, err_get(T + lane));
                        table[T + lane] = 0ull;
                        moved = true;
                    }
                }
                slive = slive && !moved;
                stash_live = uniform(stash_live - popc64(ballot(moved)));
                wave_sync();
            }
        }

        const uint32_t wl = (uint32_t)((end - pos) < kWave ? (end - pos) : kWave);
        const bool valid = lane < wl;
        const uint32_t x = valid ? xn : 0u;

        // victims for this window (list entries list_ptr + lane), fetched early
        // when the last window needed them.  The loads are unconditional on
        // clamped indices: no divergent branch may separate the wave-wide
        // operations of the victim loop below.
        bool vinb = false;
        uint32_t vs = 0, vcnt = 0;
        auto fetch_victims = [&]() {
            const uint32_t li = list_ptr + lane;
            vinb = li < list_len;
            const uint32_t e = list[vinb ? li : 0u];
            vs = vinb ? e : 0u;
            vcnt = words[2 * vs + 1];
        };
        const bool early = last_slow && full && list_ptr < list_len;
        if (early) fetch_victims();

        // 1. look up against the state at window start: the item's buckets
        //    (four 16-byte loads each, branch-free), then the stash while it
        //    is used
        bool hit = false, miss = false, bad = false, nofree = false;
        uint32_t slot = 0, hp = kNone;
        const uint32_t b1 = home_bucket(x, NB, hk);
        const uint32_t b2 = alt_bucket(x, NB, b1, hk);
        const uint32_t b3 = bucket3(x, b1, b2);
        Bucket B1 = load_bucket(tbl4, b1), B2 = load_bucket(tbl4, b2);
        Bucket B3;
        if constexpr (NCH == 3) B3 = load_bucket(tbl4, b3);
        {
            const uint32_t h1 = match_mask(B1, x), h2 = match_mask(B2, x);
            uint32_t h3 = 0u;
            if constexpr (NCH == 3) h3 = match_mask(B3, x);
            const uint32_t hb = h1 ? b1 : h2 ? b2 : b3;
            const uint32_t hm = h1 ? h1 : h2 ? h2 : h3;
            slot = kBucketSlots * hb + ((uint32_t)__builtin_ctz(hm | (1u << kBucketSlots)) & (kBucketSlots - 1));
            hit = valid && (h1 | h2 | h3) != 0u;
        }
        KSTAT_ADD(16, stash_live ? 1 : 0);
        // the stash's live keys, one by one from the lanes holding them
        for (uint64_t sm = ballot(slive); sm; sm &= sm - 1) {
            const uint32_t j = (uint32_t)__builtin_ctzll(sm);
            if (x == (uint32_t)__builtin_amdgcn_readlane((int)skey, (int)j)) {
                hit = valid;
                slot = T + j;
            }
        }
        miss = valid && !hit;

        const uint64_t missmask = ballot(miss);
        KSTAT_ADD(15, KSTAT_NOW() - tw);
        if (missmask == 0) {
            // all hits: increments commute
            pos += wl;
            xn = ring[(uint32_t)(pos + lane) & (kRing - 1)];
            if (hit) atomicAdd(&words[2 * slot + 1], 1u);
            last_slow = 0;
            KSTAT_ADD(1, 1);
            KSTAT_ADD(2, KSTAT_NOW() - tw);
            continue;
        }
        last_slow = 1;

        // 2. group unmonitored items by value: one claimed slot per value,
        //    tagged with the lowest lane holding it
        const unsigned long long tp = KSTAT_NOW();
        //    Each lane claims a free slot of its emptiest bucket (else of the
        //    stash) with a compare-and-swap, working from the buckets as the
        //    lookup read them: no claim exists at window start, and a lost
        //    swap returns the slot's new entry -- a claim of the same value
        //    (the lane joins it, lowering the claim's lane) or of another one
        //    (the slot leaves the lane's view).  Lanes holding equal values
        //    see the same buckets and the same outcomes, so they pick the same
        //    slots.  Every lost swap removes a slot from the view, so the loop
        //    ends within 8 NCH + 64 rounds.  The claimed slot becomes the new
        //    counter if the item is installed.
#ifdef PSS_KERNEL_STATS
        uint32_t steps_seen = 0;
#endif
        if (miss) {
            const uint64_t mine = make_entry(x, kTagPend + lane);
            uint32_t e1 = empty_mask(B1), e2 = empty_mask(B2), e3 = 0u;
            if constexpr (NCH == 3) e3 = empty_mask(B3);
            uint32_t steps = 0;
            for (;;) {
                uint32_t h = kNone;
                bool join = false;
                if (e1 | e2 | e3) {
                    h = claim_slot(e1, e2, e3, b1, b2, b3, x, hk.pick);
                } else {
                    // all its buckets full: the value's claim, or a free slot, in the stash
                    uint32_t fe = kNone;
                    for (uint32_t i = 0; i < kStash / 2; ++i) {
                        const uint4 e = stash4[i];
                        if (e.x == x && e.y >= kTagPend) {
                            h = T + 2 * i;
                            join = true;
                        }
                        if (e.z == x && e.w >= kTagPend) {
                            h = T + 2 * i + 1;
                            join = true;
                        }
                        if (fe == kNone && e.y == kTagEmpty) fe = T + 2 * i;
                        if (fe == kNone && e.w == kTagEmpty) fe = T + 2 * i + 1;
                    }
                    if (!join) h = fe;
                }
                if (h == kNone) {  // no free slot in the item's buckets or the stash
                    bad = true;
                    nofree = true;
                    break;
                }
                if (!join) {
                    const uint64_t emp = empty_entry<NCH>(ekey, h);
                    const uint64_t old =
                        atomicCAS((unsigned long long*)&table[h], (unsigned long long)emp, (unsigned long long)mine);
                    if (old == emp) {
                        hp = h;
                        break;
                    }
                    join = (uint32_t)old == x && (uint32_t)(old >> 32) >= kTagPend;
                    if (!join && h < T) {  // taken by another value
                        const uint32_t bit = 1u << (h % kBucketSlots);
                        const uint32_t hb = h / kBucketSlots;
                        if (hb == b1)
                            e1 &= ~bit;
                        else if (hb == b2)
                            e2 &= ~bit;
                        else
                            e3 &= ~bit;
                    }
                }
                if (join) {
                    atomicMin(&words[2 * h + 1], kTagPend + lane);
                    hp = h;
                    break;
                }
                if (++steps > (uint32_t)NCH * kBucketSlots + kStash) {
                    bad = true;
                    break;
                }
            }
#ifdef PSS_KERNEL_STATS
            steps_seen = steps + 1;
#endif
        }
        KSTAT_ADD(26, KSTAT_NOW() - tp);
#ifdef PSS_KERNEL_STATS
        KSTAT_ADD(27, wave_max_u32(steps_seen));
#endif
        if (ballot(bad)) {
            failed = ballot(nofree) ? 2u : 1u;  // 2: the hash functions, not the algorithm
            continue;
        }
        KSTAT_ADD(17, popc64(ballot(miss && hp >= T)));
        KSTAT_ADD(18, popc64(ballot(miss)));

        KSTAT_ADD(13, KSTAT_NOW() - tp);
        const unsigned long long tv = KSTAT_NOW();
        // 3. victims: the counters of level m in id order, from the list
        uint32_t avail = 0, vr = 0;
        uint64_t vmask = 0;
        bool vv = false;
        if (!full) {
            avail = k - size;
        } else {
            if (!early) fetch_victims();
            // at most one pass over the listed entries plus one rebuild
            uint32_t guard = list_len / kWave + 3;
            for (;;) {
                vv = vinb && (vcnt & cmask) == m;
                vmask = ballot(vv);
                if (vmask) break;
                if (guard-- == 0) {
                    failed = 1;
                    break;
                }
                if (list_ptr + kWave < list_len) {
                    list_ptr = uniform(list_ptr + kWave);
                } else {
                    // level exhausted: list the new minimum level, by id
                    const unsigned long long tl = KSTAT_NOW();
                    KSTAT_ADD(5, 1);
                    uint32_t len = 0;
                    const unsigned long long tsrt = KSTAT_NOW();
                    if constexpr (G) {
                        const uint64_t rr = build_level_global(sb, lds, L, m, lane);
                        m = uniform((uint32_t)(rr >> 32));
                        len = uniform((uint32_t)rr);
                    } else {
                        uint64_t rr;
                        if constexpr (P >= 16)
                            rr = build_level_lds<P>((uint32_t)(sb - smem), L, m, lane);
                        else
                            rr = level_lds_body<P>((uint32_t)(sb - smem), L, m, lane);
                        m = uniform((uint32_t)(rr >> 32));
                        len = uniform((uint32_t)rr);
                    }
                    list_len = len;
                    list_ptr = 0;
                    KSTAT_ADD(8, KSTAT_NOW() - tsrt);
                    KSTAT_ADD(4, KSTAT_NOW() - tl);
                }
                fetch_victims();
            }
            if (failed) continue;
            avail = popc64(vmask);
            vr = mbcnt(vmask);
            // tag them with their rank for the conflict test (their count is m)
            if (vv) words[2 * vs + 1] = kTagVict + vr;
        }
        wave_sync();
        KSTAT_ADD(6, KSTAT_NOW() - tv);
        const unsigned long long tq = KSTAT_NOW();

        const uint32_t rep = miss ? (tag_word<G>(words, 2 * hp + 1) - kTagPend) : lane;
        // a hit on a counter tagged as the j-th victim: jmark = j + 1
        uint32_t jmark = 0;
        if (hit && full) {
            const uint32_t c = tag_word<G>(words, 2 * slot + 1);
            jmark = (c >= kTagVict && c < kTagPend) ? c - kTagVict + 1u : 0u;
        }
        const uint64_t newmask = ballot(miss && rep == lane);
        const bool newf = (newmask >> lane) & 1ull;
        const uint32_t r = popc64(newmask);
        const uint32_t nrank = mbcnt(newmask);

        // 4. longest prefix with no conflict
        uint32_t cpos = wl;
        if (newf && nrank >= avail) cpos = lane;
        if (jmark != 0 && jmark - 1 < r) {
            // the hit and the eviction of the same counter cannot both be applied
            uint64_t mm = newmask;
            for (uint32_t t = 0; t + 1 < jmark; ++t) mm &= mm - 1;
            cpos = max(lane, (uint32_t)__builtin_ctzll(mm));
        }
        const uint32_t p = uniform(ballot(cpos < wl) ? wave_min_u32(cpos) : wl);
        if (p == 0) {  // the first item of a window is always applicable
            failed = 1;
            continue;
        }
        const bool in = lane < p;

        // 5. apply the prefix: the first rp victims empty their slots, the
        //    others get their count m back; then hits add 1; a new item
        //    becomes the counter in its claimed slot (count 1, or m + 1 with
        //    error m when it replaces a victim); a repeat adds 1 to its
        //    value's new counter; claims past the prefix are released
        KSTAT_ADD(24, KSTAT_NOW() - tq);
        const unsigned long long ta = KSTAT_NOW();
        const uint64_t inmask = (p >= kWave) ? ~0ull : ((1ull << p) - 1ull);
        const uint32_t rp = popc64(newmask & inmask);
        if (full) {
            if (vv) {
                if (vr < rp)
                    table[vs] = empty_entry<NCH>(ekey, vs);
                else
                    words[2 * vs + 1] = vcnt;  // its count word as fetched: count m (and its error)
            }
            wave_sync();
        }
        if (in && hit) atomicAdd(&words[2 * slot + 1], 1u);
        if (newf) {
            if (in) {
                err_put(hp, full ? m : 0u);
                table[hp] = make_entry(x, full ? (PK ? (m << kCountBits) | (m + 1u) : m + 1u) : 1u);
            } else {
                table[hp] = empty_entry<NCH>(ekey, hp);
            }
        }
        const bool repeat = in && miss && !newf;
        if (ballot(repeat)) {
            wave_sync();
            const uint32_t rslot = (uint32_t)__shfl((int)hp, (int)rep);
            if (repeat) atomicAdd(&words[2 * rslot + 1], 1u);
        }

        // stash occupancy: new counters placed there, evicted victims removed from there
        const uint32_t sadd = popc64(ballot(newf && in && hp >= T));
        const uint32_t sdel = popc64(ballot(vv && vr < rp && vs >= T));
        stash_live = uniform(stash_live + sadd - sdel);
        if (!full) {
            size = uniform(size + rp);
            if (size == k) {
                full = 1;
                list_len = 0;
                list_ptr = 0;
            }
        } else if (rp > 0) {
            const uint64_t lastm = ballot(vv && vr == rp - 1);
            list_ptr = uniform(list_ptr + (uint32_t)__builtin_ctzll(lastm) + 1u);
        }
        pos += p;
        xn = ring[(uint32_t)(pos + lane) & (kRing - 1)];
        wave_sync();
        KSTAT_ADD(25, KSTAT_NOW() - ta);
        KSTAT_ADD(3, KSTAT_NOW() - tw);
        KSTAT_ADD(11, p < wl ? 1 : 0);
        KSTAT_ADD(14, r);
    }
    KSTAT_ADD(12, KSTAT_NOW() - t_start);
    KSTAT_FLUSH();

    // write the summary, compacted from the slots, and its minimum (0 while
    // fewer than k counters are used)
    wave_sync();
    if (failed == 2) return kOverflow;
    if (failed) {
        if (lane == 0) {
            *o_size = kBlockFailed;
            *o_min = 0;
        }
        return kDone;
    }
    uint32_t mn = 0xFFFFFFFFu, outn = 0;
    for (uint32_t b = 0; b < S; b += kWave) {
        const uint32_t s = b + lane;
        const uint64_t e = s < S ? table[s] : 0ull;
        const uint32_t c = (uint32_t)(e >> 32);
        const bool live = s < S && live_tag(c);
        const uint64_t bm = ballot(live);
        if (live) {
            const uint32_t o = outn + mbcnt(bm);
            o_item[o] = (uint32_t)e;
            o_cnt[o] = c & cmask;
            o_err[o] = PK ? c >> kCountBits : err_get(s);
            mn = min(mn, c & cmask);
        }
        outn = uniform(outn + popc64(bm));
    }
    const uint32_t mo = full ? wave_min_u32(mn) : 0u;
    if (lane == 0) {
        *o_size = outn == size ? size : kBlockFailed;  // the slots hold exactly the counters
        *o_min = mo;
    }
    return kDone;
}

// A block under the attempts' hash functions in turn; after the last one
// overflows, the block is marked failed (the caller sees a device error).
template <int P, bool G, bool PK = false>
__device__ __forceinline__ void summarize_block_any(const uint32_t* __restrict__ items, uint64_t n, uint64_t begin,
                                                    uint64_t end, const ChunkLayout& L, int vec_ok,
                                                    unsigned char* sb, unsigned char* lds,
                                                    uint32_t* __restrict__ errs, uint32_t* __restrict__ o_item,
                                                    uint32_t* __restrict__ o_cnt, uint32_t* __restrict__ o_err,
                                                    uint32_t* __restrict__ o_size, uint32_t* __restrict__ o_min) {
    for (uint32_t attempt = 0; attempt < kHashAttempts; ++attempt) {
        if (summarize_block<P, G, PK>(items, n, begin, end, L, vec_ok, sb, lds, errs, o_item, o_cnt, o_err, o_size,
                                      o_min, hash_keys(attempt)) == kDone)
            return;
        wave_sync();  // the next attempt clears the table this one used
    }
    if (lane_id() == 0) {
        *o_size = kBlockFailed;
        *o_min = 0;
    }
}

// One wave per block c of C: [floor(c n / C), floor((c+1) n / C)) (Algorithm
// 1's block bounds, 64-bit products, n < 2^32).  G: state slab gstate +
// c * state_bytes.  Error scratch of block c: errs + c * err_stride.  PK:
// the layout packs each error in its counter's count word (no scratch).
template <int P, bool G, bool PK>
__global__ __launch_bounds__(64) void chunk_summary_kernel(const uint32_t* __restrict__ items, uint64_t n,
                                                           uint32_t chunks, ChunkLayout L, int vec_ok,
                                                           uint32_t* __restrict__ o_item,
                                                           uint32_t* __restrict__ o_cnt,
                                                           uint32_t* __restrict__ o_err,
                                                           uint32_t* __restrict__ o_size,
                                                           uint32_t* __restrict__ o_min,
                                                           unsigned char* __restrict__ gstate,
                                                           uint32_t* __restrict__ errs) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t c = blockIdx.x;
    unsigned char* sb = G ? gstate + (size_t)c * L.state_bytes : smem;
    const uint64_t begin = (uint64_t)c * n / chunks;
    const uint64_t end = (uint64_t)(c + 1) * n / chunks;
    const uint64_t ob = (uint64_t)c * L.k;
    summarize_block_any<P, G, PK>(items, n, begin, end, L, vec_ok, sb, smem, errs + (size_t)c * L.err_stride,
                                  o_item + ob, o_cnt + ob, o_err + ob, o_size + c, o_min + c);
}

// Batched form: every wave of a persistent grid takes blocks from a queue
// (one counter per launch, zeroed before it) until the list is exhausted.
// Blocks of one launch share P (their k fall in one size class); each block
// carries its own stream, bounds, k, hash load factor and error scratch
// (errs + eoff).  W waves per workgroup, each with its own LDS slab of
// lds_stride bytes.
template <int P, int W>
__global__ __launch_bounds__(64 * W) void batch_blocks_kernel(const BatchBlock* __restrict__ blocks,
                                                              uint32_t nblocks, uint32_t* __restrict__ queue,
                                                              uint32_t lds_stride, uint32_t* __restrict__ o_item,
                                                              uint32_t* __restrict__ o_cnt,
                                                              uint32_t* __restrict__ o_err,
                                                              uint32_t* __restrict__ o_size,
                                                              uint32_t* __restrict__ o_min,
                                                              uint32_t* __restrict__ errs) {
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned char* lds = smem + (threadIdx.x / kWave) * lds_stride;
    const uint32_t lane = lane_id();
    for (;;) {
        uint32_t b = 0;
        if (lane == 0) b = atomicAdd(queue, 1u);
        b = __builtin_amdgcn_readlane(b, 0);
        if (b >= nblocks) break;
        const BatchBlock bb = blocks[b];
        const ChunkLayout L = ChunkLayout::make(bb.k, false, bb.slots_x16).with_error_width(bb.end - bb.begin);
        const int vec_ok = ((uintptr_t)bb.items & 15u) == 0;
        summarize_block_any<P, false>(bb.items, bb.n, bb.begin, bb.end, L, vec_ok, lds, lds, errs + bb.eoff,
                                  o_item + bb.out, o_cnt + bb.out, o_err + bb.out, o_size + b, o_min + b);
        wave_sync();  // the slab is reused by the next block
    }
}

template <int P, int W>
static hipError_t launch_batch_pw(const BatchBlock* blocks, uint32_t nblocks, uint32_t* queue, uint32_t lds_stride,
                                  uint32_t grid, const BlockSummaries& out, uint32_t* errs, hipStream_t stream) {
    (void)hipGetLastError();  // a stale error of an earlier, unrelated call is not this launch's
    const uint32_t lds = W * lds_stride;
    hipFuncSetAttribute((const void*)batch_blocks_kernel<P, W>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((batch_blocks_kernel<P, W>), dim3(grid), dim3(64 * W), lds, stream, blocks, nblocks, queue,
                       lds_stride, out.item, out.cnt, out.err, out.size, out.min, errs);
    return hipGetLastError();
}

template <int P>
static hipError_t launch_batch_p(const BatchBlock* blocks, uint32_t nblocks, uint32_t* queue, uint32_t lds_stride,
                                 uint32_t waves_per_group, uint32_t grid, const BlockSummaries& out, uint32_t* errs,
                                 hipStream_t stream) {
    switch (waves_per_group) {
    case 1: return launch_batch_pw<P, 1>(blocks, nblocks, queue, lds_stride, grid, out, errs, stream);
    case 2:
        if constexpr (P <= 16) return launch_batch_pw<P, 2>(blocks, nblocks, queue, lds_stride, grid, out, errs, stream);
        return hipErrorInvalidValue;
    case 4:
        if constexpr (P <= 8) return launch_batch_pw<P, 4>(blocks, nblocks, queue, lds_stride, grid, out, errs, stream);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_blocks(const BatchBlock* blocks, uint32_t nblocks, uint32_t* queue, uint32_t sort_lanes,
                               uint32_t lds_stride, uint32_t waves_per_group, uint32_t grid,
                               const BlockSummaries& out, uint32_t* errs, hipStream_t stream) {
    if (nblocks == 0) return hipSuccess;
    if (!errs) return hipErrorInvalidValue;
    switch (sort_lanes) {
    case 1:
    case 2: return launch_batch_p<2>(blocks, nblocks, queue, lds_stride, waves_per_group, grid, out, errs, stream);
    case 4: return launch_batch_p<4>(blocks, nblocks, queue, lds_stride, waves_per_group, grid, out, errs, stream);
    case 8: return launch_batch_p<8>(blocks, nblocks, queue, lds_stride, waves_per_group, grid, out, errs, stream);
    case 16: return launch_batch_p<16>(blocks, nblocks, queue, lds_stride, waves_per_group, grid, out, errs, stream);
    case 32: return launch_batch_p<32>(blocks, nblocks, queue, lds_stride, waves_per_group, grid, out, errs, stream);
    case 64: return launch_batch_p<64>(blocks, nblocks, queue, lds_stride, waves_per_group, grid, out, errs, stream);
    default: return hipErrorInvalidValue;
    }
}

#ifdef PSS_KERNEL_STATS
extern "C" int pss_debug_kstats(unsigned long long* out, int reset) {
    if (hipMemcpyFromSymbol(out, HIP_SYMBOL(g_kstats), sizeof(g_kstats)) != hipSuccess) return -6;
    if (reset) {
        unsigned long long z[32] = {0};
        if (hipMemcpyToSymbol(HIP_SYMBOL(g_kstats), z, sizeof(z)) != hipSuccess) return -6;
    }
    return 0;
}
#endif

template <int P, bool G, bool PK>
static hipError_t launch_pe(const uint32_t* d_items, uint64_t n, uint32_t chunks, const ChunkLayout& L, int vec_ok,
                            const BlockSummaries& out, unsigned char* gstate, uint32_t* errs, hipStream_t stream) {
    (void)hipGetLastError();  // a stale error of an earlier, unrelated call is not this launch's
    hipFuncSetAttribute((const void*)chunk_summary_kernel<P, G, PK>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)L.lds_bytes);
    hipLaunchKernelGGL((chunk_summary_kernel<P, G, PK>), dim3(chunks), dim3(64), L.lds_bytes, stream, d_items, n,
                       chunks, L, vec_ok, out.item, out.cnt, out.err, out.size, out.min, gstate, errs);
    return hipGetLastError();
}

// Errors packed in the count words (the common case: blocks of fewer than
// 2^22 items and at most 1022 k) get their own instance of the LDS-state
// kernels, with no error scratch and no width switch in the window loop
template <int P, bool G>
static hipError_t launch_p(const uint32_t* d_items, uint64_t n, uint32_t chunks, const ChunkLayout& L, int vec_ok,
                           const BlockSummaries& out, unsigned char* gstate, uint32_t* errs, hipStream_t stream) {
    if constexpr (!G) {
        if (L.err_bytes == 0) return launch_pe<P, G, true>(d_items, n, chunks, L, vec_ok, out, gstate, errs, stream);
    }
    return launch_pe<P, G, false>(d_items, n, chunks, L, vec_ok, out, gstate, errs, stream);
}

// Waves per CU for blocks whose state lives in device memory.  Their table
// accesses miss the L2, and with every CU full of waves (16 by registers)
// the blocks' states (284 KiB each at k = 10^4) far exceed the last-level
// cache, so every access went to HBM; with four waves per CU the k = 10^4
// states (~290 MiB) mostly stay in it.  Measured on the 2^31-item high-k
// streams: 4 waves per CU are 25-34% faster at k = 10^4 than 16 and equal at
// k = 5 x 10^4; 2 and 8 are slower.  The layout asks for a quarter of the
// CU's LDS so that no more waves fit.
constexpr uint32_t kGlobalStateWavesPerCu = 4;

ChunkLayout chunk_layout(uint32_t k, size_t lds_max) {
    const ChunkLayout L = ChunkLayout::make(k, false);
    if (L.fits_lds_indices() && L.lds_bytes <= lds_max && sort_lanes_per_k(k) <= 64) return L;
    ChunkLayout G = ChunkLayout::make(k, true);
    const uint32_t quarter = (uint32_t)(lds_max / kGlobalStateWavesPerCu) / kLdsUnit * kLdsUnit;
    if (quarter > G.lds_bytes) G.lds_bytes = quarter;
    return G;
}

hipError_t launch_chunk_summary(const uint32_t* d_items, uint64_t n, uint32_t chunks, const ChunkLayout& L0,
                                const BlockSummaries& out, unsigned char* gstate, uint32_t* errs,
                                hipStream_t stream) {
    const int vec_ok = ((uintptr_t)d_items & 15u) == 0;
    if (chunks == 0) return hipErrorInvalidValue;
    // blocks hold at most ceil(n / chunks) items
    const ChunkLayout L = L0.with_error_width((n + chunks - 1) / chunks, true);
    if (!errs) return hipErrorInvalidValue;
    if (L.global_state) {
        if (!gstate) return hipErrorInvalidValue;
        return launch_p<1, true>(d_items, n, chunks, L, vec_ok, out, gstate, errs, stream);
    }
    switch (sort_lanes_per_k(L.k)) {
    case 1:
    case 2: return launch_p<2, false>(d_items, n, chunks, L, vec_ok, out, nullptr, errs, stream);
    case 4: return launch_p<4, false>(d_items, n, chunks, L, vec_ok, out, nullptr, errs, stream);
    case 8: return launch_p<8, false>(d_items, n, chunks, L, vec_ok, out, nullptr, errs, stream);
    case 16: return launch_p<16, false>(d_items, n, chunks, L, vec_ok, out, nullptr, errs, stream);
    case 32: return launch_p<32, false>(d_items, n, chunks, L, vec_ok, out, nullptr, errs, stream);
    case 64: return launch_p<64, false>(d_items, n, chunks, L, vec_ok, out, nullptr, errs, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace pss
