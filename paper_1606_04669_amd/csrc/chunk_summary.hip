// Block summaries: sequential Space Saving over each of C contiguous blocks
// of the input (Section 3, second paragraph; Algorithm 1, SpaceSaving on
// [left, right]).  One wave owns one block and keeps its k counters in LDS.
//
// The wave consumes its block in windows of up to 64 consecutive items, one
// item per lane, and reproduces the sequential algorithm exactly:
//
//  * every lane looks its item up in an open-addressed hash (item -> counter)
//    holding the state at window start;
//  * items not monitored are grouped by value; the first occurrence of each
//    value ("new item") will take a counter, later occurrences add 1 to it;
//  * while counters are free, the j-th new item takes free counter size+j;
//    once all k are used, the j-th new item evicts the j-th victim, where the
//    victims are the counters of the current minimum count m taken in
//    increasing item id (the sequential rule: minimum count, then smallest
//    id), installed with count m+1 and error m;
//  * hits add 1 and commute with each other; the only interactions with the
//    evictions are a hit on a counter that is also evicted in the window, and
//    running out of free counters or of counters at level m.  The wave takes
//    the longest prefix of the window free of both, applies it at once and
//    starts the next window at the first item it did not apply.  The first
//    item of a window is always applicable, so every window makes progress.
//
// The counters at the minimum level are kept as a list sorted by item id,
// built when the level is first needed; an entry stays usable while its
// counter still holds that item at count m (counts never decrease and new
// items enter at m+1, so nothing joins level m after the list is built).
#include "pss_device.h"
#include "pss_layout.h"
#include "pss_kernels.h"

namespace pss {

constexpr uint32_t kTagEmpty = 0u;
constexpr uint32_t kTagTomb = 0xFFFFFFFFu;
constexpr uint32_t kTagPend = 0x80000000u;

__device__ __forceinline__ uint64_t make_entry(uint32_t key, uint32_t tag) {
    return ((uint64_t)tag << 32) | key;
}

// Bitonic sort (ascending) of P (power of two) uint64 values by one wave.
__device__ void wave_bitonic_sort_u64(uint64_t* a, uint32_t P, uint32_t lane) {
    for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t t = lane; t < P / 2; t += kWave) {
                uint32_t i = 2 * t - (t & (stride - 1));
                uint32_t j = i + stride;
                bool up = (i & size) == 0;
                uint64_t x = a[i], y = a[j];
                if ((x > y) == up) {
                    a[i] = y;
                    a[j] = x;
                }
            }
            wave_sync();
        }
    }
}

// Four consecutive items at idx (a multiple of 4), zero beyond the array.
__device__ __forceinline__ uint4 load4(const uint32_t* __restrict__ items, uint64_t idx, uint64_t n, uint64_t stop,
                                       int vec_ok) {
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (idx >= stop) return v;
    if (vec_ok && idx + 3 < n) {
        v = *(const uint4*)(items + idx);
    } else {
        if (idx < n) v.x = items[idx];
        if (idx + 1 < n) v.y = items[idx + 1];
        if (idx + 2 < n) v.z = items[idx + 2];
        if (idx + 3 < n) v.w = items[idx + 3];
    }
    return v;
}

struct Prefetch {
    uint4 a, b;
};

__device__ __forceinline__ Prefetch fetch_half(const uint32_t* __restrict__ items, uint64_t tile, uint64_t n,
                                               uint64_t stop, int vec_ok, uint32_t lane) {
    Prefetch p;
    p.a = load4(items, tile + 4 * lane, n, stop, vec_ok);
    p.b = load4(items, tile + 256 + 4 * lane, n, stop, vec_ok);
    return p;
}

__device__ __forceinline__ void store_half(uint32_t* ring, uint64_t tile, const Prefetch& p, uint32_t lane) {
    uint32_t base = (uint32_t)tile & (kRing - 1);
    *(uint4*)(ring + base + 4 * lane) = p.a;
    *(uint4*)(ring + base + 256 + 4 * lane) = p.b;
}

__global__ __launch_bounds__(64) void chunk_summary_kernel(const uint32_t* __restrict__ items, uint64_t n,
                                                           uint32_t chunks, ChunkLayout L, int vec_ok,
                                                           uint32_t* __restrict__ o_item,
                                                           uint32_t* __restrict__ o_cnt,
                                                           uint32_t* __restrict__ o_err,
                                                           uint32_t* __restrict__ o_size,
                                                           uint32_t* __restrict__ o_min) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t lane = threadIdx.x;
    const uint32_t c = blockIdx.x;
    const uint32_t k = L.k;
    uint64_t* table = (uint64_t*)(smem + L.off_table);
    uint64_t* list = (uint64_t*)(smem + L.off_list);
    uint32_t* cnt = (uint32_t*)(smem + L.off_cnt);
    uint32_t* item = (uint32_t*)(smem + L.off_item);
    uint32_t* err = (uint32_t*)(smem + L.off_err);
    uint32_t* hpos = (uint32_t*)(smem + L.off_hpos);
    uint8_t* mark = (uint8_t*)(smem + L.off_mark);
    uint32_t* ring = (uint32_t*)(smem + L.off_ring);
    uint32_t* vbuf = (uint32_t*)(smem + L.off_scratch);
    uint32_t* posbuf = vbuf + 64;

    // block bounds (Algorithm 1): [floor(c n / C), floor((c+1) n / C)), n < 2^32
    const uint64_t begin = (uint64_t)c * n / chunks;
    const uint64_t end = (uint64_t)(c + 1) * n / chunks;
    const uint32_t tmask = L.tsize - 1;
    const uint32_t tlimit = L.tsize - 65;  // keep >= 65 empty slots before each window

    for (uint32_t i = lane; i < L.tsize; i += kWave) table[i] = 0ull;
    for (uint32_t i = lane; i < k; i += kWave) mark[i] = 0;

    uint32_t size = 0, full = 0, m = 0, list_len = 0, list_ptr = 0, tused = 0;

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

    uint64_t pos = begin;
    while (pos < end) {
        if (pos >= rbase + kRingHalf) {
            store_half(ring, rbase + kRing, pf, lane);  // overwrites the consumed half
            rbase += kRingHalf;
            pf = fetch_half(items, rbase + kRing, n, end, vec_ok, lane);
            wave_sync();
        }
        if (tused > tlimit) {
            // drop tombstones: rebuild the hash from the live counters
            for (uint32_t i = lane; i < L.tsize; i += kWave) table[i] = 0ull;
            wave_sync();
            for (uint32_t s = lane; s < size; s += kWave) {
                uint32_t x = item[s];
                uint32_t h = hash_slot(x, L.tbits);
                while (atomicCAS((unsigned long long*)&table[h], 0ull, (unsigned long long)make_entry(x, s + 1)) != 0ull)
                    h = (h + 1) & tmask;
                hpos[s] = h;
            }
            wave_sync();
            tused = size;
        }

        const uint32_t wl = (uint32_t)((end - pos) < kWave ? (end - pos) : kWave);
        const bool valid = lane < wl;
        const uint32_t x = valid ? ring[(uint32_t)(pos + lane) & (kRing - 1)] : 0u;

        // 1. look up against the state at window start
        bool hit = false, miss = false;
        uint32_t slot = 0, hp = 0;
        if (valid) {
            uint32_t h = hash_slot(x, L.tbits);
            for (;;) {
                uint64_t e = table[h];
                uint32_t tag = (uint32_t)(e >> 32);
                if (tag == kTagEmpty) {
                    miss = true;
                    break;
                }
                if (tag != kTagTomb && (uint32_t)e == x) {
                    hit = true;
                    slot = tag - 1u;
                    break;
                }
                h = (h + 1) & tmask;
            }
            hp = h;
        }

        // 2. group unmonitored items by value: one pending hash entry per
        //    value, tagged with the lowest lane holding it
        const uint64_t missmask = ballot(miss);
        uint32_t rep = lane;
        uint64_t newmask = 0;
        if (missmask) {
            if (miss) {
                const uint64_t mine = make_entry(x, kTagPend | lane);
                uint32_t h = hp;
                for (;;) {
                    uint64_t old = atomicCAS((unsigned long long*)&table[h], 0ull, (unsigned long long)mine);
                    if (old == 0ull) break;
                    uint32_t otag = (uint32_t)(old >> 32);
                    if (otag != kTagTomb && (otag & kTagPend) && (uint32_t)old == x) {
                        atomicMin(((uint32_t*)&table[h]) + 1, kTagPend | lane);
                        break;
                    }
                    h = (h + 1) & tmask;
                }
                hp = h;
            }
            wave_sync();
            if (miss) rep = ((const volatile uint32_t*)&table[hp])[1] & 63u;
            newmask = ballot(miss && rep == lane);
        }
        const bool newf = (newmask >> lane) & 1ull;
        const uint32_t r = popc64(newmask);
        const uint32_t nrank = mbcnt(newmask);

        // 3. counters the new items will take: free ones, or victims at level m
        uint32_t avail = 0;
        uint64_t vmask = 0;
        uint32_t vs = 0, vr = 0;
        bool vv = false;
        if (r > 0) {
            if (newf) posbuf[nrank] = lane;
            if (!full) {
                avail = k - size;
            } else {
                for (;;) {
                    if (list_ptr >= list_len) {
                        // (re)build the minimum level: all counters at the minimum count, by id
                        uint32_t mn = 0xFFFFFFFFu;
                        for (uint32_t s = lane; s < k; s += kWave) mn = min(mn, cnt[s]);
                        mn = wave_min_u32(mn);
                        uint32_t len = 0;
                        for (uint32_t b = 0; b < k; b += kWave) {
                            uint32_t s = b + lane;
                            bool is = s < k && cnt[s] == mn;
                            uint64_t bm = ballot(is);
                            if (is) list[len + mbcnt(bm)] = ((uint64_t)item[s] << 32) | s;
                            len += popc64(bm);
                        }
                        uint32_t P = next_pow2(len);
                        if (P < 2) P = 2;
                        for (uint32_t i = len + lane; i < P; i += kWave) list[i] = ~0ull;
                        wave_sync();
                        wave_bitonic_sort_u64(list, P, lane);
                        m = mn;
                        list_len = len;
                        list_ptr = 0;
                    }
                    uint32_t li = list_ptr + lane;
                    bool inb = li < list_len;
                    uint64_t le = inb ? list[li] : 0ull;
                    vs = (uint32_t)le;
                    vv = inb && item[vs] == (uint32_t)(le >> 32) && cnt[vs] == m;
                    vmask = ballot(vv);
                    if (vmask) break;
                    list_ptr = (list_ptr + kWave < list_len) ? list_ptr + kWave : list_len;
                }
                avail = popc64(vmask);
                vr = mbcnt(vmask);
                if (vv && vr < r) {
                    vbuf[vr] = vs;
                    mark[vs] = (uint8_t)(vr + 1);
                }
            }
            wave_sync();
        }

        // 4. longest prefix with no conflict
        uint32_t cpos = wl;
        if (newf && nrank >= avail) cpos = lane;
        if (hit && full && r > 0) {
            uint32_t j = mark[slot];
            if (j) cpos = max(lane, posbuf[j - 1]);
        }
        const uint32_t p = wave_min_u32(cpos);
        const bool in = lane < p;

        // 5. apply the prefix
        uint32_t myslot = 0;
        if (in && hit) atomicAdd(&cnt[slot], 1u);
        if (newf) {
            if (in) {
                if (!full) {
                    myslot = size + nrank;
                    cnt[myslot] = 1u;
                    err[myslot] = 0u;
                } else {
                    myslot = vbuf[nrank];
                    table[hpos[myslot]] = make_entry(0u, kTagTomb);
                    cnt[myslot] = m + 1u;
                    err[myslot] = m;
                }
                item[myslot] = x;
                hpos[myslot] = hp;
                table[hp] = make_entry(x, myslot + 1u);
            } else {
                table[hp] = make_entry(0u, kTagTomb);  // not applied: retire the pending entry
            }
        }
        wave_sync();
        const uint32_t rslot = (uint32_t)__shfl((int)myslot, (int)rep);
        if (in && miss && !newf) atomicAdd(&cnt[rslot], 1u);
        if (vv && vr < r) mark[vs] = 0;

        const uint64_t inmask = (p >= kWave) ? ~0ull : ((1ull << p) - 1ull);
        const uint32_t rp = popc64(newmask & inmask);
        if (!full) {
            size += rp;
            if (size == k) {
                full = 1;
                list_len = 0;
                list_ptr = 0;
            }
        } else if (rp > 0) {
            uint64_t lastm = ballot(vv && vr == rp - 1);
            list_ptr += (uint32_t)__builtin_ctzll(lastm) + 1u;
        }
        tused += r;
        pos += p;
        wave_sync();
    }

    // write the summary and its minimum (0 while fewer than k counters are used)
    uint32_t mo = 0;
    if (full) {
        uint32_t mn = 0xFFFFFFFFu;
        for (uint32_t s = lane; s < k; s += kWave) mn = min(mn, cnt[s]);
        mo = wave_min_u32(mn);
    }
    const uint64_t ob = (uint64_t)c * k;
    for (uint32_t s = lane; s < size; s += kWave) {
        o_item[ob + s] = item[s];
        o_cnt[ob + s] = cnt[s];
        o_err[ob + s] = err[s];
    }
    if (lane == 0) {
        o_size[c] = size;
        o_min[c] = mo;
    }
}

hipError_t launch_chunk_summary(const uint32_t* d_items, uint64_t n, uint32_t chunks, uint32_t k,
                                const BlockSummaries& out, hipStream_t stream) {
    ChunkLayout L = ChunkLayout::make(k);
    int vec_ok = ((uintptr_t)d_items & 15u) == 0;
    hipFuncSetAttribute((const void*)chunk_summary_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.bytes);
    hipLaunchKernelGGL(chunk_summary_kernel, dim3(chunks), dim3(64), L.bytes, stream, d_items, n, chunks, L, vec_ok,
                       out.item, out.cnt, out.err, out.size, out.min);
    return hipGetLastError();
}

uint32_t chunk_summary_lds_bytes(uint32_t k) { return ChunkLayout::make(k).bytes; }

}  // namespace pss
