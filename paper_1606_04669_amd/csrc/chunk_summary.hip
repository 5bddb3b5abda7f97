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
// The counters at the minimum level are consumed through a list of at most
// kListCap entries sorted by item id: the smallest ids of level m above the
// last id already listed.  An entry stays usable while its counter still
// holds that item at count m: counts never decrease and new items enter at
// m+1, so no counter joins level m after the level is first listed.
#include "pss_device.h"
#include "pss_layout.h"
#include "pss_kernels.h"

namespace pss {

constexpr uint32_t kTagEmpty = 0u;
constexpr uint32_t kTagTomb = 0xFFFFFFFFu;
constexpr uint32_t kTagPend = 0x80000000u;
constexpr uint64_t kTombEntry = (uint64_t)kTagTomb << 32;

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

// Four consecutive items at idx (a multiple of 4), zero at and beyond stop.
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

// Lane holding the bucket of a 256-bin histogram (4 bins per lane) that
// contains the rank-th element; returns the bin and the rank inside it.
__device__ __forceinline__ void hist_select(const uint32_t* hist, uint32_t rank, uint32_t lane, uint32_t* bin_out,
                                            uint32_t* rank_out) {
    uint32_t b0 = hist[4 * lane], b1 = hist[4 * lane + 1], b2 = hist[4 * lane + 2], b3 = hist[4 * lane + 3];
    uint32_t s = b0 + b1 + b2 + b3, incl = s;
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t t = (uint32_t)__shfl_up((int)incl, off);
        if ((int)lane >= off) incl += t;
    }
    uint32_t excl = incl - s;
    bool here = excl <= rank && rank < incl;
    uint32_t bin = 0, rr = 0;
    if (here) {
        rr = rank - excl;
        bin = 4 * lane;
        if (rr >= b0) {
            rr -= b0;
            ++bin;
            if (rr >= b1) {
                rr -= b1;
                ++bin;
                if (rr >= b2) {
                    rr -= b2;
                    ++bin;
                }
            }
        }
    }
    const uint64_t hm = ballot(here);
    const uint32_t src = (uint32_t)__builtin_ctzll(hm);
    *bin_out = __builtin_amdgcn_readlane(bin, src);
    *rank_out = __builtin_amdgcn_readlane(rr, src);
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
    uint32_t* hist = (uint32_t*)(smem + L.off_list);  // aliases the list while it is rebuilt
    uint32_t* cnt = (uint32_t*)(smem + L.off_cnt);
    uint32_t* item = (uint32_t*)(smem + L.off_item);
    uint32_t* err = (uint32_t*)(smem + L.off_err);
    uint16_t* hpos = (uint16_t*)(smem + L.off_hpos);
    uint8_t* mark = (uint8_t*)(smem + L.off_mark);
    uint32_t* ring = (uint32_t*)(smem + L.off_ring);
    uint32_t* vbuf = (uint32_t*)(smem + L.off_scratch);
    uint8_t* posbuf = (uint8_t*)(vbuf + 64);

    // block bounds (Algorithm 1): [floor(c n / C), floor((c+1) n / C)), n < 2^32
    const uint64_t begin = (uint64_t)c * n / chunks;
    const uint64_t end = (uint64_t)(c + 1) * n / chunks;
    const uint32_t tmask = L.tsize - 1;
    // rebuild the hash when live + tombstone slots pass 3/4 (always >= 65 empty)
    const uint32_t tlimit = min(L.tsize - L.tsize / 4, L.tsize - 65);

    for (uint32_t i = lane; i < L.tsize; i += kWave) table[i] = 0ull;
    for (uint32_t i = lane; i < k; i += kWave) mark[i] = 0;

    uint32_t size = 0, full = 0, tused = 0;
    // minimum level: count m, listed entries [list_ptr, list_len), last id listed,
    // and whether level m may hold counters with larger ids not yet listed
    uint32_t m = 0, list_len = 0, list_ptr = 0, last_id = 0, more = 0;

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
            wave_sync();
            for (uint32_t i = lane; i < L.tsize; i += kWave) table[i] = 0ull;
            wave_sync();
            for (uint32_t s = lane; s < size; s += kWave) {
                uint32_t x = item[s];
                uint32_t h = hash_slot(x, L.tbits);
                while (atomicCAS((unsigned long long*)&table[h], 0ull, (unsigned long long)make_entry(x, s + 1)) != 0ull)
                    h = (h + 1) & tmask;
                hpos[s] = (uint16_t)h;
            }
            wave_sync();
            tused = size;
        }

        const uint32_t wl = (uint32_t)((end - pos) < kWave ? (end - pos) : kWave);
        const bool valid = lane < wl;
        const uint32_t x = valid ? ring[(uint32_t)(pos + lane) & (kRing - 1)] : 0u;

        // 1. look up against the state at window start; remember the first
        //    tombstone on the probe path as the insertion point of a miss
        bool hit = false, miss = false;
        uint32_t slot = 0, hp = 0;
        if (valid) {
            uint32_t h = hash_slot(x, L.tbits);
            uint32_t first_free = 0xFFFFFFFFu;
            for (;;) {
                const uint64_t e = table[h];
                const uint32_t tag = (uint32_t)(e >> 32);
                if (tag == kTagEmpty) {
                    miss = true;
                    break;
                }
                if (tag == kTagTomb) {
                    if (first_free == 0xFFFFFFFFu) first_free = h;
                } else if ((uint32_t)e == x) {
                    hit = true;
                    slot = tag - 1u;
                    break;
                }
                h = (h + 1) & tmask;
            }
            hp = (miss && first_free != 0xFFFFFFFFu) ? first_free : h;
        }

        const uint64_t missmask = ballot(miss);
        if (missmask == 0) {
            // all hits: increments commute
            if (hit) atomicAdd(&cnt[slot], 1u);
            pos += wl;
            continue;
        }

        // 2. group unmonitored items by value: one pending hash entry per value,
        //    tagged with the lowest lane holding it
        bool took_empty = false;
        if (miss) {
            const uint64_t mine = make_entry(x, kTagPend | lane);
            uint32_t h = hp;
            for (;;) {
                uint64_t e = table[h];
                uint32_t tag = (uint32_t)(e >> 32);
                if (tag == kTagEmpty || tag == kTagTomb) {
                    const uint64_t old = atomicCAS((unsigned long long*)&table[h], (unsigned long long)e,
                                                   (unsigned long long)mine);
                    if (old == e) {
                        took_empty = tag == kTagEmpty;
                        break;
                    }
                    e = old;
                    tag = (uint32_t)(old >> 32);
                }
                if (tag != kTagTomb && (tag & kTagPend) && (uint32_t)e == x) {
                    atomicMin(((uint32_t*)&table[h]) + 1, kTagPend | lane);
                    break;
                }
                h = (h + 1) & tmask;
            }
            hp = h;
        }
        wave_sync();
        const uint32_t rep = miss ? (((const volatile uint32_t*)&table[hp])[1] & 63u) : lane;
        const uint64_t newmask = ballot(miss && rep == lane);
        const bool newf = (newmask >> lane) & 1ull;
        const uint32_t r = popc64(newmask);
        const uint32_t nrank = mbcnt(newmask);
        tused += popc64(ballot(took_empty));
        if (newf) posbuf[nrank] = (uint8_t)lane;

        // 3. counters the new items will take: free ones, or victims at level m
        uint32_t avail = 0;
        uint64_t vmask = 0;
        uint32_t vs = 0, vr = 0;
        bool vv = false;
        if (!full) {
            avail = k - size;
        } else {
            for (;;) {
                if (list_ptr >= list_len) {
                    // list the next counters of the minimum level, by id
                    uint32_t lo = 0;
                    bool fresh = !more || last_id == 0xFFFFFFFFu;
                    if (!fresh) lo = last_id + 1;
                    uint32_t cand = 0;
                    for (int attempt = 0; attempt < 2; ++attempt) {
                        if (fresh) {
                            uint32_t mn = 0xFFFFFFFFu;
                            for (uint32_t s = lane; s < k; s += kWave) mn = min(mn, cnt[s]);
                            m = wave_min_u32(mn);
                            lo = 0;
                        }
                        uint32_t cl = 0;
                        for (uint32_t s = lane; s < k; s += kWave) cl += (cnt[s] == m && item[s] >= lo) ? 1u : 0u;
                        cand = wave_add_u32(cl);
                        if (cand > 0) break;
                        fresh = true;  // level m holds nothing above lo: move to the new minimum
                    }
                    // ids above lo at level m: take the kListCap smallest
                    uint32_t hi = 0xFFFFFFFFu;
                    if (cand > kListCap) {
                        uint32_t prefix = 0, rank = kListCap - 1;
                        for (int d = 3; d >= 0; --d) {
                            const uint32_t sh = 8u * (uint32_t)d;
                            const uint32_t pm = (d == 3) ? 0u : (0xFFFFFFFFu << (sh + 8));
                            for (uint32_t i = lane; i < 256; i += kWave) hist[i] = 0u;
                            wave_sync();
                            for (uint32_t s = lane; s < k; s += kWave) {
                                const uint32_t it = item[s];
                                if (cnt[s] == m && it >= lo && (it & pm) == prefix)
                                    atomicAdd(&hist[(it >> sh) & 255u], 1u);
                            }
                            wave_sync();
                            uint32_t bin, rr;
                            hist_select(hist, rank, lane, &bin, &rr);
                            prefix |= bin << sh;
                            rank = rr;
                            wave_sync();
                        }
                        hi = prefix;
                    }
                    uint32_t len = 0;
                    for (uint32_t b = 0; b < k; b += kWave) {
                        const uint32_t s = b + lane;
                        bool take = false;
                        uint32_t it = 0;
                        if (s < k) {
                            it = item[s];
                            take = cnt[s] == m && it >= lo && it <= hi;
                        }
                        const uint64_t bm = ballot(take);
                        if (take) list[len + mbcnt(bm)] = ((uint64_t)it << 32) | s;
                        len += popc64(bm);
                    }
                    uint32_t P = next_pow2(len);
                    if (P < 2) P = 2;
                    for (uint32_t i = len + lane; i < P; i += kWave) list[i] = ~0ull;
                    wave_sync();
                    wave_bitonic_sort_u64(list, P, lane);
                    list_len = len;
                    list_ptr = 0;
                    last_id = (uint32_t)(list[len - 1] >> 32);
                    more = cand > len;
                }
                const uint32_t li = list_ptr + lane;
                const bool inb = li < list_len;
                const uint64_t le = inb ? list[li] : 0ull;
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

        // 4. longest prefix with no conflict
        uint32_t cpos = wl;
        if (newf && nrank >= avail) cpos = lane;
        if (hit && full) {
            const uint32_t j = mark[slot];
            if (j) cpos = max(lane, (uint32_t)posbuf[j - 1]);
        }
        const uint32_t p = ballot(cpos < wl) ? wave_min_u32(cpos) : wl;
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
                    table[hpos[myslot]] = kTombEntry;
                    cnt[myslot] = m + 1u;
                    err[myslot] = m;
                }
                item[myslot] = x;
                hpos[myslot] = (uint16_t)hp;
                table[hp] = make_entry(x, myslot + 1u);
            } else {
                table[hp] = kTombEntry;  // not applied: retire the pending entry
            }
        }
        const bool repeat = in && miss && !newf;
        if (ballot(repeat)) {
            wave_sync();
            const uint32_t rslot = (uint32_t)__shfl((int)myslot, (int)rep);
            if (repeat) atomicAdd(&cnt[rslot], 1u);
        }
        if (vv && vr < r) mark[vs] = 0;

        const uint64_t inmask = (p >= kWave) ? ~0ull : ((1ull << p) - 1ull);
        const uint32_t rp = popc64(newmask & inmask);
        if (!full) {
            size += rp;
            if (size == k) {
                full = 1;
                list_len = 0;
                list_ptr = 0;
                more = 0;
            }
        } else if (rp > 0) {
            const uint64_t lastm = ballot(vv && vr == rp - 1);
            list_ptr += (uint32_t)__builtin_ctzll(lastm) + 1u;
        }
        pos += p;
        wave_sync();
    }

    // write the summary and its minimum (0 while fewer than k counters are used)
    wave_sync();
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

uint32_t chunk_summary_lds_bytes(uint32_t k) {
    ChunkLayout L = ChunkLayout::make(k);
    return L.tsize <= 65536 ? L.bytes : 0xFFFFFFFFu;
}

}  // namespace pss
