// The Frequent (Misra-Gries) summary that Section 2 of the paper names as
// the counter-based method the authors merged in parallel before Space
// Saving, in the same pipeline: Algorithm 1's blocks, one wave per block
// reproducing the sequential summary exactly, a fixed binary tree of merges,
// and a report.
//
// Frequent for the k-majority problem keeps k - 1 counters: a monitored item
// adds 1; an unmonitored item takes a free counter with count 1, or, when all
// are used, every counter loses 1 (those reaching 0 are freed) and the item
// is dropped.  D counts those decrement steps (f - D <= f^ <= f).  The merge
// is the mergeable-summaries combine: add the counts of the union; beyond
// k - 1 items subtract the k-th largest count c and keep the positive ones;
// D adds up, plus c.  The report keeps the items with (f^ + D) * k > n.
//
// The block kernel reads its block in windows of up to 64 items, one per
// lane, looked up against the counters at window start (the Space Saving
// kernel's multiple-choice table).  Hits commute.  New items (first occurrences
// of unmonitored values) take free counters in window order; the first new
// item beyond the free counters is a decrement step, so the wave applies the
// window up to it, decrements every counter (one pass over the table, at
// most n / k times per block), drops that item and starts the next window
// after it.
#include "pss_device.h"
#include "pss_kernels.h"
#include "pss_layout.h"
#include "pss_table.h"

namespace pss {

namespace {

extern __shared__ __align__(16) unsigned char smem[];

// Sequential Frequent over items[begin, end) by one wave, k - 1 counters in
// the hash table at `tbl` (LDS), NCH buckets per item.  Returns kOverflow
// when a new item found no free slot under the hash functions hk (nothing
// written), else writes the summary (entries, size, D) and returns kDone.
constexpr uint32_t kFqDone = 0, kFqOverflow = 1;

template <int NCH>
__device__ __forceinline__ uint32_t frequent_block(const uint32_t* __restrict__ items, uint64_t n, uint64_t begin,
                                                   uint64_t end, const FreqLayout& L, int vec_ok,
                                                   unsigned char* lds, uint32_t* __restrict__ o_item,
                                                   uint32_t* __restrict__ o_cnt, uint32_t* __restrict__ o_err,
                                                   uint32_t* __restrict__ o_size, uint32_t* __restrict__ o_dec,
                                                   const HashKeys hk) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t K1 = L.counters;
    const uint32_t T = L.tsize;
    const uint32_t S = L.slots;
    const uint32_t NB = L.nbuckets;
    uint64_t* table = (uint64_t*)(lds + L.off_table);
    uint32_t* words = (uint32_t*)(lds + L.off_table);  // count of slot s: words[2 s + 1]
    const uint4* tbl4 = (const uint4*)(lds + L.off_table);
    const uint4* stash4 = tbl4 + T / 2;
    uint32_t* ring = (uint32_t*)(lds + L.off_ring);

    // the item's third bucket, or none (its mask stays 0)
    auto bucket3 = [&](uint32_t y, uint32_t c1, uint32_t c2) -> uint32_t {
        if constexpr (NCH == 3) return third_bucket(y, NB, c1, c2, hk);
        return 0u;
    };
    const uint32_t ekey = uniform(empty_key_e1<NCH>(NB, hk));  // key of empty slots in the first NCH buckets
    if (ekey == 0u) return kFqOverflow;  // unusable hash functions: the caller tries others
    for (uint32_t i = lane; i < S; i += kWave) table[i] = empty_entry<NCH>(ekey, i);

    // wave-uniform state (readfirstlane-anchored, see the Space Saving kernel)
    uint32_t size = 0, dec = 0, failed = 0, stash_live = 0;

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
    uint32_t xn = ring[(uint32_t)(pos + lane) & (kRing - 1)];
    while (pos < end && !failed) {
        if (pos >= rbase + kRingHalf) {
            store_half(ring, rbase + kRing, pf, lane);
            rbase += kRingHalf;
            pf = fetch_half(items, rbase + kRing, n, end, vec_ok, lane);
            wave_sync();
        }
        // the stash, lane i holding slot T + i; its entries go back to a
        // bucket with room whenever one has some
        uint32_t skey = 0;
        bool slive = false;
        if (stash_live) {
            const uint64_t e = table[T + lane];
            skey = (uint32_t)e;
            slive = live_tag((uint32_t)(e >> 32));
            if (ballot(slive)) {
                const uint32_t s1 = home_bucket(skey, NB, hk), s2 = alt_bucket(skey, NB, s1, hk);
                const uint32_t s3 = bucket3(skey, s1, s2);
                const Bucket B1 = load_bucket(tbl4, s1), B2 = load_bucket(tbl4, s2);
                const uint32_t e1 = empty_mask(B1), e2 = empty_mask(B2);
                uint32_t e3 = 0u;
                if constexpr (NCH == 3) e3 = empty_mask(load_bucket(tbl4, s3));
                bool moved = false;
                if (slive && (e1 | e2 | e3)) {
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

        // 1. look up against the counters at window start
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
        for (uint64_t sm = ballot(slive); sm; sm &= sm - 1) {
            const uint32_t j = (uint32_t)__builtin_ctzll(sm);
            if (x == (uint32_t)__builtin_amdgcn_readlane((int)skey, (int)j)) {
                hit = valid;
                slot = T + j;
            }
        }
        miss = valid && !hit;
        if (ballot(miss) == 0) {  // all hits: increments commute
            pos += wl;
            xn = ring[(uint32_t)(pos + lane) & (kRing - 1)];
            if (hit) atomicAdd(&words[2 * slot + 1], 1u);
            continue;
        }

        // 2. group unmonitored items by value: each claims a free slot of its
        //    emptier bucket (else of the stash) with a compare-and-swap; a
        //    lost swap to the same value joins that claim (lowest lane wins),
        //    a lost swap to another value removes the slot from the view
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
                if (h == kNone) {
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
        }
        if (ballot(bad)) {
            failed = ballot(nofree) ? 2u : 1u;
            continue;
        }
        wave_sync();

        // 3. new items (the lowest lane of each claimed value) in window
        //    order; the one beyond the free counters is a decrement step
        const uint32_t rep = miss ? (lds_reread(words + 2 * hp + 1) - kTagPend) : lane;
        const uint64_t newmask = ballot(miss && rep == lane);
        const bool newf = (newmask >> lane) & 1ull;
        const uint32_t nrank = mbcnt(newmask);
        const uint32_t freec = K1 - size;
        const bool trig = newf && nrank == freec;
        const uint64_t tmask = ballot(trig);
        const uint32_t p = tmask ? (uint32_t)__builtin_ctzll(tmask) : wl;  // items applied
        const bool in = lane < p;

        // 4. apply the prefix: hits add 1, new items take their claimed slots
        //    with count 1, repeats add 1 to their value's new counter; claims
        //    past the prefix (the dropped item's among them) are released
        if (in && hit) atomicAdd(&words[2 * slot + 1], 1u);
        if (newf) table[hp] = in ? make_entry(x, 1u) : empty_entry<NCH>(ekey, hp);
        const bool repeat = in && miss && !newf;
        if (ballot(repeat)) {
            wave_sync();
            const uint32_t rslot = (uint32_t)__shfl((int)hp, (int)rep);
            if (repeat) atomicAdd(&words[2 * rslot + 1], 1u);
        }
        const uint64_t inmask = (p >= kWave) ? ~0ull : ((1ull << p) - 1ull);
        size = uniform(size + popc64(newmask & inmask));
        stash_live = uniform(stash_live + popc64(ballot(newf && in && hp >= T)));
        wave_sync();

        if (tmask) {
            // 5. decrement step: every counter loses 1, those at 0 are freed;
            //    the item at p is dropped
            uint32_t freed = 0, sfreed = 0;
            for (uint32_t b = 0; b < S; b += 4 * kWave) {
                uint32_t cv[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t s = b + j * kWave + lane;
                    cv[j] = s < S ? words[2 * s + 1] : 0u;
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t s = b + j * kWave + lane;
                    if (live_tag(cv[j])) {
                        if (cv[j] == 1u) {
                            table[s] = empty_entry<NCH>(ekey, s);
                            freed += 1;
                            sfreed += s >= T ? 1u : 0u;
                        } else {
                            words[2 * s + 1] = cv[j] - 1u;
                        }
                    }
                }
            }
            size = uniform(size - wave_add_u32(freed));
            stash_live = uniform(stash_live - wave_add_u32(sfreed));
            dec = uniform(dec + 1u);
            pos += p + 1;
        } else {
            pos += wl;
        }
        xn = ring[(uint32_t)(pos + lane) & (kRing - 1)];
        wave_sync();
    }

    wave_sync();
    if (failed == 2) return kFqOverflow;
    if (failed) {
        if (lane == 0) {
            *o_size = kBlockFailed;
            *o_dec = 0;
        }
        return kFqDone;
    }
    uint32_t outn = 0;
    for (uint32_t b = 0; b < S; b += kWave) {
        const uint32_t s = b + lane;
        const uint64_t e = s < S ? table[s] : 0ull;
        const uint32_t c = (uint32_t)(e >> 32);
        const bool live = s < S && live_tag(c);
        const uint64_t bm = ballot(live);
        if (live) {
            const uint32_t o = outn + mbcnt(bm);
            o_item[o] = (uint32_t)e;
            o_cnt[o] = c;
            o_err[o] = 0u;
        }
        outn = uniform(outn + popc64(bm));
    }
    if (lane == 0) {
        *o_size = outn == size ? size : kBlockFailed;
        *o_dec = dec;
    }
    return kFqDone;
}

// One wave per block c of C (Algorithm 1's bounds, 64-bit products).
template <int NCH>
__global__ __launch_bounds__(64) void frequent_block_kernel(const uint32_t* __restrict__ items, uint64_t n,
                                                            uint32_t chunks, FreqLayout L, int vec_ok,
                                                            BlockSummaries out) {
    const uint32_t c = blockIdx.x;
    const uint64_t begin = (uint64_t)c * n / chunks;
    const uint64_t end = (uint64_t)(c + 1) * n / chunks;
    const uint64_t ob = (uint64_t)c * L.k;
    for (uint32_t attempt = 0; attempt < kHashAttempts; ++attempt) {
        if (frequent_block<NCH>(items, n, begin, end, L, vec_ok, smem, out.item + ob, out.cnt + ob, out.err + ob,
                           out.size + c, out.min + c, hash_keys(attempt)) == kFqDone)
            return;
        wave_sync();
    }
    if (lane_id() == 0) {
        out.size[c] = kBlockFailed;
        out.min[c] = 0;
    }
}

// ---------------------------------------------------------------------------
// Merge: S_C = union with added counts; beyond k - 1 items subtract the
// k-th largest count c; D = D1 + D2 + c.  One workgroup per pair.
// ---------------------------------------------------------------------------

// 256 threads per pair where many pairs share the chip, 1024 on levels of at
// most 512 pairs, where few pairs leave CUs idle.
constexpr uint32_t kMergeThreads = 256;
constexpr uint32_t kMergeThreadsWide = 1024;
constexpr uint32_t kMergeWidePairs = 512;

struct FqMergeLds {
    uint32_t cap, hsize;
    uint32_t off_cc, off_ci, off_flag, off_hash, off_hist, off_misc, bytes;
    __host__ __device__ static FqMergeLds make(uint32_t k) {
        FqMergeLds L;
        L.cap = 2 * k;
        L.hsize = next_pow2(2 * k);
        if (L.hsize < 64) L.hsize = 64;
        uint32_t o = 0;
        L.off_cc = o;   o = align16(o + 4 * L.cap);
        L.off_ci = o;   o = align16(o + 4 * L.cap);
        L.off_flag = o; o = align16(o + L.cap);
        L.off_hash = o; o = align16(o + 4 * L.hsize);
        L.off_hist = o; o = align16(o + 2 * 4 * 256);  // two select histograms, used in turn
        L.off_misc = o; o = align16(o + 64);
        L.bytes = o;
        return L;
    }
};

template <uint32_t NT>
__device__ void frequent_merge_node(const uint32_t* i1, const uint32_t* c1, uint32_t n1, uint32_t d1,
                                    const uint32_t* i2, const uint32_t* c2, uint32_t n2, uint32_t d2, uint32_t k,
                                    uint32_t* io, uint32_t* co, uint32_t* eo, uint32_t* osize, uint32_t* odec) {
    const FqMergeLds L = FqMergeLds::make(k);
    uint32_t* cc = (uint32_t*)(smem + L.off_cc);
    uint32_t* ci = (uint32_t*)(smem + L.off_ci);
    uint8_t* flag = (uint8_t*)(smem + L.off_flag);
    uint32_t* hash = (uint32_t*)(smem + L.off_hash);
    uint32_t* hist = (uint32_t*)(smem + L.off_hist);
    uint32_t* misc = (uint32_t*)(smem + L.off_misc);
    const uint32_t tid = threadIdx.x;
    const uint32_t hbits = log2_pow2(L.hsize);
    const uint32_t hmask = L.hsize - 1;
    const uint32_t K1 = k - 1;
    if (n1 > K1 || n2 > K1) {  // an input carries a block's failure mark
        if (tid == 0) {
            *osize = kBlockFailed;
            *odec = 0;
        }
        return;
    }
    const uint32_t nc = n1 + n2;
    for (uint32_t j = tid; j < n2; j += NT) {
        ci[n1 + j] = i2[j];
        cc[n1 + j] = c2[j];
        flag[n1 + j] = 1;
    }
    for (uint32_t h = tid; h < L.hsize; h += NT) hash[h] = 0u;
    __syncthreads();
    for (uint32_t j = tid; j < n2; j += NT) {
        uint32_t h = hash_slot(ci[n1 + j], hbits);
        while (atomicCAS(&hash[h], 0u, j + 1u) != 0u) h = (h + 1) & hmask;
    }
    __syncthreads();
    for (uint32_t i = tid; i < n1; i += NT) {
        const uint32_t x = i1[i];
        uint32_t h = hash_slot(x, hbits);
        uint32_t c = c1[i];
        for (;;) {
            const uint32_t v = hash[h];
            if (v == 0u) break;
            if (ci[n1 + v - 1] == x) {
                c += cc[n1 + v - 1];
                flag[n1 + v - 1] = 0;
                break;
            }
            h = (h + 1) & hmask;
        }
        ci[i] = x;
        cc[i] = c;
        flag[i] = 1;
    }
    if (tid < 8) misc[tid] = tid == 5 ? ~0u : 0u;
    __syncthreads();
    // distinct candidates, and the OR and AND of their inverted counts (a
    // byte on which all agree selects nothing)
    uint32_t live = 0, ov = 0u, av = ~0u;
    for (uint32_t i = tid; i < nc; i += NT) {
        if (flag[i]) {
            live += 1;
            ov |= ~cc[i];
            av &= ~cc[i];
        }
    }
    live = wave_sum_u32(live);
    ov = wave_or_u32(ov);
    av = wave_and_u32(av);
    if (lane_id() == 0) {
        atomicAdd(&misc[0], live);
        atomicOr(&misc[4], ov);
        atomicAnd(&misc[5], av);
    }
    __syncthreads();
    const uint32_t ns = misc[0];
    const uint32_t differ = misc[4] ^ misc[5], common = ~misc[5];
    __syncthreads();

    // the k-th largest count (rank K1 from the top), by an MSD radix select
    // over the bytes of ~count where the candidates differ; candidates still
    // in the running carry flag bit 2.  Each pass filters by its byte and
    // counts the next one in the other histogram; the select stops once the
    // bin holding the k-th count holds nothing else.
    uint32_t cut = 0;
    if (ns > K1) {
        uint32_t vary = 0;
        for (uint32_t p = 0; p < 4; ++p) vary |= ((differ >> (8u * (3u - p))) & 255u ? 1u : 0u) << p;
        if (vary == 0u) {
            cut = common;  // every candidate has this count
        } else {
            uint32_t p = (uint32_t)__builtin_ctz(vary);
            uint32_t* hcur = hist;
            uint32_t* hnext = hist + 256;
            static_assert(NT >= 256, "a histogram bin per thread of the first 256");
            if (tid < 256) {
                hcur[tid] = 0u;
                hnext[tid] = 0u;
            }
            for (uint32_t i = tid; i < nc; i += NT) flag[i] = flag[i] ? 3 : 0;
            __syncthreads();
            for (uint32_t i = tid; i < nc; i += NT)
                if (flag[i] & 2) atomicAdd(&hcur[((~cc[i]) >> (8u * (3u - p))) & 255u], 1u);
            __syncthreads();
            uint32_t rank = K1;
            for (;;) {
                if (tid < kWave) {
                    const uint32_t b0 = hcur[4 * tid], b1 = hcur[4 * tid + 1], b2 = hcur[4 * tid + 2],
                                   b3 = hcur[4 * tid + 3];
                    const uint32_t s = b0 + b1 + b2 + b3;
                    uint32_t incl = s;
                    for (int off = 1; off < 64; off <<= 1) {
                        const uint32_t t = (uint32_t)__shfl_up((int)incl, off);
                        if ((int)tid >= off) incl += t;
                    }
                    const uint32_t excl = incl - s;
                    if (excl <= rank && rank < incl) {
                        uint32_t rr = rank - excl, bin = 4 * tid;
                        if (rr >= b0) { rr -= b0; ++bin;
                            if (rr >= b1) { rr -= b1; ++bin;
                                if (rr >= b2) { rr -= b2; ++bin; } } }
                        misc[1] = bin;
                        misc[2] = rr;
                        misc[6] = hcur[bin];
                    }
                }
                __syncthreads();
                const uint32_t sel = misc[1];
                rank = misc[2];
                const bool alone = misc[6] == 1u;
                vary &= ~((2u << p) - 1u);  // bytes after p
                const bool last = alone || vary == 0u;
                const uint32_t pn = last ? p : (uint32_t)__builtin_ctz(vary);
                if (tid < 256) hcur[tid] = 0u;  // read by the scan only: free for the pass after next
                for (uint32_t i = tid; i < nc; i += NT) {
                    if (flag[i] & 2) {
                        const uint32_t v = ~cc[i];
                        if (((v >> (8u * (3u - p))) & 255u) != sel)
                            flag[i] &= 1;
                        else if (!last)
                            atomicAdd(&hnext[(v >> (8u * (3u - pn))) & 255u], 1u);
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
                if (flag[i] & 2) misc[3] = cc[i];  // every candidate left has that count
            __syncthreads();
            cut = misc[3];
        }
    }
    // keep the counts above the cut, lowered by it, in candidate order: rows
    // of NT candidates, up to 32 rows per segment, each wave's kept count per
    // row in a table over the histograms
    constexpr uint32_t kWaves = NT / kWave;
    constexpr uint32_t kRows = 32;
    static_assert(kRows * kWaves <= 2 * 256, "the count table lies over the histograms");
    uint32_t* rowcnt = hist;
    const uint32_t w = tid / kWave;
    uint32_t kept = 0;
    __syncthreads();  // the select's last reads of the histograms are done
    for (uint32_t seg = 0; seg < nc; seg += kRows * NT) {
        const uint32_t rows = min(kRows, (nc - seg + NT - 1) / NT);
        uint32_t keepbits = 0;
        for (uint32_t q = 0; q < rows; ++q) {
            const uint32_t i = seg + q * NT + tid;
            const bool keep = i < nc && (flag[i] & 1) && cc[i] > cut;
            const uint64_t bm = ballot(keep);
            if (lane_id() == 0) rowcnt[kWaves * q + w] = popc64(bm);
            keepbits |= (keep ? 1u : 0u) << q;
        }
        __syncthreads();
        for (uint32_t q = 0; q < rows; ++q) {
            const bool keep = (keepbits >> q) & 1u;
            const uint64_t bm = ballot(keep);
            uint32_t before = kept;
            for (uint32_t u = 0; u < w; ++u) before += rowcnt[kWaves * q + u];
            if (keep) {
                const uint32_t i = seg + q * NT + tid;
                const uint32_t o = before + mbcnt(bm);
                io[o] = ci[i];
                co[o] = cc[i] - cut;
                eo[o] = 0u;
            }
            for (uint32_t u = 0; u < kWaves; ++u) kept += rowcnt[kWaves * q + u];
        }
        __syncthreads();  // the table is read before the next segment rewrites it
    }
    if (tid == 0) {
        *osize = kept;
        *odec = d1 + d2 + cut;
    }
}

template <uint32_t NT>
__global__ __launch_bounds__(NT) void frequent_level_kernel(BlockSummaries v, uint32_t k, uint32_t step) {
    const uint64_t a = 2ull * step * blockIdx.x;
    const uint64_t b = a + step;
    frequent_merge_node<NT>(v.item + a * k, v.cnt + a * k, v.size[a], v.min[a], v.item + b * k, v.cnt + b * k, v.size[b],
                        v.min[b], k, v.item + a * k, v.cnt + a * k, v.err + a * k, &v.size[a], &v.min[a]);
}

}  // namespace

uint32_t frequent_merge_lds_bytes(uint32_t k) { return FqMergeLds::make(k).bytes; }

hipError_t launch_frequent_blocks(const uint32_t* d_items, uint64_t n, uint32_t chunks, const FreqLayout& L,
                                  const BlockSummaries& out, hipStream_t stream) {
    (void)hipGetLastError();  // a stale error of an earlier, unrelated call is not this launch's
    const int vec_ok = ((uintptr_t)d_items & 15u) == 0;
    auto launch = [&](auto kern) {
        hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds_bytes);
        hipLaunchKernelGGL(kern, dim3(chunks), dim3(64), L.lds_bytes, stream, d_items, n, chunks, L, vec_ok, out);
    };
    if (L.choices == 3)
        launch(frequent_block_kernel<3>);
    else if (L.choices == 2)
        launch(frequent_block_kernel<2>);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_frequent_level(const BlockSummaries& v, uint32_t k, uint32_t count, uint32_t step,
                                 hipStream_t stream) {
    (void)hipGetLastError();
    if (step >= count) return hipSuccess;
    const uint32_t pairs = (uint32_t)(((uint64_t)count - step + 2ull * step - 1) / (2ull * step));
    const uint32_t lds = FqMergeLds::make(k).bytes;
    auto launch = [&](auto kern, uint32_t nt) {
        hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, dim3(pairs), dim3(nt), lds, stream, v, k, step);
    };
    if (pairs <= kMergeWidePairs)
        launch(frequent_level_kernel<kMergeThreadsWide>, kMergeThreadsWide);
    else
        launch(frequent_level_kernel<kMergeThreads>, kMergeThreads);
    return hipGetLastError();
}

}  // namespace pss
