// The block kernels' hash table of counters and their input staging, shared
// by the Space Saving and the Frequent block kernels.
//
// A counter is a slot of a multiple-choice hash table: its 64-bit entry
// holds the item id (low word) and the count (high word); count 0 marks an
// empty slot and the top 128 count values are tags a window uses for
// victims and claims.  An item lives in one of the 8-slot buckets its two
// (or three) hash functions pick, or in a 64-slot stash after them when they
// are all full.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "pss_device.h"
#include "pss_layout.h"

namespace pss {

// Table entry: key | tag << 32 with tag 0 = empty, 1 .. kTagVict - 1 = a
// counter and its count; during a window, kTagVict + j = the counter of
// count m that the window's j-th new item would evict, kTagPend + lane =
// claimed by a lane (so a block holds fewer than kTagVict items).
constexpr uint32_t kTagEmpty = 0u;
constexpr uint32_t kTagVict = 0xFFFFFF80u;
constexpr uint32_t kTagPend = 0xFFFFFFC0u;
static_assert(kTagVict == kStreamBound, "every count of a block stays below the window tags");
constexpr uint32_t kNone = 0xFFFFFFFFu;
// Block summary size written when a loop bound that the algorithm guarantees
// is exceeded (an internal invariant failed): the host reports a device error
// instead of the kernel spinning.
constexpr uint32_t kBlockFailed = 0xFFFFFFFFu;

__device__ __forceinline__ uint64_t make_entry(uint32_t key, uint32_t tag) {
    return ((uint64_t)tag << 32) | key;
}

// The hash functions of one attempt at a block.  The table only indexes the
// counters, so every choice of multipliers gives the same summary; the first
// attempt uses fixed ones, and a block whose items overflow a bucket pair
// and the stash under them (possible for ids chosen to collide) is run again
// from its start with other odd multipliers (SplitMix64 of the attempt).
struct HashKeys {
    uint32_t h1, h2, h3, pick, h4;
};

constexpr uint32_t kHashAttempts = 4;

__device__ __forceinline__ HashKeys hash_keys(uint32_t attempt) {
    if (attempt == 0) return HashKeys{0x9E3779B1u, 0x85EBCA77u, 0xC2B2AE3Du, 0x2C1B3C6Du, 0x27D4EB2Fu};
    uint64_t z = (uint64_t)attempt * 0x9E3779B97F4A7C15ull;
    uint64_t a = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    a = (a ^ (a >> 27)) * 0x94D049BB133111EBull;
    a ^= a >> 31;
    uint64_t b = (a + 0x9E3779B97F4A7C15ull) * 0xBF58476D1CE4E5B9ull;
    b = (b ^ (b >> 27)) * 0x94D049BB133111EBull;
    b ^= b >> 31;
    uint64_t c = (b + 0x9E3779B97F4A7C15ull) * 0xBF58476D1CE4E5B9ull;
    c = (c ^ (c >> 27)) * 0x94D049BB133111EBull;
    c ^= c >> 31;
    return HashKeys{(uint32_t)a | 1u, (uint32_t)(a >> 32) | 1u, (uint32_t)b | 1u, (uint32_t)(b >> 32) | 1u,
                    (uint32_t)c | 1u};
}

// The two buckets of an item: multiplicative hashes scaled to nb buckets;
// the second is moved to the neighbour of the first when they coincide.
__device__ __forceinline__ uint32_t home_bucket(uint32_t x, uint32_t nb, const HashKeys& hk) {
    return (uint32_t)(((uint64_t)(x * hk.h1) * nb) >> 32);
}

__device__ __forceinline__ uint32_t alt_bucket(uint32_t x, uint32_t nb, uint32_t b1, const HashKeys& hk) {
    uint32_t h = x * hk.h2;
    h = (h << 15) | (h >> 17);
    const uint32_t b2 = (uint32_t)(((uint64_t)(h * hk.h3) * nb) >> 32);
    return b2 != b1 ? b2 : (b1 + 1 == nb ? 0u : b1 + 1);
}

// The third bucket of a three-choice table: a third multiplicative hash,
// stepped past the first two buckets when it meets one of them (nb >= 3).
__device__ __forceinline__ uint32_t third_bucket(uint32_t x, uint32_t nb, uint32_t b1, uint32_t b2,
                                                 const HashKeys& hk) {
    uint32_t h = x * hk.h4;
    h = (h << 9) | (h >> 23);
    uint32_t b = (uint32_t)(((uint64_t)(h * hk.h3) * nb) >> 32);
    b = (b == b1 || b == b2) ? (b + 1 == nb ? 0u : b + 1) : b;
    b = (b == b1 || b == b2) ? (b + 1 == nb ? 0u : b + 1) : b;
    return b;
}

__device__ __forceinline__ bool live_tag(uint32_t tag) { return tag - 1u < kTagVict - 1u; }

// Keys of empty bucket slots.  A lookup compares an item only with the keys
// of its own buckets, so an empty slot of bucket b may hold any id whose
// buckets all differ from b: no lookup that reads bucket b can match it,
// and lookups need not test count words.  Id 0 has buckets 0 and 1 (and 2
// with three choices) under any multipliers (0 times anything is 0, and a
// later bucket equal to an earlier one steps to the next), so empty slots of
// every other bucket hold 0, and those of the first NCH buckets hold an id
// e1 whose buckets are none of them.  (Stash slots are compared only while
// live; they keep 0.)
//
// e1 for nb buckets under hk, or 0 when none was found among the first ids
// (the caller then treats the hash functions as unusable).
template <int NCH>
__device__ __forceinline__ uint32_t empty_key_e1(uint32_t nb, const HashKeys& hk) {
    for (uint32_t e1 = 1u; e1 < 1024u; ++e1) {
        const uint32_t c = home_bucket(e1, nb, hk), d = alt_bucket(e1, nb, c, hk);
        bool ok = c >= (uint32_t)NCH && d >= (uint32_t)NCH;
        if constexpr (NCH == 3) ok = ok && third_bucket(e1, nb, c, d, hk) >= 3u;
        if (ok) return e1;
    }
    return 0u;
}

// The entry of an empty slot s.
template <int NCH>
__device__ __forceinline__ uint64_t empty_entry(uint32_t e1, uint32_t s) {
    return s < (uint32_t)NCH * kBucketSlots ? (uint64_t)e1 : 0ull;
}

// One bucket: kBucketSlots key/tag pairs, read with kBucketSlots / 2
// 16-byte loads.
constexpr int kBucketQuads = (int)kBucketSlots / 2;
static_assert(kBucketQuads == 4, "the quad rotation below assumes four 16-byte loads per bucket");

// A bucket as one lane read it.  Buckets are 64 bytes, so with every lane
// reading its quads in the same order the four loads of a wave would fall on
// a quarter of the LDS banks; lane l reads its quads starting at l mod 4
// instead, which spreads each load over all of them.  q[j] holds slots
// 2r and 2r + 1 with r = (j + rot) mod 4.
struct Bucket {
    uint4 q[kBucketQuads];
    uint32_t rot;
};

__device__ __forceinline__ Bucket load_bucket(const uint4* tbl4, uint32_t b) {
    Bucket r;
    r.rot = __lane_id() & (uint32_t)(kBucketQuads - 1);
#pragma unroll
    for (int i = 0; i < kBucketQuads; ++i)
        r.q[i] = tbl4[kBucketQuads * b + (((uint32_t)i + r.rot) & (uint32_t)(kBucketQuads - 1))];
    return r;
}

// Slot order from load order: a left rotation of the 8-bit mask by 2 rot.
__device__ __forceinline__ uint32_t unrotate_mask(uint32_t m, uint32_t rot) {
    const uint32_t sh = 2u * rot;
    return ((m << sh) | (m >> (kBucketSlots - sh))) & ((1u << kBucketSlots) - 1u);
}

// Slot masks (bit i = slot i of the bucket).  At a window's lookups a bucket
// slot holds a counter or is empty with a key no lookup of that bucket can
// match (empty_entry), so a matching key is a counter of the item.
__device__ __forceinline__ uint32_t match_mask(const Bucket& B, uint32_t x) {
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < kBucketQuads; ++i) {
        m |= (B.q[i].x == x ? 1u : 0u) << (2 * i);
        m |= (B.q[i].z == x ? 1u : 0u) << (2 * i + 1);
    }
    return unrotate_mask(m, B.rot);
}

__device__ __forceinline__ uint32_t empty_mask(const Bucket& B) {
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < kBucketQuads; ++i) {
        m |= (B.q[i].y == kTagEmpty ? 1u : 0u) << (2 * i);
        m |= (B.q[i].w == kTagEmpty ? 1u : 0u) << (2 * i + 1);
    }
    return unrotate_mask(m, B.rot);
}

// The free slot an item claims in a bucket with free-slot mask e (nonzero):
// the (h mod popcount(e))-th free slot for a hash h of the item, so that
// equal items pick the same slot and different items spread over the free
// ones.
__device__ __forceinline__ uint32_t pick_free(uint32_t e, uint32_t x, uint32_t mult) {
    static_assert(kBucketSlots == 8, "the rank search below covers 8 slots");
    const uint32_t n = (uint32_t)__builtin_popcount(e);
    uint32_t r = (((x * mult) >> 16) * n) >> 16;  // in [0, n)
    // the r-th set bit: halve the window three times by popcounts
    uint32_t base = 0;
    uint32_t c = (uint32_t)__builtin_popcount(e & 0xFu);
    bool up = r >= c;
    base = up ? 4u : 0u;
    r = up ? r - c : r;
    e = up ? e >> 4 : e;
    c = (uint32_t)__builtin_popcount(e & 0x3u);
    up = r >= c;
    base += up ? 2u : 0u;
    r = up ? r - c : r;
    e = up ? e >> 2 : e;
    return base + ((r >= (e & 1u)) ? 1u : 0u);
}

// The slot a missing item claims: a free slot of the emptiest of its
// buckets (the earliest on ties), chosen by pick_free; kNone when all are
// full.  Two choices: e3 = 0.
__device__ __forceinline__ uint32_t claim_slot(uint32_t e1, uint32_t e2, uint32_t e3, uint32_t b1, uint32_t b2,
                                               uint32_t b3, uint32_t x, uint32_t mult) {
    const uint32_t n1 = __builtin_popcount(e1), n2 = __builtin_popcount(e2), n3 = __builtin_popcount(e3);
    const bool first = n1 >= n2;
    uint32_t e = first ? e1 : e2, b = first ? b1 : b2;
    const bool third = n3 > (first ? n1 : n2);
    e = third ? e3 : e;
    b = third ? b3 : b;
    return e ? kBucketSlots * b + pick_free(e, x, mult) : kNone;
}



// ---------------------------------------------------------------------------
// Input staging
// ---------------------------------------------------------------------------

// Four consecutive items at idx (a multiple of 4), zero at and beyond stop.
// The input is read once: loads are marked non-temporal so that the stream
// does not push the blocks' error scratch out of the L2.
#ifndef PSS_INPUT_TEMPORAL
#define PSS_NT_LOAD(p) __builtin_nontemporal_load(p)
#else
#define PSS_NT_LOAD(p) (*(p))
#endif
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint4 load4(const uint32_t* __restrict__ items, uint64_t idx, uint64_t n, uint64_t stop,
                                       int vec_ok) {
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (idx >= stop) return v;
    if (vec_ok && idx + 3 < n) {
        const u32x4_t t = PSS_NT_LOAD((const u32x4_t*)(items + idx));
        v = make_uint4(t[0], t[1], t[2], t[3]);
    } else {
        if (idx < n) v.x = PSS_NT_LOAD(items + idx);
        if (idx + 1 < n) v.y = PSS_NT_LOAD(items + idx + 1);
        if (idx + 2 < n) v.z = PSS_NT_LOAD(items + idx + 2);
        if (idx + 3 < n) v.w = PSS_NT_LOAD(items + idx + 3);
    }
    return v;
}

// Two consecutive items at idx (even), zero at and beyond stop.
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint2 load2(const uint32_t* __restrict__ items, uint64_t idx, uint64_t n, uint64_t stop,
                                       int vec_ok) {
    uint2 v = make_uint2(0u, 0u);
    if (idx >= stop) return v;
    if (vec_ok && idx + 1 < n) {
        const u32x2_t t = PSS_NT_LOAD((const u32x2_t*)(items + idx));
        v = make_uint2(t[0], t[1]);
    } else {
        if (idx < n) v.x = PSS_NT_LOAD(items + idx);
        if (idx + 1 < n) v.y = PSS_NT_LOAD(items + idx + 1);
    }
    return v;
}

// One half of the ring: kRingHalf items, kRingPerLane per lane (one 8- or
// 16-byte load).
constexpr uint32_t kRingPerLane = kRingHalf / kWave;
static_assert(kRingPerLane == 2 || kRingPerLane == 4, "one uint2 or uint4 per lane per ring half");
struct Prefetch {
    typename std::conditional<kRingPerLane == 4, uint4, uint2>::type a;
};

__device__ __forceinline__ void load_lane(uint4& a, const uint32_t* __restrict__ items, uint64_t tile, uint64_t n,
                                          uint64_t stop, int vec_ok, uint32_t lane) {
    a = load4(items, tile + 4 * lane, n, stop, vec_ok);
}

__device__ __forceinline__ void load_lane(uint2& a, const uint32_t* __restrict__ items, uint64_t tile, uint64_t n,
                                          uint64_t stop, int vec_ok, uint32_t lane) {
    a = load2(items, tile + 2 * lane, n, stop, vec_ok);
}

__device__ __forceinline__ void load_lane_whole(uint4& a, const uint32_t* __restrict__ items, uint64_t tile,
                                                uint32_t lane) {
    const u32x4_t t = PSS_NT_LOAD((const u32x4_t*)(items + tile) + lane);
    a = make_uint4(t[0], t[1], t[2], t[3]);
}

__device__ __forceinline__ void load_lane_whole(uint2& a, const uint32_t* __restrict__ items, uint64_t tile,
                                                uint32_t lane) {
    const u32x2_t t = PSS_NT_LOAD((const u32x2_t*)(items + tile) + lane);
    a = make_uint2(t[0], t[1]);
}

__device__ __forceinline__ Prefetch fetch_half(const uint32_t* __restrict__ items, uint64_t tile, uint64_t n,
                                               uint64_t stop, int vec_ok, uint32_t lane) {
    Prefetch p;
    if (vec_ok && tile + kRingHalf <= stop) {
        // the whole half is in the block (stop <= n): one load per lane, no
        // per-lane bounds (a wave-uniform test)
        load_lane_whole(p.a, items, tile, lane);
    } else {
        load_lane(p.a, items, tile, n, stop, vec_ok, lane);
    }
    return p;
}

__device__ __forceinline__ void store_half(uint32_t* ring, uint64_t tile, const Prefetch& p, uint32_t lane) {
    uint32_t base = (uint32_t)tile & (kRing - 1);
    *(decltype(p.a)*)(ring + base + kRingPerLane * lane) = p.a;
}

}  // namespace pss
