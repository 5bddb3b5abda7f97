// Memory layout of one block summary, shared by the host launcher and the
// chunk_summary kernel.  One wave owns one layout.  The per-block state (hash
// table, counts, minimum-level list) lives in LDS when it fits, otherwise in
// a global-memory slab of state_bytes per block; the input ring and a few
// small per-window arrays always live in LDS.  A counter is a hash-table
// slot: its entry holds the item id and the count, so there is no separate
// counter array; errors go to a per-block scratch array in device memory
// (written at installs, read at the end).
#pragma once

#include <stdint.h>

#ifndef __HIPCC__
#define PSS_HD
#else
#define PSS_HD __host__ __device__
#endif

namespace pss {

// Items staged per half of the LDS input ring (two halves): two per lane,
// which keeps a window (at most 64 items from a position in the first half)
// inside the ring.
#ifndef PSS_RING_HALF
#define PSS_RING_HALF 128
#endif
constexpr uint32_t kRingHalf = PSS_RING_HALF;
constexpr uint32_t kRing = 2 * kRingHalf;
static_assert(kRingHalf == 128 || kRingHalf == 256, "two or four items per lane");
// LDS is given to workgroups in units of this many bytes on MI355X (gfx950):
// a CU of 160 KiB holds floor(163840 / (bytes rounded up to a unit))
// one-wave workgroups, measured with workgroups of every size used here
// (the runtime's occupancy query assumes finer units and overestimates).
constexpr uint32_t kLdsUnit = 1280;
PSS_HD inline uint32_t lds_waves(uint64_t lds_per_cu, uint32_t bytes) {
    const uint64_t alloc = (bytes + kLdsUnit - 1) / kLdsUnit * kLdsUnit;
    return (uint32_t)(lds_per_cu / (alloc ? alloc : kLdsUnit));
}
// Largest hash table whose slot positions fit uint16 (LDS-resident state).
constexpr uint32_t kMaxLdsTableSlots = 65536;
// Slots per hash bucket (key/tag pairs of 8 bytes).
#ifndef PSS_BUCKET_SLOTS
#define PSS_BUCKET_SLOTS 8
#endif
constexpr uint32_t kBucketSlots = PSS_BUCKET_SLOTS;
// Hash slots per counter x16: 1.875 per counter up to k = 1024, 1.625 above
// with two bucket choices, 1.3125 with three (a speed / memory trade that
// never changes results: at k = 500 and 2000 these are the largest tables
// with which 16 and 6 waves share a CU's LDS).
#ifndef PSS_SLOTS_X16
#define PSS_SLOTS_X16 26
#endif
#ifndef PSS_SLOTS_X16_SMALLK
#define PSS_SLOTS_X16_SMALLK 30
#endif
#ifndef PSS_SLOTS_X16_THREE
#define PSS_SLOTS_X16_THREE 21
#endif
// Overflow slots after the buckets, for items whose buckets are all full.
constexpr uint32_t kStash = 64;
// Streams hold fewer than kStreamBound items: a count word of a hash slot
// keeps its top 128 values for the victims and claims of a window.
constexpr uint64_t kStreamBound = (1ull << 32) - 128;
// The level sort's histogram: 257 words.
constexpr uint32_t kHistBytes = 4 * 257;
// A counter's count word may carry its error above the count: the count in
// the low kCountBits bits, the error (at most kPackedErrMax) above them, so
// that packed words stay below the window tags.
constexpr uint32_t kCountBits = 22;
constexpr uint32_t kCountMask = (1u << kCountBits) - 1u;
constexpr uint32_t kPackedErrMax = 1022;
static_assert((((uint64_t)kPackedErrMax << kCountBits) | kCountMask) < kStreamBound,
              "packed count words stay below the window tags");

PSS_HD inline uint32_t next_pow2(uint32_t v) {
    uint32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

PSS_HD inline uint32_t log2_pow2(uint32_t p) {
    uint32_t b = 0;
    while ((1u << b) < p) ++b;
    return b;
}

PSS_HD inline uint32_t align16(uint32_t v) { return (v + 15u) & ~15u; }

// Registers per lane the in-register level sort needs for k counters.
PSS_HD inline uint32_t sort_lanes_per_k(uint32_t k) {
    return next_pow2((k + 63) / 64);
}

// Buckets an item may live in: three for the LDS-state classes above
// k = 1024 (a fuller table, so that more waves fit a CU's LDS, at one more
// bucket read per lookup), two elsewhere.  The block kernels derive the same
// number from their register class.
PSS_HD inline uint32_t hash_choices(uint32_t k, bool global_state) {
    return !global_state && sort_lanes_per_k(k) >= 32 ? 3u : 2u;
}

struct ChunkLayout {
    uint32_t k;
    uint32_t nbuckets;      // hash buckets of kBucketSlots slots
    uint32_t tsize;         // kBucketSlots * nbuckets slots (the stash follows them)
    uint32_t slots;         // tsize + kStash: every slot can hold a counter
    uint32_t global_state;  // 1: state in global memory, 32-bit indices; 0: LDS, 16-bit indices
    // state offsets (bytes from the state base)
    uint32_t off_table, off_list, off_tkey, off_list2, off_tkey2;
    uint32_t state_bytes;
    // LDS offsets (bytes from the LDS base; the state comes first when it is in LDS)
    uint32_t off_ring, off_hist;
    uint32_t lds_bytes;
    // per-block error scratch in device memory: one error per slot, blocks
    // err_stride words apart (a multiple of 32: each block starts a cache
    // line); err_bytes per error (4, or 2 / 1 by with_error_width; 0: the
    // errors are packed in the count words and count_mask selects the count)
    uint32_t err_stride, err_bytes, count_mask;
    uint32_t choices;  // buckets per item (hash_choices)

    // Default hash slots per counter (x16) for tables with `choices` buckets
    // per item.
    PSS_HD static uint32_t default_slots_x16(uint32_t k, uint32_t choices) {
        return choices == 3 ? PSS_SLOTS_X16_THREE : k <= 1024 ? PSS_SLOTS_X16_SMALLK : PSS_SLOTS_X16;
    }

    // slots_per_counter_x16: hash slots per counter (x16), a speed / memory
    // knob that never changes results (0 = default).  global_state selects
    // where the per-block state lives.
    PSS_HD static ChunkLayout make(uint32_t k, bool global_state, uint32_t slots_per_counter_x16 = 0) {
        ChunkLayout L;
        L.k = k;
        L.global_state = global_state ? 1u : 0u;
        L.choices = hash_choices(k, global_state);
        if (slots_per_counter_x16 == 0) slots_per_counter_x16 = default_slots_x16(k, L.choices);
        uint32_t want = (uint32_t)(((uint64_t)k * slots_per_counter_x16 + 15) / 16);
        if (want < 256) want = 256;
        L.nbuckets = (want + kBucketSlots - 1) / kBucketSlots;
        L.tsize = kBucketSlots * L.nbuckets;
        L.slots = L.tsize + kStash;
        const uint32_t idx = global_state ? 4u : 2u;
        uint32_t o = 0;
        // the counters: uint64 entries key | count << 32 (count 0: empty; the
        // top 128 values: victims and claims of a window), 64-B buckets, then
        // the stash
        L.off_table = o; o = align16(o + 8 * L.slots);
        // with LDS state the level sort holds the list in registers from its
        // first read to its scatter and lays its histogram over it
        const bool hist_over_list = !global_state;
        const uint32_t list_bytes = idx * k;
        L.off_list = o;                                  // slots of the minimum level, by id
        o = align16(o + (hist_over_list && list_bytes < kHistBytes ? kHistBytes : list_bytes));
        // the radix sort of a level (state in global memory) keeps the ids
        // beside the slots and ping-pongs both; the LDS sorts read each
        // slot's id from the table
        L.off_tkey = o;
        L.off_list2 = o;
        L.off_tkey2 = o;
        if (global_state) {
            o = align16(o + 4 * k);
            L.off_list2 = o; o = align16(o + 4 * k);
            L.off_tkey2 = o; o = align16(o + 4 * k);
        }
        L.state_bytes = o;
        uint32_t l = global_state ? 0u : o;
        L.off_ring = l;  l = align16(l + 4 * kRing);     // staged input items
        // bucket counts / starts while a level is sorted
        if (hist_over_list) {
            L.off_hist = L.off_list;
        } else {
            L.off_hist = l;  l = align16(l + kHistBytes);
        }
        L.lds_bytes = l;
        L.err_stride = (L.slots + 31u) & ~31u;
        L.err_bytes = 4;
        L.count_mask = 0xFFFFFFFFu;
        return L;
    }

    // This layout with the narrowest errors that hold every error of blocks
    // of at most max_block items: an error is a count of the minimum level at
    // an install, at most max_block / k.  Narrow errors shrink a block's
    // scratch footprint, so fewer of its lines are written back to memory
    // while the input stream passes through the L2.  With allow_packed and the
    // state in LDS, blocks whose counts fit kCountBits bits and whose errors
    // are at most kPackedErrMax keep each error in its counter's count word
    // (err_bytes 0): no scratch at all.
    PSS_HD ChunkLayout with_error_width(uint64_t max_block, bool allow_packed = false) const {
        ChunkLayout R = *this;
        const uint64_t top = max_block / k;
        if (allow_packed && !global_state && max_block <= kCountMask && top <= kPackedErrMax) {
            R.err_bytes = 0;
            R.count_mask = kCountMask;
            return R;
        }
        R.err_bytes = top < 255u ? 1u : top < 65535u ? 2u : 4u;
        R.count_mask = 0xFFFFFFFFu;
        return R;
    }

    PSS_HD bool fits_lds_indices() const { return slots <= kMaxLdsTableSlots && k <= 65535u; }
};

// Layout of one Frequent block (k - 1 counters for the k-majority problem):
// the same two-choice hash table as ChunkLayout (slots sized for k), then the
// input ring; all in LDS.
struct FreqLayout {
    uint32_t k, counters;
    uint32_t nbuckets, tsize, slots;
    uint32_t off_table, off_ring, lds_bytes;
    uint32_t choices;  // buckets per item, as in the Space Saving table of the same k

    PSS_HD static FreqLayout make(uint32_t k) {
        FreqLayout L;
        L.k = k;
        L.counters = k - 1;
        L.choices = hash_choices(k, false);
        uint32_t want = (uint32_t)(((uint64_t)k * ChunkLayout::default_slots_x16(k, L.choices) + 15) / 16);
        if (want < 256) want = 256;
        L.nbuckets = (want + kBucketSlots - 1) / kBucketSlots;
        L.tsize = kBucketSlots * L.nbuckets;
        L.slots = L.tsize + kStash;
        uint32_t o = 0;
        L.off_table = o; o = align16(o + 8 * L.slots);
        L.off_ring = o;  o = align16(o + 4 * kRing);
        L.lds_bytes = o;
        return L;
    }
};

}  // namespace pss
