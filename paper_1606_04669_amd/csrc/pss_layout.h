// Memory layout of one block summary, shared by the host launcher and the
// chunk_summary kernel.  One wave owns one layout.  The per-block state (hash
// table, counts, minimum-level list) lives in LDS when it fits, otherwise in
// a global-memory slab of state_bytes per block; the input ring and a few
// small per-window arrays always live in LDS.  A counter's item id is the
// key of its hash-table entry, and errors are written straight to the
// block's output array in device memory (read only at the end), which keeps
// both out of LDS.
#pragma once

#include <stdint.h>

#ifndef __HIPCC__
#define PSS_HD
#else
#define PSS_HD __host__ __device__
#endif

namespace pss {

// Items staged per half of the LDS input ring (two halves).
constexpr uint32_t kRingHalf = 256;
constexpr uint32_t kRing = 2 * kRingHalf;
// Largest hash table whose slot positions fit uint16 (LDS-resident state).
constexpr uint32_t kMaxLdsTableSlots = 65536;
// Slots per hash bucket (key/tag pairs of 8 bytes).
#ifndef PSS_BUCKET_SLOTS
#define PSS_BUCKET_SLOTS 8
#endif
constexpr uint32_t kBucketSlots = PSS_BUCKET_SLOTS;
// Hash slots per counter x16: 2 per counter up to k = 1024, 1.5 above (a
// speed / memory trade that never changes results: at k = 2000 the smaller
// table lets three waves share a CU's LDS instead of two).
#ifndef PSS_SLOTS_X16
#define PSS_SLOTS_X16 24
#endif
#ifndef PSS_SLOTS_X16_SMALLK
#define PSS_SLOTS_X16_SMALLK 32
#endif
// Overflow slots after the buckets, for items whose two buckets are full.
constexpr uint32_t kStash = 64;
// The level sort's histogram: 257 words.
constexpr uint32_t kHistBytes = 4 * 257;

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

struct ChunkLayout {
    uint32_t k;
    uint32_t nbuckets;      // hash buckets of kBucketSlots slots
    uint32_t tsize;         // kBucketSlots * nbuckets slots (the stash follows them)
    uint32_t global_state;  // 1: state in global memory, 32-bit indices; 0: LDS, 16-bit indices
    // state offsets (bytes from the state base)
    uint32_t off_table, off_cnt, off_hpos, off_list, off_mark, off_tkey, off_list2, off_tkey2;
    uint32_t state_bytes;
    // LDS offsets (bytes from the LDS base; the state comes first when it is in LDS)
    uint32_t off_ring, off_vslot, off_vhpos, off_hist;
    uint32_t lds_bytes;

    // Default hash slots per counter (x16).
    PSS_HD static uint32_t default_slots_x16(uint32_t k) { return k <= 1024 ? PSS_SLOTS_X16_SMALLK : PSS_SLOTS_X16; }

    // slots_per_counter_x16: hash slots per counter (x16), a speed / memory
    // knob that never changes results (0 = default).  global_state selects
    // where the per-block state lives.
    PSS_HD static ChunkLayout make(uint32_t k, bool global_state, uint32_t slots_per_counter_x16 = 0) {
        ChunkLayout L;
        L.k = k;
        L.global_state = global_state ? 1u : 0u;
        if (slots_per_counter_x16 == 0) slots_per_counter_x16 = default_slots_x16(k);
        uint32_t slots = (uint32_t)(((uint64_t)k * slots_per_counter_x16 + 15) / 16);
        if (slots < 256) slots = 256;
        L.nbuckets = (slots + kBucketSlots - 1) / kBucketSlots;
        L.tsize = kBucketSlots * L.nbuckets;
        const uint32_t idx = global_state ? 4u : 2u;
        uint32_t o = 0;
        L.off_table = o; o = align16(o + 8 * (L.tsize + kStash));  // uint64 entries (key | tag << 32): 64-B buckets, then the stash
        L.off_cnt = o;   o = align16(o + 4 * k);
        L.off_hpos = o;  o = align16(o + idx * k);       // table slot of each counter
        L.off_list = o;  o = align16(o + idx * k);       // counters of the minimum level, by id
        // uint8 victim ranks; with LDS state also the sort histogram (all marks
        // are zero while a level is sorted and are cleared again after it)
        L.off_mark = o;  o = align16(o + (global_state ? k : (k > kHistBytes ? k : kHistBytes)));
        L.off_tkey = o;  o = align16(o + 4 * k);         // ids while a level is sorted
        L.off_list2 = o;
        L.off_tkey2 = o;
        if (global_state) {                              // ping-pong buffers of the radix sort
            L.off_list2 = o; o = align16(o + 4 * k);
            L.off_tkey2 = o; o = align16(o + 4 * k);
        }
        L.state_bytes = o;
        uint32_t l = global_state ? 0u : o;
        L.off_ring = l;  l = align16(l + 4 * kRing);     // staged input items
        L.off_vslot = l; l = align16(l + 4 * 64);        // victim counter per rank
        L.off_vhpos = l; l = align16(l + 4 * 64);        // its table slot
        L.off_hist = global_state ? l : L.off_mark;      // bucket counts / starts while a level is sorted
        if (global_state) l = align16(l + kHistBytes);
        L.lds_bytes = l;
        return L;
    }

    PSS_HD bool fits_lds_indices() const { return tsize + kStash <= kMaxLdsTableSlots && k <= 65535u; }
};

}  // namespace pss
