// LDS layout of one block summary, shared by the host launcher and the
// chunk_summary kernel.  One wave owns one layout.
#pragma once

#include <stdint.h>

#ifndef __HIPCC__
#define PSS_HD
#else
#define PSS_HD __host__ __device__
#endif

namespace pss {

// Items staged per half of the LDS input ring (two halves).
constexpr uint32_t kRingHalf = 512;
constexpr uint32_t kRing = 2 * kRingHalf;
// Largest hash table (slot positions are stored as uint16).
constexpr uint32_t kMaxTableSlots = 65536;

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

// Registers per lane the victim-list sort needs for k counters.
PSS_HD inline uint32_t sort_lanes_per_k(uint32_t k) {
    return next_pow2((k + 63) / 64);
}

struct ChunkLayout {
    uint32_t k;
    uint32_t nbuckets;  // hash buckets of 4 slots
    uint32_t tsize;     // 4 * nbuckets slots
    // byte offsets inside the wave's LDS block
    uint32_t off_table, off_cnt, off_item, off_err, off_hpos, off_list, off_mark, off_ring, off_scratch, off_tkey,
        off_hist;
    uint32_t bytes;

    // Default hash slots per counter (x16): more room (shorter probes, fewer
    // rebuilds) while the LDS footprint is small, 2 per counter for large k.
    PSS_HD static uint32_t default_slots_x16(uint32_t k) { return k <= 1024 ? 64 : 32; }

    // slots_per_counter (x16): hash slots per counter; a speed / LDS knob
    // that never changes results (0 = default_slots_x16).
    PSS_HD static ChunkLayout make(uint32_t k, uint32_t slots_per_counter_x16 = 0) {
        ChunkLayout L;
        L.k = k;
        if (slots_per_counter_x16 == 0) slots_per_counter_x16 = default_slots_x16(k);
        uint32_t slots = (k * slots_per_counter_x16 + 15) / 16;
        if (slots < 256) slots = 256;
        L.nbuckets = (slots + 3) / 4;
        L.tsize = 4 * L.nbuckets;
        uint32_t o = 0;
        L.off_table = o;   o += 8 * L.tsize;           // uint64 entries (key | tag << 32), 32 B buckets
        L.off_cnt = o;     o += 4 * ((k + 3) & ~3u);
        L.off_item = o;    o += 4 * ((k + 3) & ~3u);
        L.off_err = o;     o += 4 * ((k + 3) & ~3u);
        L.off_hpos = o;    o += 2 * ((k + 7) & ~7u);   // uint16 table slot of each counter
        L.off_list = o;    o += 2 * ((k + 7) & ~7u);   // uint16 counters of the minimum level, by id
        L.off_mark = o;    o += (k + 15) & ~15u;       // uint8 victim ranks
        L.off_ring = o;    o += 4 * kRing;             // staged input items
        L.off_scratch = o; o += 4 * 64;                // victim slot | table slot << 16, per rank
        L.off_tkey = o;    o += 4 * ((k + 3) & ~3u);   // ids in bucket order while a level is sorted
        L.off_hist = o;    o += 4 * 257;               // bucket counts / starts while a level is sorted
        o = (o + 15) & ~15u;
        L.bytes = o;
        return L;
    }

    PSS_HD bool valid() const { return tsize <= kMaxTableSlots; }
};

}  // namespace pss
