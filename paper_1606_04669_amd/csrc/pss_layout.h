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
// Capacity of the sorted list of minimum-level counters (victims in order).
constexpr uint32_t kListCap = 512;

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

struct ChunkLayout {
    uint32_t k;
    uint32_t tbits;   // hash table has 2^tbits slots
    uint32_t tsize;
    // byte offsets inside the wave's LDS block
    uint32_t off_table, off_list, off_cnt, off_item, off_err, off_hpos, off_mark, off_ring, off_scratch;
    uint32_t bytes;

    // hash_shift: table size = next_pow2(2k) << hash_shift (load factor knob;
    // it changes speed and LDS use, never results)
    PSS_HD static ChunkLayout make(uint32_t k, uint32_t hash_shift = 0) {
        ChunkLayout L;
        L.k = k;
        L.tsize = next_pow2(2 * k) << hash_shift;
        if (L.tsize < 256) L.tsize = 256;
        L.tbits = log2_pow2(L.tsize);
        uint32_t o = 0;
        L.off_table = o;   o += 8 * L.tsize;           // uint64 entries (key | tag << 32)
        L.off_list = o;    o += 8 * kListCap;          // uint64 (item << 32 | slot); histogram while rebuilding
        L.off_cnt = o;     o += 4 * ((k + 3) & ~3u);
        L.off_item = o;    o += 4 * ((k + 3) & ~3u);
        L.off_err = o;     o += 4 * ((k + 3) & ~3u);
        L.off_hpos = o;    o += 2 * ((k + 7) & ~7u);   // uint16 table position of each counter
        L.off_mark = o;    o += (k + 15) & ~15u;       // uint8 victim ranks
        L.off_ring = o;    o += 4 * kRing;             // staged input items
        L.off_scratch = o; o += 4 * 64 + 64;           // victim slots [64] (u32), positions [64] (u8)
        L.bytes = o;
        return L;
    }
};

}  // namespace pss
