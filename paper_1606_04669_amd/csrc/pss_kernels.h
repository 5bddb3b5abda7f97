// Internal launch interface between the C-ABI host code and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pss_layout.h"

namespace pss {

// A set of summaries stored at stride k (entries of summary p start at p*k),
// with per-summary size and minimum (0 while fewer than k counters are used).
// Persistent summaries also keep on the device the stream length N they
// cover and a fault word: a fold or merge whose input carries a block's
// failure mark leaves the summary and N as they were and sets the fault
// word instead (block and tree summaries leave both null).
template <typename CT>
struct SummaryView {
    uint32_t* item;
    CT* cnt;
    CT* err;
    uint32_t* size;
    CT* min;
    uint64_t* total = nullptr;
    uint32_t* fault = nullptr;
};

using BlockSummaries = SummaryView<uint32_t>;
using WideSummary = SummaryView<uint64_t>;

// Result entry as written by the extract kernel (same layout as pss_entry).
struct DevEntry {
    uint32_t item;
    uint32_t reserved;
    uint64_t count;
    uint64_t error;
};

// Layout of one block summary for k counters: state in LDS when it fits in
// lds_max bytes (with 16-bit indices), else in a global slab per block, with
// an LDS request that leaves room for four such waves per CU.
ChunkLayout chunk_layout(uint32_t k, size_t lds_max);
// gstate: chunks * L.state_bytes bytes of device memory when L.global_state;
// errs: chunks * L.err_stride words of device memory (error scratch; the
// launch packs each error in its counter's count word when its blocks allow
// it, else stores it in the fewest bytes that hold every error of its
// blocks, ChunkLayout::with_error_width).  chunks >= 1.
hipError_t launch_chunk_summary(const uint32_t* d_items, uint64_t n, uint32_t chunks, const ChunkLayout& L,
                                const BlockSummaries& out, unsigned char* gstate, uint32_t* errs,
                                hipStream_t stream);

// ---- batched form: many independent streams in one launch sequence ----

// One block of a batch: items[begin, end) of a stream of n items, k counters.
struct BatchBlock {
    const uint32_t* items;  // the stream (device memory)
    uint64_t n;             // stream length: bounds every load
    uint64_t begin, end;    // block bounds within the stream (Algorithm 1)
    uint64_t out;           // entry offset of the block summary (capacity k)
    uint64_t eoff;          // word offset of the block's error scratch (err_stride of its layout)
    uint32_t k;
    uint32_t slots_x16;     // hash slots per counter (x16), result-neutral
};

// One COMBINE of a batch level: summaries a and b (entry offsets a_off,
// b_off, header indices a, b) into a, with k counters.
struct BatchNode {
    uint64_t a_off, b_off;
    uint32_t a, b, k, pad;
};

// The report of one stream of a batch: the root summary (entry offset,
// header index), k, the stream length n, and where its entries go.
struct BatchReport {
    uint64_t root_off;
    uint64_t n;
    uint64_t out_off;
    uint32_t root, k;
};

// Persistent launch over nblocks blocks whose k share sort_lanes_per_k;
// queue: one zeroed counter; waves_per_group waves per workgroup, each with
// lds_stride bytes of LDS (>= the layout of every block's k and load factor);
// errs: base of the blocks' error scratch.
hipError_t launch_batch_blocks(const BatchBlock* blocks, uint32_t nblocks, uint32_t* queue, uint32_t sort_lanes,
                               uint32_t lds_stride, uint32_t waves_per_group, uint32_t grid,
                               const BlockSummaries& out, uint32_t* errs, hipStream_t stream);
// One tree level of a batch (all streams): nodes[0, count), kmax bounds LDS.
hipError_t launch_batch_combine(const BatchNode* nodes, uint32_t count, uint32_t kmax, const BlockSummaries& base,
                                hipStream_t stream);
// Majority reports of a batch: one workgroup per stream; out_count[s] is the
// number of entries written at out + out_off.
hipError_t launch_batch_extract(const BatchReport* reps, uint32_t count, uint32_t kmax, const BlockSummaries& base,
                                DevEntry* out, uint32_t* out_count, hipStream_t stream);
// ---- served form: appends and queries on a pool of persistent summaries ----
// Pool: summary sid's entries at offset s_off of item/cnt/err, header at
// size[sid], min[sid].

// S_sid <- COMBINE(S_sid, block summary `root`) with k counters.
struct ServeFold {
    uint64_t s_off, root_off;
    uint32_t sid, root, k, pad;
};

// Report of summary sid (kind 0: count * k > n; 1: first cap), entries to
// out + out_off.
struct ServeQuery {
    uint64_t s_off, n, out_off;
    uint32_t sid, k, kind, cap;
};

// A fold whose block-tree root carries the failure mark leaves its summary
// as it was and sets *failed.
hipError_t launch_serve_fold(const ServeFold* f, uint32_t count, uint32_t kmax, const WideSummary& pool,
                             const BlockSummaries& blocks, uint32_t* failed, hipStream_t stream);
hipError_t launch_serve_query(const ServeQuery* q, uint32_t count, uint32_t kmax, const WideSummary& pool,
                              DevEntry* out, uint32_t* out_count, hipStream_t stream);

// Zero `count` words (a kernel, safe inside captured graphs).
hipError_t launch_zero_words(uint32_t* p, uint32_t count, hipStream_t stream);

// One level of the fixed tree over `count` block summaries: node j combines
// summaries 2*step*j and 2*step*j + step into position 2*step*j.
// in_lds: the O(k) arrays of a COMBINE fit LDS (combine_lds_bytes <= limit);
// otherwise scratch holds `slabs` slabs of combine_scratch_bytes and at most
// that many workgroups run, each merging several pairs in turn.
hipError_t launch_combine_level(const BlockSummaries& v, uint32_t k, uint32_t count, uint32_t step, bool in_lds,
                                unsigned char* scratch, uint32_t slabs, hipStream_t stream);
// dst <- COMBINE(dst, src) for a narrow (block/tree) src at position 0, and
// N(dst) += n; when src carries the failure mark, dst and N(dst) stay as
// they were and dst's fault word is set.
hipError_t launch_fold(const WideSummary& dst, const BlockSummaries& src, uint32_t k, uint64_t n, bool in_lds,
                       unsigned char* scratch, hipStream_t stream);
// dst <- COMBINE(dst, src) for two wide summaries, N(dst) += N(src).
hipError_t launch_merge(const WideSummary& dst, const WideSummary& src, uint32_t k, bool in_lds,
                        unsigned char* scratch, hipStream_t stream);
uint32_t combine_lds_bytes(uint32_t k, bool wide);
size_t combine_scratch_bytes(uint32_t k, bool wide);

// Canonically ordered report of a wide summary: kind 0 = count*k > N with
// the summary's own N, kind 1 = first `cap`.  Writes entries to out and the
// reported count (before truncation to cap for kind 0) to out_count[0], the
// summary's fault word to out_count[1] (then clears it) and its N to
// out_count[2..3].
// in_lds: the sort arrays fit LDS (extract_lds_bytes <= limit); otherwise
// scratch holds extract_scratch_bytes bytes.
hipError_t launch_extract(const WideSummary& s, uint32_t k, int kind, uint32_t cap, DevEntry* out,
                          uint32_t* out_count, bool in_lds, unsigned char* scratch, hipStream_t stream);
uint32_t extract_lds_bytes(uint32_t k);
size_t extract_scratch_bytes(uint32_t k);

// Majority report (count * k > N) of the tree root v (block summary 0):
// at most cap entries to out, the reported count (or 0xFFFFFFFF when the root
// carries a block's failure mark) to *out_count.  The sort arrays in LDS
// (extract_lds_bytes(k) <= the device's limit).
hipError_t launch_root_extract(const BlockSummaries& v, uint32_t k, uint64_t N, uint32_t cap, DevEntry* out,
                               uint32_t* out_count, hipStream_t stream);

// ---- Frequent (Misra-Gries) summaries: block summaries at stride k with
// k - 1 counters each, size[] and, in min[], the decrement steps D ----
hipError_t launch_frequent_blocks(const uint32_t* d_items, uint64_t n, uint32_t chunks, const FreqLayout& L,
                                  const BlockSummaries& out, hipStream_t stream);
// One tree level: node j merges summaries 2*step*j and 2*step*j + step.
hipError_t launch_frequent_level(const BlockSummaries& v, uint32_t k, uint32_t count, uint32_t step,
                                 hipStream_t stream);
uint32_t frequent_merge_lds_bytes(uint32_t k);
// Report of the root (summary 0) for a stream of N items: kind 0 = entries
// with (count + D) * k > N, kind 1 = the first cap; canonical order (count
// desc, item asc).  out_count[0] = the count before truncation (0xFFFFFFFF
// for a failed block), out_count[2..3] = D.
hipError_t launch_frequent_report(const BlockSummaries& v, uint32_t k, uint64_t N, int kind, uint32_t cap,
                                  DevEntry* out, uint32_t* out_count, hipStream_t stream);

// Set a wide summary to the empty summary (N = 0, fault cleared).
hipError_t launch_reset(const WideSummary& s, hipStream_t stream);

}  // namespace pss
