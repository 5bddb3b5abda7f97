// Internal launch interface between the C-ABI host code and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pss {

// A set of summaries stored at stride k (entries of summary p start at p*k),
// with per-summary size and minimum (0 while fewer than k counters are used).
template <typename CT>
struct SummaryView {
    uint32_t* item;
    CT* cnt;
    CT* err;
    uint32_t* size;
    CT* min;
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

hipError_t launch_chunk_summary(const uint32_t* d_items, uint64_t n, uint32_t chunks, uint32_t k,
                                const BlockSummaries& out, hipStream_t stream);
uint32_t chunk_summary_lds_bytes(uint32_t k);

// One level of the fixed tree over `count` block summaries: node j combines
// summaries 2*step*j and 2*step*j + step into position 2*step*j.
hipError_t launch_combine_level(const BlockSummaries& v, uint32_t k, uint32_t count, uint32_t step,
                                hipStream_t stream);
// dst <- COMBINE(dst, src) for a narrow (block/tree) src at position 0.
hipError_t launch_fold(const WideSummary& dst, const BlockSummaries& src, uint32_t k, hipStream_t stream);
// dst <- COMBINE(dst, src) for two wide summaries.
hipError_t launch_merge(const WideSummary& dst, const WideSummary& src, uint32_t k, hipStream_t stream);
uint32_t combine_lds_bytes(uint32_t k, bool wide);

// Canonically ordered report of a wide summary: kind 0 = count*k > N,
// kind 1 = first `cap`.  Writes entries to out and the reported count
// (before truncation to cap for kind 0) to *out_count.
hipError_t launch_extract(const WideSummary& s, uint32_t k, uint64_t N, int kind, uint32_t cap, DevEntry* out,
                          uint32_t* out_count, hipStream_t stream);
uint32_t extract_lds_bytes(uint32_t k);

// Set a wide summary to the empty summary.
hipError_t launch_reset(const WideSummary& s, hipStream_t stream);

}  // namespace pss
