// Launcher of the proxy energy / EDP kernels (proxy.hip).
#pragma once

#include "magus_internal.h"

namespace magus {

// Per-chunk summary of the fused proxy pass (jump-to-bound configs), free of
// the level entering the chunk: the steps whose interval runs at the entering
// level (up to and including the chunk's first decisive step) are kept with
// their excess at each of the three levels a chunk can be entered at
// (level_min, level_max, level_init); every later step's level is fixed by
// the chunk's own decisive steps.  80 bytes.
struct ProxySum {
    uint32_t len;        // steps in the chunk
    uint32_t ppre;       // steps whose interval runs at the entering level
    uint32_t has_dec;    // the chunk has a decisive step
    uint32_t end_up;     // level after the chunk's last step is level_max (if has_dec)
    uint32_t n_lo, n_hi; // other steps whose interval runs at level_min / level_max
    uint64_t pre_x[3];   // excess of the entering-level steps at cap[min], cap[max], cap[init]
    uint64_t x_lo, x_hi; // excess of the other steps at their level
    uint64_t ex_max;     // excess of every step at cap[level_max] (always-max policy)
    uint64_t ex_min;     // ... at cap[level_min] (always-min policy)
};
static_assert(sizeof(ProxySum) == 80, "ProxySum layout");

// Fused proxy pass for batches whose configs all jump to the bound: one read
// of the samples per step after the plan (chunk_base from launch_plan),
// per-chunk summaries into psums (max_chunks), one wave per trace folds them
// into stats and derives the metrics (optional) from the same sums.  For a
// batch the plan rejected the fold writes zero statistics and metrics are not
// written.  redo (max_chunks + 1 words, device) is the queue of chunks for
// the exact pass: redo[0] must be 0 when the call starts, and the fold sets
// it to 0 again.
hipError_t launch_proxy_fused(const uint32_t* samples, const uint64_t* offsets, uint32_t n_traces,
                              const uint32_t* chunk_base, uint32_t max_chunks,
                              const DevCfg* cfgs, const uint32_t* cfg_of_trace, uint32_t chunk,
                              const magus_proxy_model* model, ProxySum* psums, uint32_t* redo,
                              magus_proxy_stats* stats, magus_proxy_metrics* metrics,
                              bool any_base, bool mid_init, hipStream_t stream);

// Sets the count of an exact-pass queue (redo[0]) to 0, with a kernel.
hipError_t launch_proxy_queue_clear(uint32_t* redo, hipStream_t stream);

// Stepped configs: runs after launch_stepped_prepare of the same batch
// (chunk plan in chunk_base, the level entering every chunk in `entering`,
// the blocks' step masks in `masks`); reads the samples once more and sums
// per level without decision bytes.  `model` is in device memory.  stats
// (n_traces) is cleared and filled; metrics (optional, n_traces) is written.
// For a batch the plan rejected (status word chunk_base[n_traces + 1] != 0)
// stats stay zero and metrics are not written.  bin_levels: the widest level
// range (level_max - level_min + 1) of the batch's configs, which sizes the
// narrow pass's per-lane excess bins (0: the wide pass only).  redo
// (max_chunks + 1 words, device): the queue of chunks for the wide pass,
// cleared by the call's first kernel and left filled.
hipError_t launch_proxy_stepped(const uint32_t* samples, uint64_t n_samples,
                                const uint64_t* offsets, uint32_t n_traces,
                                const uint32_t* chunk_base, uint32_t max_chunks,
                                const DevCfg* cfgs, const uint32_t* cfg_of_trace, uint32_t chunk,
                                const uint32_t* entering, const uint64_t* masks,
                                const magus_proxy_model* model, magus_proxy_stats* stats,
                                magus_proxy_metrics* metrics, uint32_t bin_levels,
                                uint32_t* redo, hipStream_t stream);

}  // namespace magus
