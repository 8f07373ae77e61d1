// Launcher of the proxy energy / EDP kernels (proxy.hip).
#pragma once

#include "magus_internal.h"

namespace magus {

// Runs after a replay of the same batch that wrote the decision bytes
// `levels` with the chunk plan in `chunk_base` (chunk steps per chunk).
// `model` is in device memory.  stats (n_traces) is cleared and filled;
// metrics (optional, n_traces) is written.  For a batch the replay rejected
// (status word chunk_base[n_traces + 1] != 0) stats stay zero and metrics
// are not written.
hipError_t launch_proxy(const uint32_t* samples, const uint64_t* offsets, uint32_t n_traces,
                        const uint32_t* chunk_base, uint32_t max_chunks, const DevCfg* cfgs,
                        const uint32_t* cfg_of_trace, uint32_t chunk, const uint8_t* levels,
                        const magus_proxy_model* model, magus_proxy_stats* stats,
                        magus_proxy_metrics* metrics, hipStream_t stream);

}  // namespace magus
