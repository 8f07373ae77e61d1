// Allocation-free replay (magus_replay_noalloc): the jump-to-bound replay of
// magus_replay with every piece of scratch memory (config table, chunk
// prefix and status, chunk summaries, per-chunk fix-up records) carved out of
// one fixed device array instead of context-owned buffers, for callers that
// cannot allocate device memory at call time.
//
// The array lives in this file.  Its device address is resolved once per
// device, with that device current, on the first call there; host code uses
// only that address (the array's own name is a host-side stand-in).

#include <mutex>

#include "host_internal.h"

namespace magus {
namespace {

constexpr size_t kScratchBytes = MAGUS_NOALLOC_SCRATCH_BYTES;
constexpr uint32_t kNoAllocChunk = 4096;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static_assert(kErrOffsets == MAGUS_DATA_OFFSETS && kErrTooLong == MAGUS_DATA_TOO_LONG &&
                  kErrCfgIndex == MAGUS_DATA_CFG_INDEX,
              "public data-check bits");

std::mutex g_mu;                       // guards the two tables below
unsigned char* g_scratch[kMaxDevices]; // device address of `scratch`, per device
// host staging of the derived config table (pageable: the copy has read it
// by the time hipMemcpyAsync returns)
DevCfg g_cfg_stage[MAGUS_NOALLOC_MAX_CFGS];

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// Device address of `scratch` on the current device `dev`, resolved on the
// first call for that device.  Caller holds g_mu.
int scratch_of(int dev, unsigned char** out) {
    if (dev < 0 || dev >= kMaxDevices)
        return fail(MAGUS_EINVAL, "device %d beyond the %d the allocation-free replay tracks",
                    dev, kMaxDevices);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MAGUS_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch[dev];
    return MAGUS_OK;
}

}  // namespace
}  // namespace magus

using namespace magus;

extern "C" int magus_replay_noalloc(const uint32_t* d_samples, uint64_t n_samples,
                                    const uint64_t* d_offsets, uint32_t n_traces,
                                    const magus_config* h_cfgs, uint32_t n_cfgs,
                                    const uint32_t* d_cfg_of_trace, magus_result* d_results,
                                    uint8_t* d_levels, uint32_t* d_status,
                                    hipStream_t stream) {
    if (!h_cfgs || n_cfgs == 0) return fail(MAGUS_EINVAL, "need at least one config");
    if (n_cfgs > MAGUS_NOALLOC_MAX_CFGS)
        return fail(MAGUS_EINVAL, "%u configs: the allocation-free replay takes at most %u",
                    n_cfgs, (unsigned)MAGUS_NOALLOC_MAX_CFGS);
    if (n_traces && (!d_offsets || !d_results))
        return fail(MAGUS_EINVAL, "offsets and results are required");
    if (n_samples && !d_samples) return fail(MAGUS_EINVAL, "samples is NULL");
    if (n_traces > (1u << 30)) return fail(MAGUS_EINVAL, "too many traces");
    // scratch layout, each part 256-byte aligned: config table, chunk prefix
    // (+ total and status), chunk summaries, fix-up records (decision bytes only)
    const uint64_t max_chunks64 = n_samples / kNoAllocChunk + (uint64_t)n_traces + 1;
    const size_t off_cfg = 0;
    const size_t off_base = off_cfg + align256((size_t)n_cfgs * sizeof(DevCfg));
    const size_t off_sums = off_base + align256(((size_t)n_traces + 2) * 4);
    const size_t off_fix = off_sums + align256((size_t)max_chunks64 * sizeof(ChunkSum));
    const size_t need = off_fix + (d_levels ? (size_t)max_chunks64 * sizeof(ChunkFix) : 0);
    if (max_chunks64 > 0xFFFFFFF0ull || need > kScratchBytes)
        return fail(MAGUS_EINVAL,
                    "batch needs %llu bytes of scratch; the allocation-free replay has %zu",
                    (unsigned long long)need, kScratchBytes);
    if (n_traces == 0 && d_status == nullptr) {
        // nothing to run; the configs are still validated
        for (uint32_t i = 0; i < n_cfgs; ++i) {
            DevCfg d;
            if (int rc = derive(&h_cfgs[i], &d); rc != MAGUS_OK)
                return fail(rc, "config %u: %s", i, std::string(last_error()).c_str());
        }
        return MAGUS_OK;
    }
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_mu);
    bool any_base = false;
    for (uint32_t i = 0; i < n_cfgs; ++i) {
        if (int rc = derive(&h_cfgs[i], &g_cfg_stage[i]); rc != MAGUS_OK)
            return fail(rc, "config %u: %s", i, std::string(last_error()).c_str());
        if (g_cfg_stage[i].up || g_cfg_stage[i].down)
            return fail(MAGUS_EINVAL, "config %u has stepped actuation; the allocation-free "
                        "replay takes jump-to-bound configs only", i);
        any_base |= g_cfg_stage[i].base != 0;
    }
    unsigned char* base = nullptr;
    if (int rc = scratch_of(dev, &base); rc != MAGUS_OK) return rc;
    if (n_traces == 0) {
        // an empty batch: the plan kernel alone writes a clean status
        HIP_TRY(launch_plan(d_offsets, 0, n_samples, nullptr, n_cfgs, kNoAllocChunk, 1,
                            reinterpret_cast<uint32_t*>(base + off_base), nullptr, stream,
                            d_status));
        return MAGUS_OK;
    }
    DevCfg* cfgs = reinterpret_cast<DevCfg*>(base + off_cfg);
    HIP_TRY(hipMemcpyAsync(cfgs, g_cfg_stage, (size_t)n_cfgs * sizeof(DevCfg),
                           hipMemcpyHostToDevice, stream));
    // the plan rewrites the chunk prefix and the status word on every call,
    // the chunk kernel every summary the fold reads, so nothing needs clearing
    HIP_TRY(launch_replay(d_samples, n_samples, d_offsets, n_traces, cfgs, n_cfgs,
                          d_cfg_of_trace, kNoAllocChunk,
                          reinterpret_cast<uint32_t*>(base + off_base),
                          reinterpret_cast<ChunkSum*>(base + off_sums), (uint32_t)max_chunks64,
                          d_levels ? reinterpret_cast<ChunkFix*>(base + off_fix) : nullptr,
                          d_results, d_levels, /*err=*/nullptr, /*persistent_blocks=*/0,
                          any_base, stream, nullptr, nullptr, d_status));
    return MAGUS_OK;
}
