// Streaming-read probe on gfx950: the rate at which the chip delivers a
// buffer read with the replay chunk kernel's access pattern and no other
// work: one wave per chunk, one dword per lane per 64-sample block, eight
// blocks per iteration with the next eight in flight, non-temporal loads
// through a bounds-checked buffer descriptor.  Over the replay's batch its
// time is the practical ceiling of that access pattern, which the chunk
// kernel's HBM rate is compared with beside the published peak.

#include "magus_internal.h"

namespace magus {
namespace {

constexpr uint32_t kReadIter = 8;      // blocks of 64 samples per iteration
constexpr int kReadWaves = 4;          // waves per workgroup

__global__ __launch_bounds__(kReadWaves * kWave) void read_probe_kernel(
    const uint32_t* __restrict__ samples, uint64_t n_samples, uint32_t chunk, uint32_t n_chunks,
    uint32_t* __restrict__ out)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t w = blockIdx.x * kReadWaves +
                       (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (w >= n_chunks) return;
    const uint64_t s = (uint64_t)w * chunk;
    const uint32_t len = (uint32_t)min<uint64_t>(chunk, n_samples - s);
    const uint64_t base = (uint64_t)(samples + s);
    const uint64_t base_u =
        ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(base >> 32)) << 32) |
        (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)base);
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)base_u, (short)0, (int)(len * 4u), 0x00020000);
    const uint32_t n_iter = ((len + 63) / 64 + kReadIter - 1) / kReadIter;
    auto load = [&](uint32_t blk) -> uint32_t {
        return __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)((blk * 64 + lane) * 4), 0,
                                                    kStreamLoad);
    };
    // loads past the chunk's end read 0 (the descriptor's bound)
    uint32_t a[kReadIter], b[kReadIter], acc = 0;
#pragma unroll
    for (uint32_t j = 0; j < kReadIter; ++j) a[j] = load(j);
    for (uint32_t it = 0; it < n_iter; it += 2) {
#pragma unroll
        for (uint32_t j = 0; j < kReadIter; ++j) b[j] = load((it + 1) * kReadIter + j);
#pragma unroll
        for (uint32_t j = 0; j < kReadIter; ++j) acc = (acc ^ a[j]) * 0x9E3779B1u;
#pragma unroll
        for (uint32_t j = 0; j < kReadIter; ++j) a[j] = load((it + 2) * kReadIter + j);
#pragma unroll
        for (uint32_t j = 0; j < kReadIter; ++j) acc = (acc ^ b[j]) * 0x9E3779B1u;
    }
    if (lane == 0) out[w] = acc;
}

}  // namespace

hipError_t launch_read_probe(const uint32_t* samples, uint64_t n_samples, uint32_t chunk,
                             uint32_t* out, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1)
{
    const uint64_t n_chunks = (n_samples + chunk - 1) / chunk;
    if (n_chunks == 0) return hipSuccess;
    if (hipError_t e = record_timing_event(ev0, stream); e != hipSuccess) return e;
    read_probe_kernel<<<(uint32_t)((n_chunks + kReadWaves - 1) / kReadWaves), kReadWaves * kWave,
                        0, stream>>>(samples, n_samples, chunk, (uint32_t)n_chunks, out);
    if (hipError_t e = record_timing_event(ev1, stream); e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace magus
