// VALU issue probe for the sweep's instruction mix on gfx950.
//
// Runs the sweep's per-evaluation step (mask_step, shared with the sweep
// kernel) `steps` times per lane on register data: the step's two quotients
// come from a scalar hash of the step index instead of an LDS tile, and
// nothing else happens in the loop (no LDS reads, no barriers, no tile
// pre-pass).  Launched with the sweep's workgroup size and enough workgroups
// to fill every compute unit, it issues the step's VALU instructions as fast
// as the machine takes them, which is the ceiling the sweep is measured
// against.

#include "sweep_step.h"

namespace magus {
namespace {

__global__ __launch_bounds__(kSweepLanes) void valu_probe_kernel(uint32_t steps, uint32_t seed,
                                                                 uint32_t* __restrict__ out)
{
    const uint32_t tid = threadIdx.x;
    // a config per lane from the sweep grid's ranges
    const int32_t inc = (int32_t)(1311u + 2097u * (tid & 15u));
    const int32_t dec = -(int32_t)(1311u + 2097u * ((tid >> 4) & 15u));
    const uint32_t H = 1u + ((tid + blockIdx.x) & 15u);
    const uint32_t hmask = (1u << H) - 1u;
    const uint32_t thr = (3u * H + 4u) / 5u;
    MaskLane L{0u, 0u, 0u, 0ull};
    uint32_t h = seed ^ (blockIdx.x * 0x9E3779B9u);
#pragma unroll 1
    for (uint32_t i = 0; i < steps; i += 4) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            h = h * 0x2C1B3C6Du + 0x297A2D39u;          // wave-uniform: scalar unit
            const int2 v = make_int2((int32_t)(h >> 17), -(int32_t)((h & 0xFFFFu) << 1));
            mask_step(L, v, inc, dec, hmask, thr);
        }
    }
    out[blockIdx.x * kSweepLanes + tid] = L.hist ^ L.trans ^ (L.cmax << 7);
}

}  // namespace

hipError_t launch_valu_probe(uint32_t workgroups, uint32_t steps, uint32_t seed, uint32_t* out,
                             hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1)
{
    if (ev0) (void)hipEventRecord(ev0, stream);
    valu_probe_kernel<<<workgroups, kSweepLanes, 0, stream>>>(steps, seed, out);
    if (ev1) (void)hipEventRecord(ev1, stream);
    return hipGetLastError();
}

}  // namespace magus
