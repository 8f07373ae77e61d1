// VALU issue-rate probe on gfx950: how many 32-bit integer VALU instructions
// a compute unit issues per clock when nothing else limits it.
//
// Every lane runs `steps` rounds of kChains independent dependency chains, so
// consecutive instructions of a wave never wait on each other, and nothing
// else happens in the loop (no memory, no LDS, no barriers).  Two mixes:
//   mode 0  one v_add_u32 per chain per round;
//   mode 1  the opcodes of the sweep's per-evaluation step, one each per
//           chain per round: a compare into a wave mask (v_cmp), an add with
//           that mask as carry-in (v_addc_co_u32), a mask (v_and_b32) and a
//           population count (v_bcnt_u32_b32).
// VALU instructions per lane and round: kChains (mode 0), 4 kChains (mode 1),
// so a launch issues workgroups * 256 * steps * that many lane-ops.  The rate
// sets the issue ceiling the sweep kernel's instruction stream is compared
// with; the published vector peak of the chip is the other bound.

#include "sweep_step.h"

namespace magus {
namespace {

constexpr int kChains = 8;

__global__ __launch_bounds__(kSweepLanes) void valu_probe_kernel(uint32_t steps, uint32_t mode,
                                                                 uint32_t seed,
                                                                 uint32_t* __restrict__ out)
{
    const uint32_t tid = threadIdx.x;
    uint32_t a[kChains], b[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) {
        a[k] = seed * (uint32_t)(k + 1) + tid;
        b[k] = (seed >> k) ^ (tid * 0x9E3779B9u) ^ blockIdx.x;
    }
    if (mode == 0) {
        // four rounds per loop iteration (steps is a multiple of 4)
#pragma unroll 1
        for (uint32_t i = 0; i < steps; i += 4) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
#pragma unroll
                for (int k = 0; k < kChains; ++k)
                    asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[k]) : "v"(b[k]));
            }
        }
    } else {
#pragma unroll 1
        for (uint32_t i = 0; i < steps; ++i) {
            uint64_t m[kChains];
#pragma unroll
            for (int k = 0; k < kChains; ++k) m[k] = __ballot((int32_t)a[k] < (int32_t)b[k]);
#pragma unroll
            for (int k = 0; k < kChains; ++k) a[k] = add_bit(a[k], a[k], m[k]);
#pragma unroll
            for (int k = 0; k < kChains; ++k)
                asm volatile("v_and_b32 %0, %0, %1" : "+v"(a[k]) : "v"(b[k]));
#pragma unroll
            for (int k = 0; k < kChains; ++k)
                asm volatile("v_bcnt_u32_b32 %0, %1, %0" : "+v"(b[k]) : "v"(a[k]));
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) r ^= a[k] + b[k];
    out[blockIdx.x * kSweepLanes + tid] = r;
}

}  // namespace

uint32_t valu_probe_ops_per_step(uint32_t mode) { return mode == 0 ? kChains : 4 * kChains; }

hipError_t launch_valu_probe(uint32_t workgroups, uint32_t steps, uint32_t mode, uint32_t seed,
                             uint32_t* out, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1)
{
    if (ev0) (void)hipEventRecord(ev0, stream);
    valu_probe_kernel<<<workgroups, kSweepLanes, 0, stream>>>(steps, mode, seed, out);
    if (ev1) (void)hipEventRecord(ev1, stream);
    return hipGetLastError();
}

}  // namespace magus
