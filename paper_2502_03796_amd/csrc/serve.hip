// Serving step of the MAGUS controller on gfx950: one thread per (slot, sample).
//
// Every live telemetry stream owns a slot whose controller state stays in
// device memory between steps: the last W-1 samples (the FIFO of Alg. 1, as a
// ring indexed by the step count), the event FIFO of Alg. 2 as a bit history,
// the level and the running counters.  A step pushes one sample per listed
// slot through the same rule as replay and writes one decision byte per pair.

#include "magus_internal.h"

namespace magus {
namespace {

__global__ __launch_bounds__(256) void serve_init_kernel(
    SlotState* __restrict__ st, SlotAcc* __restrict__ acc, DevCfg* __restrict__ slot_cfg,
    const ServeInit* __restrict__ inits, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t slot = inits[i].slot;
    const DevCfg c = inits[i].cfg;
    slot_cfg[slot] = c;
    st[slot].ticks = 0;
    SlotAcc a;
    a.level_sum = 0;
    a.transitions = 0;
    a.ticks_high = 0;
    a.hist = 0;
    a.level = c.linit;
    acc[slot] = a;
}

__global__ __launch_bounds__(256) void serve_step_kernel(
    SlotState* __restrict__ st, SlotAcc* __restrict__ acc,
    const DevCfg* __restrict__ slot_cfg, const uint32_t* __restrict__ pairs, uint32_t n,
    uint8_t* __restrict__ decisions)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t slot = pairs[i];
    const uint32_t b = pairs[n + i];
    const DevCfg c = slot_cfg[slot];
    SlotAcc A = acc[slot];
    const uint32_t k = st[slot].ticks;
    const uint32_t w1 = c.W - 1;
    const uint32_t pos = k % w1;

    int pred = 0;
    if (k >= w1) {
        const uint32_t a = st[slot].ring[pos];                  // sample k-W+1
        const uint32_t d = max(a, b) - min(a, b);
        const uint32_t lov = derivative_base(a, b, c.base, c.ref);
        const bool rising = b > a;
        const uint32_t m = rising ? c.mu : c.md;
        if (((uint64_t)d << 16) > (uint64_t)lov * m) pred = rising ? 1 : -1;
    }
    st[slot].ring[pos] = b;
    st[slot].ticks = k + 1;

    const uint32_t hmask = c.H >= 32 ? 0xFFFFFFFFu : ((1u << c.H) - 1u);
    A.hist = ((A.hist << 1) | (uint32_t)(pred != 0)) & hmask;
    const bool high = (uint32_t)__popc(A.hist) >= c.thr;
    uint32_t next = A.level;
    if (high) next = c.lmax;
    else if (pred == 1) next = c.up ? min(A.level + c.up, (uint32_t)c.lmax) : c.lmax;
    else if (pred == -1)
        next = c.down ? (A.level < (uint32_t)c.lmin + c.down ? c.lmin : A.level - c.down)
                      : c.lmin;
    A.transitions += (next != A.level);
    A.level = next;
    A.level_sum += next;
    A.ticks_high += high;
    acc[slot] = A;
    decisions[i] = (uint8_t)(next | ((uint32_t)high << 5) | ((uint32_t)(pred + 1) << 6));
}

}  // namespace

hipError_t launch_serve(SlotState* st, SlotAcc* acc, DevCfg* slot_cfg, const ServeInit* inits,
                        uint32_t n_inits, const uint32_t* pairs, uint32_t n,
                        uint8_t* decisions, hipStream_t stream, hipEvent_t ev0,
                        hipEvent_t ev1)
{
    if (n_inits)
        serve_init_kernel<<<(n_inits + 255) / 256, 256, 0, stream>>>(st, acc, slot_cfg, inits,
                                                                     n_inits);
    if (ev0) (void)hipEventRecord(ev0, stream);
    if (n)
        serve_step_kernel<<<(n + 255) / 256, 256, 0, stream>>>(st, acc, slot_cfg, pairs, n,
                                                               decisions);
    if (ev1) (void)hipEventRecord(ev1, stream);
    return hipGetLastError();
}

}  // namespace magus
