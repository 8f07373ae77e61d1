// One step of the controller for a whole wave of sweep lanes (one config per
// lane) whose configs jump to the bounds and whose level is at a bound: the
// decisions of all lanes are wave masks, so the decision logic is scalar and
// each mask bit enters the lane's event history and counters as the carry-in
// of one add.  The add with a mask as carry-in is shared with the VALU
// issue-rate probe.
#pragma once

#include "magus_internal.h"

namespace magus {

// v + w + this lane's bit of the wave-uniform mask m, as one add with carry-in
// (the mask is the carry), so a lane-mask bit needs no conversion to 0/1.
__device__ __forceinline__ uint32_t add_bit(uint32_t v, uint32_t w, uint64_t m) {
    uint32_t r;
    uint64_t carry_out;
    asm("v_addc_co_u32_e64 %0, %1, %2, %3, %4"
        : "=v"(r), "=s"(carry_out) : "v"(v), "v"(w), "s"(m));
    return r;
}

struct MaskLane {
    uint32_t hist;      // event flags of the last H steps (newest in bit 0)
    uint32_t trans;     // level changes
    uint32_t cmax;      // steps at the maximum level
    uint64_t lvl_m;     // level bit of every lane (1 = at the maximum)
};

// Alg. 1 for this lane's thresholds against the step's shared quotients
// v = (U, D) (inc < U: +1; dec > D: -1), the event FIFO, Alg. 2 (events
// among the last H >= thr) and the jump-to-bound decision.
__device__ __forceinline__ void mask_step(MaskLane& L, int2 v, int32_t inc, int32_t dec,
                                          uint32_t hmask, uint32_t thr) {
    const uint32_t zero = 0;
    const uint64_t up = __ballot(inc < v.x), dn = __ballot(dec > v.y);
    L.hist = add_bit(L.hist, L.hist, up | dn) & hmask;
    const uint64_t high = __ballot((uint32_t)__popc(L.hist) >= thr);
    const uint64_t nl = high | up | (L.lvl_m & ~dn);
    L.trans = add_bit(L.trans, zero, nl ^ L.lvl_m);
    L.cmax = add_bit(L.cmax, zero, nl);
    L.lvl_m = nl;
}

}  // namespace magus
