// Alg. 1 and Alg. 2 for 64 consecutive steps of one trace at once (one step
// per lane of a wavefront), as 64-bit lane masks.  Shared by the stepped-
// actuation kernels.
#pragma once

#include "magus_internal.h"

namespace magus {

__device__ __forceinline__ uint64_t lane_ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint64_t mask_below(uint32_t n) {   // n in [0, 64]
    return n >= 64 ? ~0ull : ((1ull << n) - 1ull);
}

__device__ __forceinline__ uint32_t bits_below_lane(uint64_t m, uint32_t acc) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, acc));
}

struct BlockMasks {
    uint64_t E;      // prediction != 0
    uint64_t R;      // rising (b > a), meaningful where E is set
    uint64_t HM;     // high state
};

// One block: x = this block's samples, xprev = the block before (lane i holds
// step tb+i).  fps carries (flags of the block before) >> 1 and is updated.
// valid = lanes whose step exists; steps before W-1 of the trace never predict.
__device__ __forceinline__ BlockMasks block_masks(uint32_t x, uint32_t xprev, uint32_t tb,
                                                  uint64_t valid, const DevCfg& c,
                                                  uint64_t& fps, uint32_t lane)
{
    const uint32_t W = c.W, H = c.H;
    const int addr = (int)(((lane - (W - 1)) & 63u) << 2);
    const uint32_t ac = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)x);
    const uint32_t ap = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)xprev);
    const uint32_t a = lane >= W - 1 ? ac : ap;      // x[t-W+1]
    const uint32_t b = x;
    const bool rising = b > a;
    const uint32_t d = max(a, b) - min(a, b);
    const uint32_t lov = derivative_base(a, b, c.base);
    const uint32_t m = rising ? c.mu : c.md;
    // r = d / (W lo) beyond q / 2^16  <=>  d 2^16 > lo (W q)
    const bool ev = ((uint64_t)d << 16) > (uint64_t)lov * m;
    uint64_t vm = valid;
    if (tb < W - 1) vm &= ~mask_below(W - 1 - tb);
    BlockMasks r;
    r.E = lane_ballot(ev) & vm;
    r.R = lane_ballot(rising);
    // events among the last H steps (this block's flags and the last H-1 of
    // the block before), for all 64 steps
    const uint64_t B = fps >> (64 - H);
    const uint64_t nG = ~((r.E << (H - 1)) | B);
    const uint32_t acc0 = (uint32_t)__popcll(B) + (uint32_t)(r.E & 1ull);
    const uint32_t cnt = bits_below_lane(nG, bits_below_lane(r.E >> 1, acc0));
    r.HM = lane_ballot(cnt >= c.thr + lane) & valid;
    fps = r.E >> 1;
    return r;
}

}  // namespace magus
