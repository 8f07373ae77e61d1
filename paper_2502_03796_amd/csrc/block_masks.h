// Alg. 1 and Alg. 2 for 64 consecutive steps of one trace at once (one step
// per lane of a wavefront), as 64-bit lane masks, and a walker over the
// blocks of a time chunk.  Shared by the stepped-actuation and proxy kernels.
#pragma once

#include <type_traits>

#include "magus_internal.h"

namespace magus {

__device__ __forceinline__ uint64_t lane_ballot(bool p) { return __ballot(p); }

// v plus the value of the lane the DPP control names, in 64 bits
template <int kCtrl, int kRowMask, bool kBound>
__device__ __forceinline__ uint64_t dpp_add64(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, kCtrl,
                                                              kRowMask, 0xf, kBound);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32),
                                                              kCtrl, kRowMask, 0xf, kBound);
    return v + (((uint64_t)hi << 32) | lo);
}

// Wave sum of 64-bit values (every lane active): row shifts of 1, 2, 4 and 8
// sum each row of 16 lanes, row broadcasts of lanes 15 and 31 carry the rows
// before, and lane 63 holds the total (no LDS traffic).
__device__ __forceinline__ uint64_t dpp_wave_sum64(uint64_t v) {
    v = dpp_add64<0x111, 0xf, true>(v);
    v = dpp_add64<0x112, 0xf, true>(v);
    v = dpp_add64<0x114, 0xf, true>(v);
    v = dpp_add64<0x118, 0xf, true>(v);
    v = dpp_add64<0x142, 0xa, false>(v);
    v = dpp_add64<0x143, 0xc, false>(v);
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
}

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

// One block: lane i holds step tb+i, b = its sample x[t] and a = x[t-W+1]
// (from this block or the one before).  fps carries (flags of the block
// before) >> 1 and is updated.
// valid = lanes whose step exists; steps before W-1 of the trace never predict.
// all_high = ~0 when the count threshold is 0 (every step is high), else 0.
// kFull: every lane's step exists and the trace's FIFO is already full (the
// block does not end the chunk and does not start the trace), so no lane mask
// is needed.  kAnyBase: the config may use another derivative base than the
// smaller sample (else that base is assumed).
template <bool kFull = false, bool kAnyBase = true>
__device__ __forceinline__ BlockMasks block_masks(uint32_t a, uint32_t b, uint32_t tb,
                                                  uint64_t valid, const DevCfg& c,
                                                  uint64_t all_high, uint32_t k16,
                                                  uint64_t& fps, uint32_t lane)
{
    const uint32_t W = c.W, H = c.H;
    uint64_t vm = kFull ? ~0ull : valid;
    if (!kFull && tb < W - 1) vm &= ~mask_below(W - 1 - tb);
    BlockMasks r;
    if (!kAnyBase || c.base == 0) {
        // the smaller sample is the base: a rise is an event iff
        // b 2^16 > a (2^16 + W q_inc), a fall iff a 2^16 > b (2^16 + W |q_dec|)
        // (k16 = 2^16 as an opaque scalar keeps x 2^16 one 32x32->64 multiply)
        const uint64_t up = lane_ballot((uint64_t)b * k16 > (uint64_t)a * (65536u + c.mu)) & vm;
        const uint64_t dn = lane_ballot((uint64_t)a * k16 > (uint64_t)b * (65536u + c.md)) & vm;
        r.E = up | dn;
        r.R = up;
    } else {
        const bool rising = b > a;
        const uint32_t d = max(a, b) - min(a, b);
        const uint32_t lov = derivative_base(a, b, c.base, c.ref);
        const uint32_t m = rising ? c.mu : c.md;
        // r = d / (W base) beyond q / 2^16  <=>  d 2^16 > base (W q)
        r.E = lane_ballot(((uint64_t)d << 16) > (uint64_t)lov * m) & vm;
        r.R = lane_ballot(rising);
    }
    // events among the last H steps (this block's flags and the last H-1 of
    // the block before), for all 64 steps; with none of them a step is high
    // only if the count threshold is 0
    const uint64_t B = fps >> (64 - H);
    if ((r.E | B) == 0) {
        r.HM = all_high & (kFull ? ~0ull : valid);
    } else {
        const uint64_t nG = ~((r.E << (H - 1)) | B);
        const uint32_t acc0 = (uint32_t)__popcll(B) + (uint32_t)(r.E & 1ull);
        const uint32_t cnt = bits_below_lane(nG, bits_below_lane(r.E >> 1, acc0));
        r.HM = lane_ballot(cnt >= c.thr + lane) & (kFull ? ~0ull : valid);
    }
    fps = r.E >> 1;
    return r;
}

// A time chunk of a trace as one wave sees it: the trace, the chunk's steps
// [s, e), the first loaded step wbeg (one warm-up block before s when s > 0),
// the config and a bounds-checked buffer descriptor over samples [wbeg, e).
struct ChunkView {
    uint32_t t, s, e, wbeg;
    uint64_t tbase;
    DevCfg c;
    uint64_t all_high;       // ~0 when the count threshold is 0
    uint32_t k16;            // 2^16, opaque to the compiler
    __amdgpu_buffer_rsrc_t rsrc;
};

__device__ __forceinline__ uint32_t bm_uniform(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ ChunkView chunk_view(
    const uint32_t* samples, const uint64_t* offsets, uint32_t n_traces,
    const uint32_t* chunk_base, const DevCfg* cfgs, const uint32_t* cfg_of_trace,
    uint32_t chunk, uint32_t g)
{
    ChunkView v;
    v.t = trace_of_chunk(chunk_base, n_traces, g, threadIdx.x & 63);
    v.tbase = offsets[v.t];
    const uint32_t n = (uint32_t)(offsets[v.t + 1] - v.tbase);
    v.s = (g - chunk_base[v.t]) * chunk;
    v.e = min(v.s + chunk, n);
    v.c = cfgs[cfg_of_trace ? cfg_of_trace[v.t] : 0];
    v.all_high = v.c.thr == 0 ? ~0ull : 0ull;
    asm volatile("s_mov_b32 %0, 0x10000" : "=s"(v.k16));
    v.wbeg = v.s >= 64 ? v.s - 64 : 0;
    const uint64_t base = (uint64_t)(samples + v.tbase + v.wbeg);
    const uint64_t base_u = ((uint64_t)bm_uniform((uint32_t)(base >> 32)) << 32) |
                            bm_uniform((uint32_t)base);
    v.rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)base_u, (short)0,
                                               (int)bm_uniform((v.e - v.wbeg) * 4u),
                                               0x00020000);
    return v;
}

struct NoGroupEnd {
    __device__ __forceinline__ void operator()() const {}
};

// Walks the blocks of a chunk, calling body(block masks, first step of the
// block, valid-lane mask, this lane's sample) for every real block (the
// warm-up block only feeds the FIFOs), and group_end() after every group of
// kAhead loaded blocks (code that should not be repeated per block goes
// there).  Lanes past the chunk's end read 0.  A group of kAhead blocks is
// loaded while the group before it is evaluated, so a wave keeps that many
// loads in flight.
template <uint32_t kAhead = 8, bool kAnyBase = true, class Body, class GroupEnd = NoGroupEnd>
__device__ __forceinline__ void for_each_block(const ChunkView& v, uint32_t lane, Body&& body,
                                               GroupEnd&& group_end = GroupEnd{}) {
    const uint32_t first_real = v.s >= 64 ? 1u : 0u;
    const uint32_t nblk = (v.e - v.wbeg + 63) >> 6;
    auto load = [&](uint32_t blk) -> uint32_t {
        return __builtin_amdgcn_raw_buffer_load_b32(v.rsrc, (int)((blk * 64 + lane) * 4), 0,
                                                    kStreamLoad);
    };
    uint64_t fps = 0;
    uint32_t xprev = 0;                 // the last block of the group before
    const int addr = (int)(((lane - (v.c.W - 1)) & 63u) << 2);
    const bool from_cur = lane >= v.c.W - 1;
    auto step = [&](uint32_t blk, uint32_t a, uint32_t x, auto full_tag) {
        constexpr bool kFull = decltype(full_tag)::value;
        const uint32_t tb = v.wbeg + blk * 64;
        const uint64_t valid = kFull ? ~0ull : mask_below(min(64u, v.e - tb));
        const BlockMasks m = block_masks<kFull, kAnyBase>(a, x, tb, valid, v.c, v.all_high,
                                                          v.k16, fps, lane);
        if (kFull || blk >= first_real) body(m, tb, valid, x);
    };
    // blocks [1, nfull) hold 64 steps each and never start the trace
    const uint32_t nfull = (v.e - v.wbeg) >> 6;
    auto group = [&](uint32_t g, const uint32_t (&cur)[kAhead]) {
        // x[t-W+1] of every step of the group, all lane exchanges issued
        // before any block is evaluated
        uint32_t a[kAhead];
#pragma unroll
        for (uint32_t k = 0; k < kAhead; ++k) {
            const uint32_t ac = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)cur[k]);
            const uint32_t ap =
                (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(k ? cur[k - 1] : xprev));
            a[k] = from_cur ? ac : ap;
        }
        if (g >= 1 && (g + 1) * kAhead <= nfull) {
#pragma unroll
            for (uint32_t k = 0; k < kAhead; ++k)
                step(g * kAhead + k, a[k], cur[k], std::true_type{});
        } else {
#pragma unroll
            for (uint32_t k = 0; k < kAhead; ++k)
                if (g * kAhead + k < nblk) step(g * kAhead + k, a[k], cur[k], std::false_type{});
        }
        xprev = cur[kAhead - 1];
        group_end();
    };
    // two alternating groups of kAhead blocks: one is evaluated while the
    // other is loaded (loads past the end read 0)
    uint32_t bufA[kAhead], bufB[kAhead];
#pragma unroll
    for (uint32_t k = 0; k < kAhead; ++k) bufA[k] = load(k);
    const uint32_t groups = (nblk + kAhead - 1) / kAhead;
    for (uint32_t g = 0; g < groups; g += 2) {
#pragma unroll
        for (uint32_t k = 0; k < kAhead; ++k) bufB[k] = load((g + 1) * kAhead + k);
        group(g, bufA);
        if (g + 1 >= groups) break;
#pragma unroll
        for (uint32_t k = 0; k < kAhead; ++k) bufA[k] = load((g + 2) * kAhead + k);
        group(g + 1, bufB);
    }
}

}  // namespace magus
