// Parameter sweep of the MAGUS controller on gfx950: one lane per config.
//
// Configs are grouped into blocks of kSweepLanes that share the derivative
// window W (and base).  A workgroup takes one trace and kLanes configs of one
// block (the whole block, or a part of it; the launch shape is tunable).  For
// each tile of kTile steps the workgroup first
// computes, once per step, the two integer quotients that decide Alg. 1 for
// every threshold at once:
//   U(t) = ceil((b-a) 2^16 / (W a))  if b > a (a = 0: INT32_MAX), else 0
//   D(t) = floor((b-a) 2^16 / (W b)) if b < a (b = 0: INT32_MIN), else 0
// with a = x[t-W+1], b = x[t].  For an integer Q16.16 threshold q,
//   (b-a) 2^16 > a W q  <=>  q < U(t)     and     (a-b) 2^16 > b W |q|  <=>  q > D(t)
// (q < R <=> q < ceil(R) and q > R <=> q > floor(R) for integer q), so each
// lane decides its prediction with two int32 compares against LDS values that
// the whole workgroup shares.  The lane then carries its own event history,
// level and counters in registers across the trace; scores and the per-trace
// arg-min are reduced at the end.

#include "sweep_step.h"

namespace magus {
namespace {

// steps of the mask loop per iteration (the loop's scalar bookkeeping is
// shared by that many steps)
#ifndef MAGUS_SWEEP_UNROLL
#define MAGUS_SWEEP_UNROLL 8
#endif
constexpr uint32_t kSweepUnroll = MAGUS_SWEEP_UNROLL;

__device__ __forceinline__ uint32_t uniform(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ uint64_t wave_mask(bool p) { return __ballot(p); }

// Quotients of step t (t >= W-1) of trace x.  The derivative's base is the
// smaller sample by default (a for a rise, b for a fall), or always the
// oldest (base 1), always the newest (base 2) sample, or the fixed reference
// `ref` (base 3).
__device__ __forceinline__ int2 step_quotients(uint32_t a, uint32_t b, uint32_t W,
                                               uint32_t base, uint32_t ref) {
    int2 r = make_int2(0, 0);
    if (b > a) {
        const uint32_t bu = base == 3 ? ref : base == 2 ? b : a;
        if (bu == 0) {
            r.x = INT32_MAX;
        } else {
            const uint64_t num = (uint64_t)(b - a) << 16;
            const uint64_t den = (uint64_t)W * bu;
            const uint64_t q = (num + den - 1) / den;
            r.x = q > (uint64_t)INT32_MAX ? INT32_MAX : (int32_t)q;
        }
    } else if (b < a) {
        const uint32_t bd = base == 3 ? ref : base == 1 ? a : b;
        if (bd == 0) {
            r.y = INT32_MIN;
        } else {
            const uint64_t num = (uint64_t)(a - b) << 16;
            const uint64_t den = (uint64_t)W * bd;
            const uint64_t q = (num + den - 1) / den;     // ceil of |R'|
            r.y = q >= (uint64_t)1 << 31 ? INT32_MIN : -(int32_t)q;
        }
    }
    return r;
}

// One workgroup per (trace, part of a config block): kLanes configs, tiles of
// kTile steps (kTile / kLanes quotient pairs per thread per tile).
template <int kLanes, int kTile>
__global__ __launch_bounds__(kLanes) void sweep_kernel(
    const uint32_t* __restrict__ samples, const uint64_t* __restrict__ offsets,
    uint32_t n_traces, uint32_t n_blocks, const uint32_t* __restrict__ chunk_status,
    const uint32_t* __restrict__ block_w, const uint32_t* __restrict__ block_ref,
    const int32_t* __restrict__ lane_inc,
    const int32_t* __restrict__ lane_dec, const uint32_t* __restrict__ lane_hmask,
    const uint32_t* __restrict__ lane_thr, const uint32_t* __restrict__ lane_lv,
    const uint32_t* __restrict__ lane_orig, const uint32_t* __restrict__ lane_steps,
    const uint32_t* __restrict__ block_stepped, uint32_t n_cfgs,
    uint64_t* __restrict__ scores, uint64_t* __restrict__ keys)
{
    static_assert(kSweepLanes % kLanes == 0 && kTile % kLanes == 0, "sweep launch shape");
    constexpr uint32_t kParts = kSweepLanes / kLanes;
    __shared__ int2 ud[2][kTile];
    __shared__ uint64_t wave_min[kLanes / kWave];
    if (chunk_status[0] != 0) return;

    // Work index, grouped so that the config blocks of one trace run on the
    // same XCD (workgroups are dealt round-robin to the 8 XCDs).
    const uint32_t n_work = n_traces * n_blocks * kParts;
    const uint32_t per_xcd = (gridDim.x + 7) / 8;
    const uint32_t work = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (work >= n_work) return;
    const uint32_t t = work / (n_blocks * kParts), bp = work % (n_blocks * kParts);
    const uint32_t blk = bp / kParts, part = bp % kParts;
    // a part of a block holding only padding lanes (they sit at the block's
    // end) has nothing to report
    if (kParts > 1 && lane_orig[blk * kSweepLanes + part * kLanes] == 0xFFFFFFFFu) return;

    const uint32_t tid = threadIdx.x;
    const uint32_t W = block_w[blk] & 255u, base = block_w[blk] >> 8, ref = block_ref[blk];
    const uint32_t li = blk * kSweepLanes + part * kLanes + tid;
    const int32_t inc = lane_inc[li], dec = lane_dec[li];
    const uint32_t hmask = lane_hmask[li], thr = lane_thr[li];
    const uint32_t lv = lane_lv[li];
    const uint32_t lmin = lv & 255u, lmax = (lv >> 8) & 255u, linit = (lv >> 16) & 255u;
    const uint32_t orig = lane_orig[li];

    const uint64_t tb = offsets[t];
    const uint32_t n = (uint32_t)(offsets[t + 1] - tb);
    const uint32_t* x = samples + tb;

    uint32_t hist = 0, trans = 0, cmax = 0, cinit = 0;
    bool lvl = linit == lmax;                       // level bit (1 = max)
    bool at_init = linit != lmin && linit != lmax;  // still at a middle initial level
    // stepped actuation (integer level) for blocks holding such configs
    const bool stepped = block_stepped[blk] != 0;
    const uint32_t st = lane_steps[li];
    const uint32_t ustep = st & 255u, dstep = (st >> 8) & 255u;
    uint32_t ilvl = linit;
    uint64_t isum = 0;

    auto prepass = [&](uint32_t tile0, int buf) {
#pragma unroll
        for (uint32_t j = 0; j < (uint32_t)kTile; j += kLanes) {
            const uint32_t step = tile0 + j + tid;
            int2 q = make_int2(0, 0);
            if (step < n && step + 1 >= W)
                q = step_quotients(x[step + 1 - W], x[step], W, base, ref);
            ud[buf][j + tid] = q;
        }
    };

    prepass(0, 0);
    __syncthreads();
    int buf = 0;
    for (uint32_t tile0 = 0; tile0 < n; tile0 += kTile) {
        const uint32_t nt = min((uint32_t)kTile, n - tile0);
        const int2* q = ud[buf];
        if (stepped) {
            for (uint32_t i = 0; i < nt; ++i) {
                const int2 v = q[i];
                const bool up = inc < v.x, dn = dec > v.y;
                hist = ((hist << 1) | (uint32_t)(up | dn)) & hmask;
                const bool high = (uint32_t)__popc(hist) >= thr;
                uint32_t nl = ilvl;
                if (high) nl = lmax;
                else if (up) nl = ustep ? min(ilvl + ustep, lmax) : lmax;
                else if (dn) nl = dstep ? (ilvl < lmin + dstep ? lmin : ilvl - dstep) : lmin;
                trans += (uint32_t)(nl != ilvl);
                isum += nl;
                ilvl = nl;
            }
        } else if (__ballot(at_init) != 0) {
            for (uint32_t i = 0; i < nt; ++i) {
                const int2 v = q[i];
                const bool up = inc < v.x, dn = dec > v.y;
                hist = ((hist << 1) | (uint32_t)(up | dn)) & hmask;
                const bool high = (uint32_t)__popc(hist) >= thr;
                const bool upx = high | up;
                const bool dnx = dn & !upx;
                const bool nl = upx | (lvl & !dnx);
                trans += (uint32_t)((nl != lvl) | (at_init & dnx));
                cmax += (uint32_t)nl;
                at_init = at_init & !(upx | dnx);
                cinit += (uint32_t)at_init;
                lvl = nl;
            }
        } else {
            // the decisions of all lanes as wave masks (every lane runs
            // every step): the logic is scalar, and each mask bit enters the
            // lane's history and counters as the carry of one add
            MaskLane L{hist, trans, cmax, wave_mask(lvl)};
            auto one_step = [&](const int2 v) { mask_step(L, v, inc, dec, hmask, thr); };
            uint32_t i = 0;
#pragma unroll 1
            for (; i + kSweepUnroll <= nt; i += kSweepUnroll) {
#pragma unroll
                for (uint32_t k = 0; k < kSweepUnroll; ++k) one_step(q[i + k]);
            }
            for (; i < nt; ++i) one_step(q[i]);
            hist = L.hist;
            trans = L.trans;
            cmax = L.cmax;
            lvl = (L.lvl_m >> (threadIdx.x & 63)) & 1ull;
        }
        if (tile0 + kTile < n) prepass(tile0 + kTile, buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }

    const uint64_t level_sum = stepped ? isum
                                       : (uint64_t)lmin * (n - cmax - cinit) +
                                             (uint64_t)lmax * cmax + (uint64_t)linit * cinit;
    const uint64_t score = level_sum + 1000ull * trans;
    uint64_t key = ~0ull;
    if (orig != 0xFFFFFFFFu) {
        if (scores) scores[(uint64_t)t * n_cfgs + orig] = score;
        key = (score << 23) | orig;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const uint64_t o = __shfl_xor(key, d, 64);
        key = o < key ? o : key;
    }
    if ((tid & 63) == 0) wave_min[tid >> 6] = key;
    __syncthreads();
    if (tid == 0) {
        uint64_t m = wave_min[0];
        for (int w = 1; w < kLanes / kWave; ++w) m = wave_min[w] < m ? wave_min[w] : m;
        atomicMin((unsigned long long*)&keys[t], (unsigned long long)m);
    }
}

__global__ void keys_init_kernel(uint64_t* keys, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) keys[i] = ~0ull;
}

__global__ void argmin_kernel(const uint64_t* __restrict__ keys, uint32_t n,
                              const uint32_t* __restrict__ chunk_status,
                              uint32_t* __restrict__ argmin) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && chunk_status[0] == 0) argmin[i] = (uint32_t)(keys[i] & 0x7FFFFFull);
}

// Validates the batch (same rules as replay) into status[0] and err.
__global__ __launch_bounds__(1024) void sweep_check_kernel(
    const uint64_t* __restrict__ offsets, uint32_t n_traces, uint64_t n_samples,
    uint32_t* __restrict__ status, uint32_t* __restrict__ err)
{
    __shared__ uint32_t s_err;
    if (threadIdx.x == 0) s_err = 0;
    __syncthreads();
    uint32_t e = 0;
    for (uint32_t t = threadIdx.x; t < n_traces; t += blockDim.x) {
        const uint64_t o0 = offsets[t], o1 = offsets[t + 1];
        if (o1 < o0 || o1 > n_samples) e |= kErrOffsets;
        else if (o1 - o0 > MAGUS_MAX_TRACE_LEN) e |= kErrTooLong;
    }
    if (e) atomicOr(&s_err, e);
    __syncthreads();
    if (threadIdx.x == 0) {
        status[0] = s_err;
        if (s_err) atomicOr(err, s_err);
    }
}

}  // namespace

hipError_t launch_sweep(const uint32_t* samples, uint64_t n_samples, const uint64_t* offsets,
                        uint32_t n_traces, const SweepPlan& plan, uint32_t n_cfgs,
                        uint64_t* scores, uint32_t* argmin, uint64_t* keys, uint32_t* err,
                        uint32_t shape, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1)
{
    if (n_traces == 0) return hipSuccess;
    if (shape >= kSweepShapeCount) return hipErrorInvalidValue;
    uint32_t* status = reinterpret_cast<uint32_t*>(keys + n_traces);
    sweep_check_kernel<<<1, 1024, 0, stream>>>(offsets, n_traces, n_samples, status, err);
    keys_init_kernel<<<(n_traces + 255) / 256, 256, 0, stream>>>(keys, n_traces);
    const uint32_t lanes = kSweepShapes[shape].lanes;
    const uint64_t n_work = (uint64_t)n_traces * plan.n_blocks * (kSweepLanes / lanes);
    const uint32_t grid = (uint32_t)((n_work + 7) / 8 * 8);
    if (ev0) (void)hipEventRecord(ev0, stream);
    auto go = [&](auto kernel, uint32_t threads) {
        kernel<<<grid, threads, 0, stream>>>(
            samples, offsets, n_traces, plan.n_blocks, status, plan.block_w, plan.block_ref,
            plan.lane_inc, plan.lane_dec, plan.lane_hmask, plan.lane_thr, plan.lane_lv,
            plan.lane_orig, plan.lane_steps, plan.block_stepped, n_cfgs, scores, keys);
    };
    static_assert(kSweepShapeCount == 6, "one launch per shape");
    switch (shape) {
    case 0: go(sweep_kernel<256, 256>, 256); break;
    case 1: go(sweep_kernel<256, 512>, 256); break;
    case 2: go(sweep_kernel<256, 1024>, 256); break;
    case 3: go(sweep_kernel<128, 256>, 128); break;
    case 4: go(sweep_kernel<128, 512>, 128); break;
    default: go(sweep_kernel<64, 256>, 64); break;
    }
    if (ev1) (void)hipEventRecord(ev1, stream);
    argmin_kernel<<<(n_traces + 255) / 256, 256, 0, stream>>>(keys, n_traces, status, argmin);
    return hipGetLastError();
}

}  // namespace magus
