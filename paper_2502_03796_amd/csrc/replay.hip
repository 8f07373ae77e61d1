// Batched replay of the MAGUS controller on gfx950.
//
// A trace is cut into time chunks; each 64-lane wavefront replays one chunk
// with one lane per step.  The prediction (Alg. 1), the event flag, the event
// count over the last H steps (Alg. 2) and the decisive steps are all pure
// functions of the samples, so a wave evaluates 64 consecutive steps at once
// and turns them into 64-bit lane masks.  Only the level is recurrent: with
// jump-to-bound actuation (Sec. 6.1) the level after a step is level_max or
// level_min as set by the most recent decisive step, which is a carry chain of
// a 64-bit addition.  Per chunk the wave therefore produces a summary that does
// not depend on the level entering the chunk, and a per-trace fold composes
// the summaries in order.
//
// Kernels, in stream order:
//   plan    prefix sum of chunks per trace + device-side data checks
//   chunks  one wave per chunk -> ChunkSum (and decision bytes if asked)
//   fold    one wave per trace -> magus_result
//   fixup   (decision bytes only) level of the steps before the first
//           decisive step of each chunk
// The plan, fold and fixup kernels are in replay_fold.hip.

#include <type_traits>

#include "magus_internal.h"

namespace magus {

namespace {

constexpr int kChunkWavesPerBlock = 4;

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t lo32(uint64_t v) { return (uint32_t)v; }
__device__ __forceinline__ uint32_t hi32(uint64_t v) { return (uint32_t)(v >> 32); }

// Number of bits of `m` strictly below this lane.
__device__ __forceinline__ uint32_t mbcnt(uint64_t m, uint32_t acc) {
    return __builtin_amdgcn_mbcnt_hi(hi32(m), __builtin_amdgcn_mbcnt_lo(lo32(m), acc));
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, uint32_t lane) {
    uint32_t l = __builtin_amdgcn_readlane((int)lo32(v), (int)lane);
    uint32_t h = __builtin_amdgcn_readlane((int)hi32(v), (int)lane);
    return ((uint64_t)h << 32) | l;
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ uint64_t low_mask(uint32_t n) {   // n in [0, 64]
    return n >= 64 ? ~0ull : ((1ull << n) - 1ull);
}

// ------------------------------------------------------------------ chunks

#ifndef MAGUS_REPLAY_ITER
#define MAGUS_REPLAY_ITER 8
#endif
constexpr uint32_t kIter = MAGUS_REPLAY_ITER;   // blocks of 64 steps per unrolled iteration
static_assert(64 % kIter == 0, "an iteration must not straddle a group of 64 blocks");

// One wave replays one chunk [s, e) of trace t, 64 steps (one "block") at a
// time, kIter blocks per iteration.  The samples of iteration i+1 are loaded
// while iteration i is evaluated.  Blocks of a group of 64 consecutive blocks
// leave their decisive-step masks in lane j = block index of VGPRs; at the end
// of the group every lane resolves the level bits of its own block.
template <bool kLevels, bool kAnyBase>
__device__ __forceinline__ void replay_chunk(
    const uint32_t* __restrict__ samples, const uint64_t* __restrict__ offsets,
    uint32_t n_traces, const uint32_t* __restrict__ chunk_base,
    const DevCfg* __restrict__ cfgs, const uint32_t* __restrict__ cfg_of_trace,
    uint32_t chunk, ChunkSum* __restrict__ sums, ChunkFix* __restrict__ fix,
    uint8_t* __restrict__ levels, const uint32_t g, const uint32_t lane)
{
    const uint32_t t = trace_of_chunk(chunk_base, n_traces, g, lane);
    const uint64_t tbase = offsets[t];
    const uint32_t n = (uint32_t)(offsets[t + 1] - tbase);
    const uint32_t s = (g - chunk_base[t]) * chunk;
    const uint32_t e = min(s + chunk, n);
    const DevCfg c = cfgs[cfg_of_trace ? cfg_of_trace[t] : 0];
    const uint32_t W = c.W, H = c.H;

    // Samples [wbeg, e) of the trace through a bounds-checked buffer
    // descriptor (loads outside return 0).  When the chunk does not start the
    // trace, block 0 of the descriptor is the warm-up block [s-64, s) that
    // fills the two FIFOs for the first steps of the chunk.
    const uint32_t wbeg = s >= 64 ? s - 64 : 0;
    // (the base and size are wave-uniform; readfirstlane lets the compiler
    // keep the descriptor in SGPRs)
    const uint64_t base = (uint64_t)(samples + tbase + wbeg);
    const uint64_t base_u = ((uint64_t)uniform((uint32_t)(base >> 32)) << 32) |
                            uniform((uint32_t)base);
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)base_u, (short)0, (int)uniform((e - wbeg) * 4u), 0x00020000);
    const uint32_t first_real = s >= 64 ? 1u : 0u;
    const uint32_t nreal = (e - s + 63) >> 6;            // real blocks, last may be partial
    const uint32_t nfull = (e - s) >> 6;                 // real blocks with 64 valid steps
    const uint32_t n_iter = (nreal + kIter - 1) / kIter;

    // per-lane constants
    const int bperm_addr = (int)(((lane - (W - 1)) & 63u) << 2);  // lane of x[t-W+1]
    const bool from_cur = lane >= W - 1;
    // Alg. 2 compare, rearranged so that the block's carried-in count can stay
    // in an SGPR: count = acc0 + X >= thr + lane  <=>  X + bias >= 2^31 - acc0
    // with the per-lane bias = 2^31 - thr - lane (X, acc0 and thr + lane are
    // all below 2^8, so nothing wraps).
    const uint32_t bias_lane = 0x80000000u - (c.thr + lane);
    // (with a zero count threshold every step is high: no block is quiet)
    const uint64_t loud = c.thr == 0 ? 1ull : 0ull;
    // thresholds as per-lane registers: a select between a VGPR and an SGPR
    // operand needs no copy inside the loop
    uint32_t mu;
    asm volatile("v_mov_b32 %0, %1" : "=v"(mu) : "s"(c.mu));
    const uint32_t md = c.md;
    // E1 with the default base: a rise is an event iff b 2^16 > a (2^16 + W q_inc),
    // a fall iff a 2^16 > b (2^16 + W |q_dec|) (both sides below 2^59)
    const uint32_t ku = 65536u + c.mu, kd = 65536u + c.md;
    // 2^16 as an opaque SGPR operand, so that x 2^16 stays one 32x32->64
    // multiply instead of a zero-extension plus a 64-bit shift
    uint32_t k16;
    asm volatile("s_mov_b32 %0, 0x10000" : "=s"(k16));

    auto load_block = [&](uint32_t desc_blk) -> uint32_t {
        return __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)((desc_blk * 64 + lane) * 4), 0,
                                                    kStreamLoad);
    };
    // Alg. 1 for the 64 steps of a block: masks of the +1 and -1 predictions.
    auto events = [&](uint32_t a, uint32_t b, uint64_t& EU, uint64_t& ED) {
        if constexpr (kAnyBase) {
            const bool rising = b > a;
            const uint32_t lov = derivative_base(a, b, c.base, c.ref);
            const uint32_t d = max(a, b) - min(a, b);
            const uint32_t m = rising ? mu : md;
            // r = d / (W base) beyond q / 2^16  <=>  d 2^16 > base (W q)
            const uint64_t E = ballot(((uint64_t)d << 16) > (uint64_t)lov * m);
            const uint64_t R = ballot(rising);
            EU = E & R;
            ED = E & ~R;
        } else {
            // the smaller sample is the base: with b > a, (b - a) 2^16 > a W q
            // <=> b 2^16 > a (2^16 + W q), which cannot hold for b <= a
            // (x 2^16 as a 64-bit product: no register pair to zero-extend into)
            EU = ballot((uint64_t)b * k16 > (uint64_t)a * ku);
            ED = ballot((uint64_t)a * k16 > (uint64_t)b * kd);
        }
    };

    uint32_t xp = 0;             // samples of the block before the current one
    uint64_t fps = 0;            // (flags of the block before) >> 1
    if (first_real) {
        const uint32_t x0 = load_block(0);
        const uint32_t ac = (uint32_t)__builtin_amdgcn_ds_bpermute(bperm_addr, (int)x0);
        uint64_t EU, ED;
        events(from_cur ? ac : 0u, x0, EU, ED);
        uint64_t E = EU | ED;
        const uint32_t tb = s - 64;
        if (tb < W - 1) E &= ~low_mask(W - 1 - tb);       // FIFO not yet full
        fps = E >> 1;
        xp = x0;
    }

    uint32_t bufA[kIter], bufB[kIter];
#pragma unroll
    for (uint32_t j = 0; j < kIter; ++j) bufA[j] = load_block(first_real + j);

    uint32_t th = 0;             // steps in the high state
    uint32_t upL = 0, upH = 0, dnL = 0, dnH = 0;          // group masks, lane j = block j
    uint32_t puL = 0, puH = 0, pdL = 0, pdH = 0, hmL = 0, hmH = 0;
    uint32_t gi = 0;             // blocks in the current group
    uint32_t g0 = s;             // first step of the current group
    uint32_t gcarry = 0;         // level bit entering the group
    uint32_t cnt_max = 0, trans0 = 0;   // per lane
    bool found = false;
    uint32_t prefix = e - s, first_up = 0;

    auto flush_group = [&]() {
        const bool act = lane < gi;
        const uint64_t up = act ? (((uint64_t)upH << 32) | upL) : 0ull;
        const uint64_t dn = act ? (((uint64_t)dnH << 32) | dnL) : 0ull;
        const uint64_t d = up | dn;
        const uint64_t HAS = ballot(d != 0);
        const uint64_t LUP = ballot(up > dn);        // the last decisive step sets max
        // level bit entering every block: the carries of ~DNB + LUP + gcarry
        const uint64_t ndnb = ~(HAS & ~LUP);
        const uint64_t s1 = ndnb + LUP;
        const uint32_t k1 = s1 < ndnb;
        const uint64_t s2 = s1 + gcarry;
        const uint32_t k2 = s2 < s1;
        const uint64_t cin_mask = ~(s2 ^ HAS);
        const uint32_t cin = (uint32_t)(cin_mask >> lane) & 1u;
        // level bits inside block `lane`: the carries of ~dn + up + cin
        const uint64_t nd = ~dn;
        const uint64_t t1 = nd + up;
        const uint64_t c1 = t1 < nd;
        const uint64_t t2 = t1 + cin;
        const uint64_t c2 = t2 < t1;
        const uint64_t C = ~(t2 ^ d);                 // level bit before each step
        const uint64_t L = (C >> 1) | ((c1 | c2) << 63);   // level bit after each step
        const uint32_t bstart = g0 + lane * 64;
        const uint32_t nvalid = (act && bstart < e) ? min(64u, e - bstart) : 0u;
        const uint64_t vm = low_mask(nvalid);
        cnt_max += __popcll(L & vm);
        trans0 += __popcll((L ^ C) & vm);
        if (!found && HAS) {
            const uint32_t j0 = (uint32_t)__builtin_ctzll(HAS);
            const uint64_t dj = readlane64(d, j0);
            const uint64_t uj = readlane64(up, j0);
            const uint32_t b0 = (uint32_t)__builtin_ctzll(dj);
            prefix = g0 + j0 * 64 + b0 - s;
            first_up = (uint32_t)(uj >> b0) & 1u;
            found = true;
        }
        if constexpr (kLevels) {
            const uint64_t pu = act ? (((uint64_t)puH << 32) | puL) : 0ull;
            const uint64_t pd = act ? (((uint64_t)pdH << 32) | pdL) : 0ull;
            const uint64_t hm = act ? (((uint64_t)hmH << 32) | hmL) : 0ull;
            for (uint32_t j = 0; j < gi; ++j) {
                const uint64_t Lj = readlane64(L, j), PUj = readlane64(pu, j);
                const uint64_t PDj = readlane64(pd, j), HMj = readlane64(hm, j);
                const uint32_t step = g0 + j * 64 + lane;
                if (step < e) {
                    const uint32_t lv = ((Lj >> lane) & 1) ? c.lmax : c.lmin;
                    const uint32_t pr = ((PUj >> lane) & 1) ? 2u : (((PDj >> lane) & 1) ? 0u : 1u);
                    const uint32_t hb = (uint32_t)(HMj >> lane) & 1u;
                    levels[tbase + step] = (uint8_t)(lv | (hb << 5) | (pr << 6));
                }
            }
        }
        gcarry = k1 | k2;
        g0 += gi * 64;
        gi = 0;
        // lanes of quiet blocks are not written: start the next group at zero
        upL = upH = dnL = dnH = 0;
        if constexpr (kLevels) puL = puH = pdL = pdH = hmL = hmH = 0;
    };

    // One iteration: blocks it*kIter .. it*kIter+kIter-1 (real-block index).
    auto iteration = [&](uint32_t it, uint32_t (&cur)[kIter], uint32_t (&nxt)[kIter],
                         auto generic_tag) {
        constexpr bool generic = decltype(generic_tag)::value;
        if (it + 1 < n_iter) {
#pragma unroll
            for (uint32_t j = 0; j < kIter; ++j)
                nxt[j] = load_block(first_real + (it + 1) * kIter + j);
        }
        // x[t-W+1] of every step, from this block or the one before
        uint32_t ac[kIter], ap[kIter];
#pragma unroll
        for (uint32_t j = 0; j < kIter; ++j) {
            ac[j] = (uint32_t)__builtin_amdgcn_ds_bpermute(bperm_addr, (int)cur[j]);
            ap[j] = (uint32_t)__builtin_amdgcn_ds_bpermute(bperm_addr, (int)(j ? cur[j - 1] : xp));
        }
#pragma unroll
        for (uint32_t j = 0; j < kIter; ++j) {
            uint64_t PU, PD;
            events(from_cur ? ac[j] : ap[j], cur[j], PU, PD);
            if constexpr (generic) {
                const uint32_t tb = s + (it * kIter + j) * 64;     // trace step of lane 0
                uint64_t vm = low_mask(tb < e ? min(64u, e - tb) : 0u);
                if (tb < W - 1) vm &= ~low_mask(W - 1 - tb);
                PU &= vm;
                PD &= vm;
            }
            const uint64_t E = PU | PD;
            // Alg. 2: events among the last H steps, for all 64 steps at once
            const uint64_t B = fps >> (64 - H);           // last H-1 flags of the block before
            // A quiet block (no event in it nor in the H-1 steps before it,
            // and a non-zero count threshold) is never high and has no
            // decisive step: its group lanes stay zero and only the flag
            // history moves on.
            if (!generic && (E | B | loud) == 0) {
                fps = 0;
                continue;
            }
            const uint64_t nG = ~((E << (H - 1)) | B);    // ~(flag H-1 steps back)
            const uint32_t acc0 = (uint32_t)__popcll(B) + (uint32_t)(E & 1ull);
            const uint32_t cnt = mbcnt(nG, mbcnt(E >> 1, bias_lane));
            uint64_t HM = ballot(cnt >= 0x80000000u - acc0);
            if constexpr (generic) {
                const uint32_t tb = s + (it * kIter + j) * 64;
                HM &= low_mask(tb < e ? min(64u, e - tb) : 0u);
            }
            fps = E >> 1;
            const uint64_t UP = HM | PU;                  // high or +1 -> max
            const uint64_t DN = PD & ~HM;                 // -1 executed -> min
            th += (uint32_t)__popcll(HM);
            const uint32_t li = gi + j;
            writelane_into(upL, lo32(UP), li);
            writelane_into(upH, hi32(UP), li);
            writelane_into(dnL, lo32(DN), li);
            writelane_into(dnH, hi32(DN), li);
            if constexpr (kLevels) {
                writelane_into(puL, lo32(PU), li);
                writelane_into(puH, hi32(PU), li);
                writelane_into(pdL, lo32(PD), li);
                writelane_into(pdH, hi32(PD), li);
                writelane_into(hmL, lo32(HM), li);
                writelane_into(hmH, hi32(HM), li);
            }
        }
        xp = cur[kIter - 1];
        gi += kIter;
        if (gi == 64) flush_group();
    };

    // The first iteration of a trace and the iterations reaching past the last
    // full block need per-step masks; all others take the unmasked path.
    auto run = [&](uint32_t it, uint32_t (&cur)[kIter], uint32_t (&nxt)[kIter]) {
        if ((it == 0 && first_real == 0) || (it + 1) * kIter > nfull)
            iteration(it, cur, nxt, std::true_type{});
        else
            iteration(it, cur, nxt, std::false_type{});
    };
    for (uint32_t it = 0; it < n_iter; it += 2) {
        run(it, bufA, bufB);
        if (it + 1 < n_iter) run(it + 1, bufB, bufA);
    }
    if (gi) flush_group();

    // wave sums of the per-lane counters
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        cnt_max += __shfl_xor(cnt_max, d, 64);
        trans0 += __shfl_xor(trans0, d, 64);
    }
    if (lane == 0) {
        ChunkSum r;
        r.len = e - s;
        r.prefix = prefix;
        r.first_up = first_up;
        r.end_up = gcarry;
        r.cnt_max = cnt_max;
        r.trans0 = trans0;
        r.ticks_high = th;
        r.pad = 0;
        sums[g] = r;
        if constexpr (kLevels) {
            fix[g].start = tbase + s;
            fix[g].prefix = prefix;
        }
    }
}

// One wave per chunk.
template <bool kLevels, bool kAnyBase>
__global__ __launch_bounds__(kChunkWavesPerBlock * kWave) void chunk_kernel(
    const uint32_t* __restrict__ samples, const uint64_t* __restrict__ offsets,
    uint32_t n_traces, const uint32_t* __restrict__ chunk_base,
    const DevCfg* __restrict__ cfgs, const uint32_t* __restrict__ cfg_of_trace,
    uint32_t chunk, ChunkSum* __restrict__ sums, ChunkFix* __restrict__ fix,
    uint8_t* __restrict__ levels)
{
    const uint32_t g = blockIdx.x * kChunkWavesPerBlock + uniform(threadIdx.x >> 6);
    if (g >= chunk_base[n_traces]) return;
    replay_chunk<kLevels, kAnyBase>(samples, offsets, n_traces, chunk_base, cfgs, cfg_of_trace,
                                    chunk, sums, fix, levels, g, threadIdx.x & 63);
}

// Persistent grid: wave w of a grid of W waves replays chunks w, w + W,
// w + 2W, ... in order.  The chunk index is a wave-uniform scalar computed
// from the grid shape alone, so the loop and its exit are scalar branches
// (every lane runs the same iterations) and no counter is shared.
template <bool kLevels, bool kAnyBase>
__global__ __launch_bounds__(kChunkWavesPerBlock * kWave) void chunk_kernel_persistent(
    const uint32_t* __restrict__ samples, const uint64_t* __restrict__ offsets,
    uint32_t n_traces, const uint32_t* __restrict__ chunk_base,
    const DevCfg* __restrict__ cfgs, const uint32_t* __restrict__ cfg_of_trace,
    uint32_t chunk, ChunkSum* __restrict__ sums, ChunkFix* __restrict__ fix,
    uint8_t* __restrict__ levels)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t total = uniform(chunk_base[n_traces]);
    const uint32_t stride = gridDim.x * kChunkWavesPerBlock;
    for (uint32_t g = blockIdx.x * kChunkWavesPerBlock + uniform(threadIdx.x >> 6); g < total;
         g += stride)
        replay_chunk<kLevels, kAnyBase>(samples, offsets, n_traces, chunk_base, cfgs,
                                        cfg_of_trace, chunk, sums, fix, levels, g, lane);
}

}  // namespace

hipError_t launch_replay(const uint32_t* samples, uint64_t n_samples, const uint64_t* offsets,
                         uint32_t n_traces, const DevCfg* cfgs, uint32_t n_cfgs,
                         const uint32_t* cfg_of_trace, uint32_t chunk, uint32_t* chunk_base,
                         ChunkSum* sums, uint32_t max_chunks, ChunkFix* fix,
                         magus_result* results, uint8_t* levels, uint32_t* err,
                         uint32_t persistent_blocks, bool any_base, hipStream_t stream,
                         hipEvent_t ev0, hipEvent_t ev1, uint32_t* status_out)
{
    if (n_traces == 0) return hipSuccess;
    (void)launch_plan(offsets, n_traces, n_samples, cfg_of_trace, n_cfgs, chunk, max_chunks,
                      chunk_base, err, stream, status_out);
    uint32_t blocks = (max_chunks + kChunkWavesPerBlock - 1) / kChunkWavesPerBlock;
    if (hipError_t e = record_timing_event(ev0, stream); e != hipSuccess) return e;
    auto go = [&](auto levels_tag, auto base_tag) {
        constexpr bool kL = decltype(levels_tag)::value, kB = decltype(base_tag)::value;
        ChunkFix* f = kL ? fix : nullptr;
        uint8_t* lv = kL ? levels : nullptr;
        if (persistent_blocks)
            chunk_kernel_persistent<kL, kB>
                <<<min(blocks, persistent_blocks), kChunkWavesPerBlock * kWave, 0, stream>>>(
                    samples, offsets, n_traces, chunk_base, cfgs, cfg_of_trace, chunk, sums, f, lv);
        else
            chunk_kernel<kL, kB><<<blocks, kChunkWavesPerBlock * kWave, 0, stream>>>(
                samples, offsets, n_traces, chunk_base, cfgs, cfg_of_trace, chunk, sums, f, lv);
    };
    if (blocks) {
        if (levels) {
            if (any_base) go(std::true_type{}, std::true_type{});
            else go(std::true_type{}, std::false_type{});
        } else {
            if (any_base) go(std::false_type{}, std::true_type{});
            else go(std::false_type{}, std::false_type{});
        }
    }
    if (hipError_t e = record_timing_event(ev1, stream); e != hipSuccess) return e;
    (void)launch_fold(offsets, n_traces, chunk_base, sums, cfgs, cfg_of_trace, results,
                      levels ? fix : nullptr, stream);
    if (levels && blocks)
        (void)launch_fixup(n_traces, chunk_base, fix, max_chunks, levels, stream);
    return hipGetLastError();
}

}  // namespace magus
