// Replay with stepped actuation on gfx950.
//
// With up_step / down_step > 0 an executed +1 / -1 moves the level by that
// many rungs (clamped to [level_min, level_max]) instead of jumping to the
// bound, so the level after a step depends on the level before it through a
// clamp-add map f(x) = min(max(x + a, lo), hi):
//   high            -> constant level_max        (a = 0,  lo = hi = max)
//   +1, step u      -> x + u clamped              (a = u,  lo = min, hi = max)
//   -1, step d      -> x - d clamped              (a = -d, lo = min, hi = max)
//   +1 / -1, step 0 -> constant max / min
//   otherwise       -> identity                   (a = 0,  lo = min, hi = max)
// Clamp-add maps are closed under composition (see compose()), so a time
// chunk has one map.  Pass 1 composes each chunk's map with a wave-wide tree
// over the 64 steps of every block; a per-trace fold applies the maps in order
// to find the level entering every chunk; pass 2 replays each chunk again with
// its entering level, turning the per-step maps into levels with a wave-wide
// inclusive scan, and accumulates the level sum and transitions.

#include "block_masks.h"

namespace magus {
namespace {

constexpr int kWaves = 4;

__device__ __forceinline__ uint32_t wave_uniform(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// g after f.  g(f(x)) = clamp(clamp(x + f.a, f.lo, f.hi) + g.a, g.lo, g.hi)
// = clamp(x + f.a + g.a, L, H): clamping into [A, B] = [f.lo+g.a, f.hi+g.a]
// and then into [g.lo, g.hi] is one clamp into [min(max(A, g.lo), g.hi),
// max(min(B, g.hi), g.lo)] (a single point when the intervals do not meet).
__device__ __forceinline__ ClampAdd compose(const ClampAdd& f, const ClampAdd& g) {
    const int32_t A = f.lo + g.a, B = f.hi + g.a;
    ClampAdd r;
    r.a = f.a + g.a;
    r.lo = min(max(A, g.lo), g.hi);
    r.hi = max(min(B, g.hi), g.lo);
    return r;
}

__device__ __forceinline__ int32_t apply(const ClampAdd& f, int32_t x) {
    return min(max(x + f.a, f.lo), f.hi);
}

// The map of this lane's step from the block masks.
__device__ __forceinline__ ClampAdd step_map(const BlockMasks& m, const DevCfg& c,
                                             uint32_t lane) {
    const int32_t lmin = c.lmin, lmax = c.lmax;
    ClampAdd f{0, lmin, lmax};
    const bool high = (m.HM >> lane) & 1ull;
    const bool ev = (m.E >> lane) & 1ull;
    const bool up = (m.R >> lane) & 1ull;
    if (high) {
        f = ClampAdd{0, lmax, lmax};
    } else if (ev && up) {
        f = c.up ? ClampAdd{(int32_t)c.up, lmin, lmax} : ClampAdd{0, lmax, lmax};
    } else if (ev) {
        f = c.down ? ClampAdd{-(int32_t)c.down, lmin, lmax} : ClampAdd{0, lmin, lmin};
    }
    return f;
}

// Pass 1: the clamp-add map of every chunk.
__global__ __launch_bounds__(kWaves * kWave) void stepped_map_kernel(
    const uint32_t* __restrict__ samples, const uint64_t* __restrict__ offsets,
    uint32_t n_traces, const uint32_t* __restrict__ chunk_base,
    const DevCfg* __restrict__ cfgs, const uint32_t* __restrict__ cfg_of_trace,
    uint32_t chunk, ClampAdd* __restrict__ funcs)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t g = blockIdx.x * kWaves + wave_uniform(threadIdx.x >> 6);
    if (g >= chunk_base[n_traces]) return;
    const ChunkView v = chunk_view(samples, offsets, n_traces, chunk_base, cfgs, cfg_of_trace,
                                   chunk, g);
    ClampAdd F{0, (int32_t)v.c.lmin, (int32_t)v.c.lmax};      // identity
    for_each_block(v, lane, [&](const BlockMasks& m, uint32_t, uint64_t, uint32_t) {
        if (((m.E | m.HM)) == 0) return;                        // 64 identity steps
        ClampAdd f = step_map(m, v.c, lane);
        // ordered tree: lane i composes the map of lanes [i, i + 2k) (k doubling)
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            ClampAdd o;
            o.a = __shfl_down(f.a, d, 64);
            o.lo = __shfl_down(f.lo, d, 64);
            o.hi = __shfl_down(f.hi, d, 64);
            if (lane + d < 64) f = compose(f, o);
        }
        ClampAdd blk;
        blk.a = __builtin_amdgcn_readfirstlane(f.a);
        blk.lo = __builtin_amdgcn_readfirstlane(f.lo);
        blk.hi = __builtin_amdgcn_readfirstlane(f.hi);
        F = compose(F, blk);
    });
    if (lane == 0) funcs[g] = F;
}

// Fold 1: the level entering every chunk.
__global__ __launch_bounds__(256) void stepped_enter_kernel(
    uint32_t n_traces, const uint32_t* __restrict__ chunk_base,
    const DevCfg* __restrict__ cfgs, const uint32_t* __restrict__ cfg_of_trace,
    const ClampAdd* __restrict__ funcs, uint32_t* __restrict__ entering)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_traces || chunk_base[n_traces + 1] != 0) return;
    int32_t x = cfgs[cfg_of_trace ? cfg_of_trace[t] : 0].linit;
    for (uint32_t k = chunk_base[t]; k < chunk_base[t + 1]; ++k) {
        entering[k] = (uint32_t)x;
        x = apply(funcs[k], x);
    }
}

// Pass 2: levels, sums and (optionally) decision bytes of every chunk.
template <bool kLevels>
__global__ __launch_bounds__(kWaves * kWave) void stepped_sum_kernel(
    const uint32_t* __restrict__ samples, const uint64_t* __restrict__ offsets,
    uint32_t n_traces, const uint32_t* __restrict__ chunk_base,
    const DevCfg* __restrict__ cfgs, const uint32_t* __restrict__ cfg_of_trace,
    uint32_t chunk, const uint32_t* __restrict__ entering, StepSum* __restrict__ sums,
    uint8_t* __restrict__ levels)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t g = blockIdx.x * kWaves + wave_uniform(threadIdx.x >> 6);
    if (g >= chunk_base[n_traces]) return;
    const ChunkView v = chunk_view(samples, offsets, n_traces, chunk_base, cfgs, cfg_of_trace,
                                   chunk, g);
    int32_t x = (int32_t)entering[g];                 // level before the block
    uint64_t lsum = 0;                                 // per lane
    uint32_t trans = 0, th = 0;
    for_each_block(v, lane, [&](const BlockMasks& m, uint32_t tb, uint64_t valid, uint32_t) {
        int32_t lv;
        if (((m.E | m.HM)) == 0) {
            lv = x;                                    // 64 identity steps
        } else {
            ClampAdd f = step_map(m, v.c, lane);
            // inclusive scan: lane i gets the map of steps 0..i of the block
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                ClampAdd o;
                o.a = __shfl_up(f.a, d, 64);
                o.lo = __shfl_up(f.lo, d, 64);
                o.hi = __shfl_up(f.hi, d, 64);
                if (lane >= (uint32_t)d) f = compose(o, f);
            }
            lv = apply(f, x);
        }
        int32_t before = __shfl_up(lv, 1, 64);
        if (lane == 0) before = x;
        const bool ok = (valid >> lane) & 1ull;
        if (ok) {
            lsum += (uint32_t)lv;
            trans += lv != before;
        }
        th += (uint32_t)__popcll(m.HM);
        if constexpr (kLevels) {
            if (ok) {
                const bool hb = (m.HM >> lane) & 1ull;
                const bool ev = (m.E >> lane) & 1ull;
                const bool up = (m.R >> lane) & 1ull;
                const uint32_t pr = ev ? (up ? 2u : 0u) : 1u;
                levels[v.tbase + tb + lane] = (uint8_t)((uint32_t)lv | ((uint32_t)hb << 5) |
                                                        (pr << 6));
            }
        }
        const uint32_t last = min(64u, v.e - tb) - 1;
        x = __builtin_amdgcn_readlane(lv, (int)last);
    });
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        lsum += __shfl_xor(lsum, d, 64);
        trans += __shfl_xor(trans, d, 64);
    }
    if (lane == 0) {
        StepSum r;
        r.level_sum = lsum;
        r.transitions = trans;
        r.ticks_high = th;
        sums[g] = r;
    }
}

__global__ __launch_bounds__(256) void stepped_fold_kernel(
    uint32_t n_traces, const uint32_t* __restrict__ chunk_base,
    const StepSum* __restrict__ sums, magus_result* __restrict__ results)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_traces || chunk_base[n_traces + 1] != 0) return;
    uint64_t level_sum = 0, trans = 0, th = 0;
    for (uint32_t k = chunk_base[t]; k < chunk_base[t + 1]; ++k) {
        level_sum += sums[k].level_sum;
        trans += sums[k].transitions;
        th += sums[k].ticks_high;
    }
    magus_result r;
    r.score = level_sum + 1000ull * trans;
    r.level_sum = level_sum;
    r.transitions = trans;
    r.ticks_high = th;
    results[t] = r;
}

}  // namespace

hipError_t launch_replay_stepped(const uint32_t* samples, uint64_t n_samples,
                                 const uint64_t* offsets, uint32_t n_traces, const DevCfg* cfgs,
                                 uint32_t n_cfgs, const uint32_t* cfg_of_trace, uint32_t chunk,
                                 uint32_t* chunk_base, uint32_t max_chunks, ClampAdd* funcs,
                                 uint32_t* entering, StepSum* sums, magus_result* results,
                                 uint8_t* levels, uint32_t* err, hipStream_t stream,
                                 hipEvent_t ev0, hipEvent_t ev1)
{
    if (n_traces == 0) return hipSuccess;
    hipError_t e = launch_plan(offsets, n_traces, n_samples, cfg_of_trace, n_cfgs, chunk,
                               max_chunks, chunk_base, err, stream);
    if (e != hipSuccess) return e;
    const uint32_t blocks = (max_chunks + kWaves - 1) / kWaves;
    if (ev0) (void)hipEventRecord(ev0, stream);
    stepped_map_kernel<<<blocks, kWaves * kWave, 0, stream>>>(
        samples, offsets, n_traces, chunk_base, cfgs, cfg_of_trace, chunk, funcs);
    stepped_enter_kernel<<<(n_traces + 255) / 256, 256, 0, stream>>>(
        n_traces, chunk_base, cfgs, cfg_of_trace, funcs, entering);
    if (levels)
        stepped_sum_kernel<true><<<blocks, kWaves * kWave, 0, stream>>>(
            samples, offsets, n_traces, chunk_base, cfgs, cfg_of_trace, chunk, entering, sums,
            levels);
    else
        stepped_sum_kernel<false><<<blocks, kWaves * kWave, 0, stream>>>(
            samples, offsets, n_traces, chunk_base, cfgs, cfg_of_trace, chunk, entering, sums,
            nullptr);
    if (ev1) (void)hipEventRecord(ev1, stream);
    stepped_fold_kernel<<<(n_traces + 255) / 256, 256, 0, stream>>>(n_traces, chunk_base, sums,
                                                                    results);
    return hipGetLastError();
}

}  // namespace magus
