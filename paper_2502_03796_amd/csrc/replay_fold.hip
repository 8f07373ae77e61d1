// Plan, fold and fix-up kernels around the replay chunk kernel (replay.hip).
//
//   plan    one workgroup: prefix sum of the chunks of every trace, data checks
//           (offsets, trace length, config index) and the per-call status word
//   fold    one wave per trace: composes the trace's chunk summaries in order
//   fixup   (decision bytes only) writes the entering level into the steps
//           before the first decisive step of each chunk

#include "magus_internal.h"

namespace magus {
namespace {

constexpr int kPlanThreads = 1024;

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t uniform(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ uint64_t low_mask(uint32_t n) {   // n in [0, 64]
    return n >= 64 ? ~0ull : ((1ull << n) - 1ull);
}

// ------------------------------------------------------------------ plan

__global__ __launch_bounds__(kPlanThreads) void plan_kernel(
    const uint64_t* __restrict__ offsets, uint32_t n_traces, uint64_t n_samples,
    const uint32_t* __restrict__ cfg_of_trace, uint32_t n_cfgs, uint32_t chunk,
    uint32_t max_chunks, uint32_t* __restrict__ chunk_base, uint32_t* __restrict__ err)
{
    // Thread i owns the contiguous traces [i*per, (i+1)*per): one pass counts
    // their chunks, one block-wide scan places them, a second pass writes.
    // Up to kCache traces per thread (8,192 traces) the offsets are loaded
    // once, all at the same time, and the counts stay in registers.
    constexpr uint32_t kCache = 8;
    __shared__ uint32_t wave_sum[kPlanThreads / kWave];
    __shared__ uint32_t s_err;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0) s_err = 0;
    const uint32_t per = (n_traces + kPlanThreads - 1) / kPlanThreads;
    const uint32_t t0 = min(tid * per, n_traces), t1 = min(t0 + per, n_traces);
    auto count = [&](uint32_t t, uint64_t o0, uint64_t o1, uint32_t& e) -> uint32_t {
        if (cfg_of_trace && cfg_of_trace[t] >= n_cfgs) e |= kErrCfgIndex;
        if (o1 < o0 || o1 > n_samples) {
            e |= kErrOffsets;
            return 0;
        }
        if (o1 - o0 > MAGUS_MAX_TRACE_LEN) {
            e |= kErrTooLong;
            return 0;
        }
        return ((uint32_t)(o1 - o0) + chunk - 1) / chunk;   // both below 2^31
    };
    const bool cached = per <= kCache;
    uint32_t cnt[kCache];
    uint32_t e = 0, mine = 0;
    if (cached) {
        uint64_t o[kCache + 1];
#pragma unroll
        for (uint32_t k = 0; k <= kCache; ++k) o[k] = t0 + k <= t1 ? offsets[t0 + k] : 0;
#pragma unroll
        for (uint32_t k = 0; k < kCache; ++k) {
            cnt[k] = t0 + k < t1 ? count(t0 + k, o[k], o[k + 1], e) : 0u;
            mine += cnt[k];
        }
    } else {
        for (uint32_t t = t0; t < t1; ++t) mine += count(t, offsets[t], offsets[t + 1], e);
    }
    __syncthreads();
    if (e) atomicOr(&s_err, e);
    // exclusive scan of `mine` over the block
    uint32_t v = mine;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(v, d, 64);
        if (lane >= (uint32_t)d) v += o;
    }
    if (lane == 63) wave_sum[wv] = v;
    __syncthreads();
    if (wv == 0) {
        uint32_t w = lane < kPlanThreads / kWave ? wave_sum[lane] : 0;
#pragma unroll
        for (int d = 1; d < kPlanThreads / kWave; d <<= 1) {
            const uint32_t o = __shfl_up(w, d, 64);
            if (lane >= (uint32_t)d) w += o;
        }
        if (lane < kPlanThreads / kWave) wave_sum[lane] = w;   // inclusive
    }
    __syncthreads();
    uint32_t run = (wv ? wave_sum[wv - 1] : 0) + v - mine;
    if (cached) {
#pragma unroll
        for (uint32_t k = 0; k < kCache; ++k)
            if (t0 + k < t1) {
                chunk_base[t0 + k] = run;
                run += cnt[k];
            }
    } else {
        for (uint32_t t = t0; t < t1; ++t) {
            uint32_t dummy = 0;
            chunk_base[t] = run;
            run += count(t, offsets[t], offsets[t + 1], dummy);
        }
    }
    if (tid == kPlanThreads - 1) {
        const uint32_t total = wave_sum[kPlanThreads / kWave - 1];
        uint32_t ee = s_err;
        if (total > max_chunks) ee |= kErrOffsets;
        chunk_base[n_traces] = ee ? 0u : total;
        chunk_base[n_traces + 1] = ee;           // status of this call
        if (ee) atomicOr(err, ee);
    }
}

// ------------------------------------------------------------------ fold

// One wave per trace; lane j takes chunk j of each group of 64 chunks.  With
// jump-to-bound actuation the level entering chunk j is the end level of the
// last earlier chunk that has a decisive step (else the level entering the
// group), so a ballot and a lane shuffle give every lane its entering level,
// and the per-chunk contributions are summed across the wave.
constexpr int kFoldWaves = 4;

__global__ __launch_bounds__(kFoldWaves * kWave) void fold_kernel(
    const uint64_t* __restrict__ offsets, uint32_t n_traces,
    const uint32_t* __restrict__ chunk_base, const ChunkSum* __restrict__ sums,
    const DevCfg* __restrict__ cfgs, const uint32_t* __restrict__ cfg_of_trace,
    magus_result* __restrict__ results, ChunkFix* __restrict__ fix)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t t = blockIdx.x * kFoldWaves + uniform(threadIdx.x >> 6);
    if (t >= n_traces || chunk_base[n_traces + 1] != 0) return;
    const DevCfg c = cfgs[cfg_of_trace ? cfg_of_trace[t] : 0];
    const uint64_t lmin = c.lmin, lmax = c.lmax;
    const uint32_t k0 = chunk_base[t], k1 = chunk_base[t + 1];
    uint64_t level = c.linit;                 // level entering the current group
    uint64_t level_sum = 0, trans = 0, th = 0;
    for (uint32_t kb = k0; kb < k1; kb += 64) {
        const uint32_t k = kb + lane;
        const bool valid = k < k1;
        ChunkSum S{};
        if (valid) S = sums[k];
        const bool dec = valid && S.prefix < S.len;
        const uint64_t E = ballot(dec);
        const uint64_t end_level = S.end_up ? lmax : lmin;
        // entering level: end level of the highest earlier lane with a
        // decisive step, else the group's entering level
        const uint64_t before = E & low_mask(lane);
        const int src = before ? 63 - __builtin_clzll(before) : (int)lane;
        const uint64_t from_src = (uint64_t)__shfl((int)end_level, src, 64);
        const uint64_t lin = before ? from_src : level;
        if (valid) {
            if (fix) fix[k].level = (uint32_t)lin;
            if (!dec) {
                level_sum += lin * S.len;
            } else {
                const uint64_t first = S.first_up ? lmax : lmin;
                level_sum += lin * S.prefix + lmax * S.cnt_max +
                             lmin * (S.len - S.prefix - S.cnt_max);
                trans += S.trans0 - S.first_up + (first != lin);
            }
            th += S.ticks_high;
        }
        if (E) level = (uint64_t)__shfl((int)end_level, 63 - __builtin_clzll(E), 64);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        level_sum += ((uint64_t)__shfl_xor((int)(level_sum >> 32), d, 64) << 32) |
                     (uint32_t)__shfl_xor((int)(uint32_t)level_sum, d, 64);
        trans += (uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)trans, d, 64);
        th += (uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)th, d, 64);
    }
    if (lane == 0) {
        magus_result r;
        r.score = level_sum + 1000ull * trans;
        r.level_sum = level_sum;
        r.transitions = trans;
        r.ticks_high = th;
        results[t] = r;
    }
}

// ------------------------------------------------------------------ fixup

__global__ __launch_bounds__(256) void fixup_kernel(
    uint32_t n_traces, const uint32_t* __restrict__ chunk_base,
    const ChunkFix* __restrict__ fix, uint8_t* __restrict__ levels)
{
    if (chunk_base[n_traces + 1] != 0) return;
    const uint32_t total = chunk_base[n_traces];
    for (uint32_t k = blockIdx.x; k < total; k += gridDim.x) {
        const ChunkFix f = fix[k];
        for (uint32_t i = threadIdx.x; i < f.prefix; i += blockDim.x) {
            uint8_t* p = levels + f.start + i;
            *p = (uint8_t)((*p & 0xE0u) | f.level);
        }
    }
}

}  // namespace

hipError_t launch_plan(const uint64_t* offsets, uint32_t n_traces, uint64_t n_samples,
                       const uint32_t* cfg_of_trace, uint32_t n_cfgs, uint32_t chunk,
                       uint32_t max_chunks, uint32_t* chunk_base, uint32_t* err,
                       hipStream_t stream)
{
    plan_kernel<<<1, kPlanThreads, 0, stream>>>(offsets, n_traces, n_samples, cfg_of_trace,
                                                n_cfgs, chunk, max_chunks, chunk_base, err);
    return hipGetLastError();
}

hipError_t launch_fold(const uint64_t* offsets, uint32_t n_traces, const uint32_t* chunk_base,
                       const ChunkSum* sums, const DevCfg* cfgs, const uint32_t* cfg_of_trace,
                       magus_result* results, ChunkFix* fix, hipStream_t stream)
{
    fold_kernel<<<(n_traces + kFoldWaves - 1) / kFoldWaves, kFoldWaves * kWave, 0, stream>>>(
        offsets, n_traces, chunk_base, sums, cfgs, cfg_of_trace, results, fix);
    return hipGetLastError();
}

hipError_t launch_fixup(uint32_t n_traces, const uint32_t* chunk_base, const ChunkFix* fix,
                        uint32_t max_chunks, uint8_t* levels, hipStream_t stream)
{
    fixup_kernel<<<std::min(max_chunks, 65535u), 256, 0, stream>>>(n_traces, chunk_base, fix,
                                                                    levels);
    return hipGetLastError();
}

}  // namespace magus
