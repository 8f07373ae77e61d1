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

// Inclusive wave scan (sum) with DPP: prefix sums within each row of 16
// lanes, then the last lane of row 0 / of rows 0-1 is added into the rows
// after it.  Lanes outside a row's shifted range read 0.
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);   // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

__device__ __forceinline__ uint64_t low_mask(uint32_t n) {   // n in [0, 64]
    return n >= 64 ? ~0ull : ((1ull << n) - 1ull);
}

// ------------------------------------------------------------------ plan

__global__ __launch_bounds__(kPlanThreads) void plan_kernel(
    const uint64_t* __restrict__ offsets, uint32_t n_traces, uint64_t n_samples,
    const uint32_t* __restrict__ cfg_of_trace, uint32_t n_cfgs, uint32_t chunk,
    uint32_t max_chunks, uint32_t* __restrict__ chunk_base, uint32_t* __restrict__ err,
    uint32_t* __restrict__ status_out)
{
    // Rows of 1,024 consecutive traces; thread i takes trace i of every row,
    // so each load and store of a row is coalesced.  Up to kRows rows (a
    // "band") are counted at once with their counts in registers; a wave scan
    // per row and one exchange of wave totals through LDS place them, and the
    // band's total carries into the next band.
    constexpr uint32_t kRows = 16;
    constexpr uint32_t kPlanWaves = kPlanThreads / kWave;
    __shared__ uint32_t wave_pre[kRows][kPlanWaves];   // wave totals, then bases
    __shared__ uint32_t band_total;
    __shared__ uint32_t s_err;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0) s_err = 0;
    // a power-of-two chunk (the usual case) divides with a shift
    const uint32_t chunk_shift = (chunk & (chunk - 1)) == 0 ? 31u - __builtin_clz(chunk) : 32u;
    // chunks of a trace from its offsets and config index, with the checks
    auto count = [&](uint64_t o0, uint64_t o1, uint32_t cfg, uint32_t& e) -> uint32_t {
        if (cfg >= n_cfgs) e |= kErrCfgIndex;
        const bool bad = o1 < o0 || o1 > n_samples;
        const bool too_long = !bad && o1 - o0 > MAGUS_MAX_TRACE_LEN;
        e |= (bad ? kErrOffsets : 0u) | (too_long ? kErrTooLong : 0u);
        const uint32_t len = bad || too_long ? 0u : (uint32_t)(o1 - o0) + chunk - 1;
        return chunk_shift < 32 ? len >> chunk_shift : len / chunk;
    };
    uint32_t e = 0, carry = 0;
    for (uint32_t band = 0; band < n_traces; band += kRows * kPlanThreads) {
        // all loads of the band first (an index past the end reads the last
        // trace again), then the counts
        uint64_t o0[kRows], o1[kRows];
        uint32_t cf[kRows];
#pragma unroll
        for (uint32_t r = 0; r < kRows; ++r) {
            const uint32_t row = band + r * kPlanThreads;   // uniform
            o0[r] = o1[r] = 0;
            cf[r] = 0;
            if (row < n_traces) {
                const uint32_t t = min(row + tid, n_traces - 1);
                o0[r] = offsets[t];
                o1[r] = offsets[t + 1];
                if (cfg_of_trace) cf[r] = cfg_of_trace[t];
            }
        }
        uint32_t excl[kRows];           // chunks of this row before the trace
#pragma unroll
        for (uint32_t r = 0; r < kRows; ++r)
            excl[r] = band + r * kPlanThreads + tid < n_traces ? count(o0[r], o1[r], cf[r], e)
                                                               : 0u;
#pragma unroll
        for (uint32_t r = 0; r < kRows; ++r) {
            const uint32_t c = excl[r];
            uint32_t v = c;
            if (band + r * kPlanThreads < n_traces) v = wave_inclusive_sum(v);
            excl[r] = v - c;
            if (lane == 63) wave_pre[r][wv] = v;
        }
        __syncthreads();
        if (wv == 0) {
            // lane r: exclusive prefix of row r's wave totals, then the rows
            uint32_t row_total = 0;
            if (lane < kRows)
                for (uint32_t w = 0; w < kPlanWaves; ++w) row_total += wave_pre[lane][w];
            uint32_t x = lane < kRows ? row_total : 0u;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t o = __shfl_up(x, d, 64);
                if (lane >= (uint32_t)d) x += o;
            }
            if (lane < kRows) {
                uint32_t run = carry + x - row_total;
                for (uint32_t w = 0; w < kPlanWaves; ++w) {
                    const uint32_t tot = wave_pre[lane][w];
                    wave_pre[lane][w] = run;
                    run += tot;
                }
            }
            if (lane == kRows - 1) band_total = x;
        }
        __syncthreads();
#pragma unroll
        for (uint32_t r = 0; r < kRows; ++r) {
            const uint32_t row = band + r * kPlanThreads;
            if (row < n_traces && row + tid < n_traces)
                chunk_base[row + tid] = wave_pre[r][wv] + excl[r];
        }
        carry += band_total;
        __syncthreads();                 // wave_pre and band_total are reused
    }
    if (e) atomicOr(&s_err, e);
    __syncthreads();
    if (tid == 0) {
        uint32_t ee = s_err;
        if (carry > max_chunks) ee |= kErrOffsets;
        chunk_base[n_traces] = ee ? 0u : carry;
        chunk_base[n_traces + 1] = ee;           // status of this call
        if (ee && err) atomicOr(err, ee);        // sticky word of a context
        if (status_out) *status_out = ee;        // the caller's copy of the status
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
    if (t >= n_traces) return;
    // the status, the chunk range and the config index load together
    const uint32_t status = chunk_base[n_traces + 1];
    const uint32_t k0 = chunk_base[t], k1 = chunk_base[t + 1];
    const uint32_t ci = cfg_of_trace ? cfg_of_trace[t] : 0;
    if (status != 0) return;
    const DevCfg c = cfgs[ci];
    const uint64_t lmin = c.lmin, lmax = c.lmax;
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
                       hipStream_t stream, uint32_t* status_out)
{
    plan_kernel<<<1, kPlanThreads, 0, stream>>>(offsets, n_traces, n_samples, cfg_of_trace,
                                                n_cfgs, chunk, max_chunks, chunk_base, err,
                                                status_out);
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
