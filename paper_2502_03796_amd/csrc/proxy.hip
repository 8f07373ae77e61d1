// Proxy energy / EDP model over replays on gfx950.
//
// Sec. 5.4 judges an uncore policy by performance loss, package power saving,
// energy saving and EDP against the default of Sec. 5.3 (uncore at its
// maximum).  With no power or performance model in the paper, this file
// evaluates a stated proxy from the per-step levels of a replay:
//   - interval t runs at the level set after step t-1 (level_init for t = 0);
//   - at level i the uncore sustains cap[i] MB/s and an interval whose sample x
//     exceeds that is stretched to interval * x / cap[i];
//   - package power core + uncore[i] and GPU power are held over the interval.
// Everything the metrics need is a handful of exact integer sums per trace:
// per level, the intervals run there and the sum of max(0, x - cap[level]);
// for the two static policies the same excess sums at level_max / level_min.
//
// Configs that jump to the bound (the paper's rule) take a fused pass that
// reads each sample once: per chunk, the level before every step follows from
// the chunk's own decisive steps except for the steps up to the first of them,
// whose interval runs at the level entering the chunk; those are summed at each
// of the three possible entering levels and a per-trace fold picks one.
//   plan        (replay_fold.hip) chunk prefix and data checks
//   fused chunk one wave per chunk: Alg. 1 / Alg. 2 per 64-step block, the
//               block's level bits from the carries of ~DN + UP + level, the
//               excess sums per level in 32 bits -> ProxySum; a chunk with a
//               sample of 2^24 or more is queued
//   exact       the queued chunks again in 64-bit sums (none on real traces)
//   fused fold  one wave per trace -> magus_proxy_stats, and the trace's
//               metrics from the same sums; empties the queue
// Stepped configs take the path over the stepped replay's pass 1 (its step
// masks and the level entering every chunk, stepped.hip):
//   zero     clears the statistics and the queue (no memset node, so the
//            sequence can be captured into a graph)
//   stepped  one wave per chunk: reads the samples and the step masks, walks
//            the level through each block in scalar registers from the chunk's
//            entering level (or takes it from raise / lower counts when no
//            move in the block is clamped), and sums per level: a block at one
//            level adds to a run at that level (per lane); a block whose level
//            changes adds each step's excess and interval to its lane's word
//            of its level's bins in LDS; a chunk with a sample of 2^22 or more
//            is queued
//   wide     the queued chunks: scans a changing block's per-step excess once
//            and takes each segment's sum from the scan at the segment's ends
//            (64-bit); one atomic add per non-zero sum per chunk in both
//   metrics  one wave per trace: the seven figures of each policy in FP64

#include "block_masks.h"
#include "proxy_internal.h"

namespace magus {
namespace {

static_assert(sizeof(magus_proxy_model) == 8 + 4 * 64 + 8, "magus_proxy_model layout");
static_assert(sizeof(magus_proxy_stats) == 16 + 8 * 64, "magus_proxy_stats layout");
static_assert(sizeof(magus_proxy_metrics) == 7 * 3 * 8, "magus_proxy_metrics layout");

constexpr int kStatsWaves = 4;
constexpr uint32_t kNarrowBound = 1u << 24;      // samples and thresholds below: narrow passes
constexpr uint32_t kNarrowChunk = 256 * 64;      // steps per chunk the narrow sums allow

__device__ __forceinline__ uint32_t uniform(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ uint32_t over(uint32_t x, uint32_t cap) { return x > cap ? x - cap : 0u; }

// Inclusive wave scan with DPP: row shifts build the scan within each row of
// 16 lanes, row broadcasts carry the totals of the rows before.
__device__ __forceinline__ uint32_t dpp_scan(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);   // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// a in the lanes whose bit of the wave-uniform mask is set, else b
__device__ __forceinline__ uint32_t lane_pick(uint64_t mask, uint32_t a, uint32_t b) {
    const uint64_t m = ((uint64_t)uniform((uint32_t)(mask >> 32)) << 32) | uniform((uint32_t)mask);
    uint32_t r;
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(r) : "v"(b), "v"(a), "s"(m));
    return r;
}

// Adds v to a word of LDS with no value returned (ds_add_u32): no wait for
// the word's old value.
__device__ __forceinline__ void lds_add(uint32_t* p, uint32_t v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

constexpr uint32_t kStepGroup = 8;     // blocks loaded ahead by the stepped pass
constexpr uint32_t kBinLanes = 16;     // words of a narrow bin row (lane l adds to word l % 16)
constexpr uint32_t kBinStride = 17;    // ... and the row's stride in words

// LDS words of one wave's narrow bins for a level range of `levels` rungs:
// an excess row per level and a row of two 16-bit counts per two levels.
__host__ __device__ constexpr uint32_t stepped_bin_words(uint32_t levels) {
    return (levels + (levels + 1) / 2) * kBinStride;
}
// The narrow stepped pass: chunks of at most 16,320 steps whose samples are
// all below 2^22.  A bin word takes at most one step a block from each of 4
// lanes: at most 1,020 steps, whose excesses (below 2^22 each) sum below
// 2^32, and whose count fits 16 bits.
constexpr uint32_t kNarrowSteppedChunk = 255 * 64;
constexpr uint32_t kNarrowSteppedBound = 1u << 22;

// Statistics of stepped configs from the stepped replay's pass 1: one wave per
// chunk.  The level before every step follows from the chunk's entering level
// and the blocks' step masks (moves up by up_step, down by down_step, set to
// level_max, each clamped to the range); the interval of step i runs at the
// level before step i.  Lane l keeps the interval counts of level l.
//
// The excess sums take one of two forms.  The narrow pass (every sample of
// the chunk below 2^22 and at most 16,320 steps) keeps them in LDS bins: a
// row of 16 words per level of the config's range and a row of two 16-bit
// counts per two levels, lane l adding to word l % 16 with LDS atomic adds
// (4 lanes a word: at most 1,020 steps, whose excess sum fits 32 bits and
// whose count fits 16; a 17-rung range takes 26 rows of 17 words, 1.8 KB a
// wave, so registers alone set the occupancy).  A block that changes the
// level adds each step's excess at its own level, and its interval, to its
// lane's words of that level, and a run of blocks at one level is added
// when it ends, per lane, without a wave reduction; the rows are summed
// once per chunk.  It tracks the largest sample; a chunk with one of 2^22
// or more is run again by the wide pass, which keeps the sums per level in lane l (64-bit) and splits a
// block that changes the level into segments of equal level with two 16-bit
// scans.  (A lane-parallel scan of the steps' clamp-add maps in place of the
// scalar walk moved the issue load from the scalar to the vector unit and
// was slower: 470 us against 425 us on the bulk traces.)
template <bool kNarrow>
__device__ __forceinline__ bool stepped_stats_pass(
    const uint32_t* __restrict__ samples, const uint64_t* __restrict__ offsets,
    uint32_t n_traces, const uint32_t* __restrict__ chunk_base,
    const DevCfg* __restrict__ cfgs, const uint32_t* __restrict__ cfg_of_trace,
    uint32_t chunk, const uint32_t* __restrict__ entering,
    const uint64_t* __restrict__ masks, uint64_t n_blocks, const uint32_t* s_cap,
    uint32_t* xb, uint32_t* cb, magus_proxy_stats* __restrict__ stats, uint32_t g,
    uint32_t lane)
{
    using acc_t = std::conditional_t<kNarrow, uint32_t, uint64_t>;
    const uint32_t t = trace_of_chunk(chunk_base, n_traces, g, lane);
    const uint64_t tbase = offsets[t];
    const uint32_t n = (uint32_t)(offsets[t + 1] - tbase);
    const uint32_t s = (g - chunk_base[t]) * chunk;
    const uint32_t len = min(s + chunk, n) - s;
    const DevCfg c = cfgs[cfg_of_trace ? cfg_of_trace[t] : 0];
    const int32_t lmin = c.lmin, lmax = c.lmax;
    const int32_t up = c.up ? (int32_t)c.up : 64, down = c.down ? (int32_t)c.down : 64;
    const uint32_t cap_hi = s_cap[lmax], cap_lo = s_cap[lmin];
    const uint32_t rows = (uint32_t)(lmax - lmin + 1);
    const uint32_t bin_word = lane & (kBinLanes - 1);    // this lane's word of a bin row
    const uint64_t mb = first_block(tbase, s, t);
    const uint64_t* m_hs = masks + mb;
    const uint64_t* m_up = masks + n_blocks + mb;
    const uint64_t* m_dn = masks + 2 * n_blocks + mb;
    const uint32_t nblk = (len + 63) >> 6;
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(samples + tbase + s), (short)0, (int)(len * 4u), 0x00020000);

    if constexpr (kNarrow) {
        if (lane < kBinLanes) {
            for (uint32_t r = 0; r < rows; ++r) xb[r * kBinStride + lane] = 0;
            for (uint32_t r = 0; r < (rows + 1) / 2; ++r) cb[r * kBinStride + lane] = 0;
        }
        // the zeros are in place before any lane adds to a word
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    int32_t cur = (int32_t)uniform(entering[g]);         // level before the next step
    // the run: the steps since the level last changed, all at run_lv == cur
    // (outside a block's walk); their excess is summed per lane
    uint32_t run_lv = (uint32_t)cur, cap_run = s_cap[cur], run_n = 0;
    acc_t ex_max = 0, ex_min = 0, run_x = 0;             // per lane
    uint32_t vmax = 0;                                   // largest sample (narrow pass)
    uint64_t bin_n = 0, bin_x = 0;                       // lane l: level l
    auto credit_n = [&](uint32_t level, uint32_t steps) { bin_n += lane == level ? steps : 0u; };
    auto credit = [&](uint32_t level, uint32_t steps, uint64_t sum) {
        const bool mine = lane == level;
        bin_n += mine ? steps : 0u;
        bin_x += mine ? sum : 0ull;
    };
    // ends the run if the level changed and starts one at the new level
    auto follow_level = [&]() {
        if ((uint32_t)cur != run_lv) {
            if (run_n) {
                if constexpr (kNarrow) {
                    credit_n(run_lv, run_n);
                    lds_add(xb + (run_lv - lmin) * kBinStride + bin_word, run_x);
                } else {
                    credit(run_lv, run_n, dpp_wave_sum64(run_x));
                }
            }
            run_n = 0;
            run_x = 0;
            run_lv = (uint32_t)cur;
            cap_run = s_cap[cur];
        }
    };
    // the step masks of a span of 2 * kStepGroup blocks: lane j holds block
    // b0 + j's (vector loads, issued a span ahead)
    struct SpanMasks {
        uint64_t hs, up, dn;
    };
    auto load_masks = [&](uint32_t b0) -> SpanMasks {
        const uint32_t b = b0 + lane;
        SpanMasks m{0, 0, 0};
        if (lane < 2 * kStepGroup && b < nblk) {
            m.hs = m_hs[b];
            m.up = m_up[b];
            m.dn = m_dn[b];
        }
        return m;
    };
    auto lane_u64 = [](uint64_t v, uint32_t k) -> uint64_t {
        return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(v >> 32), (int)k) << 32) |
               (uint32_t)__builtin_amdgcn_readlane((int)v, (int)k);
    };
    const int32_t neg_down = -down;
    // a block of nv steps that holds a move (lane k of the span's masks)
    auto moving_block = [&](uint32_t k, uint32_t x, const SpanMasks& sm, uint32_t nv) {
        const uint64_t hs = lane_u64(sm.hs, k), mu = lane_u64(sm.up, k),
                       md = lane_u64(sm.dn, k);
        uint64_t moves = hs | mu | md;
        // the level before each step of the block: a move at step p that
        // changes the level sets it for the steps after p (bit p of `chg`)
        uint32_t lv = (uint32_t)cur;
        uint64_t chg = 0;
        if (hs == 0) {
            // no set to level_max: unless a move is clamped, the level before
            // step i is cur + up_step (raises before i) - down_step (lowers
            // before i), and every move changes it.  No move is clamped iff
            // every such partial sum, and the one after the block, lies in
            // the range; then the walk below is not needed.
            const int32_t li = cur + up * (int32_t)bits_below_lane(mu, 0) -
                               down * (int32_t)bits_below_lane(md, 0);
            const int32_t after = cur + up * __builtin_popcountll(mu) -
                                  down * __builtin_popcountll(md);
            if (after >= lmin && after <= lmax && !__ballot(li < lmin || li > lmax)) {
                lv = (uint32_t)li;
                chg = moves;
                cur = after;
                moves = 0;
            }
        }
        while (moves) {
            // p: the next move; d: its rung move (up_step, -down_step, or 64
            // for the set to level_max); the move leaves `moves`
            uint32_t p;
            int32_t d;
            asm("s_ff1_i32_b64 %0, %2\n\t"
                "s_bitcmp1_b64 %3, %0\n\t"
                "s_cselect_b32 %1, %5, %6\n\t"
                "s_bitcmp1_b64 %4, %0\n\t"
                "s_cselect_b32 %1, 64, %1\n\t"
                "s_bitset0_b64 %2, %0"
                : "=&s"(p), "=&s"(d), "+s"(moves)
                : "s"(mu), "s"(hs), "s"(up), "s"(neg_down)
                : "scc");
            const int32_t nl = min(max(cur + d, lmin), lmax);
            if (nl != cur) {
                lv = lane_pick(~1ull << p, (uint32_t)nl, lv);
                chg |= 1ull << p;
                cur = nl;
            }
        }
        // segments of steps at one level end at the changes before the
        // block's last step, and at its last step
        const uint64_t last = 1ull << (nv - 1);
        const uint64_t ends = (chg & (last - 1)) | last;
        if (ends == last) {
            // one level, the run's (a change at the last step only sets the
            // level of the next block)
            run_x += over(x, cap_run);
            run_n += nv;
        } else if constexpr (kNarrow) {
            // each step's excess at its own level into its lane's bin (0
            // past the end), and its interval into its lane's count
            const uint32_t r = lv - (uint32_t)lmin;
            lds_add(xb + r * kBinStride + bin_word, over(x, s_cap[lv]));
            if (lane < nv) lds_add(cb + (r >> 1) * kBinStride + bin_word, 1u << (16 * (r & 1)));
        } else {
            // the excess of each step at its own level (0 past the end),
            // scanned in 16-bit halves; a segment's sum is the difference of
            // the scans at its two ends
            const uint32_t e = over(x, s_cap[lv]);
            const uint32_t p_lo = dpp_scan(e & 0xFFFFu), p_hi = dpp_scan(e >> 16);
            uint32_t prev_lo = 0, prev_hi = 0, prev_end = 0;   // prev_end: first step
            uint64_t rest = ends;
            while (rest) {
                const uint32_t p = (uint32_t)__builtin_ctzll(rest);
                rest &= rest - 1;
                const uint32_t level = (uint32_t)__builtin_amdgcn_readlane((int)lv, (int)p);
                const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)p_lo, (int)p);
                const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)p_hi, (int)p);
                credit(level, p + 1 - prev_end,
                       ((uint64_t)(hi - prev_hi) << 16) + (lo - prev_lo));
                prev_lo = lo;
                prev_hi = hi;
                prev_end = p + 1;
            }
        }
        follow_level();
    };
    // groups of kStepGroup blocks; the next group's samples load while one
    // group is summed (loads past the chunk's end read 0), the next span's
    // masks while a span is summed
    auto load = [&](uint32_t b) -> uint32_t {
        return __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)((b * 64 + lane) * 4), 0,
                                                    kStreamLoad);
    };
    // a group of kStepGroup blocks starting at block b, lanes kb.. of the
    // span's masks; a block without a move adds to the run
    const uint32_t full = len >> 6;                      // blocks of 64 steps
    auto group = [&](uint32_t b, uint32_t kb, const uint32_t (&x)[kStepGroup],
                     const SpanMasks& sm, uint64_t moving) {
        const uint32_t gm = (uint32_t)(moving >> kb) & ((1u << kStepGroup) - 1);
#pragma unroll
        for (uint32_t k = 0; k < kStepGroup; ++k) {
            ex_max += over(x[k], cap_hi);                // lanes past the end read 0
            ex_min += over(x[k], cap_lo);
            if constexpr (kNarrow) vmax = max(vmax, x[k]);
        }
        if (b + kStepGroup <= full) {                    // whole blocks only
            if (gm == 0) {
#pragma unroll
                for (uint32_t k = 0; k < kStepGroup; ++k) run_x += over(x[k], cap_run);
                run_n += kStepGroup * 64;
                return;
            }
#pragma unroll
            for (uint32_t k = 0; k < kStepGroup; ++k) {
                if ((gm >> k) & 1u) {
                    moving_block(kb + k, x[k], sm, 64);
                } else {
                    run_x += over(x[k], cap_run);
                    run_n += 64;
                }
            }
            return;
        }
#pragma unroll
        for (uint32_t k = 0; k < kStepGroup; ++k) {
            if (b + k >= nblk) break;
            const uint32_t nv = min(64u, len - (b + k) * 64);
            if ((gm >> k) & 1u) {
                moving_block(kb + k, x[k], sm, nv);
            } else {
                run_x += over(x[k], cap_run);
                run_n += nv;
            }
        }
    };
    uint32_t xa[kStepGroup], xc[kStepGroup];
    SpanMasks sm = load_masks(0);
#pragma unroll
    for (uint32_t k = 0; k < kStepGroup; ++k) xa[k] = load(k);
    for (uint32_t b0 = 0; b0 < nblk; b0 += 2 * kStepGroup) {
#pragma unroll
        for (uint32_t k = 0; k < kStepGroup; ++k) xc[k] = load(b0 + kStepGroup + k);
        const SpanMasks next = load_masks(b0 + 2 * kStepGroup);
        const uint64_t moving = __ballot((sm.hs | sm.up | sm.dn) != 0);
        group(b0, 0, xa, sm, moving);
        if (b0 + kStepGroup >= nblk) break;
#pragma unroll
        for (uint32_t k = 0; k < kStepGroup; ++k) xa[k] = load(b0 + 2 * kStepGroup + k);
        group(b0 + kStepGroup, kStepGroup, xc, sm, moving);
        sm = next;
    }
    if constexpr (kNarrow) {
        // a sample of 2^22 or more: nothing is written, the wide pass takes it
        if (__ballot(vmax >= kNarrowSteppedBound)) return false;
        if (run_n) {
            credit_n(run_lv, run_n);
            lds_add(xb + (run_lv - lmin) * kBinStride + bin_word, run_x);
        }
        // the other lanes' adds are done before their words are read
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // lane l < rows: the sums of level lmin + l's rows (its counts are the
        // 16-bit halves l & 1 of count row l / 2)
        uint64_t xs = 0;
        uint32_t ns = 0;
        if (lane < rows) {
            const uint32_t* crow = cb + (lane >> 1) * kBinStride;
            const uint32_t sh = 16 * (lane & 1);
#pragma unroll
            for (uint32_t k = 0; k < kBinLanes; ++k) {
                xs += xb[lane * kBinStride + k];
                ns += (crow[k] >> sh) & 0xFFFFu;
            }
        }
        bin_x = xs;
        // the bins' counts, from lane l (level lmin + l) to lane lmin + l
        const uint32_t from = (uint32_t)max((int32_t)lane - lmin, 0);
        const uint32_t nmoved = (uint32_t)__shfl((int)ns, (int)from, 64);
        if (lane >= (uint32_t)lmin && lane < (uint32_t)lmin + rows) bin_n += nmoved;
    } else {
        if (run_n) credit(run_lv, run_n, dpp_wave_sum64(run_x));
    }
    const uint64_t ex_max_w = dpp_wave_sum64(ex_max);
    const uint64_t ex_min_w = dpp_wave_sum64(ex_min);
    unsigned long long* st = reinterpret_cast<unsigned long long*>(stats + t);
    if (lane == 0) {
        if (ex_max_w) atomicAdd(st + 0, (unsigned long long)ex_max_w);
        if (ex_min_w) atomicAdd(st + 1, (unsigned long long)ex_min_w);
    }
    if (lane < MAGUS_PROXY_LEVELS) {
        if (bin_n) atomicAdd(st + 2 + lane, (unsigned long long)bin_n);
    }
    // the excess sums: lane l holds level l's (wide) or level lmin + l's (narrow)
    const uint32_t xlevel = kNarrow ? lmin + lane : lane;
    if (xlevel < MAGUS_PROXY_LEVELS && bin_x)
        atomicAdd(st + 2 + MAGUS_PROXY_LEVELS + xlevel, (unsigned long long)bin_x);
    return true;
}

// The narrow pass, one wave per chunk (its bins in dynamic LDS).  A chunk it
// cannot take (no bins, a chunk longer than the narrow pass allows, or a
// sample of 2^24 or more) is appended to the wide pass's queue: redo[0]
// counts the entries, redo[1..] holds their chunk indices.  Alone the narrow
// pass takes 62 VGPRs, so the bins of a 17-rung range (5.6 KB a wave) set
// the occupancy: 7 waves per SIMD (6 with the wide pass in the kernel).
__global__ __launch_bounds__(kStatsWaves * kWave) void proxy_stepped_kernel(
    const uint32_t* __restrict__ samples, const uint64_t* __restrict__ offsets,
    uint32_t n_traces, const uint32_t* __restrict__ chunk_base,
    const DevCfg* __restrict__ cfgs, const uint32_t* __restrict__ cfg_of_trace,
    uint32_t chunk, const uint32_t* __restrict__ entering,
    const uint64_t* __restrict__ masks, uint64_t n_blocks,
    const magus_proxy_model* __restrict__ model, magus_proxy_stats* __restrict__ stats,
    uint32_t bin_levels, uint32_t* __restrict__ redo)
{
    __shared__ uint32_t s_cap[MAGUS_PROXY_LEVELS];
    extern __shared__ uint32_t s_bins[];                 // bin_levels rows per wave
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x < MAGUS_PROXY_LEVELS) s_cap[threadIdx.x] = model->cap_mbps[threadIdx.x];
    __syncthreads();
    if (chunk_base[n_traces + 1] != 0) return;            // the plan rejected the batch
    const uint32_t g = blockIdx.x * kStatsWaves + uniform(wv);
    if (g >= chunk_base[n_traces]) return;
    // this wave's bins: bin_levels excess rows, then (bin_levels + 3) / 4 count rows
    uint32_t* xb = s_bins + uniform(wv) * stepped_bin_words(bin_levels);
    uint32_t* cb = xb + bin_levels * kBinStride;
    if (bin_levels && chunk <= kNarrowSteppedChunk &&
        stepped_stats_pass<true>(samples, offsets, n_traces, chunk_base, cfgs, cfg_of_trace,
                                 chunk, entering, masks, n_blocks, s_cap, xb, cb, stats, g,
                                 lane))
        return;
    if (lane == 0) redo[1 + atomicAdd(redo, 1u)] = g;   // (a vector atomic)
}

// The wide pass over the queued chunks: the grid's waves take the entries
// round-robin with a scalar entry index, so every wave leaves the loop
// together.
__global__ __launch_bounds__(kStatsWaves * kWave) void proxy_stepped_wide_kernel(
    const uint32_t* __restrict__ samples, const uint64_t* __restrict__ offsets,
    uint32_t n_traces, const uint32_t* __restrict__ chunk_base,
    const DevCfg* __restrict__ cfgs, const uint32_t* __restrict__ cfg_of_trace,
    uint32_t chunk, const uint32_t* __restrict__ entering,
    const uint64_t* __restrict__ masks, uint64_t n_blocks,
    const magus_proxy_model* __restrict__ model, magus_proxy_stats* __restrict__ stats,
    const uint32_t* __restrict__ redo)
{
    __shared__ uint32_t s_cap[MAGUS_PROXY_LEVELS];
    const uint32_t lane = threadIdx.x & 63;
    if (threadIdx.x < MAGUS_PROXY_LEVELS) s_cap[threadIdx.x] = model->cap_mbps[threadIdx.x];
    __syncthreads();
    const uint32_t n = uniform(redo[0]);
    const uint32_t waves = gridDim.x * kStatsWaves;
    for (uint32_t i = blockIdx.x * kStatsWaves + uniform(threadIdx.x >> 6); i < n; i += waves) {
        const uint32_t g = uniform(redo[1 + i]);
        if (g >= chunk_base[n_traces]) continue;        // (never: every entry is this call's)
        stepped_stats_pass<false>(samples, offsets, n_traces, chunk_base, cfgs, cfg_of_trace,
                                  chunk, entering, masks, n_blocks, s_cap, nullptr, nullptr,
                                  stats, g, lane);
    }
}

// Zeroes p[0, n); with `queue`, also sets queue[0] (a queue's count) to 0.
__global__ __launch_bounds__(256) void proxy_zero_kernel(uint64_t* __restrict__ p, uint64_t n,
                                                         uint32_t* __restrict__ queue) {
    if (queue && blockIdx.x == 0 && threadIdx.x == 0) queue[0] = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Stretched length of `steps` intervals of which the samples exceed `cap` by
// `excess` in total, in units of one interval.
__device__ __forceinline__ double stretched(uint64_t steps, uint64_t excess, uint32_t cap) {
    return (double)steps + (double)excess / (double)cap;
}

// FP64 sum across the wave (butterfly: every lane gets the total).
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// The seven figures of each policy for one trace from its statistics, by
// one wave: lane l passes level l's intervals and excess sum (lanes past the
// model's levels pass zeros).  Each lane forms its level's stretched length
// and package energy, two wave sums give MAGUS's totals, and every lane then
// derives the same figures (FP64).
__device__ __forceinline__ magus_proxy_metrics metrics_of(const magus_proxy_model* model,
                                                         const DevCfg& c, uint64_t n,
                                                         uint64_t excess_max, uint64_t excess_min,
                                                         uint64_t steps_l, uint64_t excess_l,
                                                         uint32_t lane)
{
    const double dt = (double)model->interval_us * 1e-6;
    const double core = (double)model->core_mw, gpu = (double)model->gpu_mw * 1e-3;
    double T[3], P[3];                       // intervals (stretched), package energy
    double len = 0.0, pw = 0.0;
    if (lane < model->n_levels && steps_l) {
        len = stretched(steps_l, excess_l, model->cap_mbps[lane]);
        pw = len * (core + (double)model->uncore_mw[lane]);
    }
    T[0] = wave_sum_f64(len);
    P[0] = wave_sum_f64(pw);
    T[1] = stretched(n, excess_max, model->cap_mbps[c.lmax]);
    P[1] = T[1] * (core + (double)model->uncore_mw[c.lmax]);
    T[2] = stretched(n, excess_min, model->cap_mbps[c.lmin]);
    P[2] = T[2] * (core + (double)model->uncore_mw[c.lmin]);
    magus_proxy_metrics r;
    for (int p = 0; p < 3; ++p) {
        r.time_s[p] = T[p] * dt;
        const double pkg_j = P[p] * dt * 1e-3;
        r.energy_j[p] = pkg_j + r.time_s[p] * gpu;
        r.pkg_power_w[p] = n ? pkg_j / r.time_s[p] : 0.0;
    }
    for (int p = 0; p < 3; ++p) {
        if (n == 0) {
            r.perf_loss[p] = r.pkg_power_saving[p] = r.energy_saving[p] = r.edp_saving[p] = 0.0;
            continue;
        }
        r.perf_loss[p] = r.time_s[p] / r.time_s[1] - 1.0;
        r.pkg_power_saving[p] = 1.0 - r.pkg_power_w[p] / r.pkg_power_w[1];
        r.energy_saving[p] = 1.0 - r.energy_j[p] / r.energy_j[1];
        r.edp_saving[p] = 1.0 - (r.energy_j[p] * r.time_s[p]) / (r.energy_j[1] * r.time_s[1]);
    }
    return r;
}

// Writes one trace's metrics from the wave: lane i < 21 stores word i.
__device__ __forceinline__ void store_metrics(magus_proxy_metrics* out,
                                              const magus_proxy_metrics& r, uint32_t lane) {
    constexpr uint32_t kWords = sizeof(magus_proxy_metrics) / 8;
    const double* w = reinterpret_cast<const double*>(&r);
    double v = 0.0;
#pragma unroll
    for (uint32_t i = 0; i < kWords; ++i) v = lane == i ? w[i] : v;
    if (lane < kWords) reinterpret_cast<double*>(out)[lane] = v;
}

// The model copied into LDS by the workgroup (the metrics read it in a
// dependent chain, each global load of which would be a full memory latency).
__device__ __forceinline__ const magus_proxy_model* model_to_lds(const magus_proxy_model* model,
                                                                 magus_proxy_model* s_model) {
    constexpr uint32_t kWords = sizeof(magus_proxy_model) / 4;
    for (uint32_t w = threadIdx.x; w < kWords; w += blockDim.x)
        reinterpret_cast<uint32_t*>(s_model)[w] = reinterpret_cast<const uint32_t*>(model)[w];
    __syncthreads();
    return s_model;
}

// One wave per trace (4 a workgroup).
__global__ __launch_bounds__(kStatsWaves * kWave) void proxy_metrics_kernel(
    const uint64_t* __restrict__ offsets, uint32_t n_traces,
    const uint32_t* __restrict__ chunk_base, const DevCfg* __restrict__ cfgs,
    const uint32_t* __restrict__ cfg_of_trace, const magus_proxy_model* __restrict__ model,
    const magus_proxy_stats* __restrict__ stats, magus_proxy_metrics* __restrict__ out)
{
    __shared__ magus_proxy_model s_model;
    model = model_to_lds(model, &s_model);
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t t = blockIdx.x * kStatsWaves + uniform(threadIdx.x >> 6);
    if (t >= n_traces || chunk_base[n_traces + 1] != 0) return;
    const DevCfg c = cfgs[cfg_of_trace ? cfg_of_trace[t] : 0];
    const magus_proxy_stats& st = stats[t];
    const bool lv = lane < MAGUS_PROXY_LEVELS;
    const magus_proxy_metrics r =
        metrics_of(model, c, offsets[t + 1] - offsets[t], st.excess_max, st.excess_min,
                   lv ? st.steps[lane] : 0ull, lv ? st.excess[lane] : 0ull, lane);
    store_metrics(out + t, r, lane);
}

__device__ __forceinline__ uint32_t sat_sub(uint32_t x, uint32_t cap) {
    return __builtin_elementwise_sub_sat(x, cap);
}


// Carries into the 64 bit positions of a + b + cin (cin 0 or 1) and the carry
// out, in scalar registers (a, b wave-uniform).
__device__ __forceinline__ uint64_t carries_into(uint64_t a, uint64_t b, uint32_t cin,
                                                 uint32_t& cout) {
    uint32_t s0, s1, k;
    asm("s_add_u32 %0, %3, %5\n\t"
        "s_addc_u32 %1, %4, %6\n\t"
        "s_cselect_b32 %2, 1, 0\n\t"
        "s_add_u32 %0, %0, %7\n\t"
        "s_addc_u32 %1, %1, 0\n\t"
        "s_cselect_b32 %2, 1, %2"
        : "=&s"(s0), "=&s"(s1), "=&s"(k)
        : "s"(uniform((uint32_t)a)), "s"(uniform((uint32_t)(a >> 32))),
          "s"(uniform((uint32_t)b)), "s"(uniform((uint32_t)(b >> 32))), "s"(uniform(cin))
        : "scc");
    cout = k;
    return ((((uint64_t)s1 << 32) | s0) ^ a) ^ b;
}

// v in the lanes whose bit of the wave-uniform mask is set, else 0
__device__ __forceinline__ uint32_t lane_sel(uint64_t mask, uint32_t v) {
    const uint64_t m = ((uint64_t)uniform((uint32_t)(mask >> 32)) << 32) | uniform((uint32_t)mask);
    uint32_t r;
    asm("v_cndmask_b32 %0, 0, %1, %2" : "=v"(r) : "v"(v), "s"(m));
    return r;
}

// Fused pass, one wave per chunk, in the replay chunk kernel's form: blocks of
// 64 steps, kProxyIter blocks per unrolled iteration with the next
// iteration's loads in flight, Alg. 1 as exact compares and Alg. 2 as mbcnt
// chains on wave masks.  Per lane, running totals of the excess at level_max
// and level_min (and level_init, kMidInit) over the chunk so far are the only
// per-step sums.  Everything a decisive block changes lives in LDS, one slot
// per lane, so a block without a decisive step touches no other register than
// the totals and the flag history:
//   level      the level after the last decisive step (kUnseen before the
//              first)
//   hacc/lacc  during a run at level_max the excess credited to it is hacc +
//              (total at level_max), at level_min lacc + (total at
//              level_min): a run is opened by subtracting its level's total
//              after the decisive block and closed by adding the total before
//              the next one (modular arithmetic)
//   nhi        the count of steps after the prefix at level_max, kept the
//              same way with step indices (the others are at level_min)
//   pre        the totals at the first decisive step (lanes up to it
//              included): the steps whose interval runs at the level entering
//              the chunk, summed at each level it can be; ppre counts them
// kMidInit: some config starts between the bounds, so a chunk can also be
// entered at level_init and its prefix needs a third total.
//
// Two widths.  A chunk whose samples are all below 2^24 (every real
// throughput trace) takes the narrow pass: per-lane sums in 32 bits (at most
// 256 blocks of excesses below 2^24 per lane, so the true per-lane values fit
// and modular intermediates are harmless) and, with the default base, the
// Alg. 1 compares in fp32 (below).  64-bit integer operations issue at half
// the rate of 32-bit ones on this chip, and the pass is bound by VALU issue.
// The narrow pass tracks the largest sample it read; a chunk that had one of
// 2^24 or more is run again by the exact 64-bit pass, which also takes the
// chunks whose thresholds or length rule the narrow pass out.  The two
// passes are separate kernels (the exact one over a queue of chunks), so
// the narrow kernel's register count is its own.
#ifndef MAGUS_PROXY_ITER
#define MAGUS_PROXY_ITER 8
#endif
constexpr uint32_t kProxyIter = MAGUS_PROXY_ITER;
constexpr uint32_t kUnseen = 2;
typedef __attribute__((address_space(3))) uint64_t lds_u64;
typedef __attribute__((address_space(3))) uint32_t lds_u32;
constexpr uint32_t kSlots = kStatsWaves * kWave;
constexpr uint32_t kExactBlocks = 2048;   // grid of the exact pass (at most)

// The decisive-block state of the waves of a workgroup (one slot per lane).
struct ProxyLds {
    uint64_t hacc[kSlots], lacc[kSlots], pre[3][kSlots];
    uint32_t level[kSlots], nhi[kSlots], ppre[kSlots];
};

// Alg. 1 with the default base in fp32: a rise is an event iff
// b 2^16 - a (2^16 + W q_inc) > 0, evaluated as fma(a, -ku, b 2^16).  With a,
// b and ku below 2^24 every operand is an exact float (b 2^16 too), the fma
// forms the product and the sum exactly and rounds once, and rounding keeps
// the sign of an integer: the compare is exact.  The same for a fall with the
// roles of a and b swapped.
__device__ __forceinline__ bool rise_f32(float a, float b16, float nku) {
    return __builtin_fmaf(a, nku, b16) > 0.0f;
}

template <bool kAnyBase, bool kMidInit, bool kNarrow>
__device__ __forceinline__ bool proxy_pass(const ChunkView& v, uint32_t lane, uint32_t slot,
                                           uint32_t g, const magus_proxy_model* __restrict__ model,
                                           ProxySum* __restrict__ psums, ProxyLds& L)
{
    using acc_t = std::conditional_t<kNarrow, uint32_t, uint64_t>;
    using lds_acc = std::conditional_t<kNarrow, lds_u32, lds_u64>;
    constexpr bool kF32 = kNarrow && !kAnyBase;
    // (volatile LDS pointers: the compiler must not forward these through
    // registers, which would put the state back into the loop's merge points,
    // nor move the narrow pass's 32-bit accesses past the exact pass's 64-bit
    // ones to the same bytes)
    // A lane's 64-bit slot holds its narrow sums in its low word (the same
    // bytes for both widths: the waves of a workgroup never overlap).
    volatile lds_acc* s_hacc = (volatile lds_acc*)(L.hacc + slot);
    volatile lds_acc* s_lacc = (volatile lds_acc*)(L.lacc + slot);
    volatile lds_acc* s_pre0 = (volatile lds_acc*)(L.pre[0] + slot);
    volatile lds_acc* s_pre1 = (volatile lds_acc*)(L.pre[1] + slot);
    volatile lds_acc* s_pre2 = (volatile lds_acc*)(L.pre[2] + slot);
    volatile lds_u32* s_level = (volatile lds_u32*)(L.level + slot);
    volatile lds_u32* s_nhi = (volatile lds_u32*)(L.nhi + slot);
    volatile lds_u32* s_ppre = (volatile lds_u32*)(L.ppre + slot);

    const DevCfg& c = v.c;
    const uint32_t W = c.W, H = c.H;
    const uint32_t c_lo = model->cap_mbps[c.lmin], c_hi = model->cap_mbps[c.lmax];
    const uint32_t c_in = model->cap_mbps[c.linit];
    const uint32_t s = v.s, e = v.e;
    const uint32_t first_real = s >= 64 ? 1u : 0u;
    const uint32_t nreal = (e - s + 63) >> 6;            // real blocks, last may be partial
    const uint32_t nfull = (e - s) >> 6;                 // real blocks with 64 valid steps
    const uint32_t n_iter = (nreal + kProxyIter - 1) / kProxyIter;

    // per-lane constants (as in the replay chunk kernel)
    const int bperm_addr = (int)(((lane - (W - 1)) & 63u) << 2);  // lane of x[t-W+1]
    const bool from_cur = lane >= W - 1;
    const uint32_t bias_lane = 0x80000000u - (c.thr + lane);
    const uint64_t loud = c.thr == 0 ? 1ull : 0ull;
    uint32_t mu;
    asm volatile("v_mov_b32 %0, %1" : "=v"(mu) : "s"(c.mu));
    const uint32_t md = c.md;
    const uint32_t ku = 65536u + c.mu, kd = 65536u + c.md;
    const uint32_t k16 = v.k16;
    const float nku = -(float)ku, nkd = -(float)kd;

    auto load_block = [&](uint32_t desc_blk) -> uint32_t {
        return __builtin_amdgcn_raw_buffer_load_b32(v.rsrc, (int)((desc_blk * 64 + lane) * 4), 0,
                                                    kStreamLoad);
    };
    // the value exchanged for x[t-W+1]: the sample, or its float in the fp32 form
    auto xchg = [&](uint32_t x) -> uint32_t {
        if constexpr (kF32) return __float_as_uint((float)x);
        else return x;
    };
    // Alg. 1 for the 64 steps of a block: masks of the +1 and -1 predictions
    // (a: x[t-W+1] as exchanged, b: x[t])
    auto events = [&](uint32_t a, uint32_t b, uint64_t& EU, uint64_t& ED) {
        if constexpr (kAnyBase) {
            const bool rising = b > a;
            const uint32_t lov = derivative_base(a, b, c.base, c.ref);
            const uint32_t d = max(a, b) - min(a, b);
            const uint32_t m = rising ? mu : md;
            const uint64_t E = lane_ballot(((uint64_t)d << 16) > (uint64_t)lov * m);
            const uint64_t R = lane_ballot(rising);
            EU = E & R;
            ED = E & ~R;
        } else if constexpr (kF32) {
            const float af = __uint_as_float(a), bf = (float)b;
            EU = lane_ballot(rise_f32(af, bf * 65536.0f, nku));
            ED = lane_ballot(rise_f32(bf, af * 65536.0f, nkd));
        } else {
            EU = lane_ballot((uint64_t)b * k16 > (uint64_t)a * ku);
            ED = lane_ballot((uint64_t)a * k16 > (uint64_t)b * kd);
        }
    };

    *s_hacc = 0;
    *s_lacc = 0;
    *s_level = kUnseen;
    *s_nhi = 0;

    uint32_t xp = 0;             // exchanged values of the block before the current one
    uint64_t fps = 0;            // (flags of the block before) >> 1
    uint32_t vmax = 0;           // largest sample read (narrow pass)
    if (first_real) {
        const uint32_t x0 = load_block(0);
        if constexpr (kNarrow) vmax = x0;
        const uint32_t x0x = xchg(x0);
        const uint32_t ac = (uint32_t)__builtin_amdgcn_ds_bpermute(bperm_addr, (int)x0x);
        uint64_t EU, ED;
        events(from_cur ? ac : xchg(0u), x0, EU, ED);
        uint64_t E = EU | ED;
        const uint32_t tb = s - 64;
        if (tb < W - 1) E &= ~mask_below(W - 1 - tb);     // FIFO not yet full
        fps = E >> 1;
        xp = x0x;
    }

    acc_t a_max = 0, a_min = 0, a_in = 0;       // totals of the chunk so far (per lane)

    // A block with a decisive step (UP: high or +1 executed, level_max after
    // the step; DN: -1 executed, level_min after; D = UP | DN): the totals
    // do not yet hold this block.
    auto decisive = [&](uint32_t tb, uint64_t valid, uint64_t UP, uint64_t DN, uint64_t D,
                        uint32_t e_hi, uint32_t e_lo, uint32_t x) {
        const uint32_t lvl = uniform(*s_level);
        acc_t ha = *s_hacc, la = *s_lacc;
        uint32_t nh = *s_nhi;
        uint64_t det = valid;                            // steps summed by their own level
        if (lvl == kUnseen) {
            // the chunk's first decisive step p: the steps up to it run at the
            // level entering the chunk
            const uint32_t p = (uint32_t)__builtin_ctzll(D);
            const uint64_t in = mask_below(p + 1);
            *s_ppre = tb + p + 1 - s;
            *s_pre0 = a_min + lane_sel(in, e_lo);
            *s_pre1 = a_max + lane_sel(in, e_hi);
            if constexpr (kMidInit) *s_pre2 = a_in + lane_sel(in, sat_sub(x, c_in));
            det &= ~in;
        } else if (lvl) {                                // close the run at level_max
            ha += a_max;
            nh += tb;
        } else {                                         // ... at level_min
            la += a_min;
        }
        // level bit before each step: the carries into the bits of
        // ~DN + UP + level (UP generates, DN kills; past the first decisive
        // step they do not depend on the level entering the block)
        uint32_t cout;
        const uint64_t C = carries_into(~DN, UP, lvl & 1u, cout);
        const uint64_t hi_m = C & det;
        ha += lane_sel(hi_m, e_hi);
        la += lane_sel(det & ~C, e_lo);
        nh += (uint32_t)__builtin_popcountll(hi_m);
        // open the run after the block at the level its last decisive step set
        if (cout) {
            ha -= a_max + e_hi;
            nh -= min(tb + 64, e);
        } else {
            la -= a_min + e_lo;
        }
        *s_level = cout;
        *s_hacc = ha;
        *s_lacc = la;
        *s_nhi = nh;
    };

    auto iteration = [&](uint32_t it, uint32_t (&cur)[kProxyIter], uint32_t (&nxt)[kProxyIter],
                         auto generic_tag) {
        constexpr bool generic = decltype(generic_tag)::value;
        if (it + 1 < n_iter) {
#pragma unroll
            for (uint32_t j = 0; j < kProxyIter; ++j)
                nxt[j] = load_block(first_real + (it + 1) * kProxyIter + j);
        }
        uint32_t xx[kProxyIter], ac[kProxyIter], ap[kProxyIter];
#pragma unroll
        for (uint32_t j = 0; j < kProxyIter; ++j) xx[j] = xchg(cur[j]);
#pragma unroll
        for (uint32_t j = 0; j < kProxyIter; ++j) {
            ac[j] = (uint32_t)__builtin_amdgcn_ds_bpermute(bperm_addr, (int)xx[j]);
            ap[j] = (uint32_t)__builtin_amdgcn_ds_bpermute(bperm_addr, (int)(j ? xx[j - 1] : xp));
        }
#pragma unroll
        for (uint32_t j = 0; j < kProxyIter; ++j) {
            const uint32_t x = cur[j];
            const uint32_t tb = s + (it * kProxyIter + j) * 64;     // trace step of lane 0
            if constexpr (kNarrow) vmax = max(vmax, x);
            uint64_t PU, PD;
            events(from_cur ? ac[j] : ap[j], x, PU, PD);
            uint64_t valid = ~0ull;
            if constexpr (generic) {
                valid = mask_below(tb < e ? min(64u, e - tb) : 0u);
                uint64_t vm = valid;
                if (tb < W - 1) vm &= ~mask_below(W - 1 - tb);
                PU &= vm;
                PD &= vm;
            }
            const uint64_t E = PU | PD;
            const uint64_t B = fps >> (64 - H);           // last H-1 flags of the block before
            // lanes past the chunk's end read 0: no excess
            const uint32_t e_hi = sat_sub(x, c_hi), e_lo = sat_sub(x, c_lo);
            // a quiet block (no event in it nor in the H-1 steps before it,
            // and a non-zero count threshold) is never high and has no
            // decisive step
            if ((E | B | loud) != 0) {
                const uint64_t nG = ~((E << (H - 1)) | B);    // ~(flag H-1 steps back)
                const uint32_t acc0 = (uint32_t)__popcll(B) + (uint32_t)(E & 1ull);
                const uint32_t cnt = bits_below_lane(nG, bits_below_lane(E >> 1, bias_lane));
                const uint64_t HM = lane_ballot(cnt >= 0x80000000u - acc0) & valid;
                const uint64_t UP = HM | PU;                  // high or +1 -> max
                const uint64_t DN = PD & ~HM;                 // -1 executed -> min
                const uint64_t D = UP | DN;
                if (D != 0) decisive(tb, valid, UP, DN, D, e_hi, e_lo, x);
            }
            fps = E >> 1;
            a_max += e_hi;
            a_min += e_lo;
            if constexpr (kMidInit) a_in += sat_sub(x, c_in);
        }
        xp = xx[kProxyIter - 1];
    };

    // the first iteration of a trace and the iterations reaching past the
    // last full block need per-step masks; all others take the unmasked path
    auto run = [&](uint32_t it, uint32_t (&cur)[kProxyIter], uint32_t (&nxt)[kProxyIter]) {
        if ((it == 0 && first_real == 0) || (it + 1) * kProxyIter > nfull)
            iteration(it, cur, nxt, std::true_type{});
        else
            iteration(it, cur, nxt, std::false_type{});
    };
    uint32_t bufA[kProxyIter], bufB[kProxyIter];
#pragma unroll
    for (uint32_t j = 0; j < kProxyIter; ++j) bufA[j] = load_block(first_real + j);
    for (uint32_t it = 0; it < n_iter; it += 2) {
        run(it, bufA, bufB);
        if (it + 1 < n_iter) run(it + 1, bufB, bufA);
    }
    if constexpr (kNarrow) {
        if (lane_ballot(vmax >= kNarrowBound)) return false;   // the exact pass takes it
    }

    const uint32_t lvl = uniform(*s_level);
    uint64_t ha = (acc_t)*s_hacc, la = (acc_t)*s_lacc;
    uint32_t nh = *s_nhi, ppre = e - s;
    uint64_t pre0, pre1, pre2 = 0;
    if (lvl == kUnseen) {
        // no decisive step: the whole chunk runs at the entering level
        pre0 = dpp_wave_sum64(a_min);
        pre1 = dpp_wave_sum64(a_max);
        if constexpr (kMidInit) pre2 = dpp_wave_sum64(a_in);
    } else {
        ppre = *s_ppre;
        pre0 = dpp_wave_sum64((acc_t)*s_pre0);
        pre1 = dpp_wave_sum64((acc_t)*s_pre1);
        if constexpr (kMidInit) pre2 = dpp_wave_sum64((acc_t)*s_pre2);
        if (lvl) {                                       // close the last run
            ha = (acc_t)(ha + a_max);
            nh += e;
        } else {
            la = (acc_t)(la + a_min);
        }
    }
    if constexpr (!kMidInit) pre2 = c.linit == c.lmax ? pre1 : pre0;
    ha = dpp_wave_sum64(ha);
    la = dpp_wave_sum64(la);
    const uint64_t ex_max = dpp_wave_sum64(a_max);
    const uint64_t ex_min = dpp_wave_sum64(a_min);
    if (lane == 0) {
        ProxySum r;
        r.len = e - s;
        r.ppre = ppre;
        r.has_dec = lvl == kUnseen ? 0u : 1u;
        r.end_up = lvl == 1u ? 1u : 0u;
        r.n_lo = e - s - ppre - nh;
        r.n_hi = nh;
        r.pre_x[0] = pre0;
        r.pre_x[1] = pre1;
        r.pre_x[2] = pre2;
        r.x_lo = la;
        r.x_hi = ha;
        r.ex_max = ex_max;
        r.ex_min = ex_min;
        psums[g] = r;
    }
    return true;
}

// The narrow pass, one wave per chunk.  A chunk it cannot take (the chunk
// length or the config's thresholds rule it out, or a sample reached 2^24)
// is appended to the exact pass's queue: redo[0] counts the entries,
// redo[1..] holds their chunk indices.  Only this pass's code is in the
// kernel, so it fits 64 VGPRs (8 waves per SIMD); with the exact pass in the
// same kernel it took 76.
template <bool kAnyBase, bool kMidInit>
__global__ __launch_bounds__(kStatsWaves * kWave) __attribute__((amdgpu_waves_per_eu(8)))
void proxy_chunk_kernel(
    const uint32_t* __restrict__ samples, const uint64_t* __restrict__ offsets,
    uint32_t n_traces, const uint32_t* __restrict__ chunk_base,
    const DevCfg* __restrict__ cfgs, const uint32_t* __restrict__ cfg_of_trace,
    uint32_t chunk, const magus_proxy_model* __restrict__ model, ProxySum* __restrict__ psums,
    uint32_t* __restrict__ redo)
{
    __shared__ ProxyLds L;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t g = blockIdx.x * kStatsWaves + uniform(threadIdx.x >> 6);
    if (chunk_base[n_traces + 1] != 0 || g >= chunk_base[n_traces]) return;
    const ChunkView v = chunk_view(samples, offsets, n_traces, chunk_base, cfgs, cfg_of_trace,
                                   chunk, g);
    const bool narrow = chunk <= kNarrowChunk &&
                        (kAnyBase || (65536u + v.c.mu <= kNarrowBound &&
                                      65536u + v.c.md <= kNarrowBound));
    if (narrow &&
        proxy_pass<kAnyBase, kMidInit, true>(v, lane, threadIdx.x, g, model, psums, L))
        return;
    if (lane == 0) redo[1 + atomicAdd(redo, 1u)] = g;   // (a vector atomic)
}

// The exact 64-bit pass over the queued chunks: the grid's waves take the
// entries round-robin (wave w: entries w, w + waves, ...); the entry index is
// a scalar, so every wave leaves the loop together.
template <bool kAnyBase, bool kMidInit>
__global__ __launch_bounds__(kStatsWaves * kWave) void proxy_exact_kernel(
    const uint32_t* __restrict__ samples, const uint64_t* __restrict__ offsets,
    uint32_t n_traces, const uint32_t* __restrict__ chunk_base,
    const DevCfg* __restrict__ cfgs, const uint32_t* __restrict__ cfg_of_trace,
    uint32_t chunk, const magus_proxy_model* __restrict__ model, ProxySum* __restrict__ psums,
    const uint32_t* __restrict__ redo)
{
    __shared__ ProxyLds L;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t n = uniform(redo[0]);
    const uint32_t waves = gridDim.x * kStatsWaves;
    for (uint32_t i = blockIdx.x * kStatsWaves + uniform(threadIdx.x >> 6); i < n; i += waves) {
        const uint32_t g = uniform(redo[1 + i]);
        if (g >= chunk_base[n_traces]) continue;        // (never: every entry is this call's)
        const ChunkView v = chunk_view(samples, offsets, n_traces, chunk_base, cfgs,
                                       cfg_of_trace, chunk, g);
        proxy_pass<kAnyBase, kMidInit, false>(v, lane, threadIdx.x, g, model, psums, L);
    }
}

// Fused fold, one wave per trace; lane j takes chunk j of each group of 64.
// The level entering chunk j is the end level of the last earlier chunk with
// a decisive step (else the group's entering level, level_init at the start).
__global__ __launch_bounds__(kStatsWaves * kWave) void proxy_fold_kernel(
    uint32_t n_traces, const uint64_t* __restrict__ offsets, const uint32_t* __restrict__ chunk_base,
    const ProxySum* __restrict__ psums, const DevCfg* __restrict__ cfgs,
    const uint32_t* __restrict__ cfg_of_trace, const magus_proxy_model* __restrict__ model,
    magus_proxy_stats* __restrict__ stats, magus_proxy_metrics* __restrict__ metrics,
    uint32_t* __restrict__ redo)
{
    __shared__ magus_proxy_model s_model;
    // the exact pass has read the queue: empty it for the next call
    if (blockIdx.x == 0 && threadIdx.x == 0) redo[0] = 0;
    if (metrics) model = model_to_lds(model, &s_model);
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t t = blockIdx.x * kStatsWaves + uniform(threadIdx.x >> 6);
    if (t >= n_traces) return;
    uint64_t* out = reinterpret_cast<uint64_t*>(stats + t);
    constexpr uint32_t kWords = sizeof(magus_proxy_stats) / 8;
    if (chunk_base[n_traces + 1] != 0) {
        // the plan rejected the batch: zero statistics, as the stepped path
        for (uint32_t w = lane; w < kWords; w += 64) out[w] = 0;
        return;
    }
    const DevCfg c = cfgs[cfg_of_trace ? cfg_of_trace[t] : 0];
    const uint32_t lmin = c.lmin, lmax = c.lmax, linit = c.linit;
    const uint32_t k0 = chunk_base[t], k1 = chunk_base[t + 1];
    uint32_t level = linit;                  // level entering the current group
    // per lane: intervals and excess at level_min (0), level_max (1), and at
    // level_init when it is neither (2); excess of the two static policies
    uint64_t n0 = 0, n1 = 0, n2 = 0, x0 = 0, x1 = 0, x2 = 0, emax = 0, emin = 0;
    for (uint32_t kb = k0; kb < k1; kb += 64) {
        const uint32_t k = kb + lane;
        const bool valid = k < k1;
        ProxySum P{};
        if (valid) P = psums[k];
        const uint64_t E = __ballot(valid && P.has_dec);
        const uint32_t end_level = P.end_up ? lmax : lmin;
        const uint64_t before = E & (lane ? (~0ull >> (64 - lane)) : 0ull);
        const int src = before ? 63 - __builtin_clzll(before) : (int)lane;
        const uint32_t from_src = (uint32_t)__shfl((int)end_level, src, 64);
        const uint32_t lin = before ? from_src : level;
        if (valid) {
            if (lin == lmin) {
                n0 += P.ppre;
                x0 += P.pre_x[0];
            } else if (lin == lmax) {
                n1 += P.ppre;
                x1 += P.pre_x[1];
            } else {
                n2 += P.ppre;
                x2 += P.pre_x[2];
            }
            n0 += P.n_lo;
            x0 += P.x_lo;
            n1 += P.n_hi;
            x1 += P.x_hi;
            emax += P.ex_max;
            emin += P.ex_min;
        }
        if (E) level = (uint32_t)__shfl((int)end_level, 63 - __builtin_clzll(E), 64);
    }
    n0 = dpp_wave_sum64(n0);
    n1 = dpp_wave_sum64(n1);
    n2 = dpp_wave_sum64(n2);
    x0 = dpp_wave_sum64(x0);
    x1 = dpp_wave_sum64(x1);
    x2 = dpp_wave_sum64(x2);
    emax = dpp_wave_sum64(emax);
    emin = dpp_wave_sum64(emin);
    // level l's intervals and excess: the bins of level_min, level_max and a
    // level_init between them
    auto level_stats = [&](uint32_t l, uint64_t& steps, uint64_t& excess) {
        steps = excess = 0;
        if (l == lmin) {
            steps += n0;
            excess += x0;
        }
        if (l == lmax) {
            steps += n1;
            excess += x1;
        }
        if (l == linit && linit != lmin && linit != lmax) {
            steps += n2;
            excess += x2;
        }
    };
    // every word of the trace's stats: 0 excess_max, 1 excess_min,
    // 2 + l steps[l], 2 + 32 + l excess[l]
    for (uint32_t w = lane; w < kWords; w += 64) {
        uint64_t val;
        if (w == 0) {
            val = emax;
        } else if (w == 1) {
            val = emin;
        } else {
            const bool is_n = w < 2 + MAGUS_PROXY_LEVELS;
            uint64_t steps, excess;
            level_stats(is_n ? w - 2 : w - 2 - MAGUS_PROXY_LEVELS, steps, excess);
            val = is_n ? steps : excess;
        }
        out[w] = val;
    }
    // the metrics from the same sums, lane l taking level l
    if (metrics) {
        uint64_t steps_l, excess_l;
        level_stats(lane, steps_l, excess_l);
        const magus_proxy_metrics r =
            metrics_of(model, c, offsets[t + 1] - offsets[t], emax, emin, steps_l, excess_l, lane);
        store_metrics(metrics + t, r, lane);
    }
}

}  // namespace

hipError_t launch_proxy_stepped(const uint32_t* samples, uint64_t n_samples,
                                const uint64_t* offsets, uint32_t n_traces,
                                const uint32_t* chunk_base, uint32_t max_chunks,
                                const DevCfg* cfgs, const uint32_t* cfg_of_trace, uint32_t chunk,
                                const uint32_t* entering, const uint64_t* masks,
                                const magus_proxy_model* model, magus_proxy_stats* stats,
                                magus_proxy_metrics* metrics, uint32_t bin_levels,
                                uint32_t* redo, hipStream_t stream)
{
    if (n_traces == 0) return hipSuccess;
    // the statistics are summed with atomics: zero them, and the queue's count
    const uint64_t words = (uint64_t)n_traces * (sizeof(magus_proxy_stats) / 8);
    proxy_zero_kernel<<<(uint32_t)std::min<uint64_t>((words + 255) / 256, 4096), 256, 0, stream>>>(
        reinterpret_cast<uint64_t*>(stats), words, redo);
    const uint32_t blocks = (max_chunks + kStatsWaves - 1) / kStatsWaves;
    if (bin_levels > MAGUS_PROXY_LEVELS) bin_levels = 0;
    if (blocks) {
        const uint64_t nb = stepped_mask_blocks(n_samples, n_traces);
        proxy_stepped_kernel<<<blocks, kStatsWaves * kWave,
                               kStatsWaves * stepped_bin_words(bin_levels) * sizeof(uint32_t),
                               stream>>>(
            samples, offsets, n_traces, chunk_base, cfgs, cfg_of_trace, chunk, entering, masks,
            nb, model, stats, bin_levels, redo);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        proxy_stepped_wide_kernel<<<std::min(blocks, kExactBlocks), kStatsWaves * kWave, 0,
                                    stream>>>(
            samples, offsets, n_traces, chunk_base, cfgs, cfg_of_trace, chunk, entering, masks,
            nb, model, stats, redo);
        const hipError_t e2 = hipGetLastError();
        if (e2 != hipSuccess) return e2;
    }
    if (metrics)
        proxy_metrics_kernel<<<(n_traces + kStatsWaves - 1) / kStatsWaves, kStatsWaves * kWave,
                               0, stream>>>(
            offsets, n_traces, chunk_base, cfgs, cfg_of_trace, model, stats, metrics);
    return hipGetLastError();
}

hipError_t launch_proxy_queue_clear(uint32_t* redo, hipStream_t stream) {
    proxy_zero_kernel<<<1, 64, 0, stream>>>(nullptr, 0, redo);
    return hipGetLastError();
}

hipError_t launch_proxy_fused(const uint32_t* samples, const uint64_t* offsets, uint32_t n_traces,
                              const uint32_t* chunk_base, uint32_t max_chunks,
                              const DevCfg* cfgs, const uint32_t* cfg_of_trace, uint32_t chunk,
                              const magus_proxy_model* model, ProxySum* psums, uint32_t* redo,
                              magus_proxy_stats* stats, magus_proxy_metrics* metrics,
                              bool any_base, bool mid_init, hipStream_t stream)
{
    if (n_traces == 0) return hipSuccess;
    const uint32_t blocks = (max_chunks + kStatsWaves - 1) / kStatsWaves;
    if (blocks) {
        auto k = any_base ? (mid_init ? proxy_chunk_kernel<true, true>
                                      : proxy_chunk_kernel<true, false>)
                          : (mid_init ? proxy_chunk_kernel<false, true>
                                      : proxy_chunk_kernel<false, false>);
        k<<<blocks, kStatsWaves * kWave, 0, stream>>>(samples, offsets, n_traces, chunk_base,
                                                      cfgs, cfg_of_trace, chunk, model, psums,
                                                      redo);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        // the queue's length is known only on the device: a grid of up to
        // kExactBlocks workgroups loops over it (none has work when every
        // chunk took the narrow pass)
        auto x = any_base ? (mid_init ? proxy_exact_kernel<true, true>
                                      : proxy_exact_kernel<true, false>)
                          : (mid_init ? proxy_exact_kernel<false, true>
                                      : proxy_exact_kernel<false, false>);
        x<<<std::min(blocks, kExactBlocks), kStatsWaves * kWave, 0, stream>>>(
            samples, offsets, n_traces, chunk_base, cfgs, cfg_of_trace, chunk, model, psums, redo);
        const hipError_t e2 = hipGetLastError();
        if (e2 != hipSuccess) return e2;
    }
    proxy_fold_kernel<<<(n_traces + kStatsWaves - 1) / kStatsWaves, kStatsWaves * kWave, 0,
                        stream>>>(n_traces, offsets, chunk_base, psums, cfgs, cfg_of_trace, model,
                                  stats, metrics, redo);
    return hipGetLastError();
}

}  // namespace magus
