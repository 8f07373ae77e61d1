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
//               excess sums per level -> ProxySum
//   fused fold  one wave per trace -> magus_proxy_stats
//   metrics     as below
// Stepped configs take the path over the stepped replay's pass 1 (its step
// masks and the level entering every chunk, stepped.hip):
//   zero     clears the statistics (no memset node, so the sequence can be
//            captured into a graph)
//   stepped  one wave per chunk: reads the samples and the step masks, walks
//            the level through each block in scalar registers from the chunk's
//            entering level, and sums per level: a block at one level adds to
//            a run at that level (per lane); a block whose level changes scans
//            its per-step excess once and takes each segment's sum from the
//            scan at the segment's ends; one atomic add per non-zero sum per
//            chunk
//   metrics  one thread per trace: the seven figures of each policy in FP64

#include "block_masks.h"
#include "proxy_internal.h"

namespace magus {
namespace {

static_assert(sizeof(magus_proxy_model) == 8 + 4 * 64 + 8, "magus_proxy_model layout");
static_assert(sizeof(magus_proxy_stats) == 16 + 8 * 64, "magus_proxy_stats layout");
static_assert(sizeof(magus_proxy_metrics) == 7 * 3 * 8, "magus_proxy_metrics layout");

constexpr int kStatsWaves = 4;

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

constexpr uint32_t kStepGroup = 8;     // blocks loaded ahead by the stepped pass

// Statistics of stepped configs from the stepped replay's pass 1: one wave per
// chunk.  The level before every step follows from the chunk's entering level
// and the blocks' step masks (moves up by up_step, down by down_step, set to
// level_max, each clamped to the range); the interval of step i runs at the
// level before step i.  Lane l keeps the sums of level l.
// (eight waves per SIMD: the register budget that keeps the scalar unit fed)
__global__ __launch_bounds__(kStatsWaves * kWave) __attribute__((amdgpu_waves_per_eu(8)))
void proxy_stepped_kernel(
    const uint32_t* __restrict__ samples, const uint64_t* __restrict__ offsets,
    uint32_t n_traces, const uint32_t* __restrict__ chunk_base,
    const DevCfg* __restrict__ cfgs, const uint32_t* __restrict__ cfg_of_trace,
    uint32_t chunk, const uint32_t* __restrict__ entering,
    const uint64_t* __restrict__ masks, uint64_t n_blocks,
    const magus_proxy_model* __restrict__ model, magus_proxy_stats* __restrict__ stats)
{
    __shared__ uint32_t s_cap[MAGUS_PROXY_LEVELS];
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x < MAGUS_PROXY_LEVELS) s_cap[threadIdx.x] = model->cap_mbps[threadIdx.x];
    __syncthreads();
    if (chunk_base[n_traces + 1] != 0) return;            // the plan rejected the batch
    const uint32_t g = blockIdx.x * kStatsWaves + uniform(wv);
    if (g >= chunk_base[n_traces]) return;

    const uint32_t t = trace_of_chunk(chunk_base, n_traces, g, lane);
    const uint64_t tbase = offsets[t];
    const uint32_t n = (uint32_t)(offsets[t + 1] - tbase);
    const uint32_t s = (g - chunk_base[t]) * chunk;
    const uint32_t len = min(s + chunk, n) - s;
    const DevCfg c = cfgs[cfg_of_trace ? cfg_of_trace[t] : 0];
    const int32_t lmin = c.lmin, lmax = c.lmax;
    const int32_t up = c.up ? (int32_t)c.up : 64, down = c.down ? (int32_t)c.down : 64;
    const uint32_t cap_hi = s_cap[lmax], cap_lo = s_cap[lmin];
    const uint64_t mb = first_block(tbase, s, t);
    const uint64_t* m_hs = masks + mb;
    const uint64_t* m_up = masks + n_blocks + mb;
    const uint64_t* m_dn = masks + 2 * n_blocks + mb;
    const uint32_t nblk = (len + 63) >> 6;
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(samples + tbase + s), (short)0, (int)(len * 4u), 0x00020000);

    int32_t cur = (int32_t)uniform(entering[g]);         // level before the next step
    // the run: the steps since the level last changed, all at run_lv == cur
    // (outside a block's walk); their excess is summed per lane
    uint32_t run_lv = (uint32_t)cur, cap_run = s_cap[cur], run_n = 0;
    uint64_t ex_max = 0, ex_min = 0, run_x = 0;          // per lane
    uint64_t bin_n = 0, bin_x = 0;                       // lane l: level l
    auto credit = [&](uint32_t level, uint32_t steps, uint64_t sum) {
        const bool mine = lane == level;
        bin_n += mine ? steps : 0u;
        bin_x += mine ? sum : 0ull;
    };
    // ends the run if the level changed and starts one at the new level
    auto follow_level = [&]() {
        if ((uint32_t)cur != run_lv) {
            if (run_n) credit(run_lv, run_n, dpp_wave_sum64(run_x));
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
    uint32_t xa[kStepGroup], xb[kStepGroup];
    SpanMasks sm = load_masks(0);
#pragma unroll
    for (uint32_t k = 0; k < kStepGroup; ++k) xa[k] = load(k);
    for (uint32_t b0 = 0; b0 < nblk; b0 += 2 * kStepGroup) {
#pragma unroll
        for (uint32_t k = 0; k < kStepGroup; ++k) xb[k] = load(b0 + kStepGroup + k);
        const SpanMasks next = load_masks(b0 + 2 * kStepGroup);
        const uint64_t moving = __ballot((sm.hs | sm.up | sm.dn) != 0);
        group(b0, 0, xa, sm, moving);
        if (b0 + kStepGroup >= nblk) break;
#pragma unroll
        for (uint32_t k = 0; k < kStepGroup; ++k) xa[k] = load(b0 + 2 * kStepGroup + k);
        group(b0 + kStepGroup, kStepGroup, xb, sm, moving);
        sm = next;
    }
    if (run_n) credit(run_lv, run_n, dpp_wave_sum64(run_x));
    ex_max = dpp_wave_sum64(ex_max);
    ex_min = dpp_wave_sum64(ex_min);
    unsigned long long* st = reinterpret_cast<unsigned long long*>(stats + t);
    if (lane == 0) {
        if (ex_max) atomicAdd(st + 0, (unsigned long long)ex_max);
        if (ex_min) atomicAdd(st + 1, (unsigned long long)ex_min);
    }
    if (lane < MAGUS_PROXY_LEVELS) {
        if (bin_n) atomicAdd(st + 2 + lane, (unsigned long long)bin_n);
        if (bin_x) atomicAdd(st + 2 + MAGUS_PROXY_LEVELS + lane, (unsigned long long)bin_x);
    }
}

__global__ __launch_bounds__(256) void proxy_zero_kernel(uint64_t* __restrict__ p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Stretched length of `steps` intervals of which the samples exceed `cap` by
// `excess` in total, in units of one interval.
__device__ __forceinline__ double stretched(uint64_t steps, uint64_t excess, uint32_t cap) {
    return (double)steps + (double)excess / (double)cap;
}

__global__ __launch_bounds__(256) void proxy_metrics_kernel(
    const uint64_t* __restrict__ offsets, uint32_t n_traces,
    const uint32_t* __restrict__ chunk_base, const DevCfg* __restrict__ cfgs,
    const uint32_t* __restrict__ cfg_of_trace, const magus_proxy_model* __restrict__ model,
    const magus_proxy_stats* __restrict__ stats, magus_proxy_metrics* __restrict__ out)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_traces || chunk_base[n_traces + 1] != 0) return;
    const DevCfg c = cfgs[cfg_of_trace ? cfg_of_trace[t] : 0];
    const magus_proxy_stats& st = stats[t];
    const uint64_t n = offsets[t + 1] - offsets[t];
    const double dt = (double)model->interval_us * 1e-6;
    const double core = (double)model->core_mw, gpu = (double)model->gpu_mw * 1e-3;
    double T[3], P[3];                       // intervals (stretched), package energy
    T[0] = 0.0;
    P[0] = 0.0;
    for (uint32_t l = 0; l < model->n_levels; ++l) {
        if (!st.steps[l]) continue;
        const double len = stretched(st.steps[l], st.excess[l], model->cap_mbps[l]);
        T[0] += len;
        P[0] += len * (core + (double)model->uncore_mw[l]);
    }
    T[1] = stretched(n, st.excess_max, model->cap_mbps[c.lmax]);
    P[1] = T[1] * (core + (double)model->uncore_mw[c.lmax]);
    T[2] = stretched(n, st.excess_min, model->cap_mbps[c.lmin]);
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
    out[t] = r;
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

// Fused pass, one wave per chunk (blocks loaded four at a time: the per-lane
// sums leave fewer registers for loads in flight than the plain replay has).
// Per lane, running totals of the excess at level_max and level_min over the
// chunk so far are the only per-step sums: a run of blocks at one level is
// credited at its end from the difference of its level's total at its two
// ends, and the steps up to the chunk's first decisive step from the totals
// at that point (summed over the wave there, once), so a block without a
// decisive step costs two saturating subtractions and two 64-bit adds.
// kMidInit: some config starts between the bounds, so a chunk can also be
// entered at level_init and its prefix needs a third total.
template <bool kAnyBase, bool kMidInit>
__global__ __launch_bounds__(kStatsWaves * kWave) void proxy_chunk_kernel(
    const uint32_t* __restrict__ samples, const uint64_t* __restrict__ offsets,
    uint32_t n_traces, const uint32_t* __restrict__ chunk_base,
    const DevCfg* __restrict__ cfgs, const uint32_t* __restrict__ cfg_of_trace,
    uint32_t chunk, const magus_proxy_model* __restrict__ model, ProxySum* __restrict__ psums)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t g = blockIdx.x * kStatsWaves + uniform(threadIdx.x >> 6);
    if (chunk_base[n_traces + 1] != 0 || g >= chunk_base[n_traces]) return;
    const ChunkView v = chunk_view(samples, offsets, n_traces, chunk_base, cfgs, cfg_of_trace,
                                   chunk, g);
    const uint32_t c_lo = model->cap_mbps[v.c.lmin], c_hi = model->cap_mbps[v.c.lmax];
    const uint32_t c_in = model->cap_mbps[v.c.linit];
    uint64_t a_max = 0, a_min = 0;   // totals of the chunk so far (per lane)
    uint64_t mark = 0;               // the current run's level total where it began
    uint64_t a_in = 0;               // total at level_init before the first decisive step
    uint64_t a_lo = 0, a_hi = 0;     // steps after the prefix, by level
    uint64_t pre0 = 0, pre1 = 0, pre2 = 0;   // prefix at min, max, init (wave sums)
    uint32_t n_lo = 0, n_hi = 0;
    bool seen = false;          // a decisive step earlier in this chunk
    uint32_t ppre = v.e - v.s;  // steps up to and including the first decisive step
    uint32_t lvl = 0;           // level bit after the last step (once seen)
    uint32_t run0 = v.s;        // first step of the current run
    for_each_block<4, kAnyBase>(v, lane, [&](const BlockMasks& m, uint32_t tb, uint64_t valid,
                                             uint32_t x) {
        const uint32_t e_hi = sat_sub(x, c_hi), e_lo = sat_sub(x, c_lo);
        if ((m.E | m.HM) == 0) {
            // no decisive step: the block runs at the level it was entered at
            a_max += e_hi;                               // lanes past the end read 0
            a_min += e_lo;
            if (kMidInit && !seen) a_in += sat_sub(x, c_in);
            return;
        }
        const uint64_t UP = m.HM | (m.E & m.R);          // high or +1 -> max
        const uint64_t DN = m.E & ~(m.R | m.HM);         // -1 executed -> min
        const uint64_t D = UP | DN;
        uint64_t det = valid;
        if (seen) {
            // the run since the last decisive block, at level lvl
            if (lvl) {
                a_hi += a_max - mark;
                n_hi += tb - run0;
            } else {
                a_lo += a_min - mark;
                n_lo += tb - run0;
            }
        } else {
            // steps up to and including the first decisive one run at the
            // level entering the chunk: the totals so far plus this block's
            // lanes up to it, at each level the chunk can be entered at
            const uint32_t p = (uint32_t)__builtin_ctzll(D);
            const uint64_t in = mask_below(p + 1);
            ppre = tb + p + 1 - v.s;
            pre0 = dpp_wave_sum64(a_min + lane_sel(in, e_lo));
            pre1 = dpp_wave_sum64(a_max + lane_sel(in, e_hi));
            if (kMidInit) pre2 = dpp_wave_sum64(a_in + lane_sel(in, sat_sub(x, c_in)));
            det &= ~in;
            seen = true;
        }
        a_max += e_hi;
        a_min += e_lo;
        // level bit before each step: the carries into the bits of
        // ~DN + UP + lvl (UP generates, DN kills)
        uint32_t cout;
        const uint64_t C = carries_into(~DN, UP, lvl, cout);
        const uint64_t hi_m = C & det, lo_m = det & ~C;
        n_hi += (uint32_t)__builtin_popcountll(hi_m);
        n_lo += (uint32_t)__builtin_popcountll(lo_m);
        a_hi += lane_sel(hi_m, e_hi);
        a_lo += lane_sel(lo_m, e_lo);
        lvl = cout;                                      // level after the block's last step
        mark = lvl ? a_max : a_min;
        run0 = tb + 64;
    });
    if (seen) {
        if (lvl) {
            a_hi += a_max - mark;
            n_hi += v.e > run0 ? v.e - run0 : 0u;
        } else {
            a_lo += a_min - mark;
            n_lo += v.e > run0 ? v.e - run0 : 0u;
        }
    }
    a_lo = dpp_wave_sum64(a_lo);
    a_hi = dpp_wave_sum64(a_hi);
    a_max = dpp_wave_sum64(a_max);
    a_min = dpp_wave_sum64(a_min);
    if (!seen) {
        // no decisive step: the whole chunk runs at the entering level
        pre0 = a_min;
        pre1 = a_max;
        if (kMidInit) pre2 = dpp_wave_sum64(a_in);
    }
    if (!kMidInit) pre2 = v.c.linit == v.c.lmax ? pre1 : pre0;
    if (lane == 0) {
        ProxySum r;
        r.len = v.e - v.s;
        r.ppre = ppre;
        r.has_dec = seen ? 1u : 0u;
        r.end_up = (uint32_t)lvl;
        r.n_lo = n_lo;
        r.n_hi = n_hi;
        r.pre_x[0] = pre0;
        r.pre_x[1] = pre1;
        r.pre_x[2] = pre2;
        r.x_lo = a_lo;
        r.x_hi = a_hi;
        r.ex_max = a_max;
        r.ex_min = a_min;
        psums[g] = r;
    }
}

// Fused fold, one wave per trace; lane j takes chunk j of each group of 64.
// The level entering chunk j is the end level of the last earlier chunk with
// a decisive step (else the group's entering level, level_init at the start).
__global__ __launch_bounds__(kStatsWaves * kWave) void proxy_fold_kernel(
    uint32_t n_traces, const uint32_t* __restrict__ chunk_base,
    const ProxySum* __restrict__ psums, const DevCfg* __restrict__ cfgs,
    const uint32_t* __restrict__ cfg_of_trace, magus_proxy_stats* __restrict__ stats)
{
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
            const uint32_t l = is_n ? w - 2 : w - 2 - MAGUS_PROXY_LEVELS;
            val = 0;
            if (l == lmin) val += is_n ? n0 : x0;
            if (l == lmax) val += is_n ? n1 : x1;
            if (l == linit && linit != lmin && linit != lmax) val += is_n ? n2 : x2;
        }
        out[w] = val;
    }
}

}  // namespace

hipError_t launch_proxy_stepped(const uint32_t* samples, uint64_t n_samples,
                                const uint64_t* offsets, uint32_t n_traces,
                                const uint32_t* chunk_base, uint32_t max_chunks,
                                const DevCfg* cfgs, const uint32_t* cfg_of_trace, uint32_t chunk,
                                const uint32_t* entering, const uint64_t* masks,
                                const magus_proxy_model* model, magus_proxy_stats* stats,
                                magus_proxy_metrics* metrics, hipStream_t stream)
{
    if (n_traces == 0) return hipSuccess;
    const uint64_t words = (uint64_t)n_traces * (sizeof(magus_proxy_stats) / 8);
    proxy_zero_kernel<<<(uint32_t)std::min<uint64_t>((words + 255) / 256, 4096), 256, 0, stream>>>(
        reinterpret_cast<uint64_t*>(stats), words);
    const uint32_t blocks = (max_chunks + kStatsWaves - 1) / kStatsWaves;
    if (blocks)
        proxy_stepped_kernel<<<blocks, kStatsWaves * kWave, 0, stream>>>(
            samples, offsets, n_traces, chunk_base, cfgs, cfg_of_trace, chunk, entering, masks,
            stepped_mask_blocks(n_samples, n_traces), model, stats);
    if (metrics)
        proxy_metrics_kernel<<<(n_traces + 255) / 256, 256, 0, stream>>>(
            offsets, n_traces, chunk_base, cfgs, cfg_of_trace, model, stats, metrics);
    return hipGetLastError();
}

hipError_t launch_proxy_fused(const uint32_t* samples, const uint64_t* offsets, uint32_t n_traces,
                              const uint32_t* chunk_base, uint32_t max_chunks,
                              const DevCfg* cfgs, const uint32_t* cfg_of_trace, uint32_t chunk,
                              const magus_proxy_model* model, ProxySum* psums,
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
                                                      cfgs, cfg_of_trace, chunk, model, psums);
    }
    proxy_fold_kernel<<<(n_traces + kStatsWaves - 1) / kStatsWaves, kStatsWaves * kWave, 0,
                        stream>>>(n_traces, chunk_base, psums, cfgs, cfg_of_trace, stats);
    if (metrics)
        proxy_metrics_kernel<<<(n_traces + 255) / 256, 256, 0, stream>>>(
            offsets, n_traces, chunk_base, cfgs, cfg_of_trace, model, stats, metrics);
    return hipGetLastError();
}

}  // namespace magus
