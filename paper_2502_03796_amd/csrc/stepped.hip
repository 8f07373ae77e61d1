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
// chunk has one map.
//
// Pass 1 streams the samples once.  Per 64-step block it parks the Alg. 1 /
// Alg. 2 lane masks (events, rises, high steps) in lane j of six registers
// for block j of a group of 64 blocks.  Per group each lane derives the steps
// of its block that can move the level, as three masks (raise by up_step,
// lower by down_step, set level_max at the start of a run of high steps),
// writes them out (24 B per block) and walks their set bits to form the
// block's map; a wave-wide tree composes the 64 block maps.  A per-trace fold applies the chunk maps in order to find
// the level entering every chunk.  Pass 2 reads only the masks: lane j
// composes its block's map again, an inclusive wave scan of the block maps
// gives the level entering every block, and lane j walks its block once more
// to add up levels and count transitions.  When the per-step decision bytes
// are asked for, pass 2 instead replays the samples of the chunk from its
// entering level (a wave-wide scan of the per-step maps of every block).

#include "block_masks.h"

namespace magus {
namespace {

constexpr int kWaves = 4;
constexpr uint32_t kGroupBlocks = 8;   // blocks the walker loads ahead

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

// The steps of a block that can move the level, as disjoint lane masks: raise
// by up_step, lower by down_step, or set level_max (hs: a high step that does
// not follow another high step; a high step after one leaves level_max where
// it is).  hm_before: bit 0 = the step before the block was high.
struct StepMasks {
    uint64_t hs, up, dn;
};

__device__ __forceinline__ StepMasks step_masks(const BlockMasks& m, uint64_t hm_before) {
    StepMasks s;
    s.hs = m.HM & ~((m.HM << 1) | hm_before);
    const uint64_t ev = m.E & ~m.HM;
    s.up = ev & m.R;
    s.dn = ev & ~m.R;
    return s;
}

// Rung moves of a config: a jump to the bound is a move of 64 rungs (beyond
// any range), so every kind of step is one clamped add.
struct Moves {
    int32_t up, down, lmin, lmax;
};

__device__ __forceinline__ Moves moves_of(const DevCfg& c) {
    return Moves{c.up ? (int32_t)c.up : 64, c.down ? (int32_t)c.down : 64, (int32_t)c.lmin,
                 (int32_t)c.lmax};
}

// The rung move of bit p of a block's masks (p is one of its set bits).
__device__ __forceinline__ int32_t move_at(const StepMasks& s, uint32_t p, const Moves& mv) {
    const bool hs = (s.hs >> p) & 1ull;
    const bool up = (s.up >> p) & 1ull;
    return hs ? 64 : (up ? mv.up : -mv.down);
}

// The map of one block: its moves composed in step order.
__device__ __forceinline__ ClampAdd block_map(const StepMasks& s, const Moves& mv) {
    ClampAdd f{0, mv.lmin, mv.lmax};
    uint64_t c = s.hs | s.up | s.dn;
    while (c) {
        const uint32_t p = (uint32_t)__builtin_ctzll(c);
        c &= c - 1;
        const int32_t d = move_at(s, p, mv);
        f.a += d;
        f.lo = min(max(f.lo + d, mv.lmin), mv.lmax);
        f.hi = min(max(f.hi + d, mv.lmin), mv.lmax);
    }
    return f;
}

// Level sum and transitions of steps [0, n) of a block entered at level x.
__device__ __forceinline__ void block_walk(const StepMasks& s, const Moves& mv, int32_t x,
                                           uint32_t n, uint32_t& lsum, uint32_t& trans) {
    uint64_t c = s.hs | s.up | s.dn;
    int32_t lv = x;
    uint32_t last = 0;
    while (c) {
        const uint32_t p = (uint32_t)__builtin_ctzll(c);
        c &= c - 1;
        lsum += (uint32_t)lv * (p - last);
        const int32_t nl = min(max(lv + move_at(s, p, mv), mv.lmin), mv.lmax);
        trans += nl != lv;
        lv = nl;
        last = p;
    }
    lsum += (uint32_t)lv * (n - last);
}

// The Alg. 1 / Alg. 2 masks of 64 blocks (events, rises, high steps), block
// j in lane j, as pairs of 32-bit halves.
struct ParkedMasks {
    uint32_t e0, e1, r0, r1, h0, h1;
    __device__ __forceinline__ BlockMasks get() const {
        BlockMasks m;
        m.E = ((uint64_t)e1 << 32) | e0;
        m.R = ((uint64_t)r1 << 32) | r0;
        m.HM = ((uint64_t)h1 << 32) | h0;
        return m;
    }
};

// f of an earlier lane picked by a DPP control (row shift or row broadcast);
// lanes with no such lane, or outside the rows of kRowMask, get `id`.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ ClampAdd dpp_earlier(const ClampAdd& f, const ClampAdd& id) {
    ClampAdd o;
    o.a = __builtin_amdgcn_update_dpp(id.a, f.a, kCtrl, kRowMask, 0xf, false);
    o.lo = __builtin_amdgcn_update_dpp(id.lo, f.lo, kCtrl, kRowMask, 0xf, false);
    o.hi = __builtin_amdgcn_update_dpp(id.hi, f.hi, kCtrl, kRowMask, 0xf, false);
    return o;
}

// Inclusive wave scan: lane i gets the composition of the maps of lanes 0..i
// (lane 0 first).  Within each row of 16 lanes by shifts of 1, 2, 4 and 8,
// then the last lane of row 0 / 2 is composed into rows 1 / 3 and the last
// lane of row 1 into rows 2 and 3.  `id` is the identity map of the level
// range; composing with it changes the representation of a map but not the
// map on that range.
__device__ __forceinline__ ClampAdd wave_scan(ClampAdd f, const ClampAdd& id) {
    f = compose(dpp_earlier<0x111, 0xf>(f, id), f);   // row_shr:1
    f = compose(dpp_earlier<0x112, 0xf>(f, id), f);   // row_shr:2
    f = compose(dpp_earlier<0x114, 0xf>(f, id), f);   // row_shr:4
    f = compose(dpp_earlier<0x118, 0xf>(f, id), f);   // row_shr:8
    f = compose(dpp_earlier<0x142, 0xa>(f, id), f);   // row_bcast:15 into rows 1, 3
    f = compose(dpp_earlier<0x143, 0xc>(f, id), f);   // row_bcast:31 into rows 2, 3
    return f;
}

// Ordered wave reduction: the composition of the maps of lanes 0..63,
// wave-uniform.
__device__ __forceinline__ ClampAdd wave_compose(ClampAdd f, const ClampAdd& id) {
    f = wave_scan(f, id);
    ClampAdd r;
    r.a = __builtin_amdgcn_readlane(f.a, 63);
    r.lo = __builtin_amdgcn_readlane(f.lo, 63);
    r.hi = __builtin_amdgcn_readlane(f.hi, 63);
    return r;
}

// A block map in one word for pass 2.  A move of 32 rungs or more saturates
// every level of a 0..31 ladder, so a in [-64, 64] represents the map
// exactly, and so does every composition with it.
__device__ __forceinline__ int32_t clamp_move(int32_t a) { return min(max(a, -64), 64); }

__device__ __forceinline__ uint32_t pack_map(const ClampAdd& f) {
    return (uint32_t)(clamp_move(f.a) + 64) | ((uint32_t)f.lo << 8) | ((uint32_t)f.hi << 16);
}

__device__ __forceinline__ ClampAdd unpack_map(uint32_t w) {
    return ClampAdd{(int32_t)(w & 0xFFu) - 64, (int32_t)((w >> 8) & 0xFFu), (int32_t)(w >> 16)};
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) { return dpp_wave_sum64(v); }

// Pass 1: masks of every block, the map and the high steps of every chunk.
template <bool kAnyBase>
__global__ __launch_bounds__(kWaves * kWave) void stepped_mask_kernel(
    const uint32_t* __restrict__ samples, const uint64_t* __restrict__ offsets,
    uint32_t n_traces, const uint32_t* __restrict__ chunk_base,
    const DevCfg* __restrict__ cfgs, const uint32_t* __restrict__ cfg_of_trace,
    uint32_t chunk, uint64_t n_blocks, ClampAdd* __restrict__ funcs,
    StepSum* __restrict__ sums, uint64_t* __restrict__ masks)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t g = blockIdx.x * kWaves + wave_uniform(threadIdx.x >> 6);
    if (g >= chunk_base[n_traces]) return;
    const ChunkView v = chunk_view(samples, offsets, n_traces, chunk_base, cfgs, cfg_of_trace,
                                   chunk, g);
    const Moves mv = moves_of(v.c);
    const uint64_t b0 = first_block(v.tbase, v.s, v.t);
    uint64_t* out = masks + b0;
    uint32_t* out_map = reinterpret_cast<uint32_t*>(masks + 3 * n_blocks) + b0;
    ClampAdd F{0, mv.lmin, mv.lmax};                   // identity
    uint32_t j = 0, th = 0;                            // th: per lane
    uint32_t hm_carry = 0;     // the last block of the previous group ended high
    // raw masks of block j in lane j (E, R, HM as halves); the step masks are
    // derived per lane at the flush, once per 64 blocks
    ParkedMasks pk{0, 0, 0, 0, 0, 0};
    auto flush = [&](uint32_t cnt) {
        const BlockMasks m = pk.get();
        th += (uint32_t)__popcll(m.HM);
        // high before the block: the last step of block j-1 (lane j-1)
        uint32_t before = (uint32_t)__shfl_up((int)(pk.h1 >> 31), 1, 64);
        if (lane == 0) before = hm_carry;
        hm_carry = (uint32_t)__builtin_amdgcn_readlane((int)(pk.h1 >> 31), (int)(cnt - 1));
        const StepMasks sm = step_masks(m, before);
        const ClampAdd f = block_map(sm, mv);
        if (lane < cnt) {
            out[lane] = sm.hs;
            out[n_blocks + lane] = sm.up;
            out[2 * n_blocks + lane] = sm.dn;
            out_map[lane] = pack_map(f);
        }
        out += cnt;
        out_map += cnt;
        F = compose(F, wave_compose(f, ClampAdd{0, mv.lmin, mv.lmax}));
        F.a = clamp_move(F.a);
        pk = ParkedMasks{0, 0, 0, 0, 0, 0};
    };
    for_each_block<kGroupBlocks, kAnyBase>(v, lane, [&](const BlockMasks& m, uint32_t, uint64_t,
                                                        uint32_t) {
        // a block with no event and no high step moves nothing; its lane
        // stays zero
        if ((m.E | m.HM) != 0) {
            writelane_into(pk.e0, (uint32_t)m.E, j);
            writelane_into(pk.e1, (uint32_t)(m.E >> 32), j);
            writelane_into(pk.r0, (uint32_t)m.R, j);
            writelane_into(pk.r1, (uint32_t)(m.R >> 32), j);
            writelane_into(pk.h0, (uint32_t)m.HM, j);
            writelane_into(pk.h1, (uint32_t)(m.HM >> 32), j);
        }
        ++j;
    }, [&]() {
        // a group adds at most kGroupBlocks blocks, so lane j stays below 64
        if (j > 64 - kGroupBlocks) {
            flush(j);
            j = 0;
        }
    });
    if (j) flush(j);
    th = (uint32_t)wave_sum_u64(th);
    if (lane == 0) {
        funcs[g] = F;
        sums[g].ticks_high = th;
    }
}

// Pass 2 from the masks: level sum and transitions of every chunk.
__global__ __launch_bounds__(kWaves * kWave) void stepped_walk_kernel(
    const uint64_t* __restrict__ offsets, uint32_t n_traces,
    const uint32_t* __restrict__ chunk_base, const DevCfg* __restrict__ cfgs,
    const uint32_t* __restrict__ cfg_of_trace, uint32_t chunk, uint64_t n_blocks,
    const uint32_t* __restrict__ entering, const uint64_t* __restrict__ masks,
    StepSum* __restrict__ sums)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t g = blockIdx.x * kWaves + wave_uniform(threadIdx.x >> 6);
    if (g >= chunk_base[n_traces]) return;
    const uint32_t t = trace_of_chunk(chunk_base, n_traces, g, lane);
    const uint64_t tbase = offsets[t];
    const uint32_t n = (uint32_t)(offsets[t + 1] - tbase);
    const uint32_t s = (g - chunk_base[t]) * chunk;
    const uint32_t len = min(s + chunk, n) - s;
    const Moves mv = moves_of(cfgs[cfg_of_trace ? cfg_of_trace[t] : 0]);
    const uint64_t b0 = first_block(tbase, s, t);
    const uint64_t* in = masks + b0;
    const uint32_t* in_map = reinterpret_cast<const uint32_t*>(masks + 3 * n_blocks) + b0;
    const uint32_t nblk = (len + 63) >> 6;
    int32_t x = (int32_t)entering[g];                  // level before the group
    uint32_t lsum = 0, trans = 0;
    for (uint32_t b0 = 0; b0 < nblk; b0 += 64) {
        const uint32_t j = b0 + lane;
        StepMasks sm{0, 0, 0};
        ClampAdd f{0, mv.lmin, mv.lmax};
        uint32_t steps = 0;
        if (j < nblk) {
            sm.hs = in[j];
            sm.up = in[n_blocks + j];
            sm.dn = in[2 * n_blocks + j];
            f = unpack_map(in_map[j]);
            steps = min(64u, len - 64 * j);
        }
        const ClampAdd incl = wave_scan(f, ClampAdd{0, mv.lmin, mv.lmax});
        int32_t after = apply(incl, x);                // level after this lane's block
        int32_t before = __shfl_up(after, 1, 64);
        if (lane == 0) before = x;
        block_walk(sm, mv, before, steps, lsum, trans);
        x = __builtin_amdgcn_readlane(after, 63);
    }
    const uint64_t ls = dpp_wave_sum64(lsum);
    trans = (uint32_t)dpp_wave_sum64(trans);
    if (lane == 0) {
        sums[g].level_sum = ls;
        sums[g].transitions = trans;
    }
}

// Fold 1: the level entering every chunk.  One wave per trace; lane k takes
// chunk k of each group of 64 chunks and an inclusive wave scan composes
// their maps.
__global__ __launch_bounds__(kWaves * kWave) void stepped_enter_kernel(
    uint32_t n_traces, const uint32_t* __restrict__ chunk_base,
    const DevCfg* __restrict__ cfgs, const uint32_t* __restrict__ cfg_of_trace,
    const ClampAdd* __restrict__ funcs, uint32_t* __restrict__ entering)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t t = blockIdx.x * kWaves + wave_uniform(threadIdx.x >> 6);
    if (t >= n_traces || chunk_base[n_traces + 1] != 0) return;
    const DevCfg c = cfgs[cfg_of_trace ? cfg_of_trace[t] : 0];
    int32_t x = (int32_t)c.linit;
    const uint32_t k1 = chunk_base[t + 1];
    for (uint32_t k0 = chunk_base[t]; k0 < k1; k0 += 64) {
        const uint32_t k = k0 + lane;
        ClampAdd f{0, (int32_t)c.lmin, (int32_t)c.lmax};
        if (k < k1) {
            f = funcs[k];
            f.a = clamp_move(f.a);
        }
        const int32_t after =
            apply(wave_scan(f, ClampAdd{0, (int32_t)c.lmin, (int32_t)c.lmax}), x);
        int32_t before = __shfl_up(after, 1, 64);
        if (lane == 0) before = x;
        if (k < k1) entering[k] = (uint32_t)before;
        x = __builtin_amdgcn_readlane(after, 63);
    }
}

// Pass 2 from the samples: levels, sums and decision bytes of every chunk.
template <bool kAnyBase>
__global__ __launch_bounds__(kWaves * kWave) void stepped_levels_kernel(
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
    for_each_block<8, kAnyBase>(v, lane, [&](const BlockMasks& m, uint32_t tb, uint64_t valid,
                                             uint32_t) {
        int32_t lv;
        if (((m.E | m.HM)) == 0) {
            lv = x;                                    // 64 identity steps
        } else {
            // lane i gets the map of steps 0..i of the block
            const ClampAdd f = wave_scan(step_map(m, v.c, lane),
                                         ClampAdd{0, (int32_t)v.c.lmin, (int32_t)v.c.lmax});
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
        if (ok) {
            const bool hb = (m.HM >> lane) & 1ull;
            const bool ev = (m.E >> lane) & 1ull;
            const bool up = (m.R >> lane) & 1ull;
            const uint32_t pr = ev ? (up ? 2u : 0u) : 1u;
            levels[v.tbase + tb + lane] = (uint8_t)((uint32_t)lv | ((uint32_t)hb << 5) |
                                                    (pr << 6));
        }
        const uint32_t last = min(64u, v.e - tb) - 1;
        x = __builtin_amdgcn_readlane(lv, (int)last);
    });
    lsum = dpp_wave_sum64(lsum);
    trans = (uint32_t)dpp_wave_sum64(trans);
    if (lane == 0) {
        StepSum r;
        r.level_sum = lsum;
        r.transitions = trans;
        r.ticks_high = th;
        sums[g] = r;
    }
}

// One wave per trace: lane k adds chunks k, k + 64, ...
__global__ __launch_bounds__(kWaves * kWave) void stepped_fold_kernel(
    uint32_t n_traces, const uint32_t* __restrict__ chunk_base,
    const StepSum* __restrict__ sums, magus_result* __restrict__ results)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t t = blockIdx.x * kWaves + wave_uniform(threadIdx.x >> 6);
    if (t >= n_traces || chunk_base[n_traces + 1] != 0) return;
    uint64_t level_sum = 0, trans = 0, th = 0;
    for (uint32_t k = chunk_base[t] + lane; k < chunk_base[t + 1]; k += 64) {
        level_sum += sums[k].level_sum;
        trans += sums[k].transitions;
        th += sums[k].ticks_high;
    }
    level_sum = wave_sum_u64(level_sum);
    trans = wave_sum_u64(trans);
    th = wave_sum_u64(th);
    if (lane == 0) {
        magus_result r;
        r.score = level_sum + 1000ull * trans;
        r.level_sum = level_sum;
        r.transitions = trans;
        r.ticks_high = th;
        results[t] = r;
    }
}

}  // namespace

hipError_t launch_stepped_prepare(const uint32_t* samples, uint64_t n_samples,
                                  const uint64_t* offsets, uint32_t n_traces, const DevCfg* cfgs,
                                  uint32_t n_cfgs, const uint32_t* cfg_of_trace, uint32_t chunk,
                                  uint32_t* chunk_base, uint32_t max_chunks, ClampAdd* funcs,
                                  uint32_t* entering, StepSum* sums, uint64_t* masks,
                                  uint32_t* err, bool any_base, hipStream_t stream,
                                  hipEvent_t ev0)
{
    if (n_traces == 0) return hipSuccess;
    hipError_t e = launch_plan(offsets, n_traces, n_samples, cfg_of_trace, n_cfgs, chunk,
                               max_chunks, chunk_base, err, stream);
    if (e != hipSuccess) return e;
    if ((e = record_timing_event(ev0, stream)) != hipSuccess) return e;
    const uint32_t blocks = (max_chunks + kWaves - 1) / kWaves;
    (any_base ? stepped_mask_kernel<true> : stepped_mask_kernel<false>)
        <<<blocks, kWaves * kWave, 0, stream>>>(samples, offsets, n_traces, chunk_base, cfgs,
                                                cfg_of_trace, chunk,
                                                stepped_mask_blocks(n_samples, n_traces), funcs,
                                                sums, masks);
    stepped_enter_kernel<<<(n_traces + kWaves - 1) / kWaves, kWaves * kWave, 0, stream>>>(
        n_traces, chunk_base, cfgs, cfg_of_trace, funcs, entering);
    return hipGetLastError();
}

hipError_t launch_replay_stepped(const uint32_t* samples, uint64_t n_samples,
                                 const uint64_t* offsets, uint32_t n_traces, const DevCfg* cfgs,
                                 uint32_t n_cfgs, const uint32_t* cfg_of_trace, uint32_t chunk,
                                 uint32_t* chunk_base, uint32_t max_chunks, ClampAdd* funcs,
                                 uint32_t* entering, StepSum* sums, uint64_t* masks,
                                 magus_result* results, uint8_t* levels, uint32_t* err,
                                 bool any_base, hipStream_t stream, hipEvent_t ev0,
                                 hipEvent_t ev1)
{
    if (n_traces == 0) return hipSuccess;
    hipError_t e = launch_stepped_prepare(samples, n_samples, offsets, n_traces, cfgs, n_cfgs,
                                          cfg_of_trace, chunk, chunk_base, max_chunks, funcs,
                                          entering, sums, masks, err, any_base, stream, ev0);
    if (e != hipSuccess) return e;
    const uint32_t blocks = (max_chunks + kWaves - 1) / kWaves;
    const uint64_t n_blocks = stepped_mask_blocks(n_samples, n_traces);
    const uint32_t trace_blocks = (n_traces + kWaves - 1) / kWaves;
    if (levels)
        (any_base ? stepped_levels_kernel<true> : stepped_levels_kernel<false>)
            <<<blocks, kWaves * kWave, 0, stream>>>(samples, offsets, n_traces, chunk_base, cfgs,
                                                    cfg_of_trace, chunk, entering, sums, levels);
    else
        stepped_walk_kernel<<<blocks, kWaves * kWave, 0, stream>>>(
            offsets, n_traces, chunk_base, cfgs, cfg_of_trace, chunk, n_blocks, entering, masks,
            sums);
    if ((e = record_timing_event(ev1, stream)) != hipSuccess) return e;
    stepped_fold_kernel<<<trace_blocks, kWaves * kWave, 0, stream>>>(n_traces, chunk_base, sums,
                                                                     results);
    return hipGetLastError();
}

}  // namespace magus
