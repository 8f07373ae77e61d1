// Internal types shared by the host side and the gfx950 kernels of libmagus.
#pragma once

#include <vector>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "magus.h"

namespace magus {

constexpr int kWave = 64;

// Cache policy of the buffer loads of samples that a pass reads once: the
// non-temporal hint (the nt bit), so the stream does not displace data that
// is reused.  Measured on the bulk replay: 2.5 % less kernel time than plain
// loads (6.1 TB/s instead of 5.95 TB/s).
constexpr int kStreamLoad = 2;

// Controller parameters in the form the kernels use (derived on the host from
// magus_config).  32 bytes.
struct DevCfg {
    uint32_t W;          // derivative window
    uint32_t H;          // event FIFO length
    uint32_t mu;         // W * inc_q16    (E1': (hi-lo) * 2^16 > lo * mu -> +1)
    uint32_t md;         // W * |dec_q16|  (E1': (hi-lo) * 2^16 > lo * md -> -1)
    uint32_t ref;        // B_ref of the fixed-reference base (base 3), else 0
    uint32_t pad;
    uint16_t thr;        // ceil(hf_num * H / hf_den): high iff events >= thr
    uint8_t up, down;    // step sizes of an executed +1 / -1 (0 = to the bound)
    uint8_t lmin, lmax, linit;
    uint8_t base;        // derivative base: 0 min(oldest, newest), 1 oldest, 2 newest,
                         // 3 the fixed reference `ref`
};
static_assert(sizeof(DevCfg) == 32, "DevCfg layout");

// Base of the derivative of Alg. 1 for one step: the smaller of the two
// samples, or (alternative readings) the oldest, the newest, or the fixed
// reference `ref` (base 3).
__device__ __forceinline__ uint32_t derivative_base(uint32_t a, uint32_t b, uint32_t base,
                                                    uint32_t ref) {
    // masking the excluded sample to all-ones turns min() into a selection
    const uint32_t mo = base >= 2 ? 0xFFFFFFFFu : 0u;
    const uint32_t mn = base == 1 || base == 3 ? 0xFFFFFFFFu : 0u;
    const uint32_t m = min(a | mo, b | mn);
    return base == 3 ? ref : m;
}

// Trace of chunk g: the last t with chunk_base[t] <= g, for a non-decreasing
// chunk_base[0..n_traces] with chunk_base[n_traces] > g.  A 64-way search:
// every lane probes one position per round, so a round shrinks the range 64x
// (two rounds for 4,096 traces instead of twelve dependent loads).  Called by
// a whole wave; the result is wave-uniform.
__device__ __forceinline__ uint32_t trace_of_chunk(const uint32_t* chunk_base,
                                                   uint32_t n_traces, uint32_t g,
                                                   uint32_t lane) {
    uint32_t lo = 0, hi = n_traces;
    while (hi - lo > 1) {
        const uint32_t step = (hi - lo + 63) >> 6;
        const uint32_t idx = lo + lane * step;
        const bool le = idx < hi && chunk_base[idx] <= g;   // a prefix of the lanes
        const uint64_t m = __ballot(le);                    // lane 0 (idx = lo) is set
        const uint32_t k = 63u - (uint32_t)__builtin_clzll(m);
        lo += k * step;
        hi = min(lo + step, hi);
        lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)lo);
        hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)hi);
    }
    return lo;
}

__device__ int llvm_writelane(int v, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

// lane `lane` of `dst` := v (lane wave-uniform)
__device__ __forceinline__ void writelane_into(uint32_t& dst, uint32_t v, uint32_t lane) {
    dst = (uint32_t)llvm_writelane((int)v, (int)lane, (int)dst);
}

// Summary of one time chunk of one trace, computed without knowing the level
// entering the chunk (taken as level_min for the bit vector).  32 bytes.
struct ChunkSum {
    uint32_t len;        // steps in the chunk
    uint32_t prefix;     // steps before the first decisive step (== len if none)
    uint32_t first_up;   // the first decisive step sets level_max (1) or level_min (0)
    uint32_t end_up;     // level after the last step is level_max (valid if prefix < len)
    uint32_t cnt_max;    // steps at level_max
    uint32_t trans0;     // level changes, counting the entering level as level_min
    uint32_t ticks_high; // steps in the high state
    uint32_t pad;
};
static_assert(sizeof(ChunkSum) == 32, "ChunkSum layout");

// Per-chunk fix-up record for per-step output: the steps before the first
// decisive step of a chunk take the level entering the chunk, known only after
// the chunk summaries of the trace are folded.
struct ChunkFix {
    uint64_t start;      // absolute index of the chunk's first sample
    uint32_t prefix;     // steps to fix
    uint32_t level;      // level entering the chunk (written by the fold)
};

// Device error word bits.
enum : uint32_t {
    kErrOffsets = 1u,    // offsets not monotone / beyond n_samples
    kErrTooLong = 2u,    // a trace longer than MAGUS_MAX_TRACE_LEN
    kErrCfgIndex = 4u,   // cfg_of_trace out of range
};

// Clamp-add map of levels, f(x) = min(max(x + a, lo), hi) with lo <= hi: the
// effect of one step (or of a run of steps) of the decision rule on the level.
struct ClampAdd {
    int32_t a, lo, hi;
};

// Per-chunk partial sums of the stepped-actuation replay (entering level known).
struct StepSum {
    uint64_t level_sum;
    uint32_t transitions;
    uint32_t ticks_high;
};

// Records a timing event on `stream` (nothing when ev is null).  Under stream
// capture it adds an event-record node after the work captured so far and
// makes the work captured next depend on it; each launch of the graph can
// then point the node at an event of its own.  The nodes added are appended
// to *capture_marks while that is set (by the thread that captures).
hipError_t record_timing_event(hipEvent_t ev, hipStream_t stream);
extern thread_local std::vector<hipGraphNode_t>* capture_marks;

// Kernel launchers (replay.hip / sweep.hip / serve.hip).  When ev0/ev1 are
// not null they are recorded on `stream` right before and after the dominant
// kernel of the call (the chunk, sweep or serve-step kernel); the replay
// launchers record them with record_timing_event.
hipError_t launch_replay(const uint32_t* samples, uint64_t n_samples, const uint64_t* offsets,
                         uint32_t n_traces, const DevCfg* cfgs, uint32_t n_cfgs,
                         const uint32_t* cfg_of_trace, uint32_t chunk, uint32_t* chunk_base,
                         ChunkSum* sums, uint32_t max_chunks, ChunkFix* fix,
                         magus_result* results, uint8_t* levels, uint32_t* err,
                         uint32_t persistent_blocks, bool any_base, hipStream_t stream,
                         hipEvent_t ev0, hipEvent_t ev1, uint32_t* status_out = nullptr);

// Around the chunk kernel (replay_fold.hip): the plan (chunk prefix per trace,
// data checks, status word chunk_base[n_traces + 1], ORed into *err and copied
// to *status_out where those are not null), the fold of the chunk summaries of every trace
// (fix: optional, receives the level entering each chunk) and the fix-up of the
// decision bytes of the steps before each chunk's first decisive step.
hipError_t launch_plan(const uint64_t* offsets, uint32_t n_traces, uint64_t n_samples,
                       const uint32_t* cfg_of_trace, uint32_t n_cfgs, uint32_t chunk,
                       uint32_t max_chunks, uint32_t* chunk_base, uint32_t* err,
                       hipStream_t stream, uint32_t* status_out = nullptr);
hipError_t launch_fold(const uint64_t* offsets, uint32_t n_traces, const uint32_t* chunk_base,
                       const ChunkSum* sums, const DevCfg* cfgs, const uint32_t* cfg_of_trace,
                       magus_result* results, ChunkFix* fix, hipStream_t stream);
hipError_t launch_fixup(uint32_t n_traces, const uint32_t* chunk_base, const ChunkFix* fix,
                        uint32_t max_chunks, uint8_t* levels, hipStream_t stream);

// Replay for configs with stepped actuation (stepped.hip): pass 1 reads the
// samples once and writes the chunk's clamp-add map, the masks of the steps
// that can move the level and each block's map (`masks`: 28 B per slot of
// stepped_mask_blocks()); pass 2 accumulates with the entering level
// that the per-trace fold derived, from the masks, or from the samples when
// `levels` is not null.
hipError_t launch_replay_stepped(const uint32_t* samples, uint64_t n_samples,
                                 const uint64_t* offsets, uint32_t n_traces, const DevCfg* cfgs,
                                 uint32_t n_cfgs, const uint32_t* cfg_of_trace, uint32_t chunk,
                                 uint32_t* chunk_base, uint32_t max_chunks, ClampAdd* funcs,
                                 uint32_t* entering, StepSum* sums, uint64_t* masks,
                                 magus_result* results, uint8_t* levels, uint32_t* err,
                                 bool any_base, hipStream_t stream, hipEvent_t ev0,
                                 hipEvent_t ev1);
// Slots per array of the stepped replay's block scratch (one slot per
// 64-step block): three uint64 step-mask arrays (moves up, down, set max) and
// one uint32 map array.
inline uint64_t stepped_mask_blocks(uint64_t n_samples, uint32_t n_traces) {
    return n_samples / 64 + n_traces + 1;
}
// Slot of the first block of a chunk starting at step s of trace t (first
// sample tbase): blocks of one trace start 64 steps apart, so
// (absolute first step) / 64 + trace is one-to-one over all blocks of a batch
// and stays below stepped_mask_blocks().
__host__ __device__ __forceinline__ uint64_t first_block(uint64_t tbase, uint32_t s, uint32_t t) {
    return (tbase + s) / 64 + t;
}
// Pass 1 of the stepped replay and the fold of the chunk maps: the step
// masks of every block, the map of every chunk and the level entering every
// chunk (what the proxy statistics need without the replay's pass 2).  ev0,
// if not null, is recorded after the plan kernel.
hipError_t launch_stepped_prepare(const uint32_t* samples, uint64_t n_samples,
                                  const uint64_t* offsets, uint32_t n_traces, const DevCfg* cfgs,
                                  uint32_t n_cfgs, const uint32_t* cfg_of_trace, uint32_t chunk,
                                  uint32_t* chunk_base, uint32_t max_chunks, ClampAdd* funcs,
                                  uint32_t* entering, StepSum* sums, uint64_t* masks,
                                  uint32_t* err, bool any_base, hipStream_t stream,
                                  hipEvent_t ev0 = nullptr);

// Counter readings to MB/s samples (frontend.hip).
hipError_t launch_counters(const uint64_t* counts, const uint64_t* ts, const uint64_t* offsets,
                           uint32_t n_traces, uint64_t n_readings, uint32_t bits, uint32_t bpc,
                           uint32_t* status, uint32_t* err, uint32_t* out, hipStream_t stream);

struct SweepPlan {
    uint32_t n_blocks;        // config blocks of kSweepLanes lanes, one window each
    const uint32_t* block_w;  // [n_blocks] window | base << 8
    const uint32_t* block_ref;// [n_blocks] B_ref of base-3 blocks (else 0)
    const int32_t* lane_inc;  // [n_blocks * kSweepLanes]
    const int32_t* lane_dec;
    const uint32_t* lane_hmask;
    const uint32_t* lane_thr;
    const uint32_t* lane_lv;  // lmin | lmax << 8 | linit << 16
    const uint32_t* lane_orig;// original config index, 0xFFFFFFFF = padding
    const uint32_t* lane_steps;   // up_step | down_step << 8
    const uint32_t* block_stepped;// [n_blocks] 1 if any lane has a step size
};
constexpr int kSweepLanes = 256;

// Launch shapes of the sweep kernel: configs per workgroup (a block of
// kSweepLanes configs, or an equal part of one) and steps per LDS tile.
// Every shape gives the same scores.
struct SweepShape {
    uint32_t lanes, tile;
};
constexpr SweepShape kSweepShapes[] = {{256, 256}, {256, 512}, {256, 1024},
                                       {128, 256}, {128, 512}, {64, 256}};
constexpr uint32_t kSweepShapeCount = sizeof(kSweepShapes) / sizeof(kSweepShapes[0]);

hipError_t launch_sweep(const uint32_t* samples, uint64_t n_samples, const uint64_t* offsets,
                        uint32_t n_traces, const SweepPlan& plan, uint32_t n_cfgs,
                        uint64_t* scores, uint32_t* argmin, uint64_t* keys, uint32_t* err,
                        uint32_t shape, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1);

// VALU issue-rate probe (valu_probe.hip): `steps` rounds per lane of
// independent 32-bit instructions (mode 0: v_add_u32; mode 1: the sweep
// step's compare / add-with-carry / and / bcnt), workgroups of kSweepLanes
// lanes, one uint32 per lane written to out.
hipError_t launch_valu_probe(uint32_t workgroups, uint32_t steps, uint32_t mode, uint32_t seed,
                             uint32_t* out, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1);
// VALU instructions per lane and round of a probe mode.
uint32_t valu_probe_ops_per_step(uint32_t mode);

// Streaming-read probe (read_probe.hip): one wave per chunk of `chunk`
// samples reads them with the replay chunk kernel's access pattern; one
// uint32 per chunk written to out.
hipError_t launch_read_probe(const uint32_t* samples, uint64_t n_samples, uint32_t chunk,
                             uint32_t* out, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1);

// Serving slot state.
struct SlotState {
    uint32_t ring[31];   // last W-1 samples, sample k at ring[k % (W-1)]
    uint32_t ticks;      // samples seen
};
static_assert(sizeof(SlotState) == 128, "SlotState layout");
struct SlotAcc {
    uint64_t level_sum;
    uint64_t transitions;
    uint64_t ticks_high;
    uint32_t hist;       // event flags, newest in bit 0
    uint32_t level;
};
static_assert(sizeof(SlotAcc) == 32, "SlotAcc layout");

struct ServeInit {       // (re)initialises one slot
    uint32_t slot;
    uint32_t pad;
    DevCfg cfg;
};

hipError_t launch_serve(SlotState* st, SlotAcc* acc, DevCfg* slot_cfg,
                        const ServeInit* inits, uint32_t n_inits,
                        const uint32_t* pairs /* slot[n] then sample[n] */, uint32_t n,
                        uint8_t* decisions, hipStream_t stream, hipEvent_t ev0,
                        hipEvent_t ev1);

}  // namespace magus
