/*
 * magus.h -- C ABI of the MI355X (gfx950) library that replays, sweeps and
 * serves the MAGUS uncore-frequency controller (arXiv 2502.03796) in batch.
 *
 * The controller, per monitoring step of one telemetry stream (Sec. 3):
 *   - Alg. 1 (memory throughput trend prediction): the derivative of the
 *     newest vs the oldest of the last `window` throughput samples, taken
 *     relative to the smaller of the two and divided by the window,
 *       r = (x[t] - x[t-W+1]) / (W * min(x[t], x[t-W+1])),
 *     gives +1 if r > inc, -1 if r < dec, else 0 (the "temporary decision").
 *     Thresholds are Q16.16 integers and the comparison is exact.  The first
 *     W-1 steps of a stream predict 0.
 *   - Sec. 3.2: a flag (prediction != 0) is pushed into the event FIFO
 *     uncore_tune_ls of length `hold` (H, zero-filled at start), also while
 *     the high state holds.
 *   - Alg. 2 (high frequency detection): high if sum/len >= hf_num/hf_den
 *     (0.6 = 3/5 in Sec. 3.2).
 *   - Decision (Sec. 3.2, Sec. 4, Sec. 6.1): high or +1 -> level_max; else -1
 *     -> level_min (straight to the lower bound); else keep.  Streams start at
 *     level_init (idle nodes sit at the minimum, Sec. 4).  Optionally an
 *     executed +1 / -1 moves by up_step / down_step rungs instead.
 *   - Accounting per step, after the decision: transitions += (level changed);
 *     level_sum += level; score = level_sum + 1000 * transitions.
 *
 * Conventions for every call:
 *   - d_* pointers are device memory (any allocator, e.g. torch tensors) owned
 *     by the caller; h_* pointers are host memory owned by the caller.
 *   - Calls return MAGUS_OK (0) or a negative MAGUS_E* code and never throw.
 *     The message of the last failure on the calling thread is available from
 *     magus_last_error().
 *   - Host-side arguments (configs, sizes) are validated synchronously.  Work
 *     is enqueued on `stream` (a hipStream_t; NULL is the default stream) and
 *     runs asynchronously; data faults found on the device (non-monotone
 *     offsets, config index out of range, trace too long) produce no output
 *     and are reported by the next magus_ctx_check().
 *   - One context serves one stream at a time: calls on the same context from
 *     different streams that overlap in time race on its scratch memory.
 */
#ifndef MAGUS_H
#define MAGUS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MAGUS_OK 0
#define MAGUS_EINVAL (-1)   /* bad argument or config                          */
#define MAGUS_ENOMEM (-2)   /* device or pinned host allocation failed         */
#define MAGUS_ENOSLOT (-3)  /* serving: no free slot within the memory budget  */
#define MAGUS_EDEVICE (-4)  /* a HIP runtime call failed                        */
#define MAGUS_EDATA (-5)    /* device-side data check failed (magus_ctx_check)  */

/* Longest trace (samples) accepted by replay and sweep. */
#define MAGUS_MAX_TRACE_LEN ((1u << 30) - 1u)

/*
 * One controller configuration (Alg. 1 and Alg. 2 arguments, Sec. 3.2 rule).
 *   window      W = direv_length of Alg. 1, 2..32.
 *   hold        H = len(uncore_tune_ls) of Alg. 2, 1..32.
 *   inc_q16     inc_threshold as a Q16.16 integer, 0..2^20 (e.g. 0.1 -> 6554).
 *   dec_q16     dec_threshold as a Q16.16 integer, -2^20..0.
 *   hf_num/den  high_freq_threshold = hf_num / hf_den, 0 <= num <= den, den >= 1
 *               (Sec. 3.2 uses 0.6 = 3/5).
 *   level_min   lower bound on the uncore ladder (level i = 800 + 100 i MHz on
 *   level_max   the 17-level 0.8-2.4 GHz ladder); min < max <= 31.
 *   level_init  level before the first step, min <= init <= max (Sec. 4: min).
 *   up_step,    0 = an executed +1 / -1 jumps to level_max / level_min (the
 *   down_step   paper's policy, Sec. 6.1); 1..31 = it moves the level by that
 *               many rungs, clamped to [level_min, level_max] (the gradual
 *               policy Sec. 6.1 contrasts with; "how much to increase or
 *               decrease", Sec. 2).  The high state always goes to level_max.
 *   base        derivative base: 0 = min(oldest, newest) (the default reading:
 *               symmetric for rises and falls), 1 = the oldest sample, 2 = the
 *               newest sample, 3 = the fixed reference base_ref (alternative
 *               readings of Alg. 1 kept for sensitivity sweeps).
 *   base_ref    B_ref in MB/s, >= 1, for base 3 (ignored otherwise): the
 *               derivative is (x[t] - x[t-W+1]) / (W * B_ref), which is
 *               Alg. 1's own absolute derivative (newest - oldest) /
 *               direv_length in units of B_ref MB/s per step; an absolute
 *               threshold of theta MB/s per step is inc = theta / B_ref.
 */
typedef struct magus_config {
    uint16_t window;
    uint16_t hold;
    int32_t inc_q16;
    int32_t dec_q16;
    uint8_t hf_num, hf_den;
    uint8_t level_min, level_max;
    uint8_t level_init;
    uint8_t up_step, down_step;
    uint8_t base;
    uint32_t base_ref;
} magus_config;

/* Per-trace replay result. */
typedef struct magus_result {
    uint64_t score;             /* level_sum + 1000 * transitions             */
    uint64_t level_sum;         /* sum over steps of the level after the step */
    uint64_t transitions;       /* steps whose level differs from the last    */
    uint64_t ticks_high;        /* steps in the high-frequency state          */
} magus_result;

typedef struct magus_ctx magus_ctx;
typedef struct magus_server magus_server;

/* Per-step decision byte: bits 0-4 level, bit 5 high, bits 6-7 prediction+1. */
#define MAGUS_DECISION_LEVEL(b) ((b) & 31u)
#define MAGUS_DECISION_HIGH(b) (((b) >> 5) & 1u)
#define MAGUS_DECISION_PRED(b) ((int)(((b) >> 6) & 3u) - 1)

/* Library version string. */
const char* magus_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char* magus_last_error(void);

/* Checks a config on the host; MAGUS_OK or MAGUS_EINVAL. */
int magus_config_check(const magus_config* h_cfg);

/*
 * Creates a context on HIP device `device`.  The context owns its scratch
 * memory (chunk summaries, config tables, device error word), grown on demand
 * and freed by magus_ctx_destroy.
 */
int magus_ctx_create(int device, magus_ctx** out);
int magus_ctx_destroy(magus_ctx* ctx);

/*
 * Time-chunk length (steps, a multiple of 64, 64..2^24) used to split long
 * traces across wavefronts; 0 restores the default (4,096).  Results never
 * depend on it.
 */
int magus_ctx_set_chunk(magus_ctx* ctx, uint32_t chunk_steps);
uint32_t magus_ctx_get_chunk(const magus_ctx* ctx);

/*
 * Launch shape of the replay chunk kernel: 0 launches one wavefront per time
 * chunk; N > 0 launches N workgroups of 4 wavefronts that replay the chunks
 * round-robin (wavefront w takes chunks w, w + 4N, w + 8N, ...; a persistent
 * grid).  Results never depend on it.
 */
int magus_ctx_set_persistent(magus_ctx* ctx, uint32_t workgroups);
uint32_t magus_ctx_get_persistent(const magus_ctx* ctx);

/*
 * hipGraph replay.  While enabled, magus_replay captures its kernels into a
 * graph the first time it sees a given set of arguments (pointers, sizes,
 * config count, chunk and launch shape) and relaunches that graph on later
 * calls with the same set; the config table is uploaded outside the graph.
 * Up to 8 graphs are kept per context, each instantiated 8 times; launches
 * take the instances in turn.  Kernel timing (below) works inside the
 * graph: two event-record nodes bracket the chunk kernel, and each instance
 * records into a pair of events of its own, read when the instance is next
 * launched or by magus_ctx_kernel_time.
 */
int magus_ctx_set_graphs(magus_ctx* ctx, int enable);

/*
 * Autotuner for magus_replay: times every candidate time-chunk length
 * (2,048..32,768 steps) and launch shape (one wave per chunk, or a persistent
 * grid of 4 or 8 workgroups per compute unit) on the given batch, checks that
 * every candidate produces exactly the same results as the first (else
 * MAGUS_EDEVICE and the context is left unchanged), and sets the fastest on
 * the context.  d_results receives the replay results.  Synchronizes `stream`.
 */
typedef struct magus_tune_result {
    uint32_t chunk_steps;        /* chosen chunk length                     */
    uint32_t persistent_blocks;  /* chosen launch shape (0 = one wave/chunk) */
    uint32_t candidates;         /* candidates timed                        */
    uint32_t reserved;
    double best_ms;              /* time per call of the chosen candidate   */
    double default_ms;           /* time per call of the default shape      */
} magus_tune_result;
int magus_autotune_replay(magus_ctx* ctx, const uint32_t* d_samples, uint64_t n_samples,
                          const uint64_t* d_offsets, uint32_t n_traces,
                          const magus_config* h_cfgs, uint32_t n_cfgs,
                          const uint32_t* d_cfg_of_trace, magus_result* d_results,
                          uint32_t reps, hipStream_t stream, magus_tune_result* h_out);

/*
 * Kernel timing.  While enabled, every call records a pair of HIP events on
 * its stream right before and after its dominant kernel (MAGUS_KERNEL_REPLAY:
 * the chunk kernel of magus_replay; MAGUS_KERNEL_SWEEP: the sweep kernel;
 * MAGUS_KERNEL_SERVE: the serve-step kernel of a server on this context;
 * MAGUS_KERNEL_PROBE: the kernel of magus_valu_probe or magus_read_probe).
 * magus_ctx_kernel_time waits for the recorded events, returns the summed
 * elapsed time and the number of launches since its last call, and resets.
 */
#define MAGUS_KERNEL_REPLAY 0
#define MAGUS_KERNEL_SWEEP 1
#define MAGUS_KERNEL_SERVE 2
#define MAGUS_KERNEL_PROBE 3   /* the VALU issue and read probes below */
int magus_ctx_set_profiling(magus_ctx* ctx, int enable);
int magus_ctx_kernel_time(magus_ctx* ctx, int kernel, double* total_ms, uint64_t* launches);

/*
 * Synchronizes `stream` and returns MAGUS_EDATA if a device-side data check
 * of an earlier call on this context failed since the last check (clearing
 * it), else MAGUS_OK.
 */
int magus_ctx_check(magus_ctx* ctx, hipStream_t stream);

/*
 * Replay: runs every trace of a CSR batch through the controller described
 * above (Alg. 1, the event FIFO and Alg. 2 of Sec. 3.2, the decision rule).
 *   d_samples       uint32 throughput samples (MB/s), n_samples of them.
 *   d_offsets       n_traces+1 uint64, non-decreasing, trace t is
 *                   samples[offsets[t] .. offsets[t+1]), offsets[n_traces] <=
 *                   n_samples, each trace at most MAGUS_MAX_TRACE_LEN long.
 *   h_cfgs          n_cfgs >= 1 configs (host memory, read before return).
 *   d_cfg_of_trace  NULL (every trace uses h_cfgs[0]) or n_traces uint32
 *                   indices into h_cfgs.
 *   d_results       n_traces magus_result (written).
 *   d_levels        NULL or n_samples bytes: the decision byte of every step,
 *                   at the sample's own index (samples outside all traces
 *                   are left untouched).
 */
int magus_replay(magus_ctx* ctx, const uint32_t* d_samples, uint64_t n_samples,
                 const uint64_t* d_offsets, uint32_t n_traces,
                 const magus_config* h_cfgs, uint32_t n_cfgs,
                 const uint32_t* d_cfg_of_trace, magus_result* d_results,
                 uint8_t* d_levels, hipStream_t stream);

/*
 * Bits of a device-side data-check status word: the checks behind
 * MAGUS_EDATA (magus_ctx_check), as magus_replay_noalloc reports them.
 */
#define MAGUS_DATA_OFFSETS 1u    /* offsets not non-decreasing, or beyond n_samples */
#define MAGUS_DATA_TOO_LONG 2u   /* a trace longer than MAGUS_MAX_TRACE_LEN         */
#define MAGUS_DATA_CFG_INDEX 4u  /* a d_cfg_of_trace index >= n_cfgs                */

/*
 * Allocation-free replay, for callers that cannot allocate device memory at
 * call time (code that must not call hipMalloc: tight serving loops, harnesses
 * that forbid allocation).  The same computation as magus_replay for configs
 * that jump to the bound (up_step = down_step = 0; stepped configs are
 * MAGUS_EINVAL), with the same argument rules and results, on the calling
 * thread's current HIP device, with no context.
 *   - Its scratch (config table, chunk prefix and status, chunk summaries,
 *     fix-up records for decision bytes) is one fixed array of
 *     MAGUS_NOALLOC_SCRATCH_BYTES in device memory, one per device, held from
 *     the library's load until the process ends.  Its address is resolved on
 *     the first call on each device.  The call itself allocates nothing: no
 *     hipMalloc, no hipFree, no pinned host memory.
 *   - A batch needs 32 B per config (at most MAGUS_NOALLOC_MAX_CFGS),
 *     4 B per trace, and 32 B per time chunk of 4,096 steps (an upper bound
 *     of n_samples / 4096 + n_traces + 1 chunks), + 16 B per chunk with
 *     d_levels; each part rounded up to 256 B.  A batch that needs more is
 *     MAGUS_EINVAL with the sizes in magus_last_error() and nothing runs.
 *     8 MiB holds the 4,096 x 100,000 batch with decision bytes, or 20,000
 *     traces of 6.6e8 samples in all with 16,384 configs without them.
 *   - d_status: NULL, or one uint32 of device memory that receives the
 *     call's data-check bits (MAGUS_DATA_*, 0 = the batch was run).  A batch
 *     whose bits are not 0 leaves d_results and d_levels unwritten; with
 *     d_status NULL nothing reports it.  The status is the call's own (no
 *     fault of an earlier call carries over).
 *   - Every call on a device shares that device's array, which keeps the last
 *     call's contents (each call rewrites every part it reads).  Calls that
 *     overlap in time on one device, from any stream or thread, race on it:
 *     the caller orders them (one stream, or events).  Host-side, calls are
 *     serialised by a lock while they validate and enqueue.
 *   - The configs are validated and derived into a fixed host array, which
 *     the copy to the device has read before the call returns (h_cfgs may be
 *     reused at once).
 */
#define MAGUS_NOALLOC_SCRATCH_BYTES ((size_t)8 << 20)
#define MAGUS_NOALLOC_MAX_CFGS 16384u
int magus_replay_noalloc(const uint32_t* d_samples, uint64_t n_samples,
                         const uint64_t* d_offsets, uint32_t n_traces,
                         const magus_config* h_cfgs, uint32_t n_cfgs,
                         const uint32_t* d_cfg_of_trace, magus_result* d_results,
                         uint8_t* d_levels, uint32_t* d_status, hipStream_t stream);

/*
 * Parameter sweep: every trace against every config (the same controller as
 * magus_replay for every pair; Alg. 1's window and thresholds and Alg. 2's
 * FIFO length are the swept parameters).
 *   d_scores   NULL or n_traces * n_cfgs uint64, row-major [trace][config].
 *   d_argmin   n_traces uint32: index of the config with the lowest score,
 *              the lowest index among equal scores.
 * Same sample/offset rules as magus_replay, and n_cfgs <= 2^23 (the arg-min
 * packs score and index into 64 bits; scores of traces of at most
 * MAGUS_MAX_TRACE_LEN steps stay below 2^41).
 */
int magus_sweep(magus_ctx* ctx, const uint32_t* d_samples, uint64_t n_samples,
                const uint64_t* d_offsets, uint32_t n_traces,
                const magus_config* h_cfgs, uint32_t n_cfgs,
                uint64_t* d_scores, uint32_t* d_argmin, hipStream_t stream);

/*
 * Launch shape of magus_sweep: configs per workgroup and steps per tile of
 * shared quotients.  Shapes 0..MAGUS_SWEEP_SHAPES-1 are, as (configs, steps):
 * (256, 256) (the default), (256, 512), (256, 1024), (128, 256), (128, 512),
 * (64, 256); magus_sweep_shape_info returns them.  Results never depend on
 * the shape.
 */
#define MAGUS_SWEEP_SHAPES 6
int magus_ctx_set_sweep_shape(magus_ctx* ctx, uint32_t shape);
uint32_t magus_ctx_get_sweep_shape(const magus_ctx* ctx);
int magus_sweep_shape_info(uint32_t shape, uint32_t* lanes, uint32_t* tile);

/*
 * Autotuner for magus_sweep: times every launch shape on the given batch and
 * configs (`reps` timed calls each, after one untimed call), checks that every
 * shape finds the same minimal score and config for every trace as shape 0
 * (else MAGUS_EDEVICE and the context is left unchanged), and sets the
 * fastest on the context.  d_argmin receives the arg-min of the calls; a
 * batch that fails the data checks is MAGUS_EDATA.  Synchronizes `stream`.
 */
typedef struct magus_sweep_tune_result {
    uint32_t shape;              /* chosen shape                             */
    uint32_t lanes, tile;        /* its configs per workgroup, steps per tile */
    uint32_t candidates;         /* shapes timed                             */
    double best_ms;              /* time per call of the chosen shape        */
    double default_ms;           /* time per call of shape 0                 */
} magus_sweep_tune_result;
int magus_autotune_sweep(magus_ctx* ctx, const uint32_t* d_samples, uint64_t n_samples,
                         const uint64_t* d_offsets, uint32_t n_traces,
                         const magus_config* h_cfgs, uint32_t n_cfgs, uint32_t* d_argmin,
                         uint32_t reps, hipStream_t stream, magus_sweep_tune_result* h_out);

/*
 * Measurement aid: the issue rate of 32-bit integer VALU instructions.  Every
 * lane of `workgroups` workgroups of 256 lanes runs `steps` rounds of 8
 * independent dependency chains, with nothing else in the loop (no memory,
 * no LDS, no barriers):
 *   mode 0  one v_add_u32 per chain and round (8 lane-ops per round);
 *   mode 1  the opcodes of the sweep's per-evaluation step, one each per
 *           chain and round: compare into a wave mask, add with that mask as
 *           carry-in, and, population count (32 lane-ops per round).
 * *h_lane_ops (optional) receives the lane-ops the launch issues; divided by
 * the kernel time it is the rate the chip sustains for that mix, the issue
 * ceiling the sweep kernel's instruction stream is compared with.  With
 * kernel timing on, the launch is timed as MAGUS_KERNEL_PROBE.
 *   steps      a positive multiple of 4.
 *   d_out      workgroups * 256 uint32 (written; values have no meaning
 *              beyond keeping the work alive).
 */
int magus_valu_probe(magus_ctx* ctx, uint32_t workgroups, uint32_t steps, uint32_t mode,
                     uint32_t* d_out, uint64_t* h_lane_ops, hipStream_t stream);

/*
 * Measurement aid: the streaming-read rate of the replay chunk kernel's
 * access pattern with no other work.  One wavefront per chunk of
 * `chunk_steps` samples of d_samples (device memory, n_samples uint32) loads
 * one dword per lane per 64-sample block, eight blocks at a time with the
 * next eight in flight (non-temporal loads), and folds them into one word.
 * n_samples / time is the practical read ceiling the chunk kernel's HBM rate
 * is compared with.  With kernel timing on, the launch is timed as
 * MAGUS_KERNEL_PROBE.
 *   chunk_steps  a multiple of 64 in 64..2^24.
 *   d_out        ceil(n_samples / chunk_steps) uint32 (written; values have no
 *                meaning beyond keeping the loads alive).
 * MAGUS_EINVAL on a NULL buffer with n_samples > 0 or a chunk out of range.
 */
int magus_read_probe(magus_ctx* ctx, const uint32_t* d_samples, uint64_t n_samples,
                     uint32_t chunk_steps, uint32_t* d_out, hipStream_t stream);

/*
 * Monitor front end (Sec. 3, Sec. 4: memory throughput is read periodically
 * through a counter API).  Turns cumulative traffic-counter readings into the
 * MB/s samples that magus_replay / magus_sweep / serving consume:
 *   d_counts, d_ts_ns  n_readings uint64 each: counter value and time (ns) of
 *                      every reading; the counter has counter_bits bits
 *                      (1..64) and wraps; each count is bytes_per_count bytes.
 *   d_offsets          n_traces+1 uint64, strictly increasing (every trace has
 *                      at least one reading), offsets[n_traces] <= n_readings.
 *   d_samples          receives trace t's samples at [offsets[t] - t,
 *                      offsets[t+1] - t - 1): one per pair of consecutive
 *                      readings, floor(delta mod 2^bits * bytes_per_count *
 *                      1000 / delta_ns) MB/s (bytes per microsecond), 0 for a
 *                      zero interval, saturated at 2^32-1 (exact).
 * Offsets that break the rules produce no output; magus_ctx_check reports them.
 */
int magus_counters_to_mbps(magus_ctx* ctx, const uint64_t* d_counts, const uint64_t* d_ts_ns,
                           uint64_t n_readings, const uint64_t* d_offsets, uint32_t n_traces,
                           uint32_t counter_bits, uint32_t bytes_per_count,
                           uint32_t* d_samples, hipStream_t stream);

/*
 * Proxy energy / EDP model over replays.  Sec. 5.4 judges an uncore policy by
 * performance loss, package power saving, energy saving (CPU package + GPU)
 * and energy-delay product, each against the default of Sec. 5.3, where the
 * uncore stays at its maximum.  The paper measures these on hardware and gives
 * no model; this call evaluates a stated proxy of them for three policies on
 * every trace: MAGUS with the trace's config (column 0), always at level_max
 * (column 1, the baseline) and always at level_min (column 2).
 *   - Interval t of a trace runs at the level set after step t-1
 *     (level_init for t = 0): a decision takes effect on the next interval.
 *   - At level i the uncore sustains cap_mbps[i]; an interval whose sample x
 *     exceeds it lasts interval_us * x / cap_mbps[i] instead of interval_us.
 *   - Package power core_mw + uncore_mw[i] and GPU power gpu_mw are held for
 *     the whole (stretched) interval.
 * magus_proxy_stats holds the exact integer statistics the metrics are made
 * from; magus_proxy_metrics the seven figures per policy in double precision
 * (all zero for an empty trace).
 */
#define MAGUS_PROXY_LEVELS 32
typedef struct magus_proxy_model {
    uint32_t n_levels;                       /* rungs described, 1..32; every   */
                                             /* config needs level_max < this   */
    uint32_t interval_us;                    /* >= 1                            */
    uint32_t cap_mbps[MAGUS_PROXY_LEVELS];   /* >= 1 for the described rungs    */
    uint32_t uncore_mw[MAGUS_PROXY_LEVELS];
    uint32_t core_mw;                        /* core_mw + uncore_mw[i] >= 1     */
    uint32_t gpu_mw;
} magus_proxy_model;

typedef struct magus_proxy_stats {
    uint64_t excess_max;                     /* sum of max(0, x - cap[level_max]) */
    uint64_t excess_min;                     /* sum of max(0, x - cap[level_min]) */
    uint64_t steps[MAGUS_PROXY_LEVELS];      /* MAGUS: intervals run at level i  */
    uint64_t excess[MAGUS_PROXY_LEVELS];     /* MAGUS: sum of max(0, x - cap[i]) */
                                             /* over those intervals             */
} magus_proxy_stats;

typedef struct magus_proxy_metrics {         /* [policy]: 0 MAGUS, 1 max, 2 min  */
    double time_s[3];                        /* stretched run time               */
    double energy_j[3];                      /* package + GPU energy             */
    double pkg_power_w[3];                   /* average package power            */
    double perf_loss[3];                     /* time / time[1] - 1               */
    double pkg_power_saving[3];              /* 1 - pkg_power / pkg_power[1]     */
    double energy_saving[3];                 /* 1 - energy / energy[1]           */
    double edp_saving[3];                    /* 1 - energy*time / (energy*time)[1] */
} magus_proxy_metrics;

/* MAGUS_OK if the model is valid (as required by magus_proxy), else MAGUS_EINVAL
 * with the reason in magus_last_error().  Host only. */
int magus_proxy_model_check(const magus_proxy_model* model);

/*
 * Evaluates the proxy for every trace under the controller of magus_replay
 * (same sample, offset and config rules), without materialising per-step
 * levels: configs that jump to the bound take one pass over the samples (in
 * time chunks of twice the context's chunk length while that is at most
 * 8,192 steps, else of the context's length);
 * stepped configs take the stepped replay's first pass (context-owned step
 * masks, 28 B per 64 steps) and one statistics pass over samples and masks.
 * Either pass runs in 32-bit sums; a chunk holding a sample of 2^24 or more
 * (2^22 for stepped configs) is queued in the context and run again in
 * 64-bit sums, with identical results.
 *   h_model    the proxy model (host memory, read before return); an invalid
 *              model, or a config with level_max >= n_levels, is MAGUS_EINVAL.
 *   d_stats    n_traces magus_proxy_stats (written).
 *   d_metrics  NULL or n_traces magus_proxy_metrics (written).
 * A batch that breaks the data rules (found on the device) leaves d_stats
 * zero and d_metrics unwritten; magus_ctx_check reports it.
 */
int magus_proxy(magus_ctx* ctx, const uint32_t* d_samples, uint64_t n_samples,
                const uint64_t* d_offsets, uint32_t n_traces,
                const magus_config* h_cfgs, uint32_t n_cfgs, const uint32_t* d_cfg_of_trace,
                const magus_proxy_model* h_model, magus_proxy_stats* d_stats,
                magus_proxy_metrics* d_metrics, hipStream_t stream);

/*
 * Serving: a pool of slots, one per live telemetry stream, whose controller
 * state stays in device memory between steps.
 *   magus_server_create   capacity = as many slots as `mem_budget_bytes` of
 *                         device memory holds (magus_server_slot_bytes() each),
 *                         at least 1; the server owns the pool and its pinned
 *                         staging buffers.
 *   magus_stream_open     admits a stream with config h_cfg into a free slot
 *                         (MAGUS_ENOSLOT if none); its state is reset by the
 *                         next magus_serve_step on the server.
 *   magus_stream_close    frees the slot (the slot may be handed out again).
 *   magus_serve_step      one step for n (slot, sample) pairs -- for each
 *                         pair, one invocation of the controller with the
 *                         stream's newest sample, as the runtime is invoked
 *                         once per monitoring interval (Sec. 3.2, Sec. 4):
 *                         Alg. 1 on the stream's FIFO, the event FIFO and
 *                         Alg. 2, then the decision rule.  h_slots and
 *                         h_samples are host arrays (copied before return),
 *                         every slot must be open and appear at most once
 *                         (MAGUS_EINVAL otherwise).  Decision bytes for the n
 *                         pairs are written to h_decisions (host memory; pinned
 *                         memory lets the copy run asynchronously) once
 *                         `stream` has completed the step.  Steps of one server
 *                         must be issued on one stream, or otherwise ordered.
 *   magus_stream_result   (synchronous) the running magus_result of a slot.
 */
size_t magus_server_slot_bytes(void);
int magus_server_create(magus_ctx* ctx, size_t mem_budget_bytes, magus_server** out);
int magus_server_destroy(magus_server* srv);
uint32_t magus_server_capacity(const magus_server* srv);
uint32_t magus_server_open_count(const magus_server* srv);
int magus_stream_open(magus_server* srv, const magus_config* h_cfg, uint32_t* slot_out);
int magus_stream_close(magus_server* srv, uint32_t slot);
int magus_serve_step(magus_server* srv, const uint32_t* h_slots, const uint32_t* h_samples,
                     uint32_t n, uint8_t* h_decisions, hipStream_t stream);
int magus_stream_result(magus_server* srv, uint32_t slot, magus_result* h_out);

/*
 * Serving loop with continuous batching (one simulated fleet of nodes).
 * Events are sorted by t_ns (nanoseconds from the start of the run):
 *   MAGUS_EV_JOIN    node `stream` asks to be served with config
 *                    h_cfgs[value]; it is admitted into a free slot at once,
 *                    or waits (oldest first) until a leave frees one.  A
 *                    join of a node that left but whose slot still serves
 *                    its earlier samples waits for that slot to close, then
 *                    waits like any other join (a leave withdraws it).  A
 *                    join of a node that is live or waiting is ignored.
 *   MAGUS_EV_SAMPLE  one throughput sample `value` of node `stream`; dropped
 *                    unless the node is admitted.
 *   MAGUS_EV_LEAVE   the node stops; its slot is freed once its pending
 *                    samples are served.
 * realtime != 0 ingests each event at its time and measures latency from that
 * time; realtime == 0 runs flat out (latency from the start of the run).
 * Every dispatch forms one batch of at most max_batch pairs (0: the server's
 * capacity) from the oldest pending sample of each admitted node, and up to
 * `depth` (1..4) batches are in flight.  The state-update kernel reads each
 * batch from pinned host memory and writes its decisions back into pinned
 * host memory directly (no copies), on a server-owned stream, so kernels
 * run in arrival order.
 * Per event i: h_decisions[i] = decision byte of a served sample (0xFF for
 * other events and dropped samples), h_latency_ns[i] = event time to
 * decision visible in host memory (UINT64_MAX if none).  Stream ids must be
 * below n_streams.  The run admits its nodes into the server's free slots and
 * closes them before it returns; streams opened outside the run keep their
 * slots but are not stepped by it.
 */
#define MAGUS_EV_SAMPLE 0u
#define MAGUS_EV_JOIN 1u
#define MAGUS_EV_LEAVE 2u

typedef struct magus_event {
    uint64_t t_ns;
    uint32_t kind;
    uint32_t stream;
    uint32_t value;
    uint32_t reserved;
} magus_event;

typedef struct magus_run_stats {
    uint64_t samples_served;
    uint64_t samples_dropped;    /* samples of nodes not admitted at the time */
    uint64_t batches;
    uint64_t max_batch;          /* largest batch dispatched                    */
    uint64_t max_in_flight;      /* most batches in flight at once              */
    uint64_t deferred;           /* samples that waited for a later batch       */
    uint64_t joins_admitted;     /* admitted on arrival                         */
    uint64_t joins_waited;       /* admitted after waiting for a slot           */
    uint64_t joins_refused;      /* left, or the run ended, while waiting       */
    double wall_s;
} magus_run_stats;

int magus_server_run(magus_server* srv, const magus_event* h_events, uint64_t n_events,
                     uint32_t n_streams, const magus_config* h_cfgs, uint32_t n_cfgs,
                     int realtime, uint32_t max_batch, uint32_t depth,
                     uint8_t* h_decisions, uint64_t* h_latency_ns, magus_run_stats* h_stats);

#ifdef __cplusplus
}
#endif
#endif /* MAGUS_H */
