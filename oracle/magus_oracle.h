/*
 * MAGUS controller oracle -- TEST INFRASTRUCTURE ONLY (tests, smoke check and
 * the CPU-baseline leg of the benchmark).  Plain single-threaded C.
 * Names follow the paper's notation: direv_length is the derivative window of
 * Alg. 1, tune_len is len(uncore_tune_ls) of Alg. 2, hf_num/hf_den is
 * high_freq_threshold (0.6 = 3/5 in Sec. 3.2).
 */
#ifndef MAGUS_ORACLE_H
#define MAGUS_ORACLE_H
#include <stdint.h>

typedef struct oracle_config {
    uint32_t direv_length;  /* W, 2..32                                   */
    uint32_t tune_len;      /* H = len(uncore_tune_ls), 1..32             */
    int32_t inc_q;          /* inc_threshold in Q16.16, 0..2^20           */
    int32_t dec_q;          /* dec_threshold in Q16.16, -2^20..0          */
    uint32_t hf_num;        /* high_freq_threshold = hf_num / hf_den      */
    uint32_t hf_den;
    uint32_t level_min;     /* uncore ladder index of the lower bound      */
    uint32_t level_max;     /* ... of the upper bound (<= 31)              */
    uint32_t level_init;    /* level before the first step                 */
    uint32_t up_step;       /* 0: an executed increase goes to level_max;  */
    uint32_t down_step;     /*    else the level moves by this many rungs  */
    uint32_t base;          /* derivative base: 0 min(oldest, newest),     */
                            /* 1 oldest sample, 2 newest sample,           */
                            /* 3 the fixed reference base_ref              */
    uint32_t base_ref;      /* B_ref in MB/s (>= 1) for base 3, else unused */
} oracle_config;

typedef struct oracle_result {
    uint64_t score;         /* level_sum + 1000 * transitions              */
    uint64_t level_sum;     /* sum over steps of the level after the step  */
    uint64_t transitions;   /* steps whose level differs from the previous */
    uint64_t ticks_high;    /* steps spent in the high-frequency state     */
} oracle_result;

int oracle_config_valid(const oracle_config* c);

/*
 * Controller state of one stream between invocations (Sec. 3.2: one
 * invocation per monitoring interval): the two FIFOs, the level and the
 * running sums.
 */
typedef struct oracle_state {
    uint32_t mem_throughput_ls[64];   /* the last `filled` samples, oldest first  */
    uint32_t filled;                  /* samples in mem_throughput_ls (<= W)      */
    uint32_t level;                   /* current uncore level                     */
    uint8_t uncore_tune_ls[64];       /* the last H event flags, oldest first      */
    uint64_t level_sum;
    uint64_t transitions;
    uint64_t ticks_high;
    uint64_t steps;                   /* invocations so far                       */
} oracle_state;

void oracle_state_init(oracle_state* s, const oracle_config* c);
/* one invocation with the newest sample; *byte (optional) = decision byte */
int oracle_step(oracle_state* s, const oracle_config* cfg, uint32_t sample, uint8_t* byte);
int oracle_state_result(const oracle_state* s, oracle_result* res);
/* one tick of many streams: bytes[i] = step of stream[i] with samples[i] */
int oracle_serve_tick(oracle_state* states, const oracle_config* cfgs, uint32_t n_cfgs,
                      const uint32_t* cfg_of_stream, const uint32_t* stream,
                      const uint32_t* samples, uint32_t n, uint8_t* bytes);

/* bytes (optional, n entries): bits 0-4 level, bit 5 high, bits 6-7 pred+1 */
int oracle_replay_trace(const uint32_t* x, uint64_t n, const oracle_config* cfg,
                        uint8_t* bytes, oracle_result* res);
int oracle_replay_trace_fp64(const uint32_t* x, uint64_t n, const oracle_config* cfg,
                             double inc_threshold, double dec_threshold,
                             uint8_t* bytes, oracle_result* res);
int oracle_replay_batch(const uint32_t* samples, const uint64_t* offsets, uint32_t n_traces,
                        const oracle_config* cfgs, uint32_t n_cfgs,
                        const uint32_t* cfg_of_trace, oracle_result* results, uint8_t* bytes);
int oracle_sweep(const uint32_t* samples, const uint64_t* offsets, uint32_t n_traces,
                 const oracle_config* cfgs, uint32_t n_cfgs,
                 uint64_t* scores, uint32_t* argmin);
/*
 * Memory-throughput monitor front end: cumulative traffic counter readings
 * (counts[i] at time ts_ns[i], a counter of counter_bits bits that wraps,
 * bytes_per_count bytes per count) to throughput samples in MB/s:
 *   out[i] = floor(((counts[i+1] - counts[i]) mod 2^bits) * bytes_per_count
 *                  * 1000 / (ts_ns[i+1] - ts_ns[i])),
 * 0 when the interval is 0, saturated at 2^32-1.  n readings give n-1 samples.
 */
int oracle_counters_to_mbps(const uint64_t* counts, const uint64_t* ts_ns, uint64_t n,
                            uint32_t counter_bits, uint32_t bytes_per_count, uint32_t* out);
/*
 * Proxy energy / EDP model (a proxy: the paper measures these on hardware).
 * Policy columns of the metrics: 0 MAGUS, 1 uncore always at level_max (the
 * default behaviour and the baseline of every saving), 2 always at level_min.
 */
typedef struct oracle_proxy_model {
    uint32_t n_levels;         /* ladder rungs described below, 1..32           */
    uint32_t interval_us;      /* monitoring interval                           */
    uint32_t cap_mbps[32];     /* throughput the uncore sustains at each level  */
    uint32_t uncore_mw[32];    /* uncore power at each level                    */
    uint32_t core_mw;          /* rest of the CPU package                       */
    uint32_t gpu_mw;           /* GPU (core and memory)                         */
} oracle_proxy_model;

typedef struct oracle_proxy_stats {   /* exact integer statistics of one trace */
    uint64_t excess_max;       /* sum over intervals of max(0, x - cap[level_max]) */
    uint64_t excess_min;       /* ... of max(0, x - cap[level_min])                */
    uint64_t steps[32];        /* MAGUS: intervals run at each level               */
    uint64_t excess[32];       /* MAGUS: sum of max(0, x - cap[i]) over those       */
} oracle_proxy_stats;

typedef struct oracle_proxy_metrics {
    double time_s[3];          /* stretched run time                             */
    double energy_j[3];        /* package + GPU energy                           */
    double pkg_power_w[3];     /* average package power                          */
    double perf_loss[3];       /* time / time[1] - 1                             */
    double pkg_power_saving[3];/* 1 - pkg_power / pkg_power[1]                   */
    double energy_saving[3];   /* 1 - energy / energy[1]                         */
    double edp_saving[3];      /* 1 - energy * time / (energy[1] * time[1])      */
} oracle_proxy_metrics;

int oracle_proxy_model_valid(const oracle_proxy_model* m);
/* metrics may be NULL; an empty trace gives zero times, energies and savings */
int oracle_proxy_trace(const uint32_t* x, uint64_t n, const oracle_config* cfg,
                       const oracle_proxy_model* m, oracle_proxy_stats* stats,
                       oracle_proxy_metrics* metrics);
#endif
