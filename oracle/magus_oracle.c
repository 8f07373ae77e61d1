/*
 * MAGUS controller oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU statement of what the MAGUS hot path
 * computes (Zheng, Sultanov, Papka, Lan: "Exploring Uncore Frequency Scaling
 * for Heterogeneous Computing", arXiv 2502.03796).  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load this code; the
 * product path never does.  It shares no code, header, table or constant with
 * the HIP library.
 *
 * Each monitoring step follows the paper's order:
 *   1. Monitor: push the new memory-throughput sample into the fixed-size FIFO
 *      mem_throughput_ls (Sec. 3.1, "fixed-size first-in first-out queue").
 *   2. Predict (Alg. 1): derivative of the FIFO's newest vs oldest entry over
 *      direv_length, compared with inc_threshold (> -> +1) and dec_threshold
 *      (< -> -1), else 0.  The result is a temporary decision (Sec. 3.1).
 *   3. Log: push a binary flag "a frequency change would be triggered" into the
 *      FIFO uncore_tune_ls (Sec. 3.2).
 *   4. Detect (Alg. 2): freq = sum(uncore_tune_ls)/len(uncore_tune_ls);
 *      high if freq >= high_freq_threshold (0.6 in Sec. 3.2).
 *   5. Decide (Sec. 3.2, Sec. 4, Sec. 6.1): in the high state the uncore goes
 *      to its maximum; otherwise the temporary decision is executed, where an
 *      increase goes to the maximum and a decrease goes directly to the lower
 *      bound; 0 keeps the level.  Nodes start idle at the minimum (Sec. 4).
 *
 * Readings taken where the paper is silent (each one is listed in the design
 * notes of the repository):
 *   - The derivative is taken relative to the smaller of the two samples,
 *       r = (ls[-1] - ls[0]) / (direv_length * min(ls[0], ls[-1])),
 *     so that thresholds are dimensionless and an up-step by k and a
 *     down-step by 1/k give the same |r|.  A zero base gives +inf / -inf, and
 *     0/0 gives no event.
 *   - Thresholds are Q16.16 integers (inc_q / 65536, dec_q / 65536) and the
 *     comparison is exact: r > inc_q/65536 is evaluated as the integer
 *     cross-product (b - a) * 65536 > inc_q * W * min(a, b).  No rounding
 *     happens anywhere; only the thresholds are quantised.
 *   - Until the FIFO holds direv_length samples the prediction is 0 (warm-up);
 *     uncore_tune_ls has a fixed length H and starts filled with zeros.
 *   - high_freq_threshold is the fraction hf_num / hf_den and the test
 *     sum/len >= num/den is evaluated as sum * den >= num * len.
 *   - The flag logged is (temporary decision != 0), also while high.
 *   - Stepped actuation (the gradual alternative that Sec. 6.1 contrasts with
 *     MAGUS's jump to the bound, and the "how much to increase or decrease"
 *     question of Sec. 2): with up_step / down_step > 0 an executed +1 / -1
 *     moves the level by that many rungs, clamped to [level_min, level_max];
 *     0 keeps the jump to the bound.  The high state still goes to the max.
 *   - The derivative's base is a reading as well; besides the default
 *     min(oldest, newest) three alternatives are kept for sensitivity studies:
 *     the oldest sample (r = (b - a) / (W a)), the newest (W b), and a fixed
 *     reference B_ref from the config (r = (b - a) / (W B_ref)).  The last is
 *     the listing's own absolute derivative, (newest - oldest) / direv_length
 *     in MB/s per step, measured in units of B_ref: an absolute threshold of
 *     theta MB/s per step is inc = theta / B_ref (B_ref = 1 is the listing's
 *     formula unscaled).
 *   - Per step the tick is accounted after the decision:
 *       transitions += (new level != old level); level_sum += new level;
 *     score = level_sum + 1000 * transitions.
 *
 * A second predictor, the "FP64 side-form", evaluates the same derivative in
 * IEEE double with decimal thresholds; it is run beside the exact form only to
 * report how often the two disagree.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "magus_oracle.h"

#define ORACLE_FIFO_MAX 64

/* ---------------------------------------------------------------- validation */

int oracle_config_valid(const oracle_config* c)
{
    if (!c) return 0;
    if (c->direv_length < 2 || c->direv_length > 32) return 0;
    if (c->tune_len < 1 || c->tune_len > 32) return 0;
    if (c->inc_q < 0 || c->inc_q > (1 << 20)) return 0;
    if (c->dec_q > 0 || c->dec_q < -(1 << 20)) return 0;
    if (c->hf_den < 1 || c->hf_num > c->hf_den) return 0;
    if (c->level_min >= c->level_max || c->level_max > 31) return 0;
    if (c->level_init < c->level_min || c->level_init > c->level_max) return 0;
    if (c->up_step > 31 || c->down_step > 31) return 0;
    if (c->base > 3) return 0;
    if (c->base == 3 && c->base_ref < 1) return 0;
    return 1;
}

/* ------------------------------------------------------- Alg. 1, exact form */

/*
 * MEM_THROUGHPUT_TREND_PREDICTION (Alg. 1) with the relative derivative and
 * Q16.16 thresholds.  ls holds direv_length samples, ls[0] oldest.
 */
static int64_t derivative_base(int64_t first, int64_t last, uint32_t which, uint32_t ref)
{
    if (which == 1) return first;
    if (which == 2) return last;
    if (which == 3) return ref;
    return first < last ? first : last;
}

static int predict_exact(int32_t inc_q, int32_t dec_q,
                         const uint32_t* ls, uint32_t direv_length, uint32_t which,
                         uint32_t ref)
{
    int64_t first = ls[0];
    int64_t last = ls[direv_length - 1];
    int64_t base = derivative_base(first, last, which, ref);
    int64_t delta = last - first;
    /* derivative = delta / (direv_length * base); compare with q / 65536
       by cross-multiplying with the positive (or zero) denominator
       (|lhs| < 2^49 and |q * den| <= 2^20 * 2^5 * 2^32 = 2^57).           */
    int64_t lhs = delta * 65536;
    int64_t den = (int64_t)direv_length * base;
    if (lhs > (int64_t)inc_q * den) return 1;        /* derivative > inc */
    if (lhs < (int64_t)dec_q * den) return -1;       /* derivative < dec */
    return 0;
}

/* ------------------------------------------------------ Alg. 1, FP64 form */

static int predict_fp64(double inc_threshold, double dec_threshold,
                        const uint32_t* ls, uint32_t direv_length, uint32_t which,
                        uint32_t ref)
{
    double first = (double)ls[0];
    double last = (double)ls[direv_length - 1];
    double base = which == 1 ? first : which == 2 ? last : which == 3 ? (double)ref
                : (first < last ? first : last);
    double derivative = (last - first) / ((double)direv_length * base);
    if (derivative > inc_threshold) return 1;
    if (derivative < dec_threshold) return -1;
    return 0;                                        /* includes 0/0 = NaN */
}

/* ------------------------------------------------------------- Alg. 2 form */

static int high_freq_detection(uint32_t hf_num, uint32_t hf_den,
                               const uint8_t* uncore_tune_ls, uint32_t len)
{
    uint32_t sum = 0;
    for (uint32_t i = 0; i < len; ++i) sum += uncore_tune_ls[i];
    /* freq = sum / len >= hf_num / hf_den */
    return (uint64_t)sum * hf_den >= (uint64_t)hf_num * len;
}

/* ----------------------------------------------------------- the controller */

void oracle_state_init(oracle_state* s, const oracle_config* c)
{
    memset(s, 0, sizeof *s);             /* both FIFOs empty, uncore_tune_ls all 0 */
    s->level = c->level_init;            /* idle nodes sit at the minimum */
}

/*
 * One invocation of the controller (Sec. 3.2: the runtime is invoked once per
 * monitoring interval with the newest throughput sample).  Returns the step's
 * decision byte: bits 0-4 level, bit 5 high, bits 6-7 pred + 1.
 */
static uint8_t controller_step(oracle_state* s, const oracle_config* c, uint32_t sample,
                               int use_fp64, double inc_threshold, double dec_threshold)
{
    uint32_t* mem_throughput_ls = s->mem_throughput_ls;
    uint8_t* uncore_tune_ls = s->uncore_tune_ls;
    const uint32_t W = c->direv_length;
    const uint32_t H = c->tune_len;
    uint32_t level = s->level;

    /* 1. monitor: FIFO of the last W samples */
    if (s->filled == W) {
        memmove(mem_throughput_ls, mem_throughput_ls + 1, (W - 1) * sizeof(uint32_t));
        mem_throughput_ls[W - 1] = sample;
    } else {
        mem_throughput_ls[s->filled++] = sample;
    }

    /* 2. predict (temporary decision) */
    int pred = 0;
    if (s->filled == W) {
        pred = use_fp64 ? predict_fp64(inc_threshold, dec_threshold, mem_throughput_ls, W,
                                       c->base, c->base_ref)
                        : predict_exact(c->inc_q, c->dec_q, mem_throughput_ls, W, c->base,
                                        c->base_ref);
    }

    /* 3. log whether a frequency change would be triggered */
    memmove(uncore_tune_ls, uncore_tune_ls + 1, H - 1);
    uncore_tune_ls[H - 1] = (uint8_t)(pred != 0);

    /* 4. detect the high-frequency state */
    int high = high_freq_detection(c->hf_num, c->hf_den, uncore_tune_ls, H);

    /* 5. decide */
    uint32_t next = level;
    if (high) {
        next = c->level_max;
    } else if (pred == 1) {
        next = c->up_step == 0 ? c->level_max
             : (level + c->up_step > c->level_max ? c->level_max : level + c->up_step);
    } else if (pred == -1) {
        next = c->down_step == 0 ? c->level_min
             : (level < c->level_min + c->down_step ? c->level_min : level - c->down_step);
    }

    s->transitions += (next != level);
    level = next;
    s->level = level;
    s->level_sum += level;
    s->ticks_high += (uint64_t)high;
    s->steps += 1;
    return (uint8_t)(level | ((uint32_t)high << 5) | ((uint32_t)(pred + 1) << 6));
}

static void state_result(const oracle_state* s, oracle_result* res)
{
    res->level_sum = s->level_sum;
    res->transitions = s->transitions;
    res->ticks_high = s->ticks_high;
    res->score = s->level_sum + 1000u * s->transitions;
}

static void run_trace(const uint32_t* x, uint64_t n, const oracle_config* c,
                      int use_fp64, double inc_threshold, double dec_threshold,
                      uint8_t* bytes, oracle_result* res)
{
    oracle_state s;
    oracle_state_init(&s, c);
    for (uint64_t t = 0; t < n; ++t) {
        const uint8_t b = controller_step(&s, c, x[t], use_fp64, inc_threshold, dec_threshold);
        if (bytes) bytes[t] = b;
    }
    state_result(&s, res);
}

int oracle_step(oracle_state* s, const oracle_config* cfg, uint32_t sample, uint8_t* byte)
{
    if (!s || !oracle_config_valid(cfg)) return -1;
    const uint8_t b = controller_step(s, cfg, sample, 0, 0.0, 0.0);
    if (byte) *byte = b;
    return 0;
}

int oracle_state_result(const oracle_state* s, oracle_result* res)
{
    if (!s || !res) return -1;
    state_result(s, res);
    return 0;
}

/*
 * One serving tick: stream i (state states[stream[i]], config
 * cfgs[cfg_of_stream[stream[i]]]) takes sample samples[i]; bytes[i] receives
 * its decision byte.  Plain loop over the pairs in order.
 */
int oracle_serve_tick(oracle_state* states, const oracle_config* cfgs, uint32_t n_cfgs,
                      const uint32_t* cfg_of_stream, const uint32_t* stream,
                      const uint32_t* samples, uint32_t n, uint8_t* bytes)
{
    if (!states || !cfgs || !cfg_of_stream || (n && (!stream || !samples || !bytes)))
        return -1;
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t k = cfg_of_stream[stream[i]];
        if (k >= n_cfgs || !oracle_config_valid(&cfgs[k])) return -1;
        bytes[i] = controller_step(&states[stream[i]], &cfgs[k], samples[i], 0, 0.0, 0.0);
    }
    return 0;
}

int oracle_replay_trace(const uint32_t* x, uint64_t n, const oracle_config* cfg,
                        uint8_t* bytes, oracle_result* res)
{
    if (!oracle_config_valid(cfg) || !res || (n && !x)) return -1;
    run_trace(x, n, cfg, 0, 0.0, 0.0, bytes, res);
    return 0;
}

int oracle_replay_trace_fp64(const uint32_t* x, uint64_t n, const oracle_config* cfg,
                             double inc_threshold, double dec_threshold,
                             uint8_t* bytes, oracle_result* res)
{
    if (!oracle_config_valid(cfg) || !res || (n && !x)) return -1;
    run_trace(x, n, cfg, 1, inc_threshold, dec_threshold, bytes, res);
    return 0;
}

/* ----------------------------------------------------------------- batches */

int oracle_replay_batch(const uint32_t* samples, const uint64_t* offsets, uint32_t n_traces,
                        const oracle_config* cfgs, uint32_t n_cfgs,
                        const uint32_t* cfg_of_trace, oracle_result* results, uint8_t* bytes)
{
    if (!offsets || !cfgs || !results || n_cfgs == 0) return -1;
    for (uint32_t i = 0; i < n_cfgs; ++i)
        if (!oracle_config_valid(&cfgs[i])) return -1;
    for (uint32_t t = 0; t < n_traces; ++t) {
        uint32_t k = cfg_of_trace ? cfg_of_trace[t] : 0;
        if (k >= n_cfgs || offsets[t + 1] < offsets[t]) return -1;
        uint64_t n = offsets[t + 1] - offsets[t];
        run_trace(samples + offsets[t], n, &cfgs[k], 0, 0.0, 0.0,
                  bytes ? bytes + offsets[t] : NULL, &results[t]);
    }
    return 0;
}

/*
 * Parameter sweep: every trace against every config.  scores[t * n_cfgs + c]
 * (optional) and argmin[t] = smallest config index among the minimal scores.
 */
int oracle_sweep(const uint32_t* samples, const uint64_t* offsets, uint32_t n_traces,
                 const oracle_config* cfgs, uint32_t n_cfgs,
                 uint64_t* scores, uint32_t* argmin)
{
    if (!offsets || !cfgs || n_cfgs == 0) return -1;
    for (uint32_t i = 0; i < n_cfgs; ++i)
        if (!oracle_config_valid(&cfgs[i])) return -1;
    for (uint32_t t = 0; t < n_traces; ++t) {
        uint64_t n = offsets[t + 1] - offsets[t];
        uint64_t best = UINT64_MAX;
        uint32_t best_c = 0;
        for (uint32_t c = 0; c < n_cfgs; ++c) {
            oracle_result r;
            run_trace(samples + offsets[t], n, &cfgs[c], 0, 0.0, 0.0, NULL, &r);
            if (scores) scores[(uint64_t)t * n_cfgs + c] = r.score;
            if (r.score < best) { best = r.score; best_c = c; }
        }
        if (argmin) argmin[t] = best_c;
    }
    return 0;
}

/* ------------------------------------------------------------ monitor front end */

int oracle_counters_to_mbps(const uint64_t* counts, const uint64_t* ts_ns, uint64_t n,
                            uint32_t counter_bits, uint32_t bytes_per_count, uint32_t* out)
{
    if (counter_bits < 1 || counter_bits > 64 || (n > 1 && (!counts || !ts_ns || !out)))
        return -1;
    for (uint64_t i = 0; i + 1 < n; ++i) {
        unsigned __int128 delta = (unsigned __int128)counts[i + 1] - counts[i];
        if (counter_bits < 64) delta &= (((unsigned __int128)1) << counter_bits) - 1;
        else delta &= (unsigned __int128)UINT64_MAX;
        uint64_t dt = ts_ns[i + 1] - ts_ns[i];
        if (dt == 0) { out[i] = 0; continue; }
        /* bytes per microsecond = MB/s */
        unsigned __int128 mbps = delta * bytes_per_count * 1000u / dt;
        out[i] = mbps > UINT32_MAX ? UINT32_MAX : (uint32_t)mbps;
    }
    return 0;
}

/* ------------------------------------------------------------ proxy energy model */
/*
 * Proxy of the four metrics of Sec. 5.4 (performance loss, package power
 * saving, energy saving, energy-delay product) for three uncore policies run on
 * the same trace: MAGUS with the trace's config, the default behaviour of
 * Sec. 5.3 (the uncore stays at its maximum, the baseline of every saving) and
 * a static minimum.  The paper measures these on hardware and gives no power
 * or performance model, so the model here is a stated proxy:
 *   - interval t (interval_us long) runs at the level the controller set after
 *     reading interval t-1, i.e. the level after step t-1 (level_init for
 *     t = 0); the static policies run at level_max / level_min throughout;
 *   - at level i the uncore sustains cap_mbps[i]; an interval whose demand
 *     x[t] exceeds that takes interval_us * x[t] / cap_mbps[i] instead of
 *     interval_us (the interval's traffic moves at the capped rate);
 *   - package power is core_mw + uncore_mw[i] and system power adds gpu_mw,
 *     both held for the whole (possibly stretched) interval.
 * The integer statistics are exact; the metrics are the plain definitions
 * summed interval by interval in double precision.
 */
int oracle_proxy_model_valid(const oracle_proxy_model* m)
{
    if (!m || m->n_levels < 1 || m->n_levels > 32 || m->interval_us < 1) return 0;
    for (uint32_t i = 0; i < m->n_levels; ++i)
        if (m->cap_mbps[i] < 1 || (uint64_t)m->core_mw + m->uncore_mw[i] < 1) return 0;
    return 1;
}

int oracle_proxy_trace(const uint32_t* x, uint64_t n, const oracle_config* cfg,
                       const oracle_proxy_model* m, oracle_proxy_stats* st,
                       oracle_proxy_metrics* out)
{
    if (!oracle_config_valid(cfg) || !oracle_proxy_model_valid(m) || !st || (n && !x))
        return -1;
    if (cfg->level_max >= m->n_levels) return -1;
    uint8_t* bytes = n ? (uint8_t*)malloc(n) : NULL;
    if (n && !bytes) return -1;
    oracle_result r;
    run_trace(x, n, cfg, 0, 0.0, 0.0, bytes, &r);

    /* per interval: the level it runs at under each policy */
    const double dt_s = m->interval_us * 1e-6;
    double time_s[3] = {0, 0, 0}, pkg_j[3] = {0, 0, 0};
    memset(st, 0, sizeof *st);
    for (uint64_t t = 0; t < n; ++t) {
        uint32_t lv[3];
        lv[0] = t == 0 ? cfg->level_init : (uint32_t)(bytes[t - 1] & 31u);
        lv[1] = cfg->level_max;
        lv[2] = cfg->level_min;
        for (int p = 0; p < 3; ++p) {
            const uint32_t cap = m->cap_mbps[lv[p]];
            const uint64_t excess = x[t] > cap ? (uint64_t)(x[t] - cap) : 0;
            if (p == 0) {
                st->steps[lv[0]] += 1;
                st->excess[lv[0]] += excess;
            } else if (p == 1) {
                st->excess_max += excess;
            } else {
                st->excess_min += excess;
            }
            /* stretched length of this interval and the package energy over it */
            const double len = x[t] > cap ? dt_s * ((double)x[t] / (double)cap) : dt_s;
            time_s[p] += len;
            pkg_j[p] += len * ((double)m->core_mw + (double)m->uncore_mw[lv[p]]) * 1e-3;
        }
    }
    free(bytes);
    if (!out) return 0;
    for (int p = 0; p < 3; ++p) {
        out->time_s[p] = time_s[p];
        out->energy_j[p] = pkg_j[p] + time_s[p] * (double)m->gpu_mw * 1e-3;
        out->pkg_power_w[p] = time_s[p] > 0 ? pkg_j[p] / time_s[p] : 0.0;
    }
    /* savings and loss relative to the default (always at the maximum) */
    for (int p = 0; p < 3; ++p) {
        if (n == 0) {
            out->perf_loss[p] = out->pkg_power_saving[p] = 0.0;
            out->energy_saving[p] = out->edp_saving[p] = 0.0;
            continue;
        }
        out->perf_loss[p] = out->time_s[p] / out->time_s[1] - 1.0;
        out->pkg_power_saving[p] = 1.0 - out->pkg_power_w[p] / out->pkg_power_w[1];
        out->energy_saving[p] = 1.0 - out->energy_j[p] / out->energy_j[1];
        out->edp_saving[p] = 1.0 - (out->energy_j[p] * out->time_s[p]) /
                                   (out->energy_j[1] * out->time_s[1]);
    }
    return 0;
}
