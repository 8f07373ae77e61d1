/*
 * Test driver for a sanitizer build of the oracle (AddressSanitizer and
 * UndefinedBehaviorSanitizer): reads one batch from a binary file, runs the
 * batch replay (with decision bytes), the sweep, the proxy and the counter
 * front end, and writes every output to another file for comparison with the
 * regular build.  Input layout (little-endian):
 *   u64 n_samples, u32 n_traces, u32 n_cfgs, u64 n_readings,
 *   u32 samples[n_samples], u64 offsets[n_traces + 1],
 *   oracle_config cfgs[n_cfgs], u32 cfg_of_trace[n_traces],
 *   oracle_proxy_model model, u64 counts[n_readings], u64 ts_ns[n_readings],
 *   u32 counter_bits, u32 bytes_per_count
 * Output: results, decision bytes, sweep scores and arg-min, per-trace proxy
 * stats and metrics (config of the trace), counter samples.
 */
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/magus_oracle.h"

static void* read_n(FILE* f, size_t size, size_t n) {
    void* p = malloc(size * n + 1);
    if (!p || fread(p, size, n, f) != n) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
    return p;
}

static void write_n(FILE* f, const void* p, size_t size, size_t n) {
    if (n && fwrite(p, size, n, f) != n) {
        fprintf(stderr, "short output\n");
        exit(2);
    }
}

int main(int argc, char** argv) {
    if (argc != 3) return 2;
    FILE* in = fopen(argv[1], "rb");
    if (!in) return 2;
    uint64_t n_samples, n_readings;
    uint32_t n_traces, n_cfgs;
    if (fread(&n_samples, 8, 1, in) != 1 || fread(&n_traces, 4, 1, in) != 1 ||
        fread(&n_cfgs, 4, 1, in) != 1 || fread(&n_readings, 8, 1, in) != 1)
        return 2;
    uint32_t* samples = read_n(in, 4, n_samples);
    uint64_t* offsets = read_n(in, 8, (size_t)n_traces + 1);
    oracle_config* cfgs = read_n(in, sizeof(oracle_config), n_cfgs);
    uint32_t* cot = read_n(in, 4, n_traces);
    oracle_proxy_model* model = read_n(in, sizeof(oracle_proxy_model), 1);
    uint64_t* counts = read_n(in, 8, n_readings);
    uint64_t* ts = read_n(in, 8, n_readings);
    uint32_t* fe = read_n(in, 4, 2);
    fclose(in);

    oracle_result* res = malloc(sizeof(oracle_result) * (n_traces + 1));
    uint8_t* bytes = malloc(n_samples + 1);
    uint64_t* scores = malloc(8 * ((size_t)n_traces * n_cfgs + 1));
    uint32_t* argmin = malloc(4 * ((size_t)n_traces + 1));
    oracle_proxy_stats* st = malloc(sizeof(oracle_proxy_stats) * (n_traces + 1));
    oracle_proxy_metrics* me = malloc(sizeof(oracle_proxy_metrics) * (n_traces + 1));
    uint32_t* mbps = malloc(4 * (n_readings + 1));
    int rc = 0;
    rc |= oracle_replay_batch(samples, offsets, n_traces, cfgs, n_cfgs, cot, res, bytes);
    rc |= oracle_sweep(samples, offsets, n_traces, cfgs, n_cfgs, scores, argmin);
    for (uint32_t t = 0; t < n_traces; ++t)
        rc |= oracle_proxy_trace(samples + offsets[t], offsets[t + 1] - offsets[t],
                                 &cfgs[cot[t]], model, &st[t], &me[t]);
    if (n_readings >= 2) rc |= oracle_counters_to_mbps(counts, ts, n_readings, fe[0], fe[1], mbps);
    if (rc) {
        fprintf(stderr, "oracle call failed\n");
        return 3;
    }
    FILE* out = fopen(argv[2], "wb");
    if (!out) return 2;
    write_n(out, res, sizeof(oracle_result), n_traces);
    write_n(out, bytes, 1, n_samples);
    write_n(out, scores, 8, (size_t)n_traces * n_cfgs);
    write_n(out, argmin, 4, n_traces);
    write_n(out, st, sizeof(oracle_proxy_stats), n_traces);
    write_n(out, me, sizeof(oracle_proxy_metrics), n_traces);
    if (n_readings >= 2) write_n(out, mbps, 4, n_readings - 1);
    fclose(out);
    free(samples); free(offsets); free(cfgs); free(cot); free(model); free(counts); free(ts);
    free(fe); free(res); free(bytes); free(scores); free(argmin); free(st); free(me); free(mbps);
    return 0;
}
