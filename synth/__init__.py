"""Seeded synthetic inputs for the MAGUS hot path.

This package generates telemetry traces and controller-config grids.  It holds
none of the controller's arithmetic: it only draws numbers.  Both the HIP
library's tests/benchmarks and the oracle consume what it produces, so the two
sides always see identical bytes.

Random numbers come from SplitMix64 (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used in counter mode: draw k of a
stream with key K is mix64(K + (k + 1) * 0x9E3779B97F4A7C15).
"""
from .rng import mix64, stream_key, purpose_key, draws_u64, uniform01
from .traces import (four_phase_trace, geometric_phase_trace, make_batch,
                     workload_small, workload_bulk, workload_sweep_traces,
                     workload_uneven, serve_stream_samples, serve_schedule,
                     serve_fleet_events, EVENT_DTYPE, EV_SAMPLE, EV_JOIN, EV_LEAVE)
from .proxy import proxy_model, LADDER_MHZ
from .grid import (default_config, THRESHOLD_TABLE_Q16, threshold_q16, sweep_grid,
                   sweep_config, config_index)

__all__ = [
    "mix64", "stream_key", "purpose_key", "draws_u64", "uniform01",
    "four_phase_trace", "geometric_phase_trace", "make_batch",
    "workload_small", "workload_bulk", "workload_sweep_traces", "workload_uneven",
    "serve_stream_samples", "serve_schedule", "serve_fleet_events", "EVENT_DTYPE",
    "EV_SAMPLE", "EV_JOIN", "EV_LEAVE",
    "default_config", "THRESHOLD_TABLE_Q16", "threshold_q16", "sweep_grid",
    "sweep_config", "config_index", "proxy_model", "LADDER_MHZ",
]
