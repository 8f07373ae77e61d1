"""Parameter tables of the proxy energy / EDP model (inputs, not arithmetic).

The paper measures energy on two Xeon + GPU machines and publishes no power or
performance model, so the tables below are a synthetic stand-in with the
shape such a model has: the uncore ladder of 17 rungs from 0.8 to 2.4 GHz in
100 MHz steps, a memory throughput the uncore sustains that grows with its
frequency, an uncore power that grows faster than linearly, and constant core
and GPU power (a GPU-heavy node whose cores are mostly idle).
"""
from __future__ import annotations

LADDER_MHZ = [800 + 100 * i for i in range(17)]


def proxy_model(cap_mbps_per_mhz: int = 50, uncore_min_mw: int = 15000,
                uncore_span_mw: int = 25000, core_mw: int = 60000, gpu_mw: int = 250000,
                interval_us: int = 100000) -> dict:
    """Model dict for the 17-rung ladder.

    cap[i] = cap_mbps_per_mhz * f_i (40,000 MB/s at 0.8 GHz, 120,000 at
    2.4 GHz by default); uncore[i] = uncore_min + uncore_span * (i / 16)^2
    rounded to the milliwatt (15 W .. 40 W); core 60 W, GPU 250 W; 100 ms
    intervals.
    """
    n = len(LADDER_MHZ)
    return {
        "n_levels": n,
        "interval_us": interval_us,
        "cap_mbps": [cap_mbps_per_mhz * f for f in LADDER_MHZ],
        "uncore_mw": [uncore_min_mw + (uncore_span_mw * i * i + (n - 1) ** 2 // 2) // (n - 1) ** 2
                      for i in range(n)],
        "core_mw": core_mw,
        "gpu_mw": gpu_mw,
    }
