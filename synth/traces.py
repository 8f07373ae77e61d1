"""Synthetic memory-throughput traces (uint32 MB/s, one sample per 100 ms tick).

The paper measures on application telemetry (Altis, ECP proxies, GROMACS,
LAMMPS, MLPerf) that was never published; these seeded traces stand in for it
with the shapes the workloads are quoted on:

* four-phase traces: 3 cut points drawn uniformly without replacement in
  [1, n-1], phase levels uniform in [1,000, 200,000] MB/s;
* geometric-phase traces: phase lengths Geometric(mean 200) samples, levels
  log-normal (median 20,000 MB/s, sigma 1.0) clipped to [500, 400,000]; the
  bursty variant makes a phase short (uniform 1..50 samples) with probability
  0.1;
* every sample gets multiplicative noise: x = round-half-even(L * (1 + u)),
  u ~ U[-0.05, 0.05], clamped to the uint32 range.

Geometric lengths are 1 + floor(ln(1-u) / ln(1 - 1/mean)); normals use
Box-Muller.  Everything is drawn from counter-mode SplitMix64 streams.
"""
from __future__ import annotations

import math

import numpy as np

from .rng import stream_key, purpose_key, uniform01

SEED_BASE = 0x4D41475553
P_NOISE, P_LEN, P_LEVEL, P_SHORT, P_CUT, P_LEN2, P_FLIP = range(7)

U32_MAX = float(2**32 - 1)


def apply_noise(levels: np.ndarray, key: int, start: int = 0) -> np.ndarray:
    u = uniform01(purpose_key(key, P_NOISE), start, len(levels))
    x = np.rint(levels * (1.0 + (u * 0.1 - 0.05)))
    return np.clip(x, 0.0, U32_MAX).astype(np.uint32)


def four_phase_trace(n: int, key: int, lo: float = 1000.0, hi: float = 200000.0,
                     phases: int = 4) -> np.ndarray:
    """Piecewise-constant trace with `phases` phases (fewer when n is tiny)."""
    if n <= 0:
        return np.zeros(0, dtype=np.uint32)
    ncut = min(phases - 1, max(n - 1, 0))
    cuts: list[int] = []
    k = 0
    ck = purpose_key(key, P_CUT)
    while len(cuts) < ncut:
        u = uniform01(ck, k, 1)[0]
        k += 1
        c = 1 + int(math.floor(u * (n - 1)))
        if c not in cuts:
            cuts.append(c)
    cuts.sort()
    bounds = [0] + cuts + [n]
    lv = lo + uniform01(purpose_key(key, P_LEVEL), 0, len(bounds) - 1) * (hi - lo)
    levels = np.repeat(lv, np.diff(bounds))
    return apply_noise(levels, key)


def _phase_lengths(n: int, key: int, mean: float, short_prob: float) -> np.ndarray:
    """Enough phase lengths to cover n samples."""
    out = []
    total = 0
    start = 0
    batch = max(16, int(2 * n / mean) + 16)
    lnq = math.log(1.0 - 1.0 / mean)
    while total < n:
        u = uniform01(purpose_key(key, P_LEN), start, batch)
        lens = 1 + np.floor(np.log1p(-u) / lnq).astype(np.int64)
        if short_prob > 0.0:
            s = uniform01(purpose_key(key, P_SHORT), start, batch)
            u2 = uniform01(purpose_key(key, P_LEN2), start, batch)
            short = 1 + np.floor(u2 * 50.0).astype(np.int64)
            lens = np.where(s < short_prob, short, lens)
        out.append(lens)
        total += int(lens.sum())
        start += batch
    lens = np.concatenate(out)
    cs = np.cumsum(lens)
    m = int(np.searchsorted(cs, n)) + 1
    return lens[:m]


def lognormal_levels(key: int, count: int, median: float = 20000.0, sigma: float = 1.0,
                     lo: float = 500.0, hi: float = 400000.0) -> np.ndarray:
    u1 = uniform01(purpose_key(key, P_LEVEL), 0, count)
    u2 = uniform01(purpose_key(key, P_LEVEL), count, count)
    z = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * math.pi * u2)
    return np.clip(median * np.exp(sigma * z), lo, hi)


def geometric_phase_trace(n: int, key: int, mean: float = 200.0, short_prob: float = 0.0,
                          median: float = 20000.0, sigma: float = 1.0) -> np.ndarray:
    if n <= 0:
        return np.zeros(0, dtype=np.uint32)
    lens = _phase_lengths(n, key, mean, short_prob)
    lv = lognormal_levels(key, len(lens), median, sigma)
    levels = np.repeat(lv, lens)[:n]
    return apply_noise(levels, key)


def make_batch(traces) -> tuple[np.ndarray, np.ndarray]:
    """CSR batch: (samples uint32[N], offsets uint64[T+1])."""
    lens = np.array([len(t) for t in traces], dtype=np.uint64)
    offsets = np.zeros(len(traces) + 1, dtype=np.uint64)
    np.cumsum(lens, out=offsets[1:])
    samples = np.empty(int(offsets[-1]), dtype=np.uint32)
    for i, t in enumerate(traces):
        samples[int(offsets[i]):int(offsets[i + 1])] = t
    return samples, offsets


# --------------------------------------------------------------- workloads

def workload_small(n: int = 10000):
    """One four-phase trace of 10,000 samples (the plain single-trace replay)."""
    key = stream_key(SEED_BASE + 1, 0)
    return make_batch([four_phase_trace(n, key)])


def workload_bulk(n_traces: int = 4096, n: int = 100000):
    """4,096 geometric-phase traces x 100,000 samples (bulk single-config replay)."""
    offsets = np.arange(n_traces + 1, dtype=np.uint64) * np.uint64(n)
    samples = np.empty(n_traces * n, dtype=np.uint32)
    for t in range(n_traces):
        samples[t * n:(t + 1) * n] = geometric_phase_trace(n, stream_key(SEED_BASE + 2, t))
    return samples, offsets


def workload_sweep_traces(n_traces: int = 1024, n: int = 50000):
    """1,024 four-phase traces x 50,000 samples (the parameter-sweep traces)."""
    offsets = np.arange(n_traces + 1, dtype=np.uint64) * np.uint64(n)
    samples = np.empty(n_traces * n, dtype=np.uint32)
    for t in range(n_traces):
        samples[t * n:(t + 1) * n] = four_phase_trace(n, stream_key(SEED_BASE + 3, t))
    return samples, offsets


def uneven_lengths(n_traces: int, seed: int = SEED_BASE + 4, median: float = 20000.0,
                   sigma: float = 1.0, lo: int = 1000, hi: int = 1000000) -> np.ndarray:
    key = stream_key(seed, 1 << 40)
    u1 = uniform01(purpose_key(key, P_LEN), 0, n_traces)
    u2 = uniform01(purpose_key(key, P_LEN), n_traces, n_traces)
    z = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * math.pi * u2)
    return np.clip(np.floor(median * np.exp(sigma * z)), lo, hi).astype(np.int64)


def workload_uneven(n_traces: int = 20000, n_cfgs: int = 16384):
    """20,000 bursty traces of log-normal length (median 20,000, 1,000..1,000,000),
    each paired with a uniformly drawn config index of the sweep grid."""
    seed = SEED_BASE + 4
    lens = uneven_lengths(n_traces, seed)
    offsets = np.zeros(n_traces + 1, dtype=np.uint64)
    np.cumsum(lens.astype(np.uint64), out=offsets[1:])
    samples = np.empty(int(offsets[-1]), dtype=np.uint32)
    for t in range(n_traces):
        samples[int(offsets[t]):int(offsets[t + 1])] = geometric_phase_trace(
            int(lens[t]), stream_key(seed, t), short_prob=0.1)
    ck = stream_key(seed, (1 << 40) + 1)
    cfg_of_trace = np.minimum(
        np.floor(uniform01(ck, 0, n_traces) * n_cfgs), n_cfgs - 1).astype(np.uint32)
    return samples, offsets, cfg_of_trace


# ----------------------------------------------------------------- serving

def serve_stream_samples(stream_id: int, n_ticks: int, seed: int = SEED_BASE + 5,
                         mean: float = 2500.0, lo: float = 1000.0, hi: float = 200000.0,
                         flip_prob: float = 0.01) -> np.ndarray:
    """Samples of one served node: phases Geometric(mean 2,500 ticks) with levels
    U[1,000, 200,000]; a flip starts with probability 0.01 per tick and lasts
    U{1..50} ticks at a fresh U[1,000, 200,000] level."""
    key = stream_key(seed, stream_id)
    lens = _phase_lengths(n_ticks, key, mean, 0.0)
    lv = lo + uniform01(purpose_key(key, P_LEVEL), 0, len(lens)) * (hi - lo)
    levels = np.repeat(lv, lens)[:n_ticks].copy()
    fk = purpose_key(key, P_FLIP)
    starts = np.nonzero(uniform01(fk, 0, n_ticks) < flip_prob)[0]
    if len(starts):
        flen = 1 + np.floor(uniform01(fk, n_ticks, len(starts)) * 50.0).astype(np.int64)
        flv = lo + uniform01(fk, n_ticks + len(starts), len(starts)) * (hi - lo)
        for s, ln, v in zip(starts, flen, flv):
            levels[s:s + ln] = v
    return apply_noise(levels, key)


def serve_schedule(n_streams: int, n_ticks: int, period_ms: float = 100.0,
                   jitter_ms: float = 10.0, seed: int = SEED_BASE + 5) -> np.ndarray:
    """Arrival time (ms, float64) of each (stream, tick): tick * period + phase
    offset of the stream + U[-jitter, +jitter]."""
    key = stream_key(seed, 1 << 41)
    phase = uniform01(purpose_key(key, 0), 0, n_streams) * period_ms
    jit = (uniform01(purpose_key(key, 1), 0, n_streams * n_ticks) * 2.0 - 1.0) * jitter_ms
    t = np.arange(n_ticks, dtype=np.float64)[None, :] * period_ms + phase[:, None]
    return t + jit.reshape(n_streams, n_ticks)


EVENT_DTYPE = np.dtype([("t_ns", "<u8"), ("kind", "<u4"), ("stream", "<u4"),
                        ("value", "<u4"), ("reserved", "<u4")])
EV_SAMPLE, EV_JOIN, EV_LEAVE = 0, 1, 2


def serve_fleet_events(n_initial: int, n_ticks: int, period_ms: float = 100.0,
                       jitter_ms: float = 10.0, join_rate: float = 50.0,
                       leave_rate: float = 50.0, n_cfgs: int = 16384,
                       seed: int = SEED_BASE + 5):
    """A fleet of simulated nodes as a time-sorted event list.

    n_initial nodes join at time 0; new nodes join as a Poisson process of
    `join_rate` per second and uniformly chosen live nodes leave at
    `leave_rate` per second.  Every live node emits one sample per period at
    its own phase offset plus U[-jitter, +jitter].  Each node gets a config
    index drawn uniformly from [0, n_cfgs).

    Returns (events: EVENT_DTYPE array sorted by time, n_streams, cfg_of_stream).
    """
    dur_ms = n_ticks * period_ms
    key = stream_key(seed, 1 << 42)
    # Poisson joins and leaves
    def poisson_times(pk, rate):
        if rate <= 0:
            return np.zeros(0)
        n_max = int(rate * dur_ms / 1000.0 * 3 + 20)
        gaps = -np.log1p(-uniform01(purpose_key(key, pk), 0, n_max)) / rate * 1000.0
        t = np.cumsum(gaps)
        return t[t < dur_ms]
    join_t = poisson_times(0, join_rate)
    leave_t = poisson_times(1, leave_rate)
    n_streams = n_initial + len(join_t)
    start = np.concatenate([np.zeros(n_initial), join_t])
    end = np.full(n_streams, np.inf)
    # each leave picks a uniformly random live node
    pick = uniform01(purpose_key(key, 2), 0, max(1, len(leave_t)))
    order = np.argsort(start, kind="stable")
    for i, tl in enumerate(leave_t):
        live = np.nonzero((start <= tl) & (end > tl))[0]
        if len(live):
            end[live[min(int(pick[i] * len(live)), len(live) - 1)]] = tl
    cfg_of_stream = np.minimum(np.floor(uniform01(purpose_key(key, 3), 0, n_streams) * n_cfgs),
                               n_cfgs - 1).astype(np.uint32)
    phase = uniform01(purpose_key(key, 4), 0, n_streams) * period_ms
    chunks = []
    for sid in range(n_streams):
        first = int(np.ceil((start[sid] - phase[sid] + jitter_ms) / period_ms))
        first = max(first, 0)
        ticks = np.arange(first, n_ticks)
        jit = (uniform01(purpose_key(stream_key(seed, sid), 9), 0, n_ticks)[ticks] * 2.0
               - 1.0) * jitter_ms
        t = ticks * period_ms + phase[sid] + jit
        keep = (t > start[sid]) & (t < end[sid]) & (t < dur_ms)
        t = t[keep]
        if len(t) == 0:
            continue
        vals = serve_stream_samples(sid, len(t), seed=seed)
        ev = np.zeros(len(t), EVENT_DTYPE)
        ev["t_ns"] = np.round(t * 1e6).astype(np.uint64)
        ev["kind"] = EV_SAMPLE
        ev["stream"] = sid
        ev["value"] = vals
        chunks.append(ev)
    jn = np.zeros(n_streams, EVENT_DTYPE)
    jn["t_ns"] = np.round(start * 1e6).astype(np.uint64)
    jn["kind"] = EV_JOIN
    jn["stream"] = np.arange(n_streams)
    jn["value"] = cfg_of_stream
    left = np.nonzero(np.isfinite(end))[0]
    lv = np.zeros(len(left), EVENT_DTYPE)
    lv["t_ns"] = np.round(end[left] * 1e6).astype(np.uint64)
    lv["kind"] = EV_LEAVE
    lv["stream"] = left
    ev = np.concatenate([jn] + chunks + [lv])
    rank = np.where(ev["kind"] == EV_JOIN, 0, np.where(ev["kind"] == EV_SAMPLE, 1, 2))
    ev = ev[np.lexsort((rank, ev["t_ns"]))]
    return ev, n_streams, cfg_of_stream
