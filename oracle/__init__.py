"""MAGUS controller oracle -- TEST INFRASTRUCTURE ONLY.

Plain single-threaded C (``magus_oracle.c``) loaded with ctypes.  Only the
tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package; the product library never does and shares no code with
it.  The C source states, step by step and in the paper's order, what the
controller of arXiv 2502.03796 computes (Alg. 1, Alg. 2 and the decision rule
of Sec. 3.2 / Sec. 4); its header lists every reading taken where the paper is
silent.

Configs are passed as plain dicts with the keys
``window, hold, inc_q16, dec_q16, hf_num, hf_den, level_min, level_max,
level_init`` and optionally ``up_step, down_step`` (steps; 0 = jump to the
bound), ``base`` (derivative base: 0 min of the two samples, 1 oldest,
2 newest, 3 the fixed reference) and ``base_ref`` (B_ref in MB/s for base 3)
-- integers; thresholds in Q16.16.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "magus_oracle.c")
_LIB = os.path.join(_HERE, "libmagus_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/libmagus_oracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
             "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(ctypes.Structure):
    _fields_ = [("direv_length", ctypes.c_uint32), ("tune_len", ctypes.c_uint32),
                ("inc_q", ctypes.c_int32), ("dec_q", ctypes.c_int32),
                ("hf_num", ctypes.c_uint32), ("hf_den", ctypes.c_uint32),
                ("level_min", ctypes.c_uint32), ("level_max", ctypes.c_uint32),
                ("level_init", ctypes.c_uint32), ("up_step", ctypes.c_uint32),
                ("down_step", ctypes.c_uint32), ("base", ctypes.c_uint32),
                ("base_ref", ctypes.c_uint32)]


class _Res(ctypes.Structure):
    _fields_ = [("score", ctypes.c_uint64), ("level_sum", ctypes.c_uint64),
                ("transitions", ctypes.c_uint64), ("ticks_high", ctypes.c_uint64)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_config_valid.argtypes = [ctypes.POINTER(_Cfg)]
        lib.oracle_replay_trace.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(_Cfg), P, ctypes.POINTER(_Res)]
        lib.oracle_replay_trace_fp64.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(_Cfg),
                                                 ctypes.c_double, ctypes.c_double, P,
                                                 ctypes.POINTER(_Res)]
        lib.oracle_replay_batch.argtypes = [P, P, ctypes.c_uint32, P, ctypes.c_uint32, P, P, P]
        lib.oracle_sweep.argtypes = [P, P, ctypes.c_uint32, P, ctypes.c_uint32, P, P]
        lib.oracle_counters_to_mbps.argtypes = [P, P, ctypes.c_uint64, ctypes.c_uint32,
                                                ctypes.c_uint32, P]
        lib.oracle_proxy_model_valid.argtypes = [P]
        lib.oracle_proxy_trace.argtypes = [P, ctypes.c_uint64, P, P, P, P]
        lib.oracle_state_init.argtypes = [P, ctypes.POINTER(_Cfg)]
        lib.oracle_state_init.restype = None
        lib.oracle_step.argtypes = [P, ctypes.POINTER(_Cfg), ctypes.c_uint32, P]
        lib.oracle_state_result.argtypes = [P, ctypes.POINTER(_Res)]
        lib.oracle_serve_tick.argtypes = [P, P, ctypes.c_uint32, P, P, P, ctypes.c_uint32, P]
        _lib = lib
    return _lib


def _cfg(d: dict) -> _Cfg:
    return _Cfg(int(d["window"]), int(d["hold"]), int(d["inc_q16"]), int(d["dec_q16"]),
                int(d["hf_num"]), int(d["hf_den"]), int(d["level_min"]),
                int(d["level_max"]), int(d["level_init"]), int(d.get("up_step", 0)),
                int(d.get("down_step", 0)), int(d.get("base", 0)), int(d.get("base_ref", 0)))


def _cfg_array(cfgs):
    arr = (_Cfg * len(cfgs))()
    for i, d in enumerate(cfgs):
        arr[i] = _cfg(d)
    return arr


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def config_valid(cfg: dict) -> bool:
    c = _cfg(cfg)
    return bool(_load().oracle_config_valid(ctypes.byref(c)))


def replay_trace(x, cfg: dict, want_bytes: bool = True):
    """Run one trace.  Returns (result dict, per-step decision bytes or None)."""
    x = np.ascontiguousarray(x, dtype=np.uint32)
    c = _cfg(cfg)
    r = _Res()
    out = np.empty(len(x), dtype=np.uint8) if want_bytes else None
    rc = _load().oracle_replay_trace(_ptr(x), len(x), ctypes.byref(c), _ptr(out), ctypes.byref(r))
    if rc != 0:
        raise ValueError("oracle: invalid config or trace")
    return _res_dict(r), out


def replay_trace_fp64(x, cfg: dict, inc_threshold: float, dec_threshold: float,
                      want_bytes: bool = True):
    """FP64 side-form of the predictor with decimal thresholds."""
    x = np.ascontiguousarray(x, dtype=np.uint32)
    c = _cfg(cfg)
    r = _Res()
    out = np.empty(len(x), dtype=np.uint8) if want_bytes else None
    rc = _load().oracle_replay_trace_fp64(_ptr(x), len(x), ctypes.byref(c),
                                          float(inc_threshold), float(dec_threshold),
                                          _ptr(out), ctypes.byref(r))
    if rc != 0:
        raise ValueError("oracle: invalid config or trace")
    return _res_dict(r), out


def _res_dict(r: _Res) -> dict:
    return {"score": r.score, "level_sum": r.level_sum,
            "transitions": r.transitions, "ticks_high": r.ticks_high}


def replay_batch(samples, offsets, cfgs, cfg_of_trace=None, want_bytes=False):
    """Run every trace of a CSR batch.  Returns (results[n,4] uint64, bytes or None).

    results columns: score, level_sum, transitions, ticks_high.
    """
    samples = np.ascontiguousarray(samples, dtype=np.uint32)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    n_traces = len(offsets) - 1
    carr = _cfg_array(cfgs)
    cot = None if cfg_of_trace is None else np.ascontiguousarray(cfg_of_trace, dtype=np.uint32)
    res = np.zeros((n_traces, 4), dtype=np.uint64)
    out = np.empty(len(samples), dtype=np.uint8) if want_bytes else None
    rc = _load().oracle_replay_batch(_ptr(samples), _ptr(offsets), n_traces, carr, len(cfgs),
                                     _ptr(cot), _ptr(res), _ptr(out))
    if rc != 0:
        raise ValueError("oracle: invalid batch")
    return res, out


def sweep(samples, offsets, cfgs, want_scores=True):
    """Every trace against every config.  Returns (scores[n_traces, n_cfgs] or None, argmin)."""
    samples = np.ascontiguousarray(samples, dtype=np.uint32)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    n_traces = len(offsets) - 1
    carr = _cfg_array(cfgs)
    scores = np.zeros((n_traces, len(cfgs)), dtype=np.uint64) if want_scores else None
    argmin = np.zeros(n_traces, dtype=np.uint32)
    rc = _load().oracle_sweep(_ptr(samples), _ptr(offsets), n_traces, carr, len(cfgs),
                              _ptr(scores), _ptr(argmin))
    if rc != 0:
        raise ValueError("oracle: invalid sweep")
    return scores, argmin


def counters_to_mbps(counts, ts_ns, counter_bits=48, bytes_per_count=64):
    """Monitor front end: cumulative counter readings to MB/s samples (n-1 of them)."""
    counts = np.ascontiguousarray(counts, dtype=np.uint64)
    ts_ns = np.ascontiguousarray(ts_ns, dtype=np.uint64)
    out = np.zeros(max(len(counts) - 1, 0), dtype=np.uint32)
    rc = _load().oracle_counters_to_mbps(_ptr(counts), _ptr(ts_ns), len(counts),
                                         int(counter_bits), int(bytes_per_count), _ptr(out))
    if rc != 0:
        raise ValueError("oracle: invalid counter arguments")
    return out


class _Model(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_uint32), ("interval_us", ctypes.c_uint32),
                ("cap_mbps", ctypes.c_uint32 * 32), ("uncore_mw", ctypes.c_uint32 * 32),
                ("core_mw", ctypes.c_uint32), ("gpu_mw", ctypes.c_uint32)]


class _Stats(ctypes.Structure):
    _fields_ = [("excess_max", ctypes.c_uint64), ("excess_min", ctypes.c_uint64),
                ("steps", ctypes.c_uint64 * 32), ("excess", ctypes.c_uint64 * 32)]


_METRIC_KEYS = ("time_s", "energy_j", "pkg_power_w", "perf_loss", "pkg_power_saving",
                "energy_saving", "edp_saving")


class _Metrics(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double * 3) for k in _METRIC_KEYS]


def _model(m: dict) -> _Model:
    out = _Model()
    out.n_levels = int(m["n_levels"])
    out.interval_us = int(m["interval_us"])
    for i, v in enumerate(m["cap_mbps"]):
        out.cap_mbps[i] = int(v)
    for i, v in enumerate(m["uncore_mw"]):
        out.uncore_mw[i] = int(v)
    out.core_mw = int(m["core_mw"])
    out.gpu_mw = int(m["gpu_mw"])
    return out


def proxy_model_valid(model: dict) -> bool:
    mm = _model(model)
    return bool(_load().oracle_proxy_model_valid(ctypes.byref(mm)))


def proxy_trace(x, cfg: dict, model: dict):
    """Proxy energy / EDP model of one trace under MAGUS, always-max and always-min.

    model: dict with n_levels, interval_us, cap_mbps[], uncore_mw[], core_mw, gpu_mw.
    Returns (stats dict of exact integers, metrics dict of 3-element lists; column 0
    MAGUS, 1 always at level_max (the baseline), 2 always at level_min).
    """
    x = np.ascontiguousarray(x, dtype=np.uint32)
    c = _cfg(cfg)
    mm = _model(model)
    st = _Stats()
    me = _Metrics()
    rc = _load().oracle_proxy_trace(_ptr(x), len(x), ctypes.byref(c), ctypes.byref(mm),
                                    ctypes.byref(st), ctypes.byref(me))
    if rc != 0:
        raise ValueError("oracle: invalid config, model or trace")
    stats = {"excess_max": st.excess_max, "excess_min": st.excess_min,
             "steps": list(st.steps), "excess": list(st.excess)}
    metrics = {k: list(getattr(me, k)) for k in _METRIC_KEYS}
    return stats, metrics


class _State(ctypes.Structure):
    _fields_ = [("mem_throughput_ls", ctypes.c_uint32 * 64), ("filled", ctypes.c_uint32),
                ("level", ctypes.c_uint32), ("uncore_tune_ls", ctypes.c_uint8 * 64),
                ("level_sum", ctypes.c_uint64), ("transitions", ctypes.c_uint64),
                ("ticks_high", ctypes.c_uint64), ("steps", ctypes.c_uint64)]


class Streams:
    """Controller states of many streams, each stepped one sample at a time
    (one invocation per monitoring interval, Sec. 3.2)."""

    def __init__(self, cfgs, cfg_of_stream):
        self.cfgs = _cfg_array(cfgs)
        self.n_cfgs = len(cfgs)
        self.cfg_of_stream = np.ascontiguousarray(cfg_of_stream, dtype=np.uint32)
        n = len(self.cfg_of_stream)
        if n and int(self.cfg_of_stream.max()) >= self.n_cfgs:
            raise ValueError("oracle: config index out of range")
        self.states = (_State * n)()
        lib = _load()
        for i in range(n):
            lib.oracle_state_init(ctypes.byref(self.states[i]),
                                  ctypes.byref(self.cfgs[int(self.cfg_of_stream[i])]))

    def reset(self, stream: int) -> None:
        _load().oracle_state_init(ctypes.byref(self.states[stream]),
                                  ctypes.byref(self.cfgs[int(self.cfg_of_stream[stream])]))

    def tick(self, streams, samples):
        """One step for each (stream, sample) pair, in order; returns the decision bytes."""
        st = np.ascontiguousarray(streams, dtype=np.uint32)
        x = np.ascontiguousarray(samples, dtype=np.uint32)
        if len(st) != len(x) or (len(st) and int(st.max()) >= len(self.cfg_of_stream)):
            raise ValueError("oracle: bad stream ids")
        out = np.empty(len(x), dtype=np.uint8)
        rc = _load().oracle_serve_tick(ctypes.cast(self.states, ctypes.c_void_p), self.cfgs,
                                       self.n_cfgs, _ptr(self.cfg_of_stream), _ptr(st), _ptr(x),
                                       len(x), _ptr(out))
        if rc != 0:
            raise ValueError("oracle: invalid tick")
        return out

    def result(self, stream: int) -> dict:
        r = _Res()
        _load().oracle_state_result(ctypes.byref(self.states[stream]), ctypes.byref(r))
        return _res_dict(r)


def decode(byte_arr):
    """Split decision bytes into (level, high, pred) arrays."""
    b = np.asarray(byte_arr, dtype=np.uint8)
    return (b & 31).astype(np.int64), ((b >> 5) & 1).astype(np.int64), \
        (b >> 6).astype(np.int64) - 1
