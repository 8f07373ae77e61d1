"""Python binding of libmagus: MAGUS (arXiv 2502.03796) replay, sweep and serving
on MI355X (gfx950).

Argument marshalling only: every step of the controller runs in the HIP
kernels behind the C ABI of ``include/magus.h``.  PyTorch supplies device
memory and streams.  There is no CPU fallback: if ``libmagus.so`` has not been
built, every entry point raises.

Configs are dicts with the keys ``window, hold, inc_q16, dec_q16, hf_num,
hf_den, level_min, level_max, level_init`` and optionally ``up_step,
down_step, base, base_ref`` (see ``include/magus.h`` for meaning and ranges).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmagus.so")

OK, EINVAL, ENOMEM, ENOSLOT, EDEVICE, EDATA = 0, -1, -2, -3, -4, -5
KERNEL_REPLAY, KERNEL_SWEEP, KERNEL_SERVE, KERNEL_PROBE = 0, 1, 2, 3
MAX_TRACE_LEN = (1 << 30) - 1
DATA_OFFSETS, DATA_TOO_LONG, DATA_CFG_INDEX = 1, 2, 4   # data-check status bits
NOALLOC_SCRATCH_BYTES = 8 << 20
NOALLOC_MAX_CFGS = 16384


class MagusError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"magus error {code}: {msg}")
        self.code = code


class MagusConfig(ctypes.Structure):
    _fields_ = [("window", ctypes.c_uint16), ("hold", ctypes.c_uint16),
                ("inc_q16", ctypes.c_int32), ("dec_q16", ctypes.c_int32),
                ("hf_num", ctypes.c_uint8), ("hf_den", ctypes.c_uint8),
                ("level_min", ctypes.c_uint8), ("level_max", ctypes.c_uint8),
                ("level_init", ctypes.c_uint8), ("up_step", ctypes.c_uint8),
                ("down_step", ctypes.c_uint8), ("base", ctypes.c_uint8),
                ("base_ref", ctypes.c_uint32)]


class MagusResult(ctypes.Structure):
    _fields_ = [("score", ctypes.c_uint64), ("level_sum", ctypes.c_uint64),
                ("transitions", ctypes.c_uint64), ("ticks_high", ctypes.c_uint64)]


class MagusRunStats(ctypes.Structure):
    _fields_ = [("samples_served", ctypes.c_uint64), ("samples_dropped", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("max_batch", ctypes.c_uint64),
                ("max_in_flight", ctypes.c_uint64), ("deferred", ctypes.c_uint64),
                ("joins_admitted", ctypes.c_uint64), ("joins_waited", ctypes.c_uint64),
                ("joins_refused", ctypes.c_uint64), ("wall_s", ctypes.c_double)]


class MagusSweepTuneResult(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_uint32), ("lanes", ctypes.c_uint32),
                ("tile", ctypes.c_uint32), ("candidates", ctypes.c_uint32),
                ("best_ms", ctypes.c_double), ("default_ms", ctypes.c_double)]


SWEEP_SHAPES = 6


class MagusTuneResult(ctypes.Structure):
    _fields_ = [("chunk_steps", ctypes.c_uint32), ("persistent_blocks", ctypes.c_uint32),
                ("candidates", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("best_ms", ctypes.c_double), ("default_ms", ctypes.c_double)]


PROXY_LEVELS = 32


class MagusProxyModel(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_uint32), ("interval_us", ctypes.c_uint32),
                ("cap_mbps", ctypes.c_uint32 * PROXY_LEVELS),
                ("uncore_mw", ctypes.c_uint32 * PROXY_LEVELS),
                ("core_mw", ctypes.c_uint32), ("gpu_mw", ctypes.c_uint32)]


class MagusProxyStats(ctypes.Structure):
    _fields_ = [("excess_max", ctypes.c_uint64), ("excess_min", ctypes.c_uint64),
                ("steps", ctypes.c_uint64 * PROXY_LEVELS),
                ("excess", ctypes.c_uint64 * PROXY_LEVELS)]


PROXY_METRIC_KEYS = ("time_s", "energy_j", "pkg_power_w", "perf_loss", "pkg_power_saving",
                     "energy_saving", "edp_saving")


class MagusProxyMetrics(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double * 3) for k in PROXY_METRIC_KEYS]


EV_SAMPLE, EV_JOIN, EV_LEAVE = 0, 1, 2
EVENT_DTYPE = np.dtype([("t_ns", "<u8"), ("kind", "<u4"), ("stream", "<u4"),
                        ("value", "<u4"), ("reserved", "<u4")])

assert ctypes.sizeof(MagusConfig) == 24 and ctypes.sizeof(MagusResult) == 32
assert ctypes.sizeof(MagusProxyModel) == 272 and ctypes.sizeof(MagusProxyStats) == 528
assert ctypes.sizeof(MagusProxyMetrics) == 168
assert EVENT_DTYPE.itemsize == 24

_lib = None

# name -> (restype, argtypes); every symbol of include/magus.h
_P = ctypes.c_void_p
SIGNATURES = {
    "magus_version": (ctypes.c_char_p, []),
    "magus_last_error": (ctypes.c_char_p, []),
    "magus_config_check": (ctypes.c_int, [_P]),
    "magus_ctx_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_P)]),
    "magus_ctx_destroy": (ctypes.c_int, [_P]),
    "magus_ctx_set_chunk": (ctypes.c_int, [_P, ctypes.c_uint32]),
    "magus_ctx_get_chunk": (ctypes.c_uint32, [_P]),
    "magus_ctx_check": (ctypes.c_int, [_P, _P]),
    "magus_ctx_set_persistent": (ctypes.c_int, [_P, ctypes.c_uint32]),
    "magus_ctx_get_persistent": (ctypes.c_uint32, [_P]),
    "magus_ctx_set_graphs": (ctypes.c_int, [_P, ctypes.c_int]),
    "magus_autotune_replay": (ctypes.c_int, [_P, _P, ctypes.c_uint64, _P, ctypes.c_uint32, _P,
                                             ctypes.c_uint32, _P, _P, ctypes.c_uint32, _P,
                                             ctypes.POINTER(MagusTuneResult)]),
    "magus_ctx_set_profiling": (ctypes.c_int, [_P, ctypes.c_int]),
    "magus_ctx_kernel_time": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_uint64)]),
    "magus_replay": (ctypes.c_int, [_P, _P, ctypes.c_uint64, _P, ctypes.c_uint32, _P,
                                    ctypes.c_uint32, _P, _P, _P, _P]),
    "magus_replay_noalloc": (ctypes.c_int, [_P, ctypes.c_uint64, _P, ctypes.c_uint32, _P,
                                            ctypes.c_uint32, _P, _P, _P, _P, _P]),
    "magus_sweep": (ctypes.c_int, [_P, _P, ctypes.c_uint64, _P, ctypes.c_uint32, _P,
                                   ctypes.c_uint32, _P, _P, _P]),
    "magus_ctx_set_sweep_shape": (ctypes.c_int, [_P, ctypes.c_uint32]),
    "magus_ctx_get_sweep_shape": (ctypes.c_uint32, [_P]),
    "magus_sweep_shape_info": (ctypes.c_int, [ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32),
                                              ctypes.POINTER(ctypes.c_uint32)]),
    "magus_autotune_sweep": (ctypes.c_int, [_P, _P, ctypes.c_uint64, _P, ctypes.c_uint32, _P,
                                            ctypes.c_uint32, _P, ctypes.c_uint32, _P,
                                            ctypes.POINTER(MagusSweepTuneResult)]),
    "magus_valu_probe": (ctypes.c_int, [_P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                        _P, ctypes.POINTER(ctypes.c_uint64), _P]),
    "magus_read_probe": (ctypes.c_int, [_P, _P, ctypes.c_uint64, ctypes.c_uint32, _P, _P]),
    "magus_counters_to_mbps": (ctypes.c_int, [_P, _P, _P, ctypes.c_uint64, _P, ctypes.c_uint32,
                                              ctypes.c_uint32, ctypes.c_uint32, _P, _P]),
    "magus_proxy_model_check": (ctypes.c_int, [ctypes.POINTER(MagusProxyModel)]),
    "magus_proxy": (ctypes.c_int, [_P, _P, ctypes.c_uint64, _P, ctypes.c_uint32, _P,
                                   ctypes.c_uint32, _P, ctypes.POINTER(MagusProxyModel), _P, _P,
                                   _P]),
    "magus_server_slot_bytes": (ctypes.c_size_t, []),
    "magus_server_create": (ctypes.c_int, [_P, ctypes.c_size_t, ctypes.POINTER(_P)]),
    "magus_server_destroy": (ctypes.c_int, [_P]),
    "magus_server_capacity": (ctypes.c_uint32, [_P]),
    "magus_server_open_count": (ctypes.c_uint32, [_P]),
    "magus_stream_open": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_uint32)]),
    "magus_stream_close": (ctypes.c_int, [_P, ctypes.c_uint32]),
    "magus_serve_step": (ctypes.c_int, [_P, _P, _P, ctypes.c_uint32, _P, _P]),
    "magus_stream_result": (ctypes.c_int, [_P, ctypes.c_uint32, ctypes.POINTER(MagusResult)]),
    "magus_server_run": (ctypes.c_int, [_P, _P, ctypes.c_uint64, ctypes.c_uint32, _P,
                                        ctypes.c_uint32, ctypes.c_int, ctypes.c_uint32,
                                        ctypes.c_uint32, _P, _P,
                                        ctypes.POINTER(MagusRunStats)]),
}


def load() -> ctypes.CDLL:
    """Load libmagus.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "paper_2502_03796_amd.build.build() (no CPU fallback exists)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != OK:
        raise MagusError(rc, load().magus_last_error().decode())


def make_config(d: dict) -> MagusConfig:
    return MagusConfig(int(d["window"]), int(d["hold"]), int(d["inc_q16"]), int(d["dec_q16"]),
                       int(d["hf_num"]), int(d["hf_den"]), int(d["level_min"]),
                       int(d["level_max"]), int(d["level_init"]), int(d.get("up_step", 0)),
                       int(d.get("down_step", 0)), int(d.get("base", 0)),
                       int(d.get("base_ref", 0)))


def config_array(cfgs) -> ctypes.Array:
    """Marshal configs (a dict, a list of dicts, or an already built array)."""
    if isinstance(cfgs, ctypes.Array):
        return cfgs
    if isinstance(cfgs, dict):
        cfgs = [cfgs]
    arr = (MagusConfig * len(cfgs))()
    for i, d in enumerate(cfgs):
        arr[i] = make_config(d)
    return arr


def sweep_shape_info(shape: int):
    """(configs per workgroup, steps per tile) of a sweep launch shape."""
    lanes, tile = ctypes.c_uint32(), ctypes.c_uint32()
    _check(load().magus_sweep_shape_info(int(shape), ctypes.byref(lanes), ctypes.byref(tile)))
    return lanes.value, tile.value


def config_check(cfg: dict) -> None:
    c = make_config(cfg)
    _check(load().magus_config_check(ctypes.byref(c)))


def _torch():
    import torch
    return torch


def _dev_ptr(t, name, dtypes):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} must have dtype in {dtypes}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream, device):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def make_proxy_model(d: dict) -> MagusProxyModel:
    """Proxy model from a dict: n_levels, interval_us, cap_mbps[], uncore_mw[],
    core_mw, gpu_mw (see include/magus.h)."""
    m = MagusProxyModel()
    m.n_levels = int(d["n_levels"])
    m.interval_us = int(d["interval_us"])
    for i, v in enumerate(d["cap_mbps"]):
        m.cap_mbps[i] = int(v)
    for i, v in enumerate(d["uncore_mw"]):
        m.uncore_mw[i] = int(v)
    m.core_mw = int(d["core_mw"])
    m.gpu_mw = int(d["gpu_mw"])
    return m


def proxy_model_check(d) -> None:
    """Raise MagusError(EINVAL) unless the proxy model is valid (host only)."""
    mm = d if isinstance(d, MagusProxyModel) else make_proxy_model(d)
    _check(load().magus_proxy_model_check(ctypes.byref(mm)))


def proxy_stats_dict(row) -> dict:
    """One row of the int64[T, 66] stats tensor returned by Context.proxy."""
    v = [int(x) & 0xFFFFFFFFFFFFFFFF for x in row]
    return {"excess_max": v[0], "excess_min": v[1], "steps": v[2:2 + PROXY_LEVELS],
            "excess": v[2 + PROXY_LEVELS:2 + 2 * PROXY_LEVELS]}


def proxy_metrics_dict(row) -> dict:
    """One row of the float64[T, 21] metrics tensor returned by Context.proxy."""
    v = [float(x) for x in row]
    return {k: v[3 * i:3 * i + 3] for i, k in enumerate(PROXY_METRIC_KEYS)}


def replay_noalloc(samples, offsets, cfgs, cfg_of_trace=None, levels: bool = False,
                   results=None, levels_out=None, status=None, stream=None):
    """magus_replay_noalloc on the tensors' device (made current for the call):
    the jump-to-bound replay without a context, with the library's fixed
    scratch array.  Returns (results int64[T, 4], levels uint8 or None,
    status int32[1]: the data-check bits, 0 = run)."""
    torch = _torch()
    arr = config_array(cfgs)
    sp = _dev_ptr(samples, "samples", (torch.int32, torch.uint32))
    op = _dev_ptr(offsets, "offsets", (torch.int64, torch.uint64))
    n_traces = offsets.numel() - 1
    dev = samples.device
    if results is None:
        results = torch.empty((n_traces, 4), dtype=torch.int64, device=dev)
    rp = _dev_ptr(results, "results", (torch.int64,))
    cp = None
    if cfg_of_trace is not None:
        cp = _dev_ptr(cfg_of_trace, "cfg_of_trace", (torch.int32, torch.uint32))
    lp = None
    if levels:
        if levels_out is None:
            levels_out = torch.zeros(samples.numel(), dtype=torch.uint8, device=dev)
        lp = _dev_ptr(levels_out, "levels", (torch.uint8,))
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=dev)
    stp = _dev_ptr(status, "status", (torch.int32,))
    with torch.cuda.device(dev):
        _check(load().magus_replay_noalloc(sp, samples.numel(), op, n_traces, arr, len(arr),
                                           cp, rp, lp, stp, _stream_handle(stream, dev)))
    return results, (levels_out if levels else None), status


class Context:
    """A libmagus context on one HIP device (owns scratch memory)."""

    def __init__(self, device: int = 0):
        lib = load()
        self.device = device
        h = ctypes.c_void_p()
        _check(lib.magus_ctx_create(device, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().magus_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def chunk(self) -> int:
        return int(load().magus_ctx_get_chunk(self._h))

    def set_chunk(self, steps: int) -> None:
        _check(load().magus_ctx_set_chunk(self._h, int(steps)))

    @property
    def persistent(self) -> int:
        return int(load().magus_ctx_get_persistent(self._h))

    def set_persistent(self, workgroups: int) -> None:
        _check(load().magus_ctx_set_persistent(self._h, int(workgroups)))

    def set_graphs(self, enable: bool) -> None:
        _check(load().magus_ctx_set_graphs(self._h, int(bool(enable))))

    def autotune_replay(self, samples, offsets, cfgs, cfg_of_trace=None, reps: int = 3,
                        results=None, stream=None) -> dict:
        """Time every chunk length / launch shape on this batch (results must agree),
        keep the fastest on the context and return what was chosen."""
        torch = _torch()
        arr = config_array(cfgs)
        n_traces = offsets.numel() - 1
        if results is None:
            results = torch.empty((n_traces, 4), dtype=torch.int64, device=samples.device)
        cp = None if cfg_of_trace is None else _dev_ptr(cfg_of_trace, "cfg_of_trace",
                                                        (torch.int32, torch.uint32))
        r = MagusTuneResult()
        _check(load().magus_autotune_replay(
            self._h, _dev_ptr(samples, "samples", (torch.int32, torch.uint32)), samples.numel(),
            _dev_ptr(offsets, "offsets", (torch.int64, torch.uint64)), n_traces, arr, len(arr),
            cp, _dev_ptr(results, "results", (torch.int64,)), int(reps),
            _stream_handle(stream, self.device), ctypes.byref(r)))
        return {f: getattr(r, f) for f, _ in MagusTuneResult._fields_ if f != "reserved"}

    @property
    def sweep_shape(self) -> int:
        return int(load().magus_ctx_get_sweep_shape(self._h))

    def set_sweep_shape(self, shape: int) -> None:
        _check(load().magus_ctx_set_sweep_shape(self._h, int(shape)))

    def autotune_sweep(self, samples, offsets, cfgs, reps: int = 2, stream=None) -> dict:
        """Time every sweep launch shape on this batch (the arg-min must agree),
        keep the fastest on the context and return what was chosen."""
        torch = _torch()
        arr = config_array(cfgs)
        n_traces = offsets.numel() - 1
        argmin = torch.empty(n_traces, dtype=torch.int32, device=samples.device)
        r = MagusSweepTuneResult()
        _check(load().magus_autotune_sweep(
            self._h, _dev_ptr(samples, "samples", (torch.int32, torch.uint32)), samples.numel(),
            _dev_ptr(offsets, "offsets", (torch.int64, torch.uint64)), n_traces, arr, len(arr),
            _dev_ptr(argmin, "argmin", (torch.int32,)), int(reps),
            _stream_handle(stream, self.device), ctypes.byref(r)))
        return {f: getattr(r, f) for f, _ in MagusSweepTuneResult._fields_}

    def set_profiling(self, enable: bool) -> None:
        _check(load().magus_ctx_set_profiling(self._h, int(bool(enable))))

    def kernel_time(self, kernel: int):
        """(total ms, launches) of the dominant kernel since the last query."""
        ms = ctypes.c_double()
        n = ctypes.c_uint64()
        _check(load().magus_ctx_kernel_time(self._h, int(kernel), ctypes.byref(ms),
                                            ctypes.byref(n)))
        return ms.value, n.value

    def valu_probe(self, workgroups: int, steps: int, mode: int = 1, out=None, stream=None):
        """The VALU issue-rate probe (see magus.h): `steps` rounds of 8
        independent instruction chains per lane in `workgroups` workgroups of
        256 lanes.  Returns (out, lane-ops issued by the launch)."""
        torch = _torch()
        if out is None:
            out = torch.empty(workgroups * 256, dtype=torch.int32, device=f"cuda:{self.device}")
        ops = ctypes.c_uint64()
        _check(load().magus_valu_probe(self._h, int(workgroups), int(steps), int(mode),
                                       _dev_ptr(out, "out", (torch.int32,)), ctypes.byref(ops),
                                       _stream_handle(stream, self.device)))
        return out, ops.value

    def read_probe(self, samples, chunk: int = 4096, out=None, stream=None):
        """The streaming-read probe (see magus.h) over `samples` (int32/uint32,
        device): one wave per chunk of `chunk` samples.  Returns out (one word
        per chunk)."""
        torch = _torch()
        sp = _dev_ptr(samples, "samples", (torch.int32, torch.uint32))
        n = samples.numel()
        n_chunks = (n + chunk - 1) // chunk if chunk > 0 else 0
        if out is None:
            out = torch.empty(max(n_chunks, 1), dtype=torch.int32,
                              device=f"cuda:{self.device}")
        if out.numel() < n_chunks:
            raise ValueError(f"out holds {out.numel()} words, the probe writes {n_chunks}")
        _check(load().magus_read_probe(self._h, sp, n, int(chunk),
                                       _dev_ptr(out, "out", (torch.int32,)),
                                       _stream_handle(stream, self.device)))
        return out

    def check(self, stream=None) -> None:
        """Synchronize and raise MagusError(EDATA) on a device-side data fault."""
        _check(load().magus_ctx_check(self._h, _stream_handle(stream, self.device)))

    def replay(self, samples, offsets, cfgs, cfg_of_trace=None, levels: bool = False,
               results=None, levels_out=None, stream=None):
        """Replay every trace; returns (results int64[n_traces, 4], levels uint8 or None).

        results columns: score, level_sum, transitions, ticks_high.
        """
        torch = _torch()
        arr = config_array(cfgs)
        sp = _dev_ptr(samples, "samples", (torch.int32, torch.uint32))
        op = _dev_ptr(offsets, "offsets", (torch.int64, torch.uint64))
        n_traces = offsets.numel() - 1
        if results is None:
            results = torch.empty((n_traces, 4), dtype=torch.int64, device=samples.device)
        rp = _dev_ptr(results, "results", (torch.int64,))
        cp = None
        if cfg_of_trace is not None:
            cp = _dev_ptr(cfg_of_trace, "cfg_of_trace", (torch.int32, torch.uint32))
        lp = None
        if levels:
            if levels_out is None:
                levels_out = torch.zeros(samples.numel(), dtype=torch.uint8, device=samples.device)
            lp = _dev_ptr(levels_out, "levels", (torch.uint8,))
        _check(load().magus_replay(self._h, sp, samples.numel(), op, n_traces, arr, len(arr),
                                   cp, rp, lp, _stream_handle(stream, self.device)))
        return results, (levels_out if levels else None)

    def proxy(self, samples, offsets, cfgs, model, cfg_of_trace=None, metrics: bool = True,
              stream=None, stats=None):
        """Proxy energy / EDP model of MAGUS vs always-max vs always-min per trace.

        Returns (stats int64[T, 66], metrics float64[T, 21] or None); decode rows
        with proxy_stats_dict / proxy_metrics_dict.  `stats` optionally gives
        the output tensor for the statistics.
        """
        torch = _torch()
        arr = config_array(cfgs)
        mm = model if isinstance(model, MagusProxyModel) else make_proxy_model(model)
        sp = _dev_ptr(samples, "samples", (torch.int32, torch.uint32))
        op = _dev_ptr(offsets, "offsets", (torch.int64, torch.uint64))
        n_traces = offsets.numel() - 1
        st = stats if stats is not None else \
            torch.empty((n_traces, 2 + 2 * PROXY_LEVELS), dtype=torch.int64,
                        device=samples.device)
        if tuple(st.shape) != (n_traces, 2 + 2 * PROXY_LEVELS) or not st.is_contiguous():
            raise ValueError("stats must be a contiguous int64 tensor [n_traces, 66]")
        me = None
        mp = None
        if metrics:
            me = torch.empty((n_traces, 21), dtype=torch.float64, device=samples.device)
            mp = _dev_ptr(me, "metrics", (torch.float64,))
        cp = None
        if cfg_of_trace is not None:
            cp = _dev_ptr(cfg_of_trace, "cfg_of_trace", (torch.int32, torch.uint32))
        _check(load().magus_proxy(self._h, sp, samples.numel(), op, n_traces, arr, len(arr),
                                  cp, ctypes.byref(mm), _dev_ptr(st, "stats", (torch.int64,)),
                                  mp, _stream_handle(stream, self.device)))
        return st, me

    def counters_to_mbps(self, counts, ts_ns, offsets, counter_bits: int = 48,
                         bytes_per_count: int = 64, stream=None):
        """Monitor front end: counter readings (CSR, >= 1 per trace) to MB/s samples.

        Returns (samples int32 tensor viewed as uint32, sample offsets int64 tensor).
        """
        torch = _torch()
        n_traces = offsets.numel() - 1
        out = torch.zeros(max(counts.numel() - n_traces, 0), dtype=torch.int32,
                          device=counts.device)
        _check(load().magus_counters_to_mbps(
            self._h, _dev_ptr(counts, "counts", (torch.int64, torch.uint64)),
            _dev_ptr(ts_ns, "ts_ns", (torch.int64, torch.uint64)), counts.numel(),
            _dev_ptr(offsets, "offsets", (torch.int64, torch.uint64)), n_traces,
            int(counter_bits), int(bytes_per_count), _dev_ptr(out, "samples", (torch.int32,)),
            _stream_handle(stream, self.device)))
        sample_offsets = offsets - torch.arange(n_traces + 1, device=offsets.device,
                                                dtype=offsets.dtype)
        return out, sample_offsets

    def sweep(self, samples, offsets, cfgs, scores: bool = False, stream=None):
        """Every trace against every config; returns (scores int64[T, C] or None, argmin int32[T])."""
        torch = _torch()
        arr = config_array(cfgs)
        sp = _dev_ptr(samples, "samples", (torch.int32, torch.uint32))
        op = _dev_ptr(offsets, "offsets", (torch.int64, torch.uint64))
        n_traces = offsets.numel() - 1
        argmin = torch.empty(n_traces, dtype=torch.int32, device=samples.device)
        sc = None
        scp = None
        if scores:
            sc = torch.empty((n_traces, len(arr)), dtype=torch.int64, device=samples.device)
            scp = _dev_ptr(sc, "scores", (torch.int64,))
        _check(load().magus_sweep(self._h, sp, samples.numel(), op, n_traces, arr, len(arr),
                                  scp, _dev_ptr(argmin, "argmin", (torch.int32,)),
                                  _stream_handle(stream, self.device)))
        return sc, argmin


class Server:
    """Serving slot pool: controller state of every live stream stays on the GPU."""

    def __init__(self, ctx: Context, mem_budget_bytes: int):
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(load().magus_server_create(ctx._h, int(mem_budget_bytes), ctypes.byref(h)))
        self._h = h

    @staticmethod
    def slot_bytes() -> int:
        return int(load().magus_server_slot_bytes())

    @property
    def capacity(self) -> int:
        return int(load().magus_server_capacity(self._h))

    @property
    def open_count(self) -> int:
        return int(load().magus_server_open_count(self._h))

    def close(self):
        if getattr(self, "_h", None):
            load().magus_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def open(self, cfg: dict) -> int:
        c = make_config(cfg)
        slot = ctypes.c_uint32()
        _check(load().magus_stream_open(self._h, ctypes.byref(c), ctypes.byref(slot)))
        return slot.value

    def try_open(self, cfg: dict):
        """Like open() but returns None when admission is refused (no free slot)."""
        try:
            return self.open(cfg)
        except MagusError as e:
            if e.code == ENOSLOT:
                return None
            raise

    def close_stream(self, slot: int) -> None:
        _check(load().magus_stream_close(self._h, int(slot)))

    def step(self, slots, samples, decisions=None, stream=None, sync: bool = True):
        """One step for the given (slot, sample) pairs; returns uint8 decisions."""
        slots = np.ascontiguousarray(slots, dtype=np.uint32)
        samples = np.ascontiguousarray(samples, dtype=np.uint32)
        if slots.shape != samples.shape:
            raise ValueError("slots and samples differ in length")
        if decisions is None:
            decisions = np.empty(len(slots), dtype=np.uint8)
        sh = _stream_handle(stream, self.ctx.device)
        _check(load().magus_serve_step(self._h, slots.ctypes.data_as(_P),
                                       samples.ctypes.data_as(_P), len(slots),
                                       decisions.ctypes.data_as(_P), sh))
        if sync:
            _torch().cuda.current_stream(self.ctx.device).synchronize() if stream is None \
                else stream.synchronize()
        return decisions

    def run(self, events, n_streams: int, cfgs, realtime: bool = True, max_batch: int = 0,
            depth: int = 2):
        """Serve a time-sorted fleet event list with continuous batching.

        Returns (decisions uint8[n_events], latency_ns uint64[n_events], stats dict);
        decisions are 0xFF and latencies 2^64-1 for non-sample events and for
        samples of nodes that were not admitted.
        """
        ev = np.ascontiguousarray(events, dtype=EVENT_DTYPE)
        arr = config_array(cfgs)
        dec = np.empty(len(ev), np.uint8)
        lat = np.empty(len(ev), np.uint64)
        st = MagusRunStats()
        _check(load().magus_server_run(self._h, ev.ctypes.data_as(_P), len(ev), int(n_streams),
                                       arr, len(arr), int(bool(realtime)), int(max_batch),
                                       int(depth), dec.ctypes.data_as(_P),
                                       lat.ctypes.data_as(_P), ctypes.byref(st)))
        stats = {f: getattr(st, f) for f, _ in MagusRunStats._fields_}
        return dec, lat, stats

    def result(self, slot: int) -> dict:
        r = MagusResult()
        _check(load().magus_stream_result(self._h, int(slot), ctypes.byref(r)))
        return {"score": r.score, "level_sum": r.level_sum,
                "transitions": r.transitions, "ticks_high": r.ticks_high}
