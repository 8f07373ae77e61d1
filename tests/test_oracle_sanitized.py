"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
host code only) runs a mixed batch through every entry point without a
report, and gives exactly the outputs of the regular build."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth
from synth import default_config

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def build_sanitized(tmp):
    exe = os.path.join(tmp, "oracle_driver_san")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           os.path.join(ROOT, "oracle", "magus_oracle.c"),
           os.path.join(HERE, "sanitize", "oracle_driver.c"), "-o", exe, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip(f"sanitizer build unavailable: {r.stderr[:200]}")
    return exe


def batch(seed):
    rng = np.random.default_rng(seed)
    lengths = [0, 1, 2, 3, 31, 64, 65, 300, 2000, 0, 5000]
    traces = []
    for i, n in enumerate(lengths):
        kind = i % 3
        if kind == 0:
            traces.append(rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32))
        elif kind == 1:
            traces.append(synth.geometric_phase_trace(n, synth.stream_key(seed, i),
                                                      short_prob=0.3) if n else
                          np.zeros(0, np.uint32))
        else:
            traces.append(np.repeat(rng.integers(1, 200000, max(n // 10, 1)), 10)[:n]
                          .astype(np.uint32))
    samples, offsets = synth.make_batch(traces)
    cfgs = [default_config(), default_config(window=2, hold=1),
            default_config(window=32, hold=32, hf_num=0, hf_den=1),
            default_config(up_step=3, down_step=1, level_init=5),
            default_config(base=1, window=5), default_config(base=2, up_step=1),
            default_config(level_min=2, level_max=31, level_init=31, inc_q16=0, dec_q16=0)]
    cot = (np.arange(len(traces)) % len(cfgs)).astype(np.uint32)
    model = dict(n_levels=32, interval_us=100000,
                 cap_mbps=[int(v) for v in rng.integers(1, 2**32, 32, dtype=np.uint64)],
                 uncore_mw=[int(v) for v in rng.integers(0, 2**32, 32, dtype=np.uint64)],
                 core_mw=60000, gpu_mw=250000)
    n_r = 400
    counts = np.cumsum(rng.integers(0, 2**40, n_r, dtype=np.uint64)).astype(np.uint64)
    ts = np.cumsum(rng.integers(0, 2 * 10**8, n_r, dtype=np.uint64)).astype(np.uint64)
    return samples, offsets, cfgs, cot, model, counts, ts


def test_sanitized_oracle_matches_regular_build(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = build_sanitized(str(tmp_path))
    samples, offsets, cfgs, cot, model, counts, ts = batch(77)
    n_t, n_c = len(offsets) - 1, len(cfgs)
    carr = oracle._cfg_array(cfgs)
    mm = oracle._model(model)
    inp = tmp_path / "in.bin"
    with open(inp, "wb") as f:
        f.write(np.array([len(samples)], np.uint64).tobytes())
        f.write(np.array([n_t, n_c], np.uint32).tobytes())
        f.write(np.array([len(counts)], np.uint64).tobytes())
        f.write(samples.astype(np.uint32).tobytes())
        f.write(offsets.astype(np.uint64).tobytes())
        f.write(bytes(carr))
        f.write(cot.tobytes())
        f.write(bytes(mm))
        f.write(counts.tobytes())
        f.write(ts.tobytes())
        f.write(np.array([40, 64], np.uint32).tobytes())
    out = tmp_path / "out.bin"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(inp), str(out)], capture_output=True, text=True, env=env,
                       timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    raw = out.read_bytes()
    pos = 0

    def take(dtype, n):
        nonlocal pos
        a = np.frombuffer(raw, dtype=dtype, count=n, offset=pos)
        pos += a.nbytes
        return a
    res = take(np.uint64, 4 * n_t).reshape(n_t, 4)
    dec = take(np.uint8, len(samples))
    scores = take(np.uint64, n_t * n_c).reshape(n_t, n_c)
    argmin = take(np.uint32, n_t)
    st = take(np.uint64, 66 * n_t).reshape(n_t, 66)
    me = take(np.float64, 21 * n_t).reshape(n_t, 21)
    mbps = take(np.uint32, len(counts) - 1)
    assert pos == len(raw)

    want_res, want_dec = oracle.replay_batch(samples, offsets, cfgs, cot, want_bytes=True)
    assert (res == want_res).all() and (dec == want_dec).all()
    want_sc, want_arg = oracle.sweep(samples, offsets, cfgs)
    assert (scores == want_sc).all() and (argmin == want_arg).all()
    for t in range(n_t):
        x = samples[int(offsets[t]):int(offsets[t + 1])]
        ws, wm = oracle.proxy_trace(x, cfgs[int(cot[t])], model)
        assert list(st[t]) == [ws["excess_max"], ws["excess_min"]] + ws["steps"] + ws["excess"]
        got_m = me[t].reshape(7, 3)
        for i, k in enumerate(oracle._METRIC_KEYS):
            assert list(got_m[i]) == wm[k], (t, k)
    assert (mbps == oracle.counters_to_mbps(counts, ts, 40, 64)).all()
