"""GPU parity of magus_sweep: scores and arg-min against the oracle, and the
sweep against the plain replay of each config on the same GPU."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import paper_2502_03796_amd as magus
import synth
from synth import default_config
from tests.gpu_util import to_dev, results_np, describe_mismatch
from tests.test_gpu_replay import mixed_traces

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = magus.Context(0)
    yield c
    c.close()


def sweep_both(ctx, oracle_mod, traces, cfgs):
    samples, offsets = synth.make_batch(traces)
    want_scores, want_arg = oracle_mod.sweep(samples, offsets, cfgs)
    s, o, _ = to_dev(samples, offsets)
    sc, arg = ctx.sweep(s, o, cfgs, scores=True)
    ctx.check()
    got = sc.cpu().numpy().view(np.uint64)
    assert (got == want_scores).all(), describe_mismatch(got.ravel(), want_scores.ravel())
    assert (arg.cpu().numpy().astype(np.uint32) == want_arg).all()
    return got


def test_grid_sample_on_mixed_traces(ctx, oracle_mod):
    grid = synth.sweep_grid()
    idx = list(range(0, 16384, 37)) + [0, 1, 4095, 4096, 8191, 16383]
    cfgs = [grid[i] for i in idx]
    traces = mixed_traces(101, [0, 1, 5, 64, 255, 256, 257, 1000, 3000, 5000])
    sweep_both(ctx, oracle_mod, traces, cfgs)


def test_unsorted_windows_and_padding(ctx, oracle_mod):
    """Configs in arbitrary window order, blocks that need padding lanes, and
    every kind of initial level."""
    rng = np.random.default_rng(4)
    cfgs = []
    for i in range(700):
        lmin = int(rng.integers(0, 10))
        lmax = int(rng.integers(lmin + 1, 32))
        den = int(rng.integers(1, 8))
        cfgs.append(default_config(window=int(rng.integers(2, 33)), hold=int(rng.integers(1, 33)),
                                   inc_q16=int(rng.integers(0, 70000)),
                                   dec_q16=-int(rng.integers(0, 70000)),
                                   hf_num=int(rng.integers(0, den + 1)), hf_den=den,
                                   level_min=lmin, level_max=lmax,
                                   level_init=int(rng.choice([lmin, lmax,
                                                              int(rng.integers(lmin, lmax + 1))]))))
    traces = mixed_traces(202, [700, 2000, 1, 0, 333])
    sweep_both(ctx, oracle_mod, traces, cfgs)


@pytest.mark.parametrize("shape", range(magus.SWEEP_SHAPES))
def test_every_launch_shape_matches_the_oracle(ctx, oracle_mod, shape):
    """Each launch shape (configs per workgroup, steps per tile): traces of
    lengths around the tile sizes (255..1025, and 2 tiles + 1), a grid
    sample, stepped and base-variant configs, and blocks with padding parts
    (700 configs: the last block of each window holds fewer than 256)."""
    grid = synth.sweep_grid()
    rng = np.random.default_rng(50 + shape)
    cfgs = [grid[int(i)] for i in rng.integers(0, len(grid), 640)]
    cfgs += [dict(default_config(up_step=2, down_step=1)), dict(default_config(base=1)),
             dict(default_config(base=3, base_ref=20000)), default_config(level_init=7)]
    cfgs += [grid[int(i)] for i in rng.integers(0, len(grid), 56)]
    traces = mixed_traces(404 + shape, [0, 1, 63, 255, 256, 257, 511, 512, 513, 1023, 1024,
                                        1025, 2049, 4000])
    ctx.set_sweep_shape(shape)
    try:
        assert ctx.sweep_shape == shape
        sweep_both(ctx, oracle_mod, traces, cfgs)
    finally:
        ctx.set_sweep_shape(0)


def test_sweep_autotune_keeps_results(ctx, oracle_mod):
    """The autotuner times every shape, requires identical arg-min keys, and
    keeps the fastest; the sweep with the chosen shape matches the oracle."""
    grid = synth.sweep_grid()
    cfgs = [grid[i] for i in range(0, 16384, 5)]
    traces = mixed_traces(505, [3000] * 8 + [777, 1])
    samples, offsets = synth.make_batch(traces)
    s, o, _ = to_dev(samples, offsets)
    r = ctx.autotune_sweep(s, o, cfgs, reps=1)
    try:
        assert r["candidates"] == magus.SWEEP_SHAPES
        assert ctx.sweep_shape == r["shape"]
        assert (r["lanes"], r["tile"]) == magus.sweep_shape_info(r["shape"])
        assert r["best_ms"] <= r["default_ms"]
        sweep_both(ctx, oracle_mod, traces, cfgs)
    finally:
        ctx.set_sweep_shape(0)


def test_ties_take_the_lowest_index(ctx, oracle_mod):
    """A constant trace scores 0 under every config: arg-min is config 0; with a
    duplicated best config the lower index wins."""
    traces = [np.full(500, 1234, np.uint32), np.array([10000, 20000] * 200, np.uint32)]
    cfgs = [synth.sweep_config(i) for i in (5000, 77, 77, 16000, 9)]
    got = sweep_both(ctx, oracle_mod, traces, cfgs)
    assert (got[0] == 0).all()


def test_sweep_equals_replay_on_the_gpu(ctx, oracle_mod):
    """Cross-form parity: scores of the sweep == scores of the plain replay of
    each config on the same traces."""
    import torch
    traces = mixed_traces(303, [4000] * 16)
    samples, offsets = synth.make_batch(traces)
    s, o, _ = to_dev(samples, offsets)
    cfgs = [synth.sweep_config(i) for i in range(0, 16384, 211)]
    sc, _ = ctx.sweep(s, o, cfgs, scores=True)
    for j, c in enumerate(cfgs):
        res, _ = ctx.replay(s, o, [c])
        assert (res[:, 0] == sc[:, j]).all(), j
    ctx.check()


def test_sweep_workload_full_size(ctx, oracle_mod):
    """The benchmark's sweep launch: 1,024 traces x 50,000 samples against all
    16,384 grid configs (four window blocks) in ONE call, checked against the
    oracle three ways:
      - every config on 16 traces, and those traces' 16,384-wide arg-min
        against the oracle's arg-min over the same configs;
      - a stratified 1/16 of the configs (every 16th, so 256 in each window
        block) on every trace;
      - every trace's arg-min is the lowest index among the minimal scores
        of the GPU score matrix (internal consistency of the arg-min
        reduction with the scores, which the two checks above pin).
    The oracle runs in host threads (its ctypes calls release the
    interpreter lock)."""
    samples, offsets = synth.workload_sweep_traces()
    grid = synth.sweep_grid()
    n_cfg = len(grid)
    assert n_cfg == 16384
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    s, o, _ = to_dev(samples, offsets)
    arr = magus.config_array(grid)
    sc, arg = ctx.sweep(s, o, arr, scores=True)
    ctx.check()
    sc = sc.cpu().numpy().view(np.uint64)
    arg = arg.cpu().numpy().astype(np.uint32)
    assert sc.shape == (1024, n_cfg)

    def part(traces):
        return synth.make_batch([samples[int(offsets[t]):int(offsets[t + 1])] for t in traces])

    rng = np.random.default_rng(2024)
    every = sorted(rng.choice(1024, 16, replace=False).tolist())
    cpick = np.arange(int(rng.integers(0, 16)), n_cfg, 16)
    assert all(((cpick >= 4096 * w) & (cpick < 4096 * (w + 1))).sum() == 256 for w in range(4))
    sub_cfgs = [grid[i] for i in cpick]

    # every config on 16 traces: one task per (trace, window block)
    def full_row_block(tw):
        t, w = tw
        b = part([t])
        return oracle_mod.sweep(b[0], b[1], grid[w * 4096:(w + 1) * 4096])[0][0]

    def stratified(t0):
        b = part(range(t0, t0 + 16))
        return oracle_mod.sweep(b[0], b[1], sub_cfgs)[0]

    with ThreadPoolExecutor(max_workers=threads) as pool:
        tasks = [(t, w) for t in every for w in range(4)]
        rows = {}
        for (t, w), r in zip(tasks, pool.map(full_row_block, tasks)):
            rows.setdefault(t, [None] * 4)[w] = r
        starts = list(range(0, 1024, 16))
        strat = list(pool.map(stratified, starts))
    for t in every:
        want = np.concatenate(rows[t])
        assert (sc[t] == want).all(), (t, describe_mismatch(sc[t], want))
        # the oracle's arg-min over all 16,384 configs: lowest index of the minimum
        assert arg[t] == int(np.argmin(want)), (t, int(arg[t]), int(np.argmin(want)))
    for t0, r in zip(starts, strat):
        assert (sc[t0:t0 + 16][:, cpick] == r).all(), (t0, describe_mismatch(
            sc[t0:t0 + 16][:, cpick].ravel(), r.ravel()))
    mins = sc.min(axis=1)
    assert (arg == np.argmax(sc == mins[:, None], axis=1)).all()
