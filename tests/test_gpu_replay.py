"""GPU parity of magus_replay against the oracle: bit-exact per-step decision
bytes and per-trace results, through the C ABI."""
import ctypes
import itertools

import numpy as np
import pytest

import paper_2502_03796_amd as magus
import synth
from synth import default_config
from tests.gpu_util import to_dev, results_np, describe_mismatch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = magus.Context(0)
    yield c
    c.close()


def run_both(ctx, oracle_mod, traces, cfgs, cot=None, chunk=None, levels=True):
    samples, offsets = synth.make_batch(traces)
    want_res, want_b = oracle_mod.replay_batch(samples, offsets, cfgs, cot, want_bytes=levels)
    s, o, c = to_dev(samples, offsets, cot)
    if chunk is not None:
        ctx.set_chunk(chunk)
    try:
        res, lv = ctx.replay(s, o, cfgs, c, levels=levels)
        ctx.check()
    finally:
        ctx.set_chunk(0)
    got_res = results_np(res)
    assert (got_res == want_res).all(), describe_mismatch(got_res[:, 0], want_res[:, 0])
    if levels:
        got_b = lv.cpu().numpy()
        assert (got_b == want_b).all(), describe_mismatch(got_b, want_b, offsets)
    return got_res


def pin_traces():
    return [
        [777] * 300, [0] * 70, [2**32 - 1] * 65,
        [10000] * 40 + [20000] * 60,
        [65536] * 4 + [91752] * 4, [65536] * 4 + [91753] * 4,
        [40000] * 40 + [10000] * 60,
        [10000, 20000] * 50,
        [10000, 20000] * 10 + [20000] * 30,
        [30000] * 20 + [10000] * 20 + [40000] * 20 + [9000] * 20,
        [1, 2], [5], [],
    ]


@pytest.mark.parametrize("cfg", [default_config(), default_config(window=16),
                                 default_config(window=2), default_config(hold=1),
                                 default_config(hf_num=0), default_config(level_init=7),
                                 default_config(level_min=3, level_max=31, level_init=31)])
def test_pin_traces(ctx, oracle_mod, cfg):
    traces = [np.array(t, np.uint32) for t in pin_traces()]
    run_both(ctx, oracle_mod, traces, [cfg])


def test_brute_force_tiny_traces(ctx, oracle_mod):
    """Every trace over {0..4} of length <= 7 (97,656 traces, one batch), for
    W in {2,3,4}, H in {1,2,3,5} and 25 threshold pairs with exact-equality
    cases: results and every decision byte against the oracle."""
    traces = [np.array(t, np.uint32) for n in range(0, 8)
              for t in itertools.product(range(5), repeat=n)]
    samples, offsets = synth.make_batch(traces)
    s, o, _ = to_dev(samples, offsets)
    for W, H, inc, dec in itertools.product((2, 3, 4), (1, 2, 3, 5),
                                            (0, 1, 16384, 32768, 65536),
                                            (0, -1, -16384, -32768, -65536)):
        cfg = default_config(window=W, hold=H, inc_q16=inc, dec_q16=dec)
        want_res, want_b = oracle_mod.replay_batch(samples, offsets, [cfg], want_bytes=True)
        res, lv = ctx.replay(s, o, [cfg], levels=True)
        ctx.check()
        got_res = results_np(res)
        assert (got_res == want_res).all(), (cfg, describe_mismatch(got_res[:, 0],
                                                                    want_res[:, 0]))
        got_b = lv.cpu().numpy()
        assert (got_b == want_b).all(), (cfg, describe_mismatch(got_b, want_b, offsets))


def test_brute_force_tiny_traces_other_bases(ctx, oracle_mod):
    """The same tiny traces under the oldest, newest and fixed-reference
    derivative bases (B_ref 1 and 2: r = 1/4 at W = 4 is an equality case)."""
    traces = [np.array(t, np.uint32) for n in range(0, 8)
              for t in itertools.product(range(5), repeat=n)]
    samples, offsets = synth.make_batch(traces)
    s, o, _ = to_dev(samples, offsets)
    for (base, bref), W, H, (inc, dec) in itertools.product(
            ((1, 0), (2, 0), (3, 1), (3, 2)), (2, 4), (1, 3),
            ((0, 0), (16384, -16384), (32768, -1))):
        cfg = default_config(window=W, hold=H, inc_q16=inc, dec_q16=dec, base=base,
                             base_ref=bref)
        want_res, want_b = oracle_mod.replay_batch(samples, offsets, [cfg], want_bytes=True)
        res, lv = ctx.replay(s, o, [cfg], levels=True)
        ctx.check()
        assert (results_np(res) == want_res).all(), cfg
        got_b = lv.cpu().numpy()
        assert (got_b == want_b).all(), (cfg, describe_mismatch(got_b, want_b, offsets))


def mixed_traces(seed, lengths):
    out = []
    for i, n in enumerate(lengths):
        key = synth.stream_key(seed, i)
        kind = i % 3
        if kind == 0:
            out.append(synth.four_phase_trace(n, key))
        elif kind == 1:
            out.append(synth.geometric_phase_trace(n, key, mean=30.0, short_prob=0.3))
        else:
            out.append(synth.geometric_phase_trace(n, key, mean=200.0, short_prob=0.1))
    return out


LENGTHS = [0, 1, 2, 31, 32, 63, 64, 65, 127, 128, 129, 4095, 4096, 4097, 8191, 8192, 8193,
           16383, 16384, 16385, 20000, 33333, 70001]


@pytest.mark.parametrize("chunk", [64, 128, 192, 4096, 4160, 16384, 65536])
def test_chunking_never_changes_results(ctx, oracle_mod, chunk):
    """Chunk boundaries at every offset class, incl. chunks of one block."""
    traces = mixed_traces(31 + chunk, LENGTHS)
    grid = synth.sweep_grid()
    rng = np.random.default_rng(chunk)
    cfgs = [grid[int(i)] for i in rng.integers(0, len(grid), 40)] + [default_config()]
    cot = rng.integers(0, len(cfgs), len(traces)).astype(np.uint32)
    run_both(ctx, oracle_mod, traces, cfgs, cot, chunk=chunk)


def test_random_configs_all_windows_and_holds(ctx, oracle_mod):
    rng = np.random.default_rng(7)
    cfgs = []
    for W in range(2, 33):
        for H in (1, 2, 7, 16, 31, 32):
            lmin = int(rng.integers(0, 20))
            lmax = int(rng.integers(lmin + 1, 32))
            den = int(rng.integers(1, 10))
            cfgs.append(default_config(window=W, hold=H,
                                       inc_q16=int(rng.integers(0, 2**20 + 1)) >> int(rng.integers(0, 12)),
                                       dec_q16=-(int(rng.integers(0, 2**20 + 1)) >> int(rng.integers(0, 12))),
                                       hf_num=int(rng.integers(0, den + 1)), hf_den=den,
                                       level_min=lmin, level_max=lmax,
                                       level_init=int(rng.integers(lmin, lmax + 1))))
    traces = mixed_traces(77, [int(v) for v in rng.integers(0, 3000, len(cfgs))])
    cot = np.arange(len(traces), dtype=np.uint32)
    for chunk in (64, 1024):
        run_both(ctx, oracle_mod, traces, cfgs, cot, chunk=chunk)


def test_extreme_sample_values(ctx, oracle_mod):
    rng = np.random.default_rng(3)
    traces = []
    for i in range(40):
        x = rng.integers(0, 2**32, size=int(rng.integers(1, 600)), dtype=np.uint64)
        x[rng.random(len(x)) < 0.1] = 0
        x[rng.random(len(x)) < 0.1] = 2**32 - 1
        traces.append(x.astype(np.uint32))
    for W, q in ((2, 2**20), (32, 2**20), (7, 1), (3, 12345), (16, 0)):
        run_both(ctx, oracle_mod, traces, [default_config(window=W, hold=3, inc_q16=q,
                                                          dec_q16=-q)], chunk=128)
    # every derivative base at the extremes of the products (the fixed
    # reference up to 2^32-1 against thresholds up to 2^20 at W = 32)
    for base, bref in ((1, 0), (2, 0), (3, 1), (3, 2**32 - 1), (3, 77777)):
        for W, q in ((2, 2**20), (32, 2**20), (7, 1), (16, 0)):
            run_both(ctx, oracle_mod, traces,
                     [default_config(window=W, hold=3, inc_q16=q, dec_q16=-q, base=base,
                                     base_ref=bref)], chunk=128)


@pytest.mark.parametrize("chunk", [128, 4096])
def test_threshold_boundaries_at_large_samples(ctx, oracle_mod, chunk):
    """Alg. 1 exactly on and next to the rise and fall thresholds with
    samples just below 2^24 (where a float product of either side would be
    off by far more than one), a chunk holding one sample of 2^24 between
    chunks without, and threshold factors 2^16 + W q of 2^24 and just above.
    Results and every decision byte against the oracle."""
    from tests.test_gpu_proxy import _alg1_boundary_trace
    lim = 1 << 24
    cfg_a = default_config(window=2, hold=4)
    ku = 65536 + 2 * cfg_a["inc_q16"]
    kd = 65536 - 2 * cfg_a["dec_q16"]
    one_big = np.full(3 * chunk + 77, lim - 2, np.uint32)
    one_big[::5] = 9000
    one_big[chunk + chunk // 2] = lim
    traces = [_alg1_boundary_trace(chunk, ku, kd), _alg1_boundary_trace(chunk + 1, ku, kd, 400),
              one_big, np.array([lim - 1, 0, lim - 1, lim // 2] * (chunk // 4 + 33), np.uint32)]
    run_both(ctx, oracle_mod, traces, [cfg_a], chunk=chunk)
    for q in ((lim - 65536) // 16, (lim - 65536) // 16 + 1):
        cfg = default_config(window=16, hold=3, inc_q16=q, dec_q16=-q)
        run_both(ctx, oracle_mod, traces, [cfg], chunk=chunk)


def test_small_workload(ctx, oracle_mod):
    """One four-phase trace of 10,000 samples, default config: every step."""
    samples, offsets = synth.workload_small()
    run_both(ctx, oracle_mod, [samples], [default_config()])


def test_run_twice_is_bitwise_identical(ctx):
    samples, offsets = synth.make_batch(mixed_traces(5, [50000] * 64))
    s, o, _ = to_dev(samples, offsets)
    r1, l1 = ctx.replay(s, o, [default_config()], levels=True)
    r2, l2 = ctx.replay(s, o, [default_config()], levels=True)
    r3, _ = ctx.replay(s, o, [default_config()])
    assert (r1 == r2).all() and (l1 == l2).all() and (r1 == r3).all()


def test_offsets_not_starting_at_zero(ctx, oracle_mod):
    """Traces are views into a larger sample array; samples before the first
    and after the last trace are never read or written."""
    traces = mixed_traces(9, [500, 700, 64, 1000])
    offs = np.array([10, 510, 1210, 1274, 2274], np.uint64)
    big = np.full(2400, 123456789, np.uint32)
    for t, x in enumerate(traces):
        big[int(offs[t]):int(offs[t + 1])] = x
    s, o, _ = to_dev(big, offs)
    res, lv = ctx.replay(s, o, [default_config()], levels=True)
    ctx.check()
    got = lv.cpu().numpy()
    for t, x in enumerate(traces):
        r, b = oracle_mod.replay_trace(x, default_config())
        assert (got[int(offs[t]):int(offs[t + 1])] == b).all()
        assert results_np(res)[t][0] == r["score"]
    assert (got[:10] == 0).all() and (got[2274:] == 0).all()


def test_device_data_faults_are_reported_not_run(ctx):
    import torch
    samples, offsets = synth.make_batch(mixed_traces(1, [100, 100]))
    s, o, _ = to_dev(samples, offsets)
    bad = torch.tensor([0, 150, 100], dtype=torch.int64, device="cuda")   # not monotone
    ctx.replay(s, bad, [default_config()])
    with pytest.raises(magus.MagusError) as ei:
        ctx.check()
    assert ei.value.code == magus.EDATA
    beyond = torch.tensor([0, 100, 201], dtype=torch.int64, device="cuda")
    ctx.replay(s, beyond, [default_config()])
    with pytest.raises(magus.MagusError):
        ctx.check()
    cot = torch.tensor([0, 5], dtype=torch.int32, device="cuda")      # index out of range
    ctx.replay(s, o, [default_config()], cfg_of_trace=cot)
    with pytest.raises(magus.MagusError):
        ctx.check()
    # a trace one sample longer than the maximum, over a real allocation of
    # its whole span (4 GiB), so that the device-side gate is the only thing
    # that keeps the kernels from running it, and a run would stay in bounds
    lib = magus.load()
    n_big = (1 << 30) + 1
    big = torch.zeros(n_big, dtype=torch.int32, device="cuda")
    huge = torch.tensor([0, 1 << 30], dtype=torch.int64, device="cuda")
    res = torch.full((1, 4), 7, dtype=torch.int64, device="cuda")
    arr = magus.config_array([default_config()])
    rc = lib.magus_replay(ctx._h, ctypes.c_void_p(big.data_ptr()), n_big,
                          ctypes.c_void_p(huge.data_ptr()), 1, arr, 1, None,
                          ctypes.c_void_p(res.data_ptr()), None,
                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    with pytest.raises(magus.MagusError):
        ctx.check()
    assert (res.cpu().numpy() == 7).all()      # not run: the results are untouched
    del big
    torch.cuda.empty_cache()
    ctx.check()                      # cleared
    r, _ = ctx.replay(s, o, [default_config()])
    ctx.check()


def test_a_data_fault_stays_with_its_call(ctx, oracle_mod):
    """A faulty batch (offsets that go backwards in the middle) writes no
    result; the next good replay on the context, before the check, is run
    and correct (the plan's status is per call); the check still reports the
    earlier fault; after it, good batches (with and without decision bytes,
    one wave per chunk and the persistent grid) match the oracle."""
    import torch
    traces = mixed_traces(41, [9000, 5000, 12000, 300, 20000, 7000])
    samples, offsets = synth.make_batch(traces)
    want, want_b = oracle_mod.replay_batch(samples, offsets, [default_config()],
                                           want_bytes=True)
    s, o, _ = to_dev(samples, offsets)
    bad_off = offsets.copy()
    bad_off[3] = offsets[1]                         # trace 2 runs backwards
    bo = torch.from_numpy(bad_off.view(np.int64)).cuda()
    sentinel = torch.full((len(traces), 4), 7, dtype=torch.int64, device="cuda")
    ctx.replay(s, bo, [default_config()], levels=True, results=sentinel)
    torch.cuda.synchronize()
    assert (sentinel.cpu().numpy() == 7).all()      # no result written
    res, _ = ctx.replay(s, o, [default_config()])
    torch.cuda.synchronize()
    assert (results_np(res) == want).all()
    with pytest.raises(magus.MagusError) as ei:
        ctx.check()
    assert ei.value.code == magus.EDATA
    for persistent in (0, 3):
        ctx.set_persistent(persistent)
        try:
            for levels in (False, True):
                res, lv = ctx.replay(s, o, [default_config()], levels=levels)
                ctx.check()
                assert (results_np(res) == want).all(), (persistent, levels)
                if levels:
                    got = lv.cpu().numpy()
                    assert (got == want_b).all(), describe_mismatch(got, want_b, offsets)
        finally:
            ctx.set_persistent(0)


@pytest.fixture(scope="module")
def bulk():
    return synth.workload_bulk()


def test_bulk_workload_full_size(ctx, oracle_mod, bulk):
    """4,096 x 100,000 samples, single default config, the benchmark's launch:
    every trace's results and every step's decision byte against the oracle."""
    samples, offsets = bulk
    s, o, _ = to_dev(samples, offsets)
    res, _ = ctx.replay(s, o, [default_config()])
    ctx.check()
    got = results_np(res)
    want_res, want = oracle_mod.replay_batch(samples, offsets, [default_config()],
                                             want_bytes=True)
    assert (got == want_res).all(), describe_mismatch(got[:, 0], want_res[:, 0])
    _, lv = ctx.replay(s, o, [default_config()], levels=True)
    ctx.check()
    b = lv.cpu().numpy()
    assert (b == want).all(), describe_mismatch(b, want, offsets)


def test_persistent_grid_and_graph_replays_match(ctx, oracle_mod):
    """The persistent launch shape and hipGraph relaunches give the eager
    results; every graph replay is checked, with eager work in between."""
    import torch
    traces = mixed_traces(404, LENGTHS * 3)
    grid = synth.sweep_grid()
    rng = np.random.default_rng(404)
    cfgs = [grid[int(i)] for i in rng.integers(0, len(grid), 30)]
    cot = rng.integers(0, len(cfgs), len(traces)).astype(np.uint32)
    samples, offsets = synth.make_batch(traces)
    want_res, want_b = oracle_mod.replay_batch(samples, offsets, cfgs, cot, want_bytes=True)
    s, o, c = to_dev(samples, offsets, cot)
    try:
        for pers in (0, 7, 512):
            ctx.set_persistent(pers)
            res, lv = ctx.replay(s, o, cfgs, c, levels=True)
            ctx.check()
            assert (results_np(res) == want_res).all() and (lv.cpu().numpy() == want_b).all()
        ctx.set_graphs(True)
        res = torch.zeros((len(traces), 4), dtype=torch.int64, device="cuda")
        lv = torch.zeros(len(samples), dtype=torch.uint8, device="cuda")
        for rep in range(4):
            res.zero_()
            lv.zero_()
            ctx.replay(s, o, cfgs, c, levels=True, results=res, levels_out=lv)
            ctx.check()
            assert (results_np(res) == want_res).all(), rep
            assert (lv.cpu().numpy() == want_b).all(), rep
            # eager work of the program between replays
            ctx.set_graphs(False)
            r2, _ = ctx.replay(s, o, [default_config()])
            ctx.set_graphs(True)
            torch.cuda.synchronize()
    finally:
        ctx.set_graphs(False)
        ctx.set_persistent(0)


@pytest.mark.parametrize("n_traces", [33000, 70000])
def test_many_short_traces(ctx, oracle_mod, n_traces):
    """More traces than the plan keeps in registers (32 per plan thread), with
    empty and one-block traces among them, every result and decision byte."""
    rng = np.random.default_rng(n_traces)
    lens = rng.integers(0, 90, n_traces)
    lens[rng.integers(0, n_traces, 50)] = rng.integers(4000, 9000, 50)
    flat = rng.integers(1000, 60000, int(lens.sum())).astype(np.uint32)
    bounds = np.concatenate([[0], np.cumsum(lens)])
    traces = [flat[bounds[i]:bounds[i + 1]] for i in range(n_traces)]
    grid = synth.sweep_grid()
    cfgs = [grid[int(i)] for i in rng.integers(0, len(grid), 64)]
    cot = rng.integers(0, len(cfgs), n_traces).astype(np.uint32)
    run_both(ctx, oracle_mod, traces, cfgs, cot)


def test_kernel_timing_inside_graphs(ctx, oracle_mod):
    """With timing on, each graph launch times its own chunk kernel: one
    launch per call, eager and graph calls alike, and the results stay right."""
    import torch
    traces = mixed_traces(505, LENGTHS * 2)
    cfgs = [default_config(), default_config(window=5, hold=2)]
    cot = (np.arange(len(traces)) % 2).astype(np.uint32)
    samples, offsets = synth.make_batch(traces)
    want_res, _ = oracle_mod.replay_batch(samples, offsets, cfgs, cot)
    s, o, c = to_dev(samples, offsets, cot)
    res = torch.zeros((len(traces), 4), dtype=torch.int64, device="cuda")
    ctx.set_profiling(True)
    try:
        ctx.kernel_time(magus.KERNEL_REPLAY)
        for graphs in (False, True, True, False, True):
            ctx.set_graphs(graphs)
            res.zero_()
            ctx.replay(s, o, cfgs, c, results=res)
            ctx.check()
            assert (results_np(res) == want_res).all(), graphs
        ms, n = ctx.kernel_time(magus.KERNEL_REPLAY)
        assert n == 5 and ms > 0
        # timing off: the graph is reused, nothing is counted
        ctx.set_profiling(False)
        ctx.replay(s, o, cfgs, c, results=res)
        ctx.check()
        assert (results_np(res) == want_res).all()
        ctx.set_profiling(True)
        ms, n = ctx.kernel_time(magus.KERNEL_REPLAY)
        assert n == 0 and ms == 0
        for rep in range(3):
            ctx.replay(s, o, cfgs, c, results=res)
        ctx.check()
        ms, n = ctx.kernel_time(magus.KERNEL_REPLAY)
        assert n == 3 and ms > 0
    finally:
        ctx.set_profiling(False)
        ctx.set_graphs(False)


def test_graph_ring_wraps_with_timing(ctx, oracle_mod):
    """A captured call relaunched more times than its ring of graph
    instances holds (8), with timing on, off and on again part-way and the
    timer read in between: every launch is counted once while timing is on,
    none while it is off, and every launch's results are right."""
    import torch
    traces = mixed_traces(611, LENGTHS)
    cfgs = [default_config()]
    samples, offsets = synth.make_batch(traces)
    want_res, _ = oracle_mod.replay_batch(samples, offsets, cfgs, None)
    s, o, _ = to_dev(samples, offsets)
    res = torch.zeros((len(traces), 4), dtype=torch.int64, device="cuda")
    ctx.set_graphs(True)
    try:
        ctx.set_profiling(True)
        ctx.kernel_time(magus.KERNEL_REPLAY)
        counted = 0
        for i in range(21):
            if i == 9:
                ctx.set_profiling(False)
            if i == 13:
                ctx.set_profiling(True)
            res.zero_()
            ctx.replay(s, o, cfgs, results=res)
            ctx.check()
            assert (results_np(res) == want_res).all(), i
            if i not in range(9, 13):
                counted += 1
            if i in (5, 17):
                ms, n = ctx.kernel_time(magus.KERNEL_REPLAY)
                assert n == counted and ms > 0, (i, n, counted)
                counted = 0
        ms, n = ctx.kernel_time(magus.KERNEL_REPLAY)
        assert n == counted and ms > 0
    finally:
        ctx.set_profiling(False)
        ctx.set_graphs(False)


@pytest.fixture(scope="module")
def uneven():
    return synth.workload_uneven()


def test_uneven_workload_full_size_with_autotune(ctx, oracle_mod, uneven):
    """20,000 bursty traces of log-normal length with a grid config each (the
    benchmark's uneven launch): autotuned shape, graph relaunch; every trace's
    results and every step's decision byte against the oracle."""
    samples, offsets, cot = uneven
    grid = synth.sweep_grid()
    s, o, c = to_dev(samples, offsets, cot)
    chosen = ctx.autotune_replay(s, o, grid, c, reps=2)
    assert chosen["candidates"] == 15 and chosen["best_ms"] <= chosen["default_ms"]
    try:
        ctx.set_graphs(True)
        for _ in range(2):
            res, _ = ctx.replay(s, o, grid, c)
            ctx.check()
        got = results_np(res)
        want_res, want = oracle_mod.replay_batch(samples, offsets, grid, cot, want_bytes=True)
        assert (got == want_res).all(), describe_mismatch(got[:, 0], want_res[:, 0])
        _, lv = ctx.replay(s, o, grid, c, levels=True)
        ctx.check()
        b = lv.cpu().numpy()
        assert (b == want).all(), describe_mismatch(b, want, offsets)
    finally:
        ctx.set_graphs(False)
        ctx.set_chunk(0)
        ctx.set_persistent(0)
