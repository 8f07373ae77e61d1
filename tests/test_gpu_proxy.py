"""GPU parity of the proxy energy / EDP model (magus_proxy) against the oracle.

The integer statistics (intervals per level, excess sums) must be identical;
the FP64 metrics are compared within a tolerance derived from the rounding of
the two evaluation orders: the oracle sums up to ~10^5 interval lengths one by
one (relative error below n * 2^-53 ~ 1.1e-11 for n = 10^5), the kernel adds at
most 32 per-level terms of exact integer sums; savings are differences of
ratios near 1, so their absolute error is below ~4e-11 times the ratio.
Tolerance: relative 1e-9 for times, energies and powers; for the four
fractions 1e-9 absolute, or relative where the fraction exceeds 1 in
magnitude (extreme models stretch intervals by up to 2^32).
"""
import numpy as np
import pytest

import paper_2502_03796_amd as magus
import synth
from synth import default_config, proxy_model
from tests.gpu_util import to_dev
from tests.test_gpu_replay import mixed_traces, LENGTHS
from tests.test_gpu_stepped import dense_traces, stepped_configs

pytestmark = pytest.mark.gpu

FRACTIONS = ("perf_loss", "pkg_power_saving", "energy_saving", "edp_saving")


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = magus.Context(0)
    yield c
    c.close()


def check_against_oracle(oracle_mod, samples, offsets, cfgs, cot, model, st, me, traces=None):
    st = st.cpu().numpy()
    me = me.cpu().numpy() if me is not None else None
    n = len(offsets) - 1
    for t in (range(n) if traces is None else traces):
        x = samples[int(offsets[t]):int(offsets[t + 1])]
        cfg = cfgs[int(cot[t])] if cot is not None else cfgs[0]
        want_st, want_me = oracle_mod.proxy_trace(x, cfg, model)
        got_st = magus.proxy_stats_dict(st[t])
        assert got_st == want_st, f"trace {t} (length {len(x)}): stats differ"
        if me is None:
            continue
        got_me = magus.proxy_metrics_dict(me[t])
        for k in magus.PROXY_METRIC_KEYS:
            for p in range(3):
                if k in FRACTIONS:
                    tol = 1e-9 * max(1.0, abs(want_me[k][p]))
                    assert abs(got_me[k][p] - want_me[k][p]) <= tol, (t, k, p)
                else:
                    assert got_me[k][p] == pytest.approx(want_me[k][p], rel=1e-9, abs=1e-300), \
                        (t, k, p)


def test_worked_examples_on_gpu(ctx, oracle_mod):
    """The hand-worked traces of the oracle's pins, through the C ABI."""
    model = dict(n_levels=17, interval_us=100000, cap_mbps=[15000] + [40000] * 16,
                 uncore_mw=[10000] + [20000] * 15 + [30000], core_mw=50000, gpu_mw=200000)
    traces = [np.array([10000] * 40 + [20000] * 60, np.uint32),
              np.array([10000] * 10 + [30000] * 20 + [10000] * 20, np.uint32),
              np.full(300, 14999, np.uint32), np.zeros(0, np.uint32)]
    samples, offsets = synth.make_batch(traces)
    s, o, _ = to_dev(samples, offsets)
    st, me = ctx.proxy(s, o, [default_config()], model)
    ctx.check()
    got = [magus.proxy_stats_dict(r) for r in st.cpu().numpy()]
    assert got[0]["steps"][0] == 41 and got[0]["steps"][16] == 59 and got[0]["excess"][0] == 5000
    assert got[1]["steps"][0] == 30 and got[1]["steps"][16] == 20 and got[1]["excess"][0] == 15000
    m0 = magus.proxy_metrics_dict(me.cpu().numpy()[0])
    assert m0["time_s"][0] == pytest.approx(10 + 0.1 / 3, rel=1e-13)
    assert m0["energy_j"][1] == pytest.approx(2800.0, rel=1e-13)
    m3 = magus.proxy_metrics_dict(me.cpu().numpy()[3])
    assert all(v == [0.0, 0.0, 0.0] for v in m3.values())
    check_against_oracle(oracle_mod, samples, offsets, [default_config()], None, model, st, me)


@pytest.mark.parametrize("chunk", [64, 192, 4096, 0])
def test_mixed_traces_grid_configs(ctx, oracle_mod, chunk):
    """Every length class across chunk boundaries, a grid config per trace."""
    traces = mixed_traces(900 + chunk, LENGTHS)
    grid = synth.sweep_grid()
    rng = np.random.default_rng(chunk)
    cfgs = [grid[int(i)] for i in rng.integers(0, len(grid), 30)] + [default_config()]
    cot = rng.integers(0, len(cfgs), len(traces)).astype(np.uint32)
    samples, offsets = synth.make_batch(traces)
    model = proxy_model()
    s, o, c = to_dev(samples, offsets, cot)
    ctx.set_chunk(chunk)
    try:
        st, me = ctx.proxy(s, o, cfgs, model, c)
        ctx.check()
    finally:
        ctx.set_chunk(0)
    check_against_oracle(oracle_mod, samples, offsets, cfgs, cot, model, st, me)


@pytest.mark.parametrize("chunk", [64, 192, 4096, 0])
def test_stepped_configs_and_inner_levels(ctx, oracle_mod, chunk):
    """Stepped actuation visits every rung; initial levels inside the range."""
    traces = mixed_traces(1300 + chunk, LENGTHS)
    cfgs = stepped_configs(chunk + 5, 20) + [default_config(level_init=7),
                                             default_config(up_step=1, down_step=2)]
    cot = (np.arange(len(traces)) % len(cfgs)).astype(np.uint32)
    samples, offsets = synth.make_batch(traces)
    rng = np.random.default_rng(chunk)
    model = dict(n_levels=20, interval_us=int(rng.integers(1, 10**6)),
                 cap_mbps=[int(v) for v in rng.integers(1000, 150000, 32)],
                 uncore_mw=[int(v) for v in rng.integers(0, 50000, 32)],
                 core_mw=30000, gpu_mw=300000)
    s, o, c = to_dev(samples, offsets, cot)
    ctx.set_chunk(chunk)
    try:
        st, me = ctx.proxy(s, o, cfgs, model, c)
        ctx.check()
        st2, _ = ctx.proxy(s, o, cfgs, model, c, metrics=False)
        ctx.check()
    finally:
        ctx.set_chunk(0)
    check_against_oracle(oracle_mod, samples, offsets, cfgs, cot, model, st, me)
    assert (st.cpu().numpy() == st2.cpu().numpy()).all()


@pytest.mark.parametrize("chunk", [64, 192, 4096, 65536])
def test_stepped_dense_events(ctx, oracle_mod, chunk):
    """Stepped configs on traces with a move at every step and long high runs:
    levels change inside blocks (several per block), blocks whose moves are
    all clamped, and chunks of one block up to many groups of blocks."""
    traces = dense_traces(chunk + 3)
    cfgs = stepped_configs(chunk + 7, 10) + [
        default_config(window=2, hold=2, up_step=1, down_step=1),
        default_config(window=2, hold=4, up_step=3, down_step=0, level_init=9),
        default_config(up_step=0, down_step=2, level_min=2, level_max=29, level_init=20)]
    cot = (np.arange(len(traces)) % len(cfgs)).astype(np.uint32)
    samples, offsets = synth.make_batch(traces)
    rng = np.random.default_rng(chunk + 5)
    model = dict(n_levels=30, interval_us=int(rng.integers(1, 10**6)),
                 cap_mbps=[int(v) for v in rng.integers(500, 6000, 32)],
                 uncore_mw=[int(v) for v in rng.integers(0, 50000, 32)],
                 core_mw=30000, gpu_mw=300000)
    s, o, c = to_dev(samples, offsets, cot)
    ctx.set_chunk(chunk)
    try:
        st, me = ctx.proxy(s, o, cfgs, model, c)
        ctx.check()
    finally:
        ctx.set_chunk(0)
    check_against_oracle(oracle_mod, samples, offsets, cfgs, cot, model, st, me)


@pytest.mark.parametrize("chunk", [64, 128, 4096])
def test_jump_to_bound_with_inner_initial_levels(ctx, oracle_mod, chunk):
    """The single-pass path (every config jumps to the bound) with initial
    levels strictly inside the range, so a chunk can be entered at level_init,
    level_min or level_max, across chunk boundaries of every kind."""
    traces = mixed_traces(1700 + chunk, LENGTHS)
    grid = synth.sweep_grid()
    rng = np.random.default_rng(chunk + 11)
    cfgs = []
    for i in rng.integers(0, len(grid), 24):
        c = dict(grid[int(i)])
        c["level_init"] = int(rng.integers(0, 17))
        cfgs.append(c)
    cfgs.append(default_config(level_min=3, level_max=9, level_init=5))
    cot = rng.integers(0, len(cfgs), len(traces)).astype(np.uint32)
    samples, offsets = synth.make_batch(traces)
    model = proxy_model()
    s, o, c = to_dev(samples, offsets, cot)
    ctx.set_chunk(chunk)
    try:
        st, me = ctx.proxy(s, o, cfgs, model, c)
        ctx.check()
    finally:
        ctx.set_chunk(0)
    check_against_oracle(oracle_mod, samples, offsets, cfgs, cot, model, st, me)


def test_full_range_samples(ctx, oracle_mod):
    rng = np.random.default_rng(99)
    traces = [rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
              for n in (1, 5, 300, 5000)]
    traces.append(np.array([0, 2**32 - 1] * 200, np.uint32))
    cfg = default_config(window=2, hold=3, level_max=31)
    model = dict(n_levels=32, interval_us=2**20, cap_mbps=[1] * 31 + [2**32 - 1],
                 uncore_mw=[2**32 - 1] * 32, core_mw=2**32 - 1, gpu_mw=2**32 - 1)
    samples, offsets = synth.make_batch(traces)
    s, o, _ = to_dev(samples, offsets)
    st, me = ctx.proxy(s, o, [cfg], model)
    ctx.check()
    check_against_oracle(oracle_mod, samples, offsets, [cfg], None, model, st, me)


def _alg1_boundary_trace(seed, ku, kd, n_pairs=3000):
    """Pairs (a, b) on both sides of the Alg. 1 thresholds with window 2:
    b 2^16 - a ku within a few 2^16 of 0 (and exactly 0 for a quarter of them)
    for rises, a 2^16 - b kd likewise for falls; every sample below 2^24 but
    large enough that a float product of either side would be off by far
    more than one."""
    rng = np.random.default_rng(seed)
    lim = 1 << 24
    out = []
    for _ in range(n_pairs):
        lo = int(rng.integers(1 << 22, (lim * 65536) // max(ku, kd) - 4))
        if rng.integers(0, 4) == 0:
            lo -= lo % 65536                              # a product that is a multiple of 2^16
        delta = int(rng.integers(-2, 3))
        if rng.integers(0, 2):
            a = lo                                        # rise: b near a ku / 2^16
            b = (a * ku) // 65536 + (delta if (a * ku) % 65536 else 0)
        else:
            b = lo                                        # fall: a near b kd / 2^16
            a = (b * kd) // 65536 + (delta if (b * kd) % 65536 else 0)
        out += [min(max(a, 0), lim - 1), min(max(b, 0), lim - 1)]
    return np.array(out, np.uint32)


@pytest.mark.parametrize("chunk", [256, 4096, 16384, 32768])
def test_narrow_pass_boundaries(ctx, oracle_mod, chunk):
    """The fused pass on samples just below 2^24, where it takes its 32-bit
    form with the fp32 Alg. 1 compares: exact-boundary pairs for rises and
    falls; a chunk that holds one sample of 2^24 (run again by the exact
    pass) between chunks that do not; all samples at 2^24 - 1 with a cap of
    1 (the largest 32-bit per-lane sums, 256 blocks a lane at chunk 16,384);
    thresholds whose 2^16 + W q is 2^24 (still narrow) and above it (exact
    only); and chunk lengths past the narrow pass's limit."""
    lim = 1 << 24
    cfg_a = default_config(window=2, hold=4)
    cfg_b = default_config(window=16, hold=3, inc_q16=(lim - 65536) // 16,
                           dec_q16=-((lim - 65536) // 16))       # 2^16 + W q = 2^24
    cfg_c = default_config(window=16, hold=3, inc_q16=(lim - 65536) // 16 + 1,
                           dec_q16=-3000)                        # above: exact pass only
    cfg_d = default_config(window=4, hold=10, level_init=5)
    cfgs = [cfg_a, cfg_b, cfg_c, cfg_d]
    ku = 65536 + 2 * cfg_a["inc_q16"]
    kd = 65536 - 2 * cfg_a["dec_q16"]
    one_big = np.full(3 * chunk + 77, lim - 2, np.uint32)
    one_big[chunk + chunk // 2] = lim                            # middle chunk only
    one_big[::7] = 1000
    traces = [_alg1_boundary_trace(chunk, ku, kd),
              _alg1_boundary_trace(chunk + 1, ku, kd, 500),
              one_big,
              np.full(2 * chunk + 64, lim - 1, np.uint32),
              np.array([lim - 1, 0] * (chunk // 2 + 40), np.uint32),
              mixed_traces(chunk, [5000])[0]]
    cot = np.array([0, 1, 0, 3, 2, 3], np.uint32)
    samples, offsets = synth.make_batch(traces)
    model = dict(proxy_model(), cap_mbps=[1] + proxy_model()["cap_mbps"][1:])
    s, o, c = to_dev(samples, offsets, cot)
    ctx.set_chunk(chunk)
    try:
        st, me = ctx.proxy(s, o, cfgs, model, c)
        ctx.check()
    finally:
        ctx.set_chunk(0)
    check_against_oracle(oracle_mod, samples, offsets, cfgs, cot, model, st, me)


def test_exact_queue_across_calls(ctx, oracle_mod):
    """The chunks that a narrow pass hands to the exact (jump-to-bound) or
    wide (stepped) pass go through one queue in the context that every call
    must start empty: one context runs a batch where most chunks hold a
    sample of 2^24 or more (a long queue), then a smaller batch with none
    (an entry left over would name a chunk of the earlier batch), then a
    mix, then the first batch again, each with a jump-to-bound and then a
    stepped config; every call matches the oracle.  (A stale entry would
    only rerun a chunk, or name none of this call's; a count never cleared
    would overrun the queue.)"""
    lim = 1 << 24
    cfgs = [default_config(window=4, hold=5),
            default_config(window=4, hold=5, up_step=2, down_step=1)]
    model = proxy_model()

    def big(n, seed):
        r = np.random.default_rng(seed)
        return r.integers(lim, 2**32, n, dtype=np.uint64).astype(np.uint32)

    batches = [
        [big(n, 1 + i) for i, n in enumerate((3000, 2500, 4096, 700))],
        mixed_traces(9, [300, 900]),
        [big(1500, 7)] + mixed_traces(11, [2000, 64]) + [big(257, 8)],
    ]
    batches.append(batches[0])
    ctx.set_chunk(256)
    try:
        for traces in batches:
            samples, offsets = synth.make_batch(traces)
            s, o, _ = to_dev(samples, offsets)
            for cfg in cfgs:
                st, me = ctx.proxy(s, o, [cfg], model)
                ctx.check()
                check_against_oracle(oracle_mod, samples, offsets, [cfg], None, model, st, me)
    finally:
        ctx.set_chunk(0)


def test_exact_queue_longer_than_its_grid(ctx, oracle_mod):
    """More queued chunks than the exact and wide kernels have waves (their
    grids stop at 2,048 workgroups of 4 waves): with chunks of 64 steps
    (128 for the single pass) 1.2 million samples of 2^24 or more queue
    9,375 chunks on the single pass and 18,750 on the stepped one, so waves
    take several queue entries each; both match the oracle."""
    rng = np.random.default_rng(7)
    traces = [rng.integers(1 << 24, 2**32, 200000, dtype=np.uint64).astype(np.uint32)
              for _ in range(6)]
    samples, offsets = synth.make_batch(traces)
    model = proxy_model()
    s, o, _ = to_dev(samples, offsets)
    ctx.set_chunk(64)
    try:
        for cfg in (default_config(window=4, hold=5),
                    default_config(window=4, hold=5, up_step=2, down_step=1)):
            st, me = ctx.proxy(s, o, [cfg], model)
            ctx.check()
            check_against_oracle(oracle_mod, samples, offsets, [cfg], None, model, st, me)
    finally:
        ctx.set_chunk(0)


@pytest.mark.parametrize("chunk", [128, 4096, 16320, 16384, 32768])
def test_stepped_narrow_and_wide_passes(ctx, oracle_mod, chunk):
    """Stepped configs through the statistics pass's two forms: the narrow
    one (32-bit excess bins and 16-bit counts in LDS, each word shared by 4
    lanes, levels from the scalar walk of each block's moves) on samples
    just below 2^22, a chunk with one sample of 2^22 (run again by the wide
    pass), the full 32-rung ladder (the largest bins), the longest narrow
    chunk (16,320 steps) and chunk lengths past the narrow limit."""
    lim = 1 << 22
    rng = np.random.default_rng(chunk + 17)
    dense = dense_traces(chunk + 9)
    # the same shapes scaled so that their largest sample is just below 2^24
    near = [(t.astype(np.uint64) * ((lim - 1) // max(int(t.max()), 1))).astype(np.uint32)
            for t in dense[:3]]
    one_big = np.concatenate(near[:1] * 3)[:3 * chunk + 50].copy()
    one_big[min(len(one_big) - 1, chunk + 5)] = lim
    traces = dense[:4] + near + [one_big]
    cfgs = [default_config(up_step=2, down_step=1, level_max=31),
            default_config(window=2, hold=3, up_step=3, down_step=2, level_min=0, level_max=31,
                           level_init=15),
            default_config(up_step=1, down_step=1, level_min=5, level_max=9, level_init=7)]
    cot = (np.arange(len(traces)) % len(cfgs)).astype(np.uint32)
    samples, offsets = synth.make_batch(traces)
    model = dict(n_levels=32, interval_us=100000,
                 cap_mbps=sorted(int(v) for v in rng.integers(lim - 300000, lim, 32)),
                 uncore_mw=[int(v) for v in rng.integers(0, 50000, 32)],
                 core_mw=30000, gpu_mw=300000)
    s, o, c = to_dev(samples, offsets, cot)
    ctx.set_chunk(chunk)
    try:
        st, me = ctx.proxy(s, o, cfgs, model, c)
        ctx.check()
    finally:
        ctx.set_chunk(0)
    check_against_oracle(oracle_mod, samples, offsets, cfgs, cot, model, st, me)


@pytest.mark.parametrize("chunk", [16320, 16384])
def test_stepped_narrow_counts_at_their_limit(ctx, oracle_mod, chunk):
    """The narrow stepped pass counts the steps of the blocks that change
    the level per level in 16-bit words, each shared by 4 lanes (l, l + 16,
    l + 32, l + 48): at most one step a block from each, 1,020 in the
    longest narrow chunk.  A period-4 trace (low, high, high, low) with
    window 2 raises the level at every rise and lowers it at every fall (two
    events in four steps stay below the 3/5 high fraction), so every block
    changes the level and lanes 0, 16, 32 and 48 are at the entering level
    in all of them: their word reaches 1,020 in a 16,320-step chunk (checked
    on the oracle's levels), and the statistics still match the oracle's."""
    pattern = np.array([1000, 2000, 2000, 1000], np.uint32)
    trace = np.tile(pattern, (2 * chunk + 640) // 4)
    cfg = default_config(window=2, hold=10, up_step=1, down_step=1, level_min=0,
                         level_max=31, level_init=5)
    _, dec = oracle_mod.replay_trace(trace, cfg)
    levels, high, _ = oracle_mod.decode(dec)
    assert not high.any()
    # the level before step i: the level after step i - 1 (level_init first)
    before = np.concatenate([[cfg["level_init"]], levels[:-1]])
    blocks = before[:chunk // 64 * 64].reshape(-1, 64)
    changing = blocks.min(axis=1) != blocks.max(axis=1)
    lanes = blocks[changing][:, [0, 16, 32, 48]]
    assert len(lanes) == chunk // 64 and (lanes == lanes[0, 0]).all()   # 4 x 255 at 16,320
    samples, offsets = synth.make_batch([trace, trace[: chunk + 64]])
    model = proxy_model()
    model = dict(model, n_levels=32, cap_mbps=[1500] * 32, uncore_mw=[20000] * 32)
    s, o, _ = to_dev(samples, offsets)
    ctx.set_chunk(chunk)
    try:
        st, me = ctx.proxy(s, o, [cfg], model)
        ctx.check()
    finally:
        ctx.set_chunk(0)
    check_against_oracle(oracle_mod, samples, offsets, [cfg], None, model, st, me)


def test_rejects_levels_the_model_does_not_describe(ctx):
    samples, offsets = synth.make_batch([np.ones(10, np.uint32)])
    s, o, _ = to_dev(samples, offsets)
    with pytest.raises(magus.MagusError) as ei:
        ctx.proxy(s, o, [default_config()], dict(proxy_model(), n_levels=16))
    assert ei.value.code == magus.EINVAL


def test_bulk_workload_full_size_sampled(ctx, oracle_mod):
    """4,096 x 100,000 at full size; sampled traces against the oracle."""
    samples, offsets = synth.workload_bulk(4096, 100000)
    s, o, _ = to_dev(samples, offsets)
    model = proxy_model()
    st, me = ctx.proxy(s, o, [default_config()], model)
    ctx.check()
    rng = np.random.default_rng(3)
    pick = sorted(set(rng.integers(0, 4096, 6).tolist()) | {0, 4095})
    check_against_oracle(oracle_mod, samples, offsets, [default_config()], None, model, st, me,
                         traces=pick)
    # every interval is counted once
    steps = st.cpu().numpy()[:, 2:2 + magus.PROXY_LEVELS].sum(axis=1)
    assert (steps == np.diff(offsets.astype(np.int64))).all()


def test_bulk_workload_full_size_stepped_sampled(ctx, oracle_mod):
    """The stepped configuration the bench times (up 2 rungs, down 1) on the
    4,096 x 100,000 bulk traces at full size; sampled traces against the
    oracle, and every interval counted once in every trace."""
    samples, offsets = synth.workload_bulk(4096, 100000)
    s, o, _ = to_dev(samples, offsets)
    model = proxy_model()
    cfg = default_config(up_step=2, down_step=1)
    st, me = ctx.proxy(s, o, [cfg], model)
    ctx.check()
    rng = np.random.default_rng(5)
    pick = sorted(set(rng.integers(0, 4096, 6).tolist()) | {0, 4095})
    check_against_oracle(oracle_mod, samples, offsets, [cfg], None, model, st, me, traces=pick)
    steps = st.cpu().numpy()[:, 2:2 + magus.PROXY_LEVELS].sum(axis=1)
    assert (steps == np.diff(offsets.astype(np.int64))).all()


@pytest.mark.parametrize("stepped", [False, True])
def test_device_data_faults_leave_stats_zero(ctx, stepped):
    """A batch the device-side checks reject (offsets not monotone, a config
    index out of range) is reported by check() and sets every word of the
    statistics to zero, on the one-pass path and on the stepped path: the
    output buffer is filled with a non-zero sentinel before each call."""
    import torch
    samples, offsets = synth.make_batch(mixed_traces(1, [100, 100]))
    s, o, _ = to_dev(samples, offsets)
    cfg = default_config(up_step=2, down_step=1) if stepped else default_config()
    model = proxy_model()
    out = torch.empty((2, 2 + 2 * magus.PROXY_LEVELS), dtype=torch.int64, device="cuda")
    bad = torch.tensor([0, 150, 100], dtype=torch.int64, device="cuda")   # not monotone
    out.fill_(0x5A5A5A5A5A5A5A5A)
    st, _ = ctx.proxy(s, bad, [cfg], model, metrics=False, stats=out)
    with pytest.raises(magus.MagusError) as ei:
        ctx.check()
    assert ei.value.code == magus.EDATA
    assert (st.cpu().numpy() == 0).all()
    cot = torch.tensor([0, 5], dtype=torch.int32, device="cuda")      # index out of range
    out.fill_(0x5A5A5A5A5A5A5A5A)
    st, _ = ctx.proxy(s, o, [cfg], model, cot, metrics=False, stats=out)
    with pytest.raises(magus.MagusError):
        ctx.check()
    assert (st.cpu().numpy() == 0).all()
    out.fill_(0x5A5A5A5A5A5A5A5A)
    st, _ = ctx.proxy(s, o, [cfg], model, stats=out)
    ctx.check()
    assert st.cpu().numpy()[:, 2:2 + magus.PROXY_LEVELS].sum() == 200
