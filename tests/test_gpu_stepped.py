"""GPU parity with stepped actuation (up_step / down_step > 0): replay, sweep
and serving against the oracle, bit for bit."""
import numpy as np
import pytest

import paper_2502_03796_amd as magus
import synth
from synth import default_config
from tests.gpu_util import to_dev, results_np, describe_mismatch
from tests.test_gpu_replay import mixed_traces, LENGTHS

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = magus.Context(0)
    yield c
    c.close()


def stepped_configs(seed, n):
    rng = np.random.default_rng(seed)
    grid = synth.sweep_grid()
    out = []
    for i in range(n):
        c = dict(grid[int(rng.integers(0, len(grid)))])
        c["up_step"] = int(rng.integers(0, 6))
        c["down_step"] = int(rng.integers(0, 6))
        if i % 5 == 0:
            c["level_init"] = int(rng.integers(0, 17))
        out.append(c)
    return out


@pytest.mark.parametrize("chunk", [64, 192, 4096, 0])
def test_stepped_replay_matches_oracle(ctx, oracle_mod, chunk):
    traces = mixed_traces(700 + chunk, LENGTHS)
    cfgs = stepped_configs(chunk, 24) + [default_config(up_step=1, down_step=1),
                                         default_config()]
    cot = (np.arange(len(traces)) % len(cfgs)).astype(np.uint32)
    samples, offsets = synth.make_batch(traces)
    want_res, want_b = oracle_mod.replay_batch(samples, offsets, cfgs, cot, want_bytes=True)
    s, o, c = to_dev(samples, offsets, cot)
    ctx.set_chunk(chunk)
    try:
        res, lv = ctx.replay(s, o, cfgs, c, levels=True)
        ctx.check()
        res2, _ = ctx.replay(s, o, cfgs, c)
        ctx.check()
    finally:
        ctx.set_chunk(0)
    got = results_np(res)
    assert (got == want_res).all(), describe_mismatch(got[:, 0], want_res[:, 0])
    assert (results_np(res2) == want_res).all()
    b = lv.cpu().numpy()
    assert (b == want_b).all(), describe_mismatch(b, want_b, offsets)


def dense_traces(seed):
    """Traces whose every step is an event (alternating samples), long high
    runs broken by single events, and plain mixed traces."""
    rng = np.random.default_rng(seed)
    out = [np.array([1000, 3000] * 5000, np.uint32),
           np.array([1000, 1000, 5000] * 3001, np.uint32)]
    x = rng.integers(1000, 1100, 20000).astype(np.uint32)
    x[rng.integers(0, 20000, 400)] = 50000
    out.append(x)
    return out + mixed_traces(seed, [70001, 16385, 8193, 4097, 65, 1])


@pytest.mark.parametrize("chunk", [64, 4096, 8192, 16384, 65536])
def test_stepped_dense_events_and_long_chunks(ctx, oracle_mod, chunk):
    """Blocks with a move at every step, chunks of one block and chunks of
    several groups of 64 blocks, with and without decision bytes."""
    traces = dense_traces(chunk)
    cfgs = stepped_configs(chunk + 1, 12) + [
        default_config(window=2, hold=2, up_step=1, down_step=1),
        default_config(window=2, hold=4, up_step=3, down_step=0, level_init=9),
        default_config(up_step=0, down_step=2, level_min=2, level_max=29, level_init=20)]
    cot = (np.arange(len(traces)) % len(cfgs)).astype(np.uint32)
    samples, offsets = synth.make_batch(traces)
    want_res, want_b = oracle_mod.replay_batch(samples, offsets, cfgs, cot, want_bytes=True)
    s, o, c = to_dev(samples, offsets, cot)
    ctx.set_chunk(chunk)
    try:
        res, _ = ctx.replay(s, o, cfgs, c)
        ctx.check()
        res2, lv = ctx.replay(s, o, cfgs, c, levels=True)
        ctx.check()
    finally:
        ctx.set_chunk(0)
    got = results_np(res)
    assert (got == want_res).all(), describe_mismatch(got[:, 0], want_res[:, 0])
    assert (results_np(res2) == want_res).all()
    assert (lv.cpu().numpy() == want_b).all()


def test_stepped_bulk_workload_full_size(ctx, oracle_mod):
    """4,096 x 100,000 with up 2 / down 1 rungs: every trace's results."""
    samples, offsets = synth.workload_bulk(4096, 100000)
    cfg = default_config(up_step=2, down_step=1)
    s, o, _ = to_dev(samples, offsets)
    res, _ = ctx.replay(s, o, [cfg])
    ctx.check()
    want, _ = oracle_mod.replay_batch(samples, offsets, [cfg])
    got = results_np(res)
    assert (got == want).all(), describe_mismatch(got[:, 0], want[:, 0])


def test_stepped_staircase_on_gpu(ctx, oracle_mod):
    cfg = default_config(window=2, hold=32, hf_num=1, hf_den=1, up_step=3)
    x = np.array([1000 * 2 ** k for k in range(20)], np.uint32)
    samples, offsets = synth.make_batch([x])
    s, o, _ = to_dev(samples, offsets)
    _, lv = ctx.replay(s, o, [cfg], levels=True)
    assert list(lv.cpu().numpy() & 31) == [min(3 * t, 16) for t in range(20)]


def test_stepped_sweep_matches_oracle(ctx, oracle_mod):
    traces = mixed_traces(808, [0, 1, 70, 300, 2000, 5000])
    cfgs = stepped_configs(9, 300) + [synth.sweep_config(i) for i in range(0, 16384, 997)]
    samples, offsets = synth.make_batch(traces)
    want_sc, want_arg = oracle_mod.sweep(samples, offsets, cfgs)
    s, o, _ = to_dev(samples, offsets)
    sc, arg = ctx.sweep(s, o, cfgs, scores=True)
    ctx.check()
    assert (sc.cpu().numpy().view(np.uint64) == want_sc).all()
    assert (arg.cpu().numpy().astype(np.uint32) == want_arg).all()


def test_stepped_serving_matches_oracle(ctx, oracle_mod):
    cfgs = stepped_configs(77, 16)
    srv = magus.Server(ctx, 16 * magus.Server.slot_bytes())
    slots = [srv.open(c) for c in cfgs]
    data = np.stack([synth.serve_stream_samples(900 + i, 300) for i in range(16)])
    out = np.zeros((300, 16), np.uint8)
    for k in range(300):
        out[k] = srv.step(slots, data[:, k])
    for i, c in enumerate(cfgs):
        _, want = oracle_mod.replay_trace(data[i], c)
        assert (out[:, i] == want).all(), i
    srv.close()
