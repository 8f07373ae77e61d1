"""GPU parity of the monitor front end (counter readings -> MB/s) and of the
alternative derivative bases, against the oracle."""
import numpy as np
import pytest

import paper_2502_03796_amd as magus
import synth
from synth import default_config, proxy_model
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


def readings(seed, lengths, bits):
    """Counter readings of traces: cumulative bytes at ~100 ms, with wraps,
    zero and very long intervals and very large deltas mixed in."""
    rng = np.random.default_rng(seed)
    cs, ts = [], []
    for n in lengths:
        dt = rng.integers(90_000_000, 110_000_000, n, dtype=np.uint64)
        dt[rng.random(n) < 0.02] = 0
        dt[rng.random(n) < 0.02] = np.uint64(1) << np.uint64(40)
        t = np.cumsum(dt).astype(np.uint64)
        d = rng.integers(0, 1 << 34, n, dtype=np.uint64)
        d[rng.random(n) < 0.03] = rng.integers(0, 2**63, 1, dtype=np.uint64)[0]
        c = np.cumsum(d).astype(np.uint64) + rng.integers(0, 2**63, 1, dtype=np.uint64)[0]
        if bits < 64:
            c &= np.uint64((1 << bits) - 1)
        cs.append(c)
        ts.append(t)
    return cs, ts


@pytest.mark.parametrize("bits,bpc", [(64, 1), (48, 64), (32, 64), (20, 1000)])
def test_counters_to_mbps_matches_oracle(ctx, oracle_mod, bits, bpc):
    import torch
    lengths = [1, 2, 3, 64, 255, 256, 257, 1000, 4097]
    cs, ts = readings(bits * 7 + bpc, lengths, bits)
    offs = np.zeros(len(lengths) + 1, np.uint64)
    offs[1:] = np.cumsum(lengths)
    c = torch.from_numpy(np.concatenate(cs).view(np.int64)).cuda()
    t = torch.from_numpy(np.concatenate(ts).view(np.int64)).cuda()
    o = torch.from_numpy(offs.view(np.int64)).cuda()
    out, so = ctx.counters_to_mbps(c, t, o, bits, bpc)
    ctx.check()
    got = out.cpu().numpy().view(np.uint32)
    so = so.cpu().numpy()
    for i in range(len(lengths)):
        want = oracle_mod.counters_to_mbps(cs[i], ts[i], bits, bpc)
        assert (got[so[i]:so[i + 1]] == want).all(), i


def test_counters_reject_empty_traces(ctx):
    import torch
    c = torch.zeros(4, dtype=torch.int64, device="cuda")
    o = torch.tensor([0, 2, 2, 4], dtype=torch.int64, device="cuda")
    ctx.counters_to_mbps(c, c, o)
    with pytest.raises(magus.MagusError):
        ctx.check()


# B_ref values of the fixed-reference base (base 3): the listing's unscaled
# derivative (1), levels inside the traces' range, and the largest reference
REFS = (1, 5000, 20000, 100000, 2**32 - 1)


@pytest.mark.parametrize("base", [1, 2, 3])
def test_base_variants_replay_sweep_serve(ctx, oracle_mod, base):
    traces = mixed_traces(50 + base, LENGTHS)
    grid = synth.sweep_grid()
    rng = np.random.default_rng(base)
    cfgs = [dict(grid[int(i)], base=base) for i in rng.integers(0, len(grid), 20)]
    cfgs += [dict(default_config(up_step=2, down_step=1), base=base), default_config()]
    if base == 3:
        # several references in one call (the sweep groups configs by them)
        for k, cf in enumerate(cfgs[:-1]):
            cf["base_ref"] = REFS[k % len(REFS)]
    cot = (np.arange(len(traces)) % len(cfgs)).astype(np.uint32)
    samples, offsets = synth.make_batch(traces)
    want_res, want_b = oracle_mod.replay_batch(samples, offsets, cfgs, cot, want_bytes=True)
    s, o, c = to_dev(samples, offsets, cot)
    res, lv = ctx.replay(s, o, cfgs, c, levels=True)
    ctx.check()
    assert (results_np(res) == want_res).all()
    b = lv.cpu().numpy()
    assert (b == want_b).all(), describe_mismatch(b, want_b, offsets)
    # without decision bytes (the stepped configs take the mask-pass walk)
    res2, _ = ctx.replay(s, o, cfgs, c)
    ctx.check()
    assert (results_np(res2) == want_res).all()
    # proxy statistics: with a stepped config in the batch (mask pass and
    # statistics pass), and with every config jumping to the bound (one pass)
    model = proxy_model()
    jump = [dict(cf, up_step=0, down_step=0) for cf in cfgs]
    for batch in (cfgs, jump):
        st, _ = ctx.proxy(s, o, batch, model, c, metrics=False)
        ctx.check()
        stn = st.cpu().numpy()
        for t in range(len(traces)):
            x = samples[int(offsets[t]):int(offsets[t + 1])]
            want_st, _ = oracle_mod.proxy_trace(x, batch[int(cot[t])], model)
            assert magus.proxy_stats_dict(stn[t]) == want_st, (t, batch[int(cot[t])])
    # sweep: base variants grouped apart from the default base
    want_sc, want_arg = oracle_mod.sweep(samples, offsets, cfgs)
    sc, arg = ctx.sweep(s, o, cfgs, scores=True)
    ctx.check()
    assert (sc.cpu().numpy().view(np.uint64) == want_sc).all()
    assert (arg.cpu().numpy().astype(np.uint32) == want_arg).all()
    # serving
    srv = magus.Server(ctx, 4 * magus.Server.slot_bytes())
    x = synth.serve_stream_samples(base, 500)
    slot = srv.open(cfgs[0])
    got = np.array([srv.step([slot], [v])[0] for v in x], np.uint8)
    _, want = oracle_mod.replay_trace(x, cfgs[0])
    assert (got == want).all()
    srv.close()


def test_counters_feed_replay_end_to_end(ctx, oracle_mod):
    """Counter readings -> MB/s on the GPU -> replay on the GPU equals the
    oracle's conversion followed by the oracle's replay."""
    import torch
    lengths = [3000, 1, 2, 5000, 777]
    cs, ts = readings(99, lengths, 48)
    offs = np.zeros(len(lengths) + 1, np.uint64)
    offs[1:] = np.cumsum(lengths)
    c = torch.from_numpy(np.concatenate(cs).view(np.int64)).cuda()
    t = torch.from_numpy(np.concatenate(ts).view(np.int64)).cuda()
    o = torch.from_numpy(offs.view(np.int64)).cuda()
    smp, so = ctx.counters_to_mbps(c, t, o, 48, 64)
    res, lv = ctx.replay(smp, so, [default_config()], levels=True)
    ctx.check()
    so = so.cpu().numpy()
    got = lv.cpu().numpy()
    for i in range(len(lengths)):
        x = oracle_mod.counters_to_mbps(cs[i], ts[i], 48, 64)
        r, want = oracle_mod.replay_trace(x, default_config())
        assert (got[so[i]:so[i + 1]] == want).all(), i
        assert results_np(res)[i][0] == r["score"]
