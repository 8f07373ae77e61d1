"""Degenerate batches on the GPU: no traces at all, and traces that are all
empty, through replay (jump and stepped actuation), sweep and proxy."""
import numpy as np
import pytest

import paper_2502_03796_amd as magus
import synth
from synth import default_config, proxy_model
from tests.gpu_util import to_dev, results_np

pytestmark = pytest.mark.gpu

CONFIGS = [default_config(), default_config(up_step=2, down_step=1)]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = magus.Context(0)
    yield c
    c.close()


def test_no_traces(ctx):
    import torch
    s = torch.zeros(0, dtype=torch.int32, device="cuda")
    o = torch.zeros(1, dtype=torch.int64, device="cuda")
    for cfg in CONFIGS:
        res, _ = ctx.replay(s, o, [cfg])
        ctx.check()
        assert tuple(res.shape) == (0, 4)
    sc, arg = ctx.sweep(s, o, synth.sweep_grid()[:100], scores=True)
    ctx.check()
    assert sc.numel() == 0 and arg.numel() == 0
    st, me = ctx.proxy(s, o, [default_config()], proxy_model())
    ctx.check()
    assert st.shape[0] == 0 and me.shape[0] == 0


def test_all_traces_empty(ctx, oracle_mod):
    """Empty traces score 0 under every config and take config 0 in the sweep."""
    samples, offsets = synth.make_batch([np.zeros(0, np.uint32)] * 5)
    s, o, _ = to_dev(samples, offsets)
    for cfg in CONFIGS:
        res, lv = ctx.replay(s, o, [cfg], levels=True)
        ctx.check()
        assert (results_np(res) == 0).all()
        assert lv.numel() == 0
    cfgs = synth.sweep_grid()[::97]
    sc, arg = ctx.sweep(s, o, cfgs, scores=True)
    ctx.check()
    assert (sc.cpu().numpy() == 0).all() and (arg.cpu().numpy() == 0).all()
    for cfg in CONFIGS:
        st, me = ctx.proxy(s, o, [cfg], proxy_model())
        ctx.check()
        for t in range(5):
            want_st, _ = oracle_mod.proxy_trace(np.zeros(0, np.uint32), cfg, proxy_model())
            assert magus.proxy_stats_dict(st.cpu().numpy()[t]) == want_st
        assert (me.cpu().numpy() == 0).all()


def test_empty_traces_between_others(ctx, oracle_mod):
    """Empty traces at the start, in the middle and at the end of a batch."""
    rng = np.random.default_rng(5)
    traces = [np.zeros(0, np.uint32)]
    for n in (1, 0, 0, 64, 0, 4097, 0):
        traces.append(rng.integers(1000, 90000, n).astype(np.uint32))
    samples, offsets = synth.make_batch(traces)
    s, o, _ = to_dev(samples, offsets)
    for cfg in CONFIGS:
        want, want_b = oracle_mod.replay_batch(samples, offsets, [cfg], want_bytes=True)
        res, lv = ctx.replay(s, o, [cfg], levels=True)
        ctx.check()
        assert (results_np(res) == want).all()
        assert (lv.cpu().numpy() == want_b).all()
