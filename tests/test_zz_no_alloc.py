"""GPU parity of the allocation-free replay (magus_replay_noalloc) against
magus_replay, through the C ABI: two calls in a row (the second on a smaller
batch, so stale contents of the shared scratch array would show), decision
bytes, a grid config per trace, an empty batch, a rejected batch and the
host-side limits."""
import ctypes

import numpy as np
import pytest

import paper_2502_03796_amd as magus
import synth
from synth import default_config
from tests.gpu_util import to_dev, results_np, describe_mismatch

pytestmark = pytest.mark.gpu


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def noalloc(s, o, cfgs, cot=None, levels=False, results=None, status=None):
    """magus_replay_noalloc on torch's current stream; returns (rc, results,
    levels, status)."""
    import torch
    arr = magus.config_array(cfgs)
    n_traces = o.numel() - 1
    if results is None:
        results = torch.full((n_traces, 4), -1, dtype=torch.int64, device="cuda")
    lv = torch.zeros(s.numel(), dtype=torch.uint8, device="cuda") if levels else None
    if status is None:
        status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    rc = magus.load().magus_replay_noalloc(
        _p(s), s.numel(), _p(o), n_traces, arr, len(arr), _p(cot), _p(results), _p(lv),
        _p(status), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return rc, results, lv, status


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = magus.Context(0)
    yield c
    c.close()


def mixed(seed, lengths):
    rng = np.random.default_rng(seed)
    out = []
    for n in lengths:
        lv = rng.choice([3000, 9000, 30000, 90000, 200000], size=max(1, n // 150 + 1))
        x = np.repeat(lv, 150)[:n] * rng.uniform(0.95, 1.05, size=n)
        out.append(np.round(x).astype(np.uint32))
    return out


def test_noalloc_matches_replay_twice_then_smaller(ctx):
    """Call 1: 40 traces (several 4,096-step chunks each, ragged tails) with
    a grid config per trace and decision bytes.  Call 2: a smaller batch with
    one config and no decision bytes.  Each against magus_replay."""
    grid = synth.sweep_grid()
    rng = np.random.default_rng(11)
    big = mixed(1, list(rng.integers(1, 30000, size=40)) + [4096, 4097, 8192, 0, 63])
    sm, om = synth.make_batch(big)
    cot = rng.integers(0, len(grid), size=len(big)).astype(np.uint32)
    s, o, c = to_dev(sm, om, cot)
    want_r, want_l = ctx.replay(s, o, grid, c, levels=True)
    ctx.check()
    rc, got_r, got_l, st = noalloc(s, o, grid, c, levels=True)
    assert rc == magus.OK, magus.load().magus_last_error()
    assert int(st.item()) == 0
    assert (results_np(got_r) == results_np(want_r)).all()
    gl, wl = got_l.cpu().numpy(), want_l.cpu().numpy()
    assert (gl == wl).all(), describe_mismatch(gl, wl, om)

    small = mixed(2, [5000, 123, 70000, 2])
    ss, os_ = synth.make_batch(small)
    s2, o2, _ = to_dev(ss, os_)
    want2, _ = ctx.replay(s2, o2, [default_config()])
    ctx.check()
    rc, got2, _, st2 = noalloc(s2, o2, [default_config()])
    assert rc == magus.OK, magus.load().magus_last_error()
    assert int(st2.item()) == 0
    assert (results_np(got2) == results_np(want2)).all()


def test_noalloc_empty_and_rejected_batches(ctx):
    import torch
    s, o, _ = to_dev(*synth.make_batch(mixed(3, [100, 100])))
    # no traces: a clean status, nothing else
    empty_o = torch.zeros(1, dtype=torch.int64, device="cuda")
    rc, _, _, st = noalloc(s, empty_o, [default_config()])
    assert rc == magus.OK and int(st.item()) == 0
    # offsets not monotone: reported in the status word, results untouched
    bad = torch.tensor([0, 150, 100], dtype=torch.int64, device="cuda")
    rc, res, _, st = noalloc(s, bad, [default_config()])
    assert rc == magus.OK
    assert int(st.item()) == magus.DATA_OFFSETS
    assert (res.cpu().numpy() == -1).all()
    cot = torch.tensor([0, 5], dtype=torch.int32, device="cuda")
    rc, res, _, st = noalloc(s, o, [default_config()], cot=cot)
    assert rc == magus.OK and int(st.item()) == magus.DATA_CFG_INDEX
    assert (res.cpu().numpy() == -1).all()
    # the next good call runs and reports a clean status
    want, _ = ctx.replay(s, o, [default_config()])
    ctx.check()
    rc, got, _, st = noalloc(s, o, [default_config()])
    assert rc == magus.OK and int(st.item()) == 0
    assert (results_np(got) == results_np(want)).all()
    # stepped configs are refused before anything runs
    rc, res, _, _ = noalloc(s, o, [default_config(up_step=2)])
    assert rc == magus.EINVAL
    assert (res.cpu().numpy() == -1).all()


def test_noalloc_bulk_batch_fits_and_matches(ctx):
    """The 4,096 x 100,000 bulk batch (the benchmark's) fits the fixed
    scratch and gives magus_replay's results."""
    sm, om = synth.workload_bulk()
    s, o, _ = to_dev(sm, om)
    want, _ = ctx.replay(s, o, [default_config()])
    ctx.check()
    rc, got, _, st = noalloc(s, o, [default_config()])
    assert rc == magus.OK, magus.load().magus_last_error()
    assert int(st.item()) == 0
    assert (results_np(got) == results_np(want)).all()
