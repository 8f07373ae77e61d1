"""Serving: each stream's decisions are the same alone, in a mix with joins
and leaves, and as a plain replay of its samples by the oracle (exact)."""
import numpy as np
import pytest

import paper_2502_03796_amd as magus
import synth
from synth import default_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = magus.Context(0)
    yield c
    c.close()


def oracle_bytes(oracle_mod, x, cfg):
    r, b = oracle_mod.replay_trace(np.asarray(x, np.uint32), cfg)
    return r, b


def test_single_stream_matches_replay(ctx, oracle_mod):
    srv = magus.Server(ctx, 1 << 20)
    cfg = default_config()
    x = synth.serve_stream_samples(0, 3000)
    slot = srv.open(cfg)
    got = np.array([srv.step([slot], [v])[0] for v in x], np.uint8)
    r, want = oracle_bytes(oracle_mod, x, cfg)
    assert (got == want).all()
    assert srv.result(slot) == r
    srv.close()


def test_mix_with_joins_and_leaves_matches_alone(ctx, oracle_mod):
    """64 streams with random configs join and leave over 400 ticks; at every
    tick only a random subset of the live streams delivers a sample (jitter),
    slots are reused after leaves, and admission is bounded by a memory budget
    of 40 slots."""
    rng = np.random.default_rng(12)
    n_streams, n_ticks = 64, 400
    grid = synth.sweep_grid()
    cfgs = [grid[int(i)] for i in rng.integers(0, len(grid), n_streams)]
    data = [synth.serve_stream_samples(100 + i, n_ticks) for i in range(n_streams)]
    join = rng.integers(0, n_ticks // 2, n_streams)
    leave = np.minimum(join + rng.integers(50, n_ticks, n_streams), n_ticks)
    srv = magus.Server(ctx, 40 * magus.Server.slot_bytes())
    assert srv.capacity == 40
    slot_of = {}
    pos = np.zeros(n_streams, np.int64)      # next sample of each stream
    got = {i: [] for i in range(n_streams)}
    refused = 0
    for tick in range(n_ticks):
        for i in range(n_streams):
            if i in slot_of and leave[i] == tick:
                srv.close_stream(slot_of.pop(i))
        for i in range(n_streams):
            if i not in slot_of and join[i] <= tick < leave[i] and pos[i] == 0:
                s = srv.try_open(cfgs[i])
                if s is None:
                    refused += 1
                else:
                    slot_of[i] = s
        live = [i for i in slot_of if rng.random() < 0.8 and pos[i] < n_ticks]
        if not live:
            continue
        slots = [slot_of[i] for i in live]
        samples = [data[i][pos[i]] for i in live]
        dec = srv.step(slots, samples)
        for i, d in zip(live, dec):
            got[i].append(d)
            pos[i] += 1
    assert refused > 0                       # admission was exercised
    checked = 0
    for i in range(n_streams):
        if not got[i]:
            continue
        x = data[i][:pos[i]]
        _, want = oracle_bytes(oracle_mod, x, cfgs[i])
        assert (np.array(got[i], np.uint8) == want).all(), i
        checked += 1
    assert checked > 30
    srv.close()


def test_step_rejects_bad_pairs(ctx):
    srv = magus.Server(ctx, 4 * magus.Server.slot_bytes())
    a = srv.open(default_config())
    with pytest.raises(magus.MagusError) as ei:
        srv.step([a, a], [1, 2])
    assert ei.value.code == magus.EINVAL
    with pytest.raises(magus.MagusError):
        srv.step([3], [1])                   # not open
    for _ in range(3):
        srv.open(default_config())
    assert srv.try_open(default_config()) is None
    with pytest.raises(magus.MagusError) as ei:
        srv.open(default_config())
    assert ei.value.code == magus.ENOSLOT
    srv.close_stream(a)
    assert srv.try_open(default_config()) == a
    srv.close()


def test_reused_slot_starts_fresh(ctx, oracle_mod):
    srv = magus.Server(ctx, 1 * magus.Server.slot_bytes())
    cfg = default_config(window=2)
    a = srv.open(cfg)
    for v in [10000, 20000] * 20:
        srv.step([a], [v])
    srv.close_stream(a)
    b = srv.open(cfg)
    assert b == a
    x = [5000] * 10 + [9000] * 10
    got = np.array([srv.step([b], [v])[0] for v in x], np.uint8)
    _, want = oracle_bytes(oracle_mod, x, cfg)
    assert (got == want).all()
    srv.close()


def test_full_fleet_tick(ctx, oracle_mod):
    """65,536 streams, 20 ticks, one batched step per tick; sampled streams
    against the oracle."""
    n, ticks = 65536, 20
    srv = magus.Server(ctx, n * magus.Server.slot_bytes())
    grid = synth.sweep_grid()
    cfg_idx = (np.arange(n) * 2654435761) % len(grid)
    slots = np.array([srv.open(grid[int(c)]) for c in cfg_idx], np.uint32)
    rng = np.random.default_rng(1)
    data = rng.integers(500, 400000, size=(ticks, n)).astype(np.uint32)
    data[:, ::7] = data[0, ::7]                       # some steady streams
    out = np.zeros((ticks, n), np.uint8)
    for k in range(ticks):
        out[k] = srv.step(slots, data[k])
    for i in list(range(0, n, 4099)) + [n - 1]:
        _, want = oracle_bytes(oracle_mod, data[:, i], grid[int(cfg_idx[i])])
        assert (out[:, i] == want).all(), i
    srv.close()


def check_fleet(oracle_mod, ev, n_streams, cfg_of_stream, grid, dec):
    """Every stream's served samples, replayed alone by the oracle, give the
    decisions the fleet run produced for it in the mix."""
    is_s = ev["kind"] == synth.EV_SAMPLE
    served = is_s & (dec != 0xFF)
    checked = 0
    for sid in np.unique(ev["stream"][served]):
        m = served & (ev["stream"] == sid)
        x = ev["value"][m]
        _, want = oracle_bytes(oracle_mod, x, grid[int(cfg_of_stream[sid])])
        assert (dec[m] == want).all(), sid
        checked += 1
    return checked


def test_fleet_flat_out_with_churn_matches_oracle(ctx, oracle_mod):
    """Continuous batching under churn: 300 nodes, joins and leaves at 200/s,
    a memory budget of 310 slots (joins wait for leaves), small batches so a
    node's samples spread over many in-flight batches."""
    grid = synth.sweep_grid()
    ev, n_streams, cfg_of_stream = synth.serve_fleet_events(
        300, 80, join_rate=200.0, leave_rate=200.0)
    srv = magus.Server(ctx, 310 * magus.Server.slot_bytes())
    dec, lat, st = srv.run(ev, n_streams, grid, realtime=False, max_batch=97, depth=3)
    n_samples = int((ev["kind"] == synth.EV_SAMPLE).sum())
    assert st["samples_served"] + st["samples_dropped"] == n_samples
    assert st["joins_waited"] > 0 and st["max_in_flight"] >= 2
    assert check_fleet(oracle_mod, ev, n_streams, cfg_of_stream, grid, dec) > 300
    # batches larger than the fleet: every node queues several samples, and a
    # batch takes only the oldest of each (the rest wait for later batches).
    # Which samples are served depends on when leaves free slots, so the two
    # runs may serve different samples; each must match the oracle on its own.
    dec2, _, st2 = srv.run(ev, n_streams, grid, realtime=False, max_batch=4096, depth=2)
    assert st2["deferred"] > 0
    assert check_fleet(oracle_mod, ev, n_streams, cfg_of_stream, grid, dec2) > 300
    assert srv.open_count == 0                 # the runs closed what they opened
    srv.close()


def test_leave_then_rejoin_same_stream(ctx, oracle_mod):
    """A node leaves and joins again (another config) while its first
    session's samples are still queued: the join is held until the old slot
    closes, then admitted as a waiting join, and the new session starts from a
    fresh state; a held join withdrawn by a leave counts as refused."""
    grid = synth.sweep_grid()
    ca, cb = 5, 9001
    x1 = synth.serve_stream_samples(3, 400)
    x2 = synth.serve_stream_samples(4, 300)

    def events(t_leave, t_join, t2, withdraw=False):
        rows = [(0, synth.EV_JOIN, 0, ca, 0)]
        rows += [(1000 + 1000 * i, synth.EV_SAMPLE, 0, int(v), 0) for i, v in enumerate(x1)]
        rows += [(t_leave, synth.EV_LEAVE, 0, 0, 0), (t_join, synth.EV_JOIN, 0, cb, 0)]
        if withdraw:
            rows += [(t_join + 1, synth.EV_LEAVE, 0, 0, 0)]
        rows += [(t2 + 1000 * i, synth.EV_SAMPLE, 0, int(v), 0) for i, v in enumerate(x2)]
        return np.array(rows, dtype=magus.EVENT_DTYPE)

    _, want1 = oracle_mod.replay_trace(x1, grid[ca])
    _, want2 = oracle_mod.replay_trace(x2, grid[cb])
    srv = magus.Server(ctx, 4 * magus.Server.slot_bytes())
    s1 = np.arange(1, 401)
    # flat out: every event is ingested before the first batch retires, so
    # the join meets the draining slot; the new session's samples arrive
    # before it is admitted and are dropped
    ev = events(401_000, 401_500, 402_000)
    dec, _, st = srv.run(ev, 1, grid, realtime=False, depth=2)
    assert (dec[s1] == want1).all()
    assert st["joins_admitted"] == 1 and st["joins_waited"] == 1 and st["joins_refused"] == 0
    assert st["samples_served"] == 400 and st["samples_dropped"] == 300
    # the held join withdrawn by a leave before the slot closes
    ev = events(401_000, 401_500, 402_000, withdraw=True)
    dec, _, st = srv.run(ev, 1, grid, realtime=False, depth=2)
    assert (dec[s1] == want1).all()
    assert st["joins_admitted"] == 1 and st["joins_waited"] == 0 and st["joins_refused"] == 1
    # real time, the new session's samples 20 ms later: both sessions are
    # served whole, each from a fresh state
    ev = events(401_000, 401_500, 20_000_000)
    dec, _, st = srv.run(ev, 1, grid, realtime=True, depth=2)
    assert (dec[s1] == want1).all()
    assert (dec[len(ev) - 300:] == want2).all()
    assert st["joins_admitted"] + st["joins_waited"] == 2 and st["samples_served"] == 700
    assert srv.open_count == 0
    srv.close()


def test_fleet_stream_alone_equals_in_mix(ctx, oracle_mod):
    grid = synth.sweep_grid()
    ev, n_streams, cfg_of_stream = synth.serve_fleet_events(64, 60, join_rate=0.0,
                                                            leave_rate=0.0)
    srv = magus.Server(ctx, 64 * magus.Server.slot_bytes())
    dec_mix, _, _ = srv.run(ev, n_streams, grid, realtime=False, max_batch=50, depth=2)
    for sid in (0, 17, 63):
        alone = ev[ev["stream"] == sid]
        dec_alone, _, st = srv.run(alone, n_streams, grid, realtime=False, depth=1)
        assert st["samples_served"] == int((alone["kind"] == synth.EV_SAMPLE).sum())
        m = (ev["stream"] == sid) & (ev["kind"] == synth.EV_SAMPLE)
        assert (dec_mix[m] == dec_alone[alone["kind"] == synth.EV_SAMPLE]).all()
    srv.close()


def test_fleet_realtime_latency(ctx, oracle_mod):
    """One simulated second of 4,096 nodes in real time: every sample of an
    admitted node is served, with finite arrival-to-decision latency."""
    grid = synth.sweep_grid()
    ev, n_streams, cfg_of_stream = synth.serve_fleet_events(4096, 10)
    srv = magus.Server(ctx, (4096 + 64) * magus.Server.slot_bytes())
    dec, lat, st = srv.run(ev, n_streams, grid, realtime=True, depth=2)
    is_s = ev["kind"] == synth.EV_SAMPLE
    served = is_s & (dec != 0xFF)
    assert served.sum() == st["samples_served"] > 0.95 * is_s.sum()
    l = lat[served].astype(np.float64) * 1e-6
    assert np.isfinite(l).all() and np.percentile(l, 50) < 50.0
    check_fleet(oracle_mod, ev, n_streams, cfg_of_stream, grid, dec)
    srv.close()
