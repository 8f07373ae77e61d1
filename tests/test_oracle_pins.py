"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: they use hand-derived closed
forms, the paper's worked example of the 0.6 threshold (Sec. 3.2), invariants
of the decision rule, scale invariance of the relative derivative, and brute
force against an exact-rational transliteration of Alg. 1 / Alg. 2.
"""
import itertools
import os

import numpy as np
import pytest

import synth
from synth import default_config
from tests import exact_reference as ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MAX = 16


def run(oracle_mod, x, cfg):
    res, b = oracle_mod.replay_trace(np.asarray(x, dtype=np.uint32), cfg)
    lv, hi, pr = oracle_mod.decode(b)
    return res, lv, hi, pr


# ---------------------------------------------------------------- P1, P2

@pytest.mark.parametrize("value", [0, 1, 777, 65536, 2**32 - 1])
@pytest.mark.parametrize("window,hold", [(2, 1), (4, 10), (16, 16), (32, 32)])
def test_constant_trace_never_moves(oracle_mod, value, window, hold):
    """Zero derivative: no prediction, no event, the node stays idle at the minimum."""
    cfg = default_config(window=window, hold=hold)
    res, lv, hi, pr = run(oracle_mod, [value] * 300, cfg)
    assert res == dict(score=0, level_sum=0, transitions=0, ticks_high=0)
    assert (pr == 0).all() and (hi == 0).all() and (lv == 0).all()


def test_constant_trace_keeps_a_non_minimal_initial_level(oracle_mod):
    cfg = default_config(level_init=7)
    res, lv, _, _ = run(oracle_mod, [5000] * 50, cfg)
    assert (lv == 7).all()
    assert res["level_sum"] == 7 * 50 and res["transitions"] == 0


@pytest.mark.parametrize("window", [2, 4, 9, 32])
def test_shorter_than_window_is_warm_up(oracle_mod, window):
    """Until the FIFO holds direv_length samples there is no prediction."""
    x = [1, 1000000, 3, 4000000, 0, 7, 1, 9, 100, 1, 10**9] * 3
    x = x[:window - 1]
    res, lv, hi, pr = run(oracle_mod, x, default_config(window=window, hold=1))
    assert res["score"] == 0 and (pr == 0).all() and (hi == 0).all()


# ---------------------------------------------------------------- P3

@pytest.mark.parametrize("window", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("s", [1, 40, 99])
def test_clean_step_up(oracle_mod, window, s):
    """10,000 -> 20,000 at tick s: r = 10000/(W*10000) = 1/W > 0.1, so the
    prediction is +1 on ticks s..s+W-2 (while the old sample is still in the
    FIFO); W-1 <= 5 events never reach 6 of 10, so no high state; the level
    jumps to MAX at s (detection delay 0) and stays: score 16(n-s) + 1000."""
    n = 100
    x = [10000] * s + [20000] * (n - s)
    res, lv, hi, pr = run(oracle_mod, x, default_config(window=window))
    expect_pred = np.zeros(n, dtype=np.int64)
    expect_pred[s:min(n, s + window - 1)] = 1
    if s < window - 1:                 # step inside the warm-up
        expect_pred[:window - 1] = 0
        expect_pred[window - 1:s + window - 1] = 1
    assert (pr == expect_pred).all()
    first = int(np.argmax(expect_pred != 0))
    assert (lv[:first] == 0).all() and (lv[first:] == MAX).all()
    assert res["transitions"] == 1 and res["ticks_high"] == 0
    assert res["score"] == 16 * (n - first) + 1000


def test_clean_step_down_goes_straight_to_the_lower_bound(oracle_mod):
    """Sec. 6.1: a decrease goes directly to the lower bound."""
    x = [10000] * 10 + [20000] * 30 + [5000] * 30
    res, lv, _, pr = run(oracle_mod, x, default_config())
    assert lv[10] == MAX and (lv[10:40] == MAX).all()
    assert pr[40] == -1 and (lv[40:] == 0).all()
    assert res["transitions"] == 2
    assert res["score"] == 16 * 30 + 2000


# ---------------------------------------------------------------- P4

def test_q16_boundary_is_strict_and_disagrees_with_fp64(oracle_mod):
    """65,536 -> 91,752 at W = 4: r = 26216 / 262144 = 6554/65536 exactly, which
    is inc_q; '>' is strict so no event.  91,753 fires.  In FP64 with the
    decimal threshold 0.1, r = 0.100006103515625 > 0.1 does fire."""
    cfg = default_config()
    r0, _ = oracle_mod.replay_trace(np.array([65536] * 4 + [91752] * 4, np.uint32), cfg)
    r1, _ = oracle_mod.replay_trace(np.array([65536] * 4 + [91753] * 4, np.uint32), cfg)
    f0, _ = oracle_mod.replay_trace_fp64(np.array([65536] * 4 + [91752] * 4, np.uint32),
                                         cfg, 0.1, -0.1)
    assert r0["score"] == 0
    assert r1["score"] == 16 * 4 + 1000
    assert f0["score"] == 16 * 4 + 1000


def test_q16_boundary_downward(oracle_mod):
    """Down: a*65536 > b*(65536 + W*|dec|).  b = 65536, W = 4, dec = -6554:
    the boundary a = 65536 + 26216 = 91752 gives no event, 91753 does."""
    cfg = default_config()
    r0, _ = oracle_mod.replay_trace(np.array([91752] * 4 + [65536] * 4, np.uint32), cfg)
    r1, b1 = oracle_mod.replay_trace(np.array([91753] * 4 + [65536] * 4, np.uint32), cfg)
    assert r0["score"] == 0
    _, _, pr = oracle_mod.decode(b1)
    assert list(pr[4:7]) == [-1, -1, -1] and r1["score"] == 0   # already at MIN


# ---------------------------------------------------------------- P5 (paper example)

def _events_trace(event_ticks, n, lo=10000, hi=20000):
    """W = 2 trace with a prediction event exactly at the given ticks."""
    v, x, ev = lo, [], set(event_ticks)
    for t in range(n):
        if t in ev:
            v = hi if v == lo else lo
        x.append(v)
    return x


def test_high_frequency_example_of_section_3_2(oracle_mod):
    rows = [tuple(int(v) for v in ln.split()) for ln in
            open(os.path.join(GOLDEN, "high_freq_example.txt")) if ln.strip() and ln[0] != "#"]
    for H, k, expect in rows:
        cfg = default_config(window=2, hold=H)
        ev = list(range(30, 30 + k))
        x = _events_trace(ev, 60)
        _, _, hi, pr = run(oracle_mod, x, cfg)
        assert (pr[ev] != 0).all() and (np.delete(pr, ev) == 0).all()
        # the window ending at the last event holds exactly k events
        t_last = 30 + k - 1 if k else 45
        assert hi[t_last] == expect, (H, k)
        assert hi.max() == expect


# ---------------------------------------------------------------- P6

def test_hold_one_locks_at_first_event(oracle_mod):
    """H = 1: the event rate is the current flag, so any event is 'high' and
    forces MAX; a -1 is never executed."""
    x = [30000] * 20 + [10000] * 20 + [40000] * 20 + [9000] * 20
    res, lv, hi, pr = run(oracle_mod, x, default_config(hold=1))
    assert ((pr != 0) == (hi == 1)).all()
    first = int(np.argmax(pr != 0))
    assert pr[first] == -1                 # the first event is a decrease ...
    assert (lv[:first] == 0).all() and (lv[first:] == MAX).all()   # ... yet MAX
    assert res["transitions"] == 1


def test_zero_high_freq_threshold_is_always_high(oracle_mod):
    """Alg. 2 with high_freq_threshold = 0: freq >= 0 holds at every step, so the
    node leaves its idle minimum on the very first step and never comes back:
    n ticks at MAX and one transition (the one out of the idle level)."""
    x = [10000, 50000, 1000, 2000] * 25
    res, lv, hi, _ = run(oracle_mod, x, default_config(hf_num=0))
    assert (hi == 1).all() and (lv == MAX).all()
    assert res == dict(score=16 * 100 + 1000, level_sum=1600, transitions=1, ticks_high=100)


# ---------------------------------------------------------------- P7, P8

def test_stuck_at_max_after_a_long_fall(oracle_mod):
    """W = 16, H = 10, 40,000 -> 10,000 at s = 40: r = -30000/(16*10000) =
    -0.1875 < -0.1 on ticks 40..54 (15 events).  The 6th event (t = 45) is
    high -> MAX; after the events stop the prediction is 0 and the level is
    kept: MAX for ever.  score = 16 * (100 - 45) + 1000 = 1880."""
    x = [40000] * 40 + [10000] * 60
    res, lv, hi, pr = run(oracle_mod, x, default_config(window=16))
    assert (pr[40:55] == -1).all() and (pr[55:] == 0).all()
    assert (lv[:45] == 0).all() and (lv[45:] == MAX).all()
    assert list(np.nonzero(hi)[0]) == list(range(45, 59))
    assert res == dict(score=1880, level_sum=880, transitions=1, ticks_high=14)


def test_alternation_locks_at_max(oracle_mod):
    """W = 2 alternating 10,000 / 20,000, low first: +1 on odd ticks, -1 on even
    ticks >= 2.  Levels MAX/MIN alternate on t = 1..5 (5 transitions), the 6th
    event (t = 6) is high and the level stays MAX (Sec. 3.2 / Sec. 6.3 lock).
    97 ticks at MAX: score = 16 * 97 + 5 * 1000 = 6552."""
    x = [10000, 20000] * 50
    res, lv, hi, pr = run(oracle_mod, x, default_config(window=2))
    assert list(lv[:7]) == [0, MAX, 0, MAX, 0, MAX, MAX]
    assert (lv[6:] == MAX).all() and (hi[6:] == 1).all() and (hi[:6] == 0).all()
    assert res == dict(score=6552, level_sum=1552, transitions=5, ticks_high=94)


def test_events_still_logged_while_high(oracle_mod):
    """Sec. 3.2: predictions keep being logged while high; the high state ends
    once fewer than 6 of the last 10 steps had an event."""
    x = [10000, 20000] * 10 + [20000] * 30
    _, lv, hi, pr = run(oracle_mod, x, default_config(window=2))
    assert (pr[1:20] != 0).all()
    # events on ticks 1..19; the window 14..23 holds 6 of them, 15..24 only 5
    assert hi[19] == 1 and hi[23] == 1 and hi[24] == 0 and (hi[24:] == 0).all()
    assert (lv[6:] == MAX).all()


# ---------------------------------------------------------------- P9

@pytest.mark.parametrize("c", [2, 3, 7, 1000])
def test_relative_derivative_is_scale_invariant(oracle_mod, c):
    """Multiplying every sample by c leaves (b-a)/(W min(a,b)) unchanged."""
    key = synth.stream_key(99, c)
    x = synth.geometric_phase_trace(3000, key, mean=20.0, short_prob=0.2,
                                    median=1000.0)
    x = np.minimum(x, (2**32 - 1) // c).astype(np.uint32)
    for cfg in (default_config(), synth.sweep_config(7777), synth.sweep_config(1234)):
        a = oracle_mod.replay_trace(x, cfg)[1]
        b = oracle_mod.replay_trace(x * np.uint32(c), cfg)[1]
        assert (a == b).all()


def test_up_by_k_and_down_by_k_are_symmetric(oracle_mod):
    """min() as the base: x -> kx and kx -> x give the same |r|."""
    for k in (1.5, 2.0, 3.0):
        base = 12345
        up = [base] * 8 + [int(base * k)] * 8
        dn = [int(base * k)] * 8 + [base] * 8
        for q in (1000, 8000, 20000, 60000):
            cfg = default_config(inc_q16=q, dec_q16=-q)
            _, _, _, pu = run(oracle_mod, up, cfg)
            _, _, _, pd = run(oracle_mod, dn, cfg)
            assert ((pu == 1) == (pd == -1)).all()


# ---------------------------------------------------------------- invariants

def _random_traces(n_traces=40, n=2000):
    out = []
    for i in range(n_traces):
        key = synth.stream_key(1234, i)
        if i % 2:
            out.append(synth.geometric_phase_trace(n, key, mean=15.0, short_prob=0.3))
        else:
            out.append(synth.four_phase_trace(n, key))
    return out


@pytest.mark.parametrize("cfg_index", [0, 1, 300, 4095, 4096 + 77, 8191, 12000, 16383])
def test_decision_rule_invariants(oracle_mod, cfg_index):
    cfg = synth.sweep_config(cfg_index)
    for x in _random_traces(12, 1500):
        res, lv, hi, pr = run(oracle_mod, x, cfg)
        assert set(np.unique(lv)) <= {0, MAX}
        assert (lv[hi == 1] == MAX).all()                 # high -> MAX
        assert (lv[pr == 1] == MAX).all()                 # +1 -> MAX
        assert (lv[(pr == -1) & (hi == 0)] == 0).all()    # executed -1 -> MIN
        keep = (pr == 0) & (hi == 0)
        prev = np.concatenate([[cfg["level_init"]], lv[:-1]])
        assert (lv[keep] == prev[keep]).all()             # 0 keeps the level
        assert res["level_sum"] == int(lv.sum())
        assert res["transitions"] == int((lv != prev).sum())
        assert res["ticks_high"] == int(hi.sum())
        assert res["score"] == res["level_sum"] + 1000 * res["transitions"]
        assert (pr[:cfg["window"] - 1] == 0).all()


def test_batch_and_sweep_agree_with_single_traces(oracle_mod):
    traces = _random_traces(10, 700) + [np.zeros(0, np.uint32), np.array([5], np.uint32)]
    samples, offsets = synth.make_batch(traces)
    cfgs = [synth.sweep_config(i) for i in (3, 999, 5000, 9000, 16000)]
    cot = np.arange(len(traces), dtype=np.uint32) % len(cfgs)
    res, b = oracle_mod.replay_batch(samples, offsets, cfgs, cot, want_bytes=True)
    scores, argmin = oracle_mod.sweep(samples, offsets, cfgs)
    for t, x in enumerate(traces):
        r, bb = oracle_mod.replay_trace(x, cfgs[cot[t]])
        assert list(res[t]) == [r["score"], r["level_sum"], r["transitions"], r["ticks_high"]]
        assert (b[int(offsets[t]):int(offsets[t + 1])] == bb).all()
        s = [oracle_mod.replay_trace(x, c, want_bytes=False)[0]["score"] for c in cfgs]
        assert list(scores[t]) == s
        assert argmin[t] == int(np.argmin(s))             # lowest index among ties


def test_invalid_configs_are_rejected(oracle_mod):
    good = default_config()
    assert oracle_mod.config_valid(good)
    for bad in (dict(window=1), dict(window=33), dict(hold=0), dict(hold=33),
                dict(inc_q16=-1), dict(dec_q16=1), dict(inc_q16=2**20 + 1),
                dict(hf_den=0), dict(hf_num=6, hf_den=5), dict(level_min=16, level_max=16),
                dict(level_max=32), dict(level_init=17)):
        assert not oracle_mod.config_valid(default_config(**bad)), bad


# ---------------------------------------------------------------- FP64 side-form

def test_fp64_side_form_agrees_away_from_boundaries(oracle_mod):
    """Decimal thresholds in FP64 vs Q16.16: decisions agree except where a
    derivative falls between v and its Q16.16 rounding."""
    for x in _random_traces(10, 3000):
        for v in (0.1, 0.25, 0.5):
            q = synth.threshold_q16(v)
            cfg = default_config(inc_q16=q, dec_q16=-q)
            _, be = oracle_mod.replay_trace(x, cfg)
            _, bf = oracle_mod.replay_trace_fp64(x, cfg, v, -v)
            if q / 65536 == v:
                assert (be == bf).all()
            else:
                assert np.mean(be != bf) < 0.01


# ---------------------------------------------------------------- P12 brute force

def _brute_traces():
    out = []
    for n in range(1, 6):
        out.extend(itertools.product(range(5), repeat=n))
    return out


def test_brute_force_against_exact_rational_transliteration(oracle_mod):
    """All traces over {0..4} of length <= 5, W in {2,3,4}, H in {1,2,3,5},
    thresholds including exact-equality cases (e.g. 1 -> 2 at W = 4 gives
    r = 1/4 = 16384/65536), against the Fraction-based Alg. 1 / Alg. 2."""
    traces = _brute_traces()
    samples, offsets = synth.make_batch([np.array(t, np.uint32) for t in traces])
    incs = (0, 1, 16384, 32768, 65536)
    decs = (0, -16384, -32768)
    checked = 0
    for W, H, inc, dec in itertools.product((2, 3, 4), (1, 2, 3, 5), incs, decs):
        cfg = default_config(window=W, hold=H, inc_q16=inc, dec_q16=dec)
        res, b = oracle_mod.replay_batch(samples, offsets, [cfg], want_bytes=True)
        for i, t in enumerate(traces):
            steps, score, ls, tr, th = ref.run(t, cfg)
            got = b[int(offsets[i]):int(offsets[i + 1])].tobytes()
            if got != ref.encode(steps) or list(res[i]) != [score, ls, tr, th]:
                raise AssertionError(f"mismatch W={W} H={H} inc={inc} dec={dec} trace={t}")
            checked += 1
    assert checked == len(traces) * 3 * 4 * len(incs) * len(decs)


def _tree_bytes(cfg):
    return ref.run_tree(range(5), 7, cfg)


def test_brute_force_length_seven_every_prefix(oracle_mod):
    """All 78,125 traces over {0..4} of length 7 -- and so, step by step,
    every trace of length <= 7, the controller being causal -- for W in
    {2,3,4}, H in {1,2,3,5} and threshold pairs with exact-equality cases,
    per-step decision bytes against the Fraction transliteration walked as a
    prefix tree (host processes in parallel)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    traces = np.array(list(itertools.product(range(5), repeat=7)), np.uint32)
    samples = traces.ravel()
    offsets = np.arange(0, len(samples) + 1, 7, dtype=np.uint64)
    pairs = ((0, 0), (1, -1), (16384, -16384), (32768, -32768), (65536, -65536),
             (0, -65536), (65536, 0), (16384, -32768))
    cfgs = [default_config(window=W, hold=H, inc_q16=i, dec_q16=d)
            for W, H, (i, d) in itertools.product((2, 3, 4), (1, 2, 3, 5), pairs)]
    workers = max(1, min(8, len(os.sched_getaffinity(0))))
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as pool:
        for cfg, tree in zip(cfgs, pool.map(_tree_bytes, cfgs)):
            _, b = oracle_mod.replay_batch(samples, offsets, [cfg], want_bytes=True)
            b = b.reshape(-1, 7)
            bad = np.nonzero((b != tree).any(axis=1))[0]
            assert len(bad) == 0, (cfg, traces[bad[0]].tolist())


def test_brute_force_hf_threshold_and_levels(oracle_mod):
    """Other high_freq_threshold fractions and ladders, against the transliteration."""
    traces = [t for t in _brute_traces() if len(t) >= 3]
    rng = np.random.default_rng(5)
    for _ in range(60):
        lmin = int(rng.integers(0, 10))
        lmax = int(rng.integers(lmin + 1, 32))
        den = int(rng.integers(1, 8))
        cfg = default_config(window=int(rng.integers(2, 5)), hold=int(rng.integers(1, 7)),
                             inc_q16=int(rng.choice([0, 9000, 16384, 40000])),
                             dec_q16=-int(rng.choice([0, 9000, 16384, 40000])),
                             hf_num=int(rng.integers(0, den + 1)), hf_den=den,
                             level_min=lmin, level_max=lmax,
                             level_init=int(rng.integers(lmin, lmax + 1)))
        for t in traces[::7]:
            steps, score, ls, tr, th = ref.run(t, cfg)
            r, b = oracle_mod.replay_trace(np.array(t, np.uint32), cfg)
            assert b.tobytes() == ref.encode(steps)
            assert [r["score"], r["level_sum"], r["transitions"], r["ticks_high"]] == \
                [score, ls, tr, th]


def test_large_values_against_transliteration(oracle_mod):
    """Random 32-bit samples incl. 0 and 2^32-1 (64-bit products near the top)."""
    rng = np.random.default_rng(11)
    for _ in range(30):
        n = 40
        x = rng.integers(0, 2**32, size=n, dtype=np.uint64)
        x[rng.integers(0, n, 5)] = 0
        x[rng.integers(0, n, 5)] = 2**32 - 1
        x[rng.integers(0, n, 5)] = 1
        for W, q in ((2, 2**20), (32, 2**20), (7, 1), (3, 12345)):
            cfg = default_config(window=W, hold=3, inc_q16=q, dec_q16=-q)
            steps, score, *_ = ref.run([int(v) for v in x], cfg)
            r, b = oracle_mod.replay_trace(x.astype(np.uint32), cfg)
            assert b.tobytes() == ref.encode(steps) and r["score"] == score


# ---------------------------------------------------------------- stepped actuation

def _doubling(n, start=1000):
    return [start * 2 ** k for k in range(n)]


@pytest.mark.parametrize("u", [1, 3, 5])
def test_stepped_staircase(oracle_mod, u):
    """W = 2 on a trace that doubles every step: r = 1/2 > 0.1, so every step
    after the first predicts +1.  With H = 32 and threshold 1/1 the high state
    needs 32 events and never comes within 20 steps; each executed +1 raises
    the level by u rungs, clamped at 16: level(t) = min(u t, 16)."""
    cfg = default_config(window=2, hold=32, hf_num=1, hf_den=1, up_step=u)
    n = 20
    res, lv, hi, pr = run(oracle_mod, _doubling(n), cfg)
    assert (hi == 0).all() and (pr[1:] == 1).all()
    want = [min(u * t, 16) for t in range(n)]
    assert list(lv) == want
    assert res["level_sum"] == sum(want)
    assert res["transitions"] == sum(1 for t in range(1, n) if want[t] != want[t - 1])


@pytest.mark.parametrize("d", [2, 4])
def test_stepped_descent(oracle_mod, d):
    """Starting at the top (level_init = 16) on a trace that halves every step:
    every step after the first predicts -1 and the level falls by d rungs,
    clamped at 0: level(t) = max(16 - d t, 0)."""
    cfg = default_config(window=2, hold=32, hf_num=1, hf_den=1, down_step=d, level_init=16)
    n = 20
    x = [2 ** (30 - k) for k in range(n)]
    res, lv, hi, pr = run(oracle_mod, x, cfg)
    assert (pr[1:] == -1).all()
    assert list(lv) == [max(16 - d * t, 0) for t in range(n)]


def test_stepped_high_state_still_locks_at_max(oracle_mod):
    """Stepped actuation does not soften the Sec. 3.2 lock: 6 of 10 events go
    straight to 16 whatever the step size."""
    cfg = default_config(window=2, up_step=1, down_step=1)
    res, lv, hi, pr = run(oracle_mod, [10000, 20000] * 20, cfg)
    assert list(lv[:7]) == [0, 1, 0, 1, 0, 1, 16] and (lv[6:] == 16).all()


def test_brute_force_stepped_actuation(oracle_mod):
    """Stepped configs against the exact-rational transliteration."""
    traces = [t for n in range(1, 7) for t in itertools.product((0, 1, 3, 4), repeat=n)]
    rng = np.random.default_rng(21)
    for _ in range(40):
        lmin = int(rng.integers(0, 6))
        lmax = int(rng.integers(lmin + 1, 20))
        cfg = default_config(window=int(rng.integers(2, 4)), hold=int(rng.integers(1, 8)),
                             inc_q16=int(rng.choice([0, 16384, 40000])),
                             dec_q16=-int(rng.choice([0, 16384, 40000])),
                             hf_num=int(rng.integers(1, 6)), hf_den=5,
                             level_min=lmin, level_max=lmax,
                             level_init=int(rng.integers(lmin, lmax + 1)),
                             up_step=int(rng.integers(0, 5)), down_step=int(rng.integers(0, 5)))
        for t in traces[::5]:
            steps, score, ls, tr, th = ref.run(t, cfg)
            r, b = oracle_mod.replay_trace(np.array(t, np.uint32), cfg)
            assert b.tobytes() == ref.encode(steps), (cfg, t)
            assert [r["score"], r["level_sum"], r["transitions"], r["ticks_high"]] == \
                [score, ls, tr, th]


# ---------------------------------------------------------------- derivative base variants

def test_oldest_sample_base_bounds_falls(oracle_mod):
    """With the oldest sample as the base a fall can never go below -1/W: the
    W = 16 fall 40,000 -> 10,000 gives r = -30000 / (16 * 40000) = -0.047,
    above dec = -0.1, so nothing happens (the min base gives -0.1875, see the
    stuck-at-max pin)."""
    x = [40000] * 40 + [10000] * 60
    res, lv, hi, pr = run(oracle_mod, x, default_config(window=16, base=1))
    assert (pr == 0).all() and res["score"] == 0
    # ... while a rise by the same factor, r = 30000 / (16 * 10000) = 0.1875, fires
    res, lv, hi, pr = run(oracle_mod, x[::-1], default_config(window=16, base=1))
    assert (pr[60:75] == 1).all()


def test_newest_sample_base_bounds_rises(oracle_mod):
    """With the newest sample as the base a rise stays below 1/W: at W = 16,
    10,000 -> 40,000 gives r = 0.047 < 0.1 (no event); the fall fires."""
    x = [10000] * 40 + [40000] * 60
    res, _, _, pr = run(oracle_mod, x, default_config(window=16, base=2))
    assert (pr == 0).all() and res["score"] == 0
    _, _, _, pr = run(oracle_mod, x[::-1], default_config(window=16, base=2))
    assert (pr[60:75] == -1).all()


def test_brute_force_base_variants(oracle_mod):
    traces = [t for n in range(1, 6) for t in itertools.product(range(5), repeat=n)]
    for which in (1, 2):
        for W, inc, dec in itertools.product((2, 3, 4), (0, 16384, 32768), (0, -16384)):
            cfg = default_config(window=W, hold=3, inc_q16=inc, dec_q16=dec, base=which)
            for t in traces[::3]:
                steps, score, *_ = ref.run(t, cfg)
                r, b = oracle_mod.replay_trace(np.array(t, np.uint32), cfg)
                assert b.tobytes() == ref.encode(steps), (which, W, inc, dec, t)


# ------------------------------------------- fixed reference base (base 3)

def test_fixed_reference_closed_form(oracle_mod):
    """Base 3: r = (b - a) / (W B_ref).  With W = 4, B_ref = 10,000 and
    inc = dec magnitude = 6554/2^16, a step of size D fires iff
    D 2^16 > 6554 * 4 * 10,000 = 262,160,000, i.e. iff D >= 4001
    (4001 * 65536 = 262,209,536; 4000 * 65536 = 262,144,000), whatever the
    level it starts from.  A clean step up at s = 40 of n = 100 then gives
    W-1 steps of +1 from s, score 16 (n - s) + 1000 = 1960."""
    cfg = default_config(base=3, base_ref=10000)
    for lo in (0, 10000, 300000, 2**32 - 4002):
        res, lv, hi, pr = run(oracle_mod, [lo] * 40 + [lo + 4001] * 60, cfg)
        assert (pr[40:43] == 1).all() and (pr[:40] == 0).all() and (pr[43:] == 0).all(), lo
        assert res["score"] == 1960 and res["transitions"] == 1, lo
        res, _, _, pr = run(oracle_mod, [lo] * 40 + [lo + 4000] * 60, cfg)
        assert res["score"] == 0 and (pr == 0).all(), lo
        # the same step down goes to the minimum from level_init = 16
        res, lv, _, pr = run(oracle_mod, [lo + 4001] * 40 + [lo] * 60,
                             default_config(base=3, base_ref=10000, level_init=16))
        assert (pr[40:43] == -1).all() and (lv[:40] == 16).all() and (lv[40:] == 0).all(), lo
        res, lv, _, pr = run(oracle_mod, [lo + 4000] * 40 + [lo] * 60,
                             default_config(base=3, base_ref=10000, level_init=16))
        assert (pr == 0).all() and (lv == 16).all(), lo


def test_fixed_reference_one_is_the_listings_absolute_derivative(oracle_mod):
    """B_ref = 1 makes r = (newest - oldest) / direv_length, Alg. 1's own
    formula in MB/s per step.  Against that formula evaluated directly with
    exact rationals on random steps (thresholds q/2^16 up to the 2^20 = 16
    MB/s per step the config allows)."""
    from fractions import Fraction
    rng = np.random.default_rng(31)
    for _ in range(300):
        W = int(rng.integers(2, 33))
        q = int(rng.integers(0, 2**20 + 1))
        a = int(rng.integers(0, 2**32 - 1000))
        d = int(rng.integers(0, 600))
        cfg = default_config(window=W, hold=1, inc_q16=q, dec_q16=-q, base=3, base_ref=1)
        for x in ([a] * W + [a + d] * W, [a + d] * W + [a] * W):
            _, _, _, pr = run(oracle_mod, x, cfg)
            for t in range(W - 1, len(x)):
                derivative = Fraction(x[t] - x[t - W + 1], W)
                want = 1 if derivative > Fraction(q, 65536) else \
                    -1 if derivative < Fraction(-q, 65536) else 0
                assert pr[t] == want, (W, q, a, d, t)


def test_fixed_reference_is_not_scale_invariant(oracle_mod):
    """Unlike the relative bases, scaling the samples changes base 3's
    decisions: the 4,001 MB/s step fires at B_ref = 10,000, half of it does
    not (while the min base gives the same bytes for both)."""
    x = np.array([10000] * 40 + [14002] * 60, np.uint64)
    c3 = default_config(base=3, base_ref=10000)
    r1, _ = oracle_mod.replay_trace(x.astype(np.uint32), c3)
    r2, _ = oracle_mod.replay_trace((x // 2).astype(np.uint32), c3)
    assert r1["transitions"] == 1 and r2["transitions"] == 0
    c0 = default_config(base=0)
    _, b1 = oracle_mod.replay_trace(x.astype(np.uint32), c0)
    _, b2 = oracle_mod.replay_trace((x // 2).astype(np.uint32), c0)
    assert (b1 == b2).all()


def test_fixed_reference_q16_and_fp64_disagree_at_the_boundary(oracle_mod):
    """W = 4, B_ref = 100,000: the step 40,001 gives r = 0.1000025, above the
    decimal 0.1 (the FP64 side-form fires) but not above 6554/2^16 =
    0.100006103515625 (the exact form does not); 40,003 fires in both."""
    cfg = default_config(base=3, base_ref=100000)
    for d, exact, fp in ((40001, 0, 1), (40002, 0, 1), (40003, 1, 1)):
        x = np.array([50000] * 10 + [50000 + d] * 10, np.uint32)
        _, be = oracle_mod.replay_trace(x, cfg)
        _, bf = oracle_mod.replay_trace_fp64(x, cfg, 0.1, -0.1)
        assert int(((be >> 6) == 2).any()) == exact, d
        assert int(((bf >> 6) == 2).any()) == fp, d


def test_fixed_reference_validation(oracle_mod):
    assert oracle_mod.config_valid(default_config(base=3, base_ref=1))
    assert not oracle_mod.config_valid(default_config(base=3, base_ref=0))
    assert not oracle_mod.config_valid(default_config(base=4, base_ref=1))


def test_brute_force_fixed_reference(oracle_mod):
    """Base 3 against the Fraction transliteration on every trace over {0..4}
    of length <= 5, B_ref in {1, 2, 3}: equality cases included (W = 4,
    B_ref = 1, a step of 1 gives r = 1/4 = 16384/2^16, no event)."""
    traces = [t for n in range(1, 6) for t in itertools.product(range(5), repeat=n)]
    for bref in (1, 2, 3):
        for W, inc, dec in itertools.product((2, 3, 4), (0, 16384, 32768), (0, -16384)):
            cfg = default_config(window=W, hold=3, inc_q16=inc, dec_q16=dec, base=3,
                                 base_ref=bref)
            for t in traces[::3]:
                steps, score, *_ = ref.run(t, cfg)
                r, b = oracle_mod.replay_trace(np.array(t, np.uint32), cfg)
                assert b.tobytes() == ref.encode(steps), (bref, W, inc, dec, t)
                assert r["score"] == score


# ---------------------------------------------------------------- monitor front end

def test_counters_constant_rate(oracle_mod):
    """1,000,000 bytes every 100 ms = 10 MB/s; 64-byte counts scale by 64."""
    ts = np.arange(50, dtype=np.uint64) * 100_000_000
    c = np.arange(50, dtype=np.uint64) * 1_000_000
    assert (oracle_mod.counters_to_mbps(c, ts, 48, 1) == 10).all()
    assert (oracle_mod.counters_to_mbps(c, ts, 48, 64) == 640).all()


def test_counters_wrap_zero_interval_and_saturation(oracle_mod):
    ts = np.array([0, 100, 200, 200, 300], np.uint64)
    c = np.array([2**32 - 10, 5, 20, 30, 2**31], np.uint64)
    out = oracle_mod.counters_to_mbps(c, ts, 32, 1)
    # 15 B / 100 ns = 150 MB/s across the 32-bit wrap; 15 B / 100 ns; dt = 0 -> 0;
    # ~2^31 B / 100 ns saturates
    assert list(out) == [150, 150, 0, 2**32 - 1]


def test_counters_against_exact_rationals(oracle_mod):
    from fractions import Fraction
    rng = np.random.default_rng(3)
    for bits in (16, 32, 48, 64):
        n = 200
        ts = np.cumsum(rng.integers(0, 10**9, n, dtype=np.uint64)).astype(np.uint64)
        c = rng.integers(0, 2**63, n, dtype=np.uint64)
        if bits < 64:
            c &= np.uint64((1 << bits) - 1)
        for bpc in (1, 64):
            out = oracle_mod.counters_to_mbps(c, ts, bits, bpc)
            for i in range(n - 1):
                d = (int(c[i + 1]) - int(c[i])) % (1 << bits)
                dt = int(ts[i + 1]) - int(ts[i])
                want = 0 if dt == 0 else min(int(Fraction(d * bpc * 1000, dt)), 2**32 - 1)
                assert out[i] == want, (bits, bpc, i)


# ------------------------------------------------ per-interval invocation form

def test_stream_steps_equal_trace_replay(oracle_mod):
    """Stepping streams one sample per tick (interleaved, one invocation per
    interval) gives the same decision bytes and results as replaying each
    trace whole."""
    rng = np.random.default_rng(12)
    grid = synth.sweep_grid()
    cfgs = [grid[int(i)] for i in rng.integers(0, len(grid), 5)] + \
        [default_config(up_step=2, down_step=1, base=1)]
    n_streams = 40
    cot = rng.integers(0, len(cfgs), n_streams)
    traces = [synth.geometric_phase_trace(int(rng.integers(0, 300)), synth.stream_key(77, i),
                                          mean=20.0, short_prob=0.3) for i in range(n_streams)]
    st = oracle_mod.Streams(cfgs, cot)
    got = [[] for _ in range(n_streams)]
    for k in range(max(len(x) for x in traces)):
        ids = [i for i in range(n_streams) if k < len(traces[i])]
        rng.shuffle(ids)
        b = st.tick(ids, [traces[i][k] for i in ids])
        for i, v in zip(ids, b):
            got[i].append(int(v))
    for i, x in enumerate(traces):
        r, want = oracle_mod.replay_trace(x, cfgs[int(cot[i])])
        assert bytes(got[i]) == want.tobytes(), i
        assert st.result(i) == r, i
    st.reset(3)
    assert st.result(3)["score"] == 0
