"""Pins of the oracle's proxy energy / EDP model (performance loss, package
power saving, energy saving and EDP of Sec. 5.4, for MAGUS against the
default uncore behaviour of Sec. 5.3 and a static minimum).

The model is a stated proxy (the paper measures on hardware): interval t runs
at the level set after step t-1, an interval whose demand exceeds the level's
capacity is stretched by demand / capacity, and package / GPU powers are held
over the stretched interval.  The pins below are worked by hand, closed forms,
and an exact-rational recomputation from an independent controller.
"""
from fractions import Fraction

import numpy as np
import pytest

from tests import exact_reference as ref

LADDER = 17


def default_cfg(**over):
    c = dict(window=4, hold=10, inc_q16=6554, dec_q16=-6554, hf_num=3, hf_den=5,
             level_min=0, level_max=16, level_init=0, up_step=0, down_step=0, base=0)
    c.update(over)
    return c


def two_level_model():
    """Capacity 15,000 MB/s at the lowest rung and 40,000 above; uncore 10 W at
    the lowest rung, 20 W in between, 30 W at the top; core 50 W; GPU 200 W;
    100 ms intervals."""
    return dict(n_levels=LADDER, interval_us=100000,
                cap_mbps=[15000] + [40000] * 16,
                uncore_mw=[10000] + [20000] * 15 + [30000],
                core_mw=50000, gpu_mw=200000)


def test_worked_step_up_example(oracle_mod):
    # 40 intervals at 10,000 MB/s, then 60 at 20,000.  MAGUS sees the rise at
    # step 40 and jumps to the top, which takes effect from interval 41:
    # interval 40 still runs at the bottom, its 20,000 MB/s over a 15,000 cap.
    x = np.array([10000] * 40 + [20000] * 60, dtype=np.uint32)
    st, m = oracle_mod.proxy_trace(x, default_cfg(), two_level_model())
    assert st["steps"][0] == 41 and st["steps"][16] == 59 and sum(st["steps"]) == 100
    assert st["excess"][0] == 5000 and st["excess"][16] == 0
    assert st["excess_max"] == 0 and st["excess_min"] == 60 * 5000
    # MAGUS: 100 intervals of 0.1 s, one of them stretched by 20/15
    # -> 10 + 0.1/3 s; package energy 60 W * (4.0 + 0.1 * 4/3) + 80 W * 5.9
    # = 248 + 472 = 720 J; system energy 720 + 200 W * T.
    t_magus = 10 + 0.1 / 3
    e_magus = 720 + 200 * t_magus
    assert m["time_s"][0] == pytest.approx(t_magus, rel=1e-13)
    assert m["energy_j"][0] == pytest.approx(e_magus, rel=1e-13)
    assert m["pkg_power_w"][0] == pytest.approx(720 / t_magus, rel=1e-13)
    # always at the top: 10 s at 80 W package + 200 W GPU = 2,800 J
    assert m["time_s"][1] == pytest.approx(10.0, rel=1e-13)
    assert m["energy_j"][1] == pytest.approx(2800.0, rel=1e-13)
    assert m["pkg_power_w"][1] == pytest.approx(80.0, rel=1e-13)
    # always at the bottom: 40 * 0.1 + 60 * 0.1 * 4/3 = 12 s at 60 W + 200 W
    assert m["time_s"][2] == pytest.approx(12.0, rel=1e-13)
    assert m["energy_j"][2] == pytest.approx(60 * 12 + 200 * 12, rel=1e-13)
    # the four metrics against the top
    assert m["perf_loss"][0] == pytest.approx(t_magus / 10 - 1, rel=1e-11)
    assert m["pkg_power_saving"][0] == pytest.approx(1 - (720 / t_magus) / 80, rel=1e-12)
    assert m["energy_saving"][0] == pytest.approx(1 - e_magus / 2800, rel=1e-12)
    assert m["edp_saving"][0] == pytest.approx(1 - e_magus * t_magus / 28000, rel=1e-12)
    assert m["perf_loss"][2] == pytest.approx(0.2, rel=1e-12)
    assert m["energy_saving"][2] == pytest.approx(1 - 3120 / 2800, rel=1e-12)
    for k in ("perf_loss", "pkg_power_saving", "energy_saving", "edp_saving"):
        assert m[k][1] == 0.0


def test_rise_and_fall_each_take_effect_one_interval_late(oracle_mod):
    # 10 intervals at 10,000, 20 at 30,000, 20 at 10,000 (W = 4, +-0.1): the
    # rise is an event at steps 10..12 (r = 0.5, three events are not "high"
    # for H = 10), so the level is at the top after steps 10..29; the fall at
    # step 30 goes straight back to the bottom.  Intervals 0..10 run at the
    # bottom (interval 10 carries 30,000 MB/s over the 15,000 cap),
    # intervals 11..30 at the top and 31..49 at the bottom.
    x = np.array([10000] * 10 + [30000] * 20 + [10000] * 20, dtype=np.uint32)
    st, m = oracle_mod.proxy_trace(x, default_cfg(), two_level_model())
    assert st["steps"][0] == 11 + 19 and st["steps"][16] == 20
    assert st["excess"][0] == 15000 and st["excess"][16] == 0
    assert st["excess_max"] == 0 and st["excess_min"] == 20 * 15000
    assert m["time_s"][0] == pytest.approx(0.1 * (49 + 2), rel=1e-13)
    # package energy: 30 bottom intervals at 60 W, one of them twice as long,
    # and 20 top intervals at 80 W
    assert m["energy_j"][0] == pytest.approx(60 * 0.1 * 31 + 80 * 0.1 * 20 + 200 * 5.1,
                                             rel=1e-13)
    assert m["time_s"][2] == pytest.approx(0.1 * (30 + 20 * 2), rel=1e-13)


def test_trace_below_every_cap_never_slows_down(oracle_mod):
    model = two_level_model()
    for lv in (700, 14999, 15000):
        x = np.full(300, lv, dtype=np.uint32)
        st, m = oracle_mod.proxy_trace(x, default_cfg(), model)
        # constant: MAGUS never moves from the bottom, so it equals always-min
        assert st["steps"][0] == 300 and st["excess"][0] == 0
        for k in m:
            assert m[k][0] == pytest.approx(m[k][2], rel=1e-13, abs=1e-15)
        assert m["perf_loss"][0] == pytest.approx(0.0, abs=1e-13)
        # package power saving = (30 W - 10 W) / (50 W + 30 W)
        assert m["pkg_power_saving"][0] == pytest.approx(20 / 80, rel=1e-12)
        # with no slowdown energy saving = power saving over the system power
        assert m["energy_saving"][0] == pytest.approx(20 / 280, rel=1e-12)
        assert m["edp_saving"][0] == pytest.approx(20 / 280, rel=1e-12)


def test_static_policies_closed_form(oracle_mod):
    rng = np.random.default_rng(7)
    model = two_level_model()
    x = rng.integers(0, 100000, 2000).astype(np.uint32)
    st, m = oracle_mod.proxy_trace(x, default_cfg(), model)
    xf = x.astype(np.float64)
    stretch_max = np.maximum(1.0, xf / 40000).sum()
    stretch_min = np.maximum(1.0, xf / 15000).sum()
    assert st["excess_max"] == int(np.maximum(0, x.astype(np.int64) - 40000).sum())
    assert st["excess_min"] == int(np.maximum(0, x.astype(np.int64) - 15000).sum())
    assert m["time_s"][1] == pytest.approx(0.1 * stretch_max, rel=1e-12)
    assert m["time_s"][2] == pytest.approx(0.1 * stretch_min, rel=1e-12)
    assert m["pkg_power_w"][1] == pytest.approx(80.0, rel=1e-12)
    assert m["pkg_power_w"][2] == pytest.approx(60.0, rel=1e-12)
    # MAGUS's intervals partition the trace
    assert sum(st["steps"]) == len(x)


def test_empty_trace_is_all_zero(oracle_mod):
    st, m = oracle_mod.proxy_trace(np.zeros(0, np.uint32), default_cfg(), two_level_model())
    assert st["excess_max"] == 0 and st["excess_min"] == 0 and sum(st["steps"]) == 0
    for k in m:
        assert m[k] == [0.0, 0.0, 0.0]


def test_model_validation(oracle_mod):
    good = two_level_model()
    assert oracle_mod.proxy_model_valid(good)
    for bad in (dict(n_levels=0), dict(n_levels=33), dict(interval_us=0),
                dict(cap_mbps=[0] + [1] * 16), dict(core_mw=0, uncore_mw=[0] * 17)):
        m = dict(good, **bad)
        assert not oracle_mod.proxy_model_valid(m), bad
    with pytest.raises(ValueError):      # level_max beyond the described ladder
        oracle_mod.proxy_trace(np.ones(4, np.uint32), default_cfg(level_max=16),
                               dict(good, n_levels=16))


def _compare_with_exact(oracle_mod, x, cfg, model):
    st, m = oracle_mod.proxy_trace(x, cfg, model)
    rst, rm = ref.proxy([int(v) for v in x], cfg, model)
    assert st == rst
    for k in m:
        for p in range(3):
            exact = float(rm[k][p])
            assert m[k][p] == pytest.approx(exact, rel=1e-10, abs=1e-12), (k, p)


def test_against_exact_rationals_random(oracle_mod):
    rng = np.random.default_rng(2025)
    for case in range(40):
        n_levels = int(rng.integers(4, 33))
        lmax = int(rng.integers(1, n_levels))
        lmin = int(rng.integers(0, lmax))
        cfg = default_cfg(window=int(rng.integers(2, 9)), hold=int(rng.integers(1, 12)),
                          inc_q16=int(rng.integers(0, 40000)),
                          dec_q16=-int(rng.integers(0, 40000)),
                          level_min=lmin, level_max=lmax,
                          level_init=int(rng.integers(lmin, lmax + 1)),
                          up_step=int(rng.integers(0, 3)) if case % 2 else 0,
                          down_step=int(rng.integers(0, 3)) if case % 2 else 0)
        model = dict(n_levels=n_levels, interval_us=int(rng.integers(1, 10**6)),
                     cap_mbps=[int(v) for v in rng.integers(1, 5000, 32)],
                     uncore_mw=[int(v) for v in rng.integers(0, 60000, 32)],
                     core_mw=int(rng.integers(1, 100000)), gpu_mw=int(rng.integers(0, 500000)))
        n = int(rng.integers(0, 120))
        # bursty levels so the controller moves
        x = np.repeat(rng.integers(0, 8000, max(1, n // 6)), 6)[:n].astype(np.uint32)
        _compare_with_exact(oracle_mod, x, cfg, model)


def test_full_range_samples_and_extreme_model(oracle_mod):
    cfg = default_cfg(window=2, hold=3)
    model = dict(n_levels=32, interval_us=4294967295 // 4096,
                 cap_mbps=[1] * 31 + [4294967295], uncore_mw=[4294967295] * 32,
                 core_mw=4294967295, gpu_mw=4294967295)
    cfg = dict(cfg, level_max=31)
    x = np.array([0, 4294967295, 1, 4294967295, 4294967295, 0, 7, 0], dtype=np.uint32)
    _compare_with_exact(oracle_mod, x, cfg, model)
