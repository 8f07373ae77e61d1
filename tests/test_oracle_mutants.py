"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of the oracle's C source (on the CPU),
compiles it, swaps it in for the real oracle and runs the pin checks of
test_oracle_pins.py; at least one of them must fail.
"""
import ctypes
import os
import subprocess
import tempfile

import pytest

import oracle
from tests import test_oracle_pins as pins
from tests import test_oracle_proxy as proxy_pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "magus_oracle.c")

MUTANTS = [
    ("inc compare not strict", "if (lhs > (int64_t)inc_q * den) return 1;",
     "if (lhs >= (int64_t)inc_q * den) return 1;"),
    ("dec compare not strict", "if (lhs < (int64_t)dec_q * den) return -1;",
     "if (lhs <= (int64_t)dec_q * den) return -1;"),
    ("derivative not divided by the window", "int64_t den = (int64_t)direv_length * base;",
     "int64_t den = base;"),
    ("oldest sample as the base", "    return first < last ? first : last;",
     "    return first;"),
    ("base variants swapped", "    if (which == 1) return first;\n    if (which == 2) return last;",
     "    if (which == 1) return last;\n    if (which == 2) return first;"),
    ("fixed reference replaced by the smaller sample", "    if (which == 3) return ref;",
     "    if (which == 3) return first < last ? first : last;"),
    ("fixed reference without the window", "    int64_t den = (int64_t)direv_length * base;",
     "    int64_t den = which == 3 ? base : (int64_t)direv_length * base;"),
    ("front end ignores the counter wrap",
     "        if (counter_bits < 64) delta &= (((unsigned __int128)1) << counter_bits) - 1;\n"
     "        else delta &= (unsigned __int128)UINT64_MAX;",
     "        delta &= (unsigned __int128)UINT64_MAX;"),
    ("front end rounds up", "        unsigned __int128 mbps = delta * bytes_per_count * 1000u / dt;",
     "        unsigned __int128 mbps = (delta * bytes_per_count * 1000u + dt - 1) / dt;"),
    ("newest sample taken one step early", "int64_t last = ls[direv_length - 1];",
     "int64_t last = ls[direv_length - 2];"),
    ("sign of dec_threshold flipped", "if (lhs < (int64_t)dec_q * den) return -1;",
     "if (lhs < -(int64_t)dec_q * den) return -1;"),
    ("Alg. 2 with > instead of >=", "return (uint64_t)sum * hf_den >= (uint64_t)hf_num * len;",
     "return (uint64_t)sum * hf_den > (uint64_t)hf_num * len;"),
    ("high state does not override", "    if (high) {\n        next = c->level_max;",
     "    if (0) {\n        next = c->level_max;"),
    ("only increases are logged", "uncore_tune_ls[H - 1] = (uint8_t)(pred != 0);",
     "uncore_tune_ls[H - 1] = (uint8_t)(pred == 1);"),
    ("decrease by one step instead of to the bound",
     "next = c->down_step == 0 ? c->level_min",
     "next = c->down_step == 0 ? (level > c->level_min ? level - 1 : level)"),
    ("stepped increase not clamped to the maximum",
     ": (level + c->up_step > c->level_max ? c->level_max : level + c->up_step);",
     ": level + c->up_step;"),
    ("stepped decrease ignores the step size",
     ": (level < c->level_min + c->down_step ? c->level_min : level - c->down_step);",
     ": (level < c->level_min + 1 ? c->level_min : level - 1);"),
    ("first transition from idle not counted", "s->transitions += (next != level);",
     "s->transitions += (s->steps > 0 && next != level);"),
    ("transition weight wrong", "res->score = s->level_sum + 1000u * s->transitions;",
     "res->score = s->level_sum + 100u * s->transitions;"),
    ("event FIFO one step short", "memmove(uncore_tune_ls, uncore_tune_ls + 1, H - 1);\n"
     "    uncore_tune_ls[H - 1] = (uint8_t)(pred != 0);",
     "memmove(uncore_tune_ls, uncore_tune_ls + 1, H - 1);\n"
     "    uncore_tune_ls[H - 1] = (uint8_t)(pred != 0); if (H > 1) uncore_tune_ls[0] = 0;"),
    ("proxy: interval runs at the level set after its own step",
     "lv[0] = t == 0 ? cfg->level_init : (uint32_t)(bytes[t - 1] & 31u);",
     "lv[0] = (uint32_t)(bytes[t] & 31u);"),
    ("proxy: package power not held over the stretch",
     "pkg_j[p] += len * ((double)m->core_mw", "pkg_j[p] += dt_s * ((double)m->core_mw"),
    ("proxy: GPU energy left out", "out->energy_j[p] = pkg_j[p] + time_s[p] * (double)m->gpu_mw * 1e-3;",
     "out->energy_j[p] = pkg_j[p];"),
    ("proxy: EDP as energy only", "out->edp_saving[p] = 1.0 - (out->energy_j[p] * out->time_s[p]) /",
     "out->edp_saving[p] = 1.0 - (out->energy_j[p] * 1.0) /"),
]


def _checks():
    om = oracle
    return [
        lambda: pins.test_constant_trace_never_moves(om, 777, 4, 10),
        lambda: [pins.test_clean_step_up(om, w, s) for w in (2, 4, 6) for s in (1, 40)],
        lambda: pins.test_clean_step_down_goes_straight_to_the_lower_bound(om),
        lambda: pins.test_q16_boundary_is_strict_and_disagrees_with_fp64(om),
        lambda: pins.test_q16_boundary_downward(om),
        lambda: pins.test_high_frequency_example_of_section_3_2(om),
        lambda: pins.test_hold_one_locks_at_first_event(om),
        lambda: pins.test_zero_high_freq_threshold_is_always_high(om),
        lambda: pins.test_stuck_at_max_after_a_long_fall(om),
        lambda: pins.test_alternation_locks_at_max(om),
        lambda: pins.test_events_still_logged_while_high(om),
        lambda: [pins.test_relative_derivative_is_scale_invariant(om, c) for c in (3, 1000)],
        lambda: pins.test_up_by_k_and_down_by_k_are_symmetric(om),
        lambda: [pins.test_decision_rule_invariants(om, i) for i in (0, 4096 + 77, 16383)],
        lambda: pins.test_large_values_against_transliteration(om),
        lambda: [pins.test_stepped_staircase(om, u) for u in (1, 3, 5)],
        lambda: [pins.test_stepped_descent(om, d) for d in (2, 4)],
        lambda: pins.test_brute_force_stepped_actuation(om),
        lambda: pins.test_oldest_sample_base_bounds_falls(om),
        lambda: pins.test_newest_sample_base_bounds_rises(om),
        lambda: pins.test_counters_wrap_zero_interval_and_saturation(om),
        lambda: pins.test_counters_against_exact_rationals(om),
        lambda: pins.test_brute_force_base_variants(om),
        lambda: pins.test_fixed_reference_closed_form(om),
        lambda: pins.test_fixed_reference_is_not_scale_invariant(om),
        lambda: pins.test_brute_force_against_exact_rational_transliteration(om),
    ]


def _proxy_checks():
    om = oracle
    return [
        lambda: proxy_pins.test_worked_step_up_example(om),
        lambda: proxy_pins.test_rise_and_fall_each_take_effect_one_interval_late(om),
        lambda: proxy_pins.test_trace_below_every_cap_never_slows_down(om),
        lambda: proxy_pins.test_against_exact_rationals_random(om),
    ]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found: {name}"
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "mut.c")
        so = os.path.join(d, "libmut.so")
        open(c, "w").write(src.replace(old, new))
        subprocess.check_call(["gcc", "-O1", "-shared", "-fPIC", "-I",
                               os.path.dirname(SRC), "-o", so, c])
        real = oracle._load()
        mut = ctypes.CDLL(so)
        for fn in ("oracle_config_valid", "oracle_replay_trace", "oracle_replay_trace_fp64",
                   "oracle_replay_batch", "oracle_sweep", "oracle_counters_to_mbps",
                   "oracle_proxy_model_valid", "oracle_proxy_trace"):
            getattr(mut, fn).argtypes = getattr(real, fn).argtypes
        oracle._lib = mut
        try:
            caught = False
            for chk in (_proxy_checks() if name.startswith("proxy:") else _checks()):
                try:
                    chk()
                except AssertionError:
                    caught = True
                    break
            assert caught, f"no pin catches: {name}"
        finally:
            oracle._lib = real
