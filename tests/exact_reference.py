"""Exact-rational transliteration of the MAGUS controller for tiny inputs.

Written independently of the C oracle, straight from the paper's two listings
and the decision rule of Sec. 3.2: Python lists are the FIFOs, the derivative is
a ``fractions.Fraction`` (an actual division, not a cross-multiplication), the
thresholds are the rationals q/65536, and Alg. 2's freq is sum/len as a
Fraction.  It is slow and meant for brute force over tiny traces only.
"""
from __future__ import annotations

from fractions import Fraction

INF = float("inf")


def trend_prediction(inc_threshold, dec_threshold, mem_throughput_ls, direv_length,
                     which_base=0, base_ref=0):
    """Alg. 1 with the derivative taken relative to the smaller end sample
    (or, as alternatives, the oldest, the newest, or a fixed reference)."""
    first, last = mem_throughput_ls[0], mem_throughput_ls[-1]
    base = (min(first, last), first, last, base_ref)[which_base]
    if base == 0:
        if last == first:
            return 0                      # 0/0: no trend
        derivative = INF if last > first else -INF
    else:
        derivative = Fraction(last - first, direv_length * base)
    if derivative > inc_threshold:
        return 1
    elif derivative < dec_threshold:
        return -1
    return 0


def high_freq_detection(high_freq_threshold, uncore_tune_ls):
    """Alg. 2."""
    freq = Fraction(sum(uncore_tune_ls), len(uncore_tune_ls))
    return freq >= high_freq_threshold


def run(trace, cfg):
    """Returns (per-step (level, high, pred) list, score, level_sum, transitions, ticks_high)."""
    inc = Fraction(cfg["inc_q16"], 65536)
    dec = Fraction(cfg["dec_q16"], 65536)
    hft = Fraction(cfg["hf_num"], cfg["hf_den"])
    W, H = cfg["window"], cfg["hold"]
    mem_throughput_ls: list[int] = []
    uncore_tune_ls = [0] * H
    level = cfg["level_init"]
    steps = []
    level_sum = transitions = ticks_high = 0
    for x in trace:
        mem_throughput_ls.append(int(x))
        if len(mem_throughput_ls) > W:
            mem_throughput_ls.pop(0)
        pred = trend_prediction(inc, dec, mem_throughput_ls, W, cfg.get("base", 0),
                                cfg.get("base_ref", 0)) \
            if len(mem_throughput_ls) == W else 0
        uncore_tune_ls.pop(0)
        uncore_tune_ls.append(1 if pred != 0 else 0)
        high = high_freq_detection(hft, uncore_tune_ls)
        up, down = cfg.get("up_step", 0), cfg.get("down_step", 0)
        if high:
            new = cfg["level_max"]
        elif pred == 1:
            new = cfg["level_max"] if up == 0 else min(level + up, cfg["level_max"])
        elif pred == -1:
            new = cfg["level_min"] if down == 0 else max(level - down, cfg["level_min"])
        else:
            new = level
        if new != level:
            transitions += 1
        level = new
        level_sum += level
        ticks_high += int(high)
        steps.append((level, int(high), pred))
    return steps, level_sum + 1000 * transitions, level_sum, transitions, ticks_high


def encode(steps):
    """Same byte layout as the oracle: level | high << 5 | (pred + 1) << 6."""
    return bytes(lv | (h << 5) | ((p + 1) << 6) for lv, h, p in steps)


def proxy(trace, cfg, model):
    """Proxy energy model in exact rationals, interval by interval.

    Interval t runs at the level set after step t-1 (level_init first) under
    MAGUS, at level_max or level_min under the static policies; its length is
    interval * max(1, x / cap[level]); package power core + uncore[level] and
    system power + gpu are held over it.  Returns (stats, metrics) in the same
    layout as the C oracle, metrics as Fractions.
    """
    steps, *_ = run(trace, cfg)
    dt = Fraction(model["interval_us"], 10**6)
    levels = [cfg["level_init"]] + [lv for lv, _, _ in steps[:-1]]
    pol = [levels, [cfg["level_max"]] * len(trace), [cfg["level_min"]] * len(trace)]
    st = {"excess_max": 0, "excess_min": 0, "steps": [0] * 32, "excess": [0] * 32}
    T = [Fraction(0)] * 3
    Epkg = [Fraction(0)] * 3
    for p in range(3):
        for x, lv in zip(trace, pol[p]):
            cap = model["cap_mbps"][lv]
            over = max(0, int(x) - cap)
            if p == 0:
                st["steps"][lv] += 1
                st["excess"][lv] += over
            elif p == 1:
                st["excess_max"] += over
            else:
                st["excess_min"] += over
            length = dt * max(Fraction(1), Fraction(int(x), cap))
            T[p] += length
            Epkg[p] += length * Fraction(model["core_mw"] + model["uncore_mw"][lv], 1000)
    E = [Epkg[p] + T[p] * Fraction(model["gpu_mw"], 1000) for p in range(3)]
    P = [Epkg[p] / T[p] if T[p] else Fraction(0) for p in range(3)]
    m = {"time_s": T, "energy_j": E, "pkg_power_w": P}
    if len(trace) == 0:
        zero = [Fraction(0)] * 3
        m.update(perf_loss=zero, pkg_power_saving=zero, energy_saving=zero, edp_saving=zero)
    else:
        m["perf_loss"] = [T[p] / T[1] - 1 for p in range(3)]
        m["pkg_power_saving"] = [1 - P[p] / P[1] for p in range(3)]
        m["energy_saving"] = [1 - E[p] / E[1] for p in range(3)]
        m["edp_saving"] = [1 - (E[p] * T[p]) / (E[1] * T[1]) for p in range(3)]
    return st, m


def run_tree(alphabet, depth, cfg):
    """Per-step decision bytes of every trace of length `depth` over
    `alphabet`, in itertools.product order, as a uint8 array [count, depth].

    The controller is causal, so the steps of a trace's prefix are the first
    steps of the trace; the traces are walked as a tree, level by level, each
    node one step of ``run``'s loop from its parent's state (same Fraction
    arithmetic), so every prefix is evaluated once.
    """
    import numpy as np
    inc = Fraction(cfg["inc_q16"], 65536)
    dec = Fraction(cfg["dec_q16"], 65536)
    hft = Fraction(cfg["hf_num"], cfg["hf_den"])
    W, H = cfg["window"], cfg["hold"]
    up, down = cfg.get("up_step", 0), cfg.get("down_step", 0)
    which, ref = cfg.get("base", 0), cfg.get("base_ref", 0)
    # state: (mem_throughput_ls, uncore_tune_ls, level)
    states = [((), (0,) * H, cfg["level_init"])]
    out = np.zeros((len(alphabet) ** depth, depth), np.uint8)
    for k in range(depth):
        nxt = []
        col = []
        for ls, tune, level in states:
            for x in alphabet:
                mem = (ls + (int(x),))[-W:]
                pred = trend_prediction(inc, dec, list(mem), W, which, ref) \
                    if len(mem) == W else 0
                tune2 = tune[1:] + ((1 if pred != 0 else 0),)
                high = high_freq_detection(hft, list(tune2))
                if high:
                    new = cfg["level_max"]
                elif pred == 1:
                    new = cfg["level_max"] if up == 0 else min(level + up, cfg["level_max"])
                elif pred == -1:
                    new = cfg["level_min"] if down == 0 else max(level - down, cfg["level_min"])
                else:
                    new = level
                nxt.append((mem, tune2, new))
                col.append(new | (int(high) << 5) | ((pred + 1) << 6))
        # node j of this level is the prefix j; its subtree spans
        # len(alphabet) ** (depth - k - 1) consecutive traces
        rep = len(alphabet) ** (depth - k - 1)
        out[:, k] = np.repeat(np.array(col, np.uint8), rep)
        states = nxt
    return out
