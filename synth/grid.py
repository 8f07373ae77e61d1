"""Controller configurations: the default config and the sweep grid.

Configs are plain dicts of integers:
  window (W, the derivative window of Alg. 1), hold (H = len(uncore_tune_ls)
  of Alg. 2), inc_q16 / dec_q16 (thresholds in Q16.16, dec <= 0),
  hf_num / hf_den (high_freq_threshold, 3/5 = 0.6 as in Sec. 3.2),
  level_min / level_max / level_init (indices on the 17-level uncore ladder
  0.8-2.4 GHz in 100 MHz steps: level i is 800 + 100 i MHz), up_step /
  down_step (0 = jump to the bound).

The sweep grid: W in {2, 4, 8, 16}; up and down thresholds each one of 16
values v_i = 0.02 + 0.032 i (i = 0..15, linear over [0.02, 0.5]) stored in
Q16.16 as round-half-even(65536 v_i); H = 1..16.  Config index
c = ((w * 16 + u) * 16 + d) * 16 + (H - 1), w indexing {2, 4, 8, 16}.
"""
from __future__ import annotations

from fractions import Fraction

WINDOWS = (2, 4, 8, 16)

# round-half-even(65536 * (0.02 + 0.032 i)), i = 0..15
THRESHOLD_TABLE_Q16 = (1311, 3408, 5505, 7602, 9699, 11796, 13894, 15991,
                       18088, 20185, 22282, 24379, 26477, 28574, 30671, 32768)


def threshold_q16(v) -> int:
    """Q16.16 of a decimal threshold, rounded half to even (exact rational)."""
    exact = Fraction(str(v)) if isinstance(v, float) else Fraction(v)
    return round(exact * 65536)


def default_config(**over) -> dict:
    """W = 4, inc = +0.1, dec = -0.1 (Q16.16 6554), H = 10, 0.6 = 3/5,
    ladder 0..16 starting idle at the minimum, jump-to-bound actuation."""
    c = dict(window=4, hold=10, inc_q16=6554, dec_q16=-6554, hf_num=3, hf_den=5,
             level_min=0, level_max=16, level_init=0, up_step=0, down_step=0)
    c.update(over)
    return c


def config_index(w_idx: int, u: int, d: int, hold: int) -> int:
    return ((w_idx * 16 + u) * 16 + d) * 16 + (hold - 1)


def sweep_config(index: int) -> dict:
    h = index % 16 + 1
    d = (index // 16) % 16
    u = (index // 256) % 16
    w = index // 4096
    return default_config(window=WINDOWS[w], hold=h, inc_q16=THRESHOLD_TABLE_Q16[u],
                          dec_q16=-THRESHOLD_TABLE_Q16[d])


def sweep_grid() -> list[dict]:
    """All 16,384 configs in index order."""
    return [sweep_config(i) for i in range(4 * 16 * 16 * 16)]
