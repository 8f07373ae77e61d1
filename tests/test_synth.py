"""The seeded input generators: determinism, shapes and the config grid."""
import os
from fractions import Fraction

import numpy as np

import synth
from synth import grid

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_reference_values():
    """SplitMix64 with state 0: the first outputs of the published generator."""
    got = [int(v) for v in synth.draws_u64(0, 0, 3)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_threshold_table_matches_rounding_rule():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "threshold_table.txt"))
            if ln.strip() and ln[0] != "#"]
    for i, v, q in rows:
        exact = Fraction(2, 100) + Fraction(32, 1000) * int(i)
        assert Fraction(v) == exact
        assert round(exact * 65536) == int(q) == grid.THRESHOLD_TABLE_Q16[int(i)]
        assert grid.threshold_q16(float(v)) == int(q)


def test_grid_index_layout():
    g = synth.sweep_grid()
    assert len(g) == 16384
    c = g[synth.config_index(2, 5, 9, 13)]
    assert (c["window"], c["inc_q16"], c["dec_q16"], c["hold"]) == \
        (8, grid.THRESHOLD_TABLE_Q16[5], -grid.THRESHOLD_TABLE_Q16[9], 13)
    assert all(g[i] == synth.sweep_config(i) for i in (0, 4095, 4096, 16383))


def test_traces_are_deterministic_and_shaped():
    s1, o1 = synth.workload_bulk(8, 5000)
    s2, o2 = synth.workload_bulk(8, 5000)
    assert (s1 == s2).all() and (o1 == o2).all() and len(s1) == 40000
    s, o = synth.workload_small()
    assert len(s) == 10000 and s.min() >= 950 and s.max() <= 210000
    lv = synth.geometric_phase_trace(200000, synth.stream_key(5, 5))
    assert lv.min() >= 475 and lv.max() <= 420000
    x = synth.four_phase_trace(1000, synth.stream_key(7, 7))
    # four distinct plateaus (noise is +-5 %)
    big = np.nonzero(np.abs(np.diff(x.astype(np.float64))) / x[:-1] > 0.12)[0]
    assert len(big) <= 3


def test_uneven_lengths_distribution():
    lens = synth.traces.uneven_lengths(20000)
    assert lens.min() >= 1000 and lens.max() <= 1000000
    assert 15000 < np.median(lens) < 25000
