"""The C ABI library: it loads, exports every symbol magus.h declares, and its
host-side validation works without a GPU (no compute calls here)."""
import ctypes
import os
import re

import pytest

import paper_2502_03796_amd as magus
from synth import default_config

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "magus.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w]+\**\s+\**(magus_\w+)\s*\(", text,
                                 flags=re.M)))


def test_library_loads_and_exports_every_declared_symbol():
    lib = magus.load()
    names = header_functions()
    assert len(names) >= 19
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(magus.SIGNATURES), set(names) ^ set(magus.SIGNATURES)
    assert b"gfx950" in lib.magus_version()


def test_struct_layouts_match_header():
    text = open(HEADER).read()
    cfg = re.search(r"typedef struct magus_config \{(.*?)\} magus_config;", text, re.S).group(1)
    fields = re.findall(r"(u?int\d+_t)\s+([\w, ]+);", cfg)
    names = [n.strip() for _, group in fields for n in group.split(",")]
    assert names == [f[0] for f in magus.MagusConfig._fields_]
    assert ctypes.sizeof(magus.MagusConfig) == 24
    res = re.search(r"typedef struct magus_result \{(.*?)\} magus_result;", text, re.S).group(1)
    assert re.findall(r"uint64_t\s+(\w+);", res) == [f[0] for f in magus.MagusResult._fields_]


def test_config_validation_on_host():
    magus.config_check(default_config())
    magus.config_check(default_config(window=32, hold=32, inc_q16=2**20, dec_q16=-2**20,
                                      hf_num=0, level_min=0, level_max=31, level_init=31))
    for bad in (dict(window=1), dict(window=33), dict(hold=0), dict(hold=33),
                dict(inc_q16=-1), dict(dec_q16=1), dict(inc_q16=2**20 + 1),
                dict(dec_q16=-2**20 - 1), dict(hf_den=0), dict(hf_num=6, hf_den=5),
                dict(level_min=16, level_max=16), dict(level_max=32),
                dict(level_init=17), dict(up_step=32), dict(down_step=40)):
        with pytest.raises(magus.MagusError) as ei:
            magus.config_check(default_config(**bad))
        assert ei.value.code == magus.EINVAL
        assert magus.load().magus_last_error()


def test_null_arguments_are_rejected_without_a_device():
    lib = magus.load()
    assert lib.magus_ctx_create(0, None) == magus.EINVAL
    assert lib.magus_replay(None, None, 0, None, 0, None, 0, None, None, None, None) == \
        magus.EINVAL
    assert lib.magus_sweep(None, None, 0, None, 0, None, 0, None, None, None) == magus.EINVAL
    assert lib.magus_server_create(None, 1 << 20, None) == magus.EINVAL
    assert lib.magus_ctx_set_chunk(None, 64) == magus.EINVAL
    assert lib.magus_server_slot_bytes() == 192


def test_sweep_shapes_on_the_host():
    lib = magus.load()
    shapes = [magus.sweep_shape_info(i) for i in range(magus.SWEEP_SHAPES)]
    assert shapes[0] == (256, 256)
    for lanes, tile in shapes:
        assert 256 % lanes == 0 and tile % lanes == 0 and lanes % 64 == 0
    with pytest.raises(magus.MagusError):
        magus.sweep_shape_info(magus.SWEEP_SHAPES)
    assert lib.magus_ctx_set_sweep_shape(None, 0) == magus.EINVAL
    assert lib.magus_ctx_get_sweep_shape(None) == 0


def test_proxy_struct_layouts_match_header():
    text = open(HEADER).read()
    for cname, pyt, size in (("magus_proxy_model", magus.MagusProxyModel, 272),
                             ("magus_proxy_stats", magus.MagusProxyStats, 528),
                             ("magus_proxy_metrics", magus.MagusProxyMetrics, 168)):
        body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (cname, cname), text, re.S).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        names = re.findall(r"(?:u?int\d+_t|double)\s+(\w+)", body)
        assert names == [f[0] for f in pyt._fields_], cname
        assert ctypes.sizeof(pyt) == size


def test_proxy_model_validation_on_host():
    from synth import proxy_model
    good = proxy_model()
    magus.proxy_model_check(good)
    for bad in (dict(n_levels=0), dict(n_levels=33), dict(interval_us=0),
                dict(cap_mbps=[0] + good["cap_mbps"][1:]),
                dict(core_mw=0, uncore_mw=[0] * 17)):
        with pytest.raises(magus.MagusError) as ei:
            magus.proxy_model_check(dict(good, **bad))
        assert ei.value.code == magus.EINVAL
    lib = magus.load()
    assert lib.magus_proxy_model_check(None) == magus.EINVAL
    assert lib.magus_proxy(None, None, 0, None, 0, None, 0, None, None, None, None, None) == \
        magus.EINVAL
