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
    assert lib.magus_read_probe(None, None, 0, 4096, None, None) == magus.EINVAL
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


def test_noalloc_host_limits_without_a_device():
    """The allocation-free replay checks its arguments and its fixed scratch
    size on the host, before it touches a device."""
    lib = magus.load()
    one = magus.config_array([default_config()])
    fake = ctypes.c_void_p(256)          # never dereferenced: rejected first
    # no configs, too many configs, missing buffers
    assert lib.magus_replay_noalloc(fake, 10, fake, 1, None, 0, None, fake, None, None,
                                    None) == magus.EINVAL
    many = magus.config_array([default_config()] * (magus.NOALLOC_MAX_CFGS + 1))
    assert lib.magus_replay_noalloc(fake, 10, fake, 1, many, len(many), None, fake, None,
                                    None, None) == magus.EINVAL
    assert b"at most 16384" in lib.magus_last_error()
    assert lib.magus_replay_noalloc(fake, 10, None, 1, one, 1, None, fake, None, None,
                                    None) == magus.EINVAL
    # a batch whose chunk summaries exceed the 8 MiB array: 2^31 samples in
    # one trace need 2^19 chunks x 32 B = 16 MiB
    assert lib.magus_replay_noalloc(fake, 1 << 31, fake, 1, one, 1, None, fake, None, None,
                                    None) == magus.EINVAL
    assert b"bytes of scratch" in lib.magus_last_error()
    # decision bytes need 16 B more per chunk: 3 x 2^28 samples are 196,610
    # chunks, 6 MiB of summaries (they fit) + 3 MiB of fix-up records (too many)
    assert lib.magus_replay_noalloc(fake, 3 << 28, fake, 1, one, 1, None, fake, fake, None,
                                    None) == magus.EINVAL
    assert b"bytes of scratch" in lib.magus_last_error()
    # no traces and no status word: only the configs are checked
    assert lib.magus_replay_noalloc(None, 0, None, 0, one, 1, None, None, None, None,
                                    None) == magus.OK
    bad = magus.config_array([default_config(window=1)])
    assert lib.magus_replay_noalloc(None, 0, None, 0, bad, 1, None, None, None, None,
                                    None) == magus.EINVAL


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
