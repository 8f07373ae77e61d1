"""The two measurement probes the bench reports beside the rooflines: the
streaming-read probe folds exactly the words it is meant to load (so the
loads are all issued and in bounds), and the VALU issue probe reports the
lane-ops its launch issues."""
import numpy as np
import pytest

import paper_2502_03796_amd as magus
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu

K = 0x9E3779B1
MASK = 0xFFFFFFFF


def read_probe_reference(x, chunk):
    """Lane 0's fold of every chunk: blocks of 64 samples in order, eight per
    iteration, an even number of iterations (blocks past the end read 0)."""
    out = []
    for s in range(0, len(x), chunk):
        n = min(chunk, len(x) - s)
        n_iter = ((n + 63) // 64 + 7) // 8
        n_iter += n_iter % 2
        acc = 0
        for blk in range(8 * n_iter):
            v = int(x[s + 64 * blk]) if 64 * blk < n else 0
            acc = ((acc ^ v) * K) & MASK
        out.append(acc)
    return np.array(out, np.uint32)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = magus.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("n,chunk", [(1, 64), (4096 * 3 + 700, 4096), (100000, 512),
                                     (64 * 8 * 2, 1024), (12345, 8192)])
def test_read_probe_folds_every_loaded_word(ctx, n, chunk):
    rng = np.random.default_rng(n + chunk)
    x = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    s, _, _ = to_dev(x, np.array([0, n], np.uint64))
    out = ctx.read_probe(s, chunk)
    got = out.cpu().numpy().view(np.uint32)[:(n + chunk - 1) // chunk]
    assert (got == read_probe_reference(x, chunk)).all()


def test_read_probe_rejects_bad_chunks(ctx):
    s, _, _ = to_dev(np.zeros(100, np.uint32), np.array([0, 100], np.uint64))
    for chunk in (0, 100, 2**24 + 64):
        with pytest.raises(magus.MagusError) as ei:
            ctx.read_probe(s, chunk)
        assert ei.value.code == magus.EINVAL


def test_valu_probe_reports_its_lane_ops(ctx):
    for mode, per_round in ((0, 8), (1, 32)):
        _, ops = ctx.valu_probe(64, 8, mode)
        ctx.check()
        assert ops == 64 * 256 * 8 * per_round
