"""Helpers shared by the GPU parity tests (marshalling only)."""
import numpy as np


def to_dev(samples, offsets, cfg_of_trace=None, device="cuda"):
    import torch
    s = torch.from_numpy(np.ascontiguousarray(samples, dtype=np.uint32).view(np.int32)).to(device)
    o = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.uint64).view(np.int64)).to(device)
    c = None
    if cfg_of_trace is not None:
        c = torch.from_numpy(np.ascontiguousarray(cfg_of_trace, dtype=np.uint32)
                             .view(np.int32)).to(device)
    return s, o, c


def results_np(res):
    return res.cpu().numpy().view(np.uint64)


def describe_mismatch(got, want, offsets=None):
    bad = np.nonzero(got != want)[0]
    msg = f"{len(bad)} mismatches, first at {bad[:5]}"
    if offsets is not None and len(bad):
        t = int(np.searchsorted(offsets, bad[0], side="right") - 1)
        msg += f" (trace {t}, step {int(bad[0] - offsets[t])})"
    return msg
