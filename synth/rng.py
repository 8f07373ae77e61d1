"""Counter-mode SplitMix64 (Steele, Lea, Flood, OOPSLA 2014), vectorised with numpy."""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_PURPOSE = np.uint64(0xD1B54A32D192ED03)
_S30, _S27, _S31, _S11 = np.uint64(30), np.uint64(27), np.uint64(31), np.uint64(11)
_INV53 = 1.0 / float(1 << 53)

MASK64 = (1 << 64) - 1


def mix64(z):
    """SplitMix64 output function on a uint64 scalar or array (wrapping arithmetic)."""
    with np.errstate(over="ignore"):
        z = np.asarray(z, dtype=np.uint64)
        z = (z ^ (z >> _S30)) * _M1
        z = (z ^ (z >> _S27)) * _M2
        return z ^ (z >> _S31)


def _u64(v: int) -> np.uint64:
    return np.uint64(v & MASK64)


def stream_key(seed: int, index: int) -> int:
    """Key of sub-stream `index` of a seed (draw index+1 of the seed's stream)."""
    return int(mix64(_u64(seed + (index + 1) * int(GAMMA))))


def purpose_key(key: int, purpose: int) -> int:
    """Independent sub-stream of `key` for one purpose (lengths, levels, noise...)."""
    return int(mix64(_u64(key + (purpose + 1) * int(_PURPOSE))))


def draws_u64(key: int, start: int, count: int) -> np.ndarray:
    """Draws start .. start+count-1 of the stream with the given key."""
    k = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(np.uint64(key & MASK64) + k * GAMMA)


def uniform01(key: int, start: int, count: int) -> np.ndarray:
    """Uniform doubles in [0, 1): (u >> 11) * 2^-53."""
    return (draws_u64(key, start, count) >> _S11).astype(np.float64) * _INV53
