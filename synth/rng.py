"""Counter-based random numbers for the synthetic inputs.

The generator is SplitMix64's output function (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014) applied to a
counter: the i-th 64-bit word of stream ``stream`` under ``seed`` is

    key  = mix64(seed * 0x9E3779B97F4A7C15 + stream * 0xD1B54A32D192ED03 + 1)
    w_i  = mix64(key + (i + 1) * 0x9E3779B97F4A7C15)

with ``mix64`` the SplitMix64 finaliser.  Every value depends only on
(seed, stream, i), so any slice of a stream can be produced on its own and in
any order.  This module holds no part of the ψ-score arithmetic.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_STREAM_MUL = np.uint64(0xD1B54A32D192ED03)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_TWO_M53 = 1.0 / 9007199254740992.0  # 2**-53


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int) -> np.uint64:
    s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    t = np.uint64(stream & 0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        k = s * _GOLDEN + t * _STREAM_MUL + np.uint64(1)
    return mix64(np.array([k], dtype=np.uint64))[0]


def words(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """64-bit words ``start .. start+count-1`` of a stream."""
    key = stream_key(seed, stream)
    idx = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(key + idx * _GOLDEN)


def uniform01(seed: int, stream: int, count: int, start: int = 0) -> np.ndarray:
    """Doubles in the open interval (0, 1): ((w >> 11) + 0.5) * 2**-53."""
    w = words(seed, stream, start, count)
    return ((w >> np.uint64(11)).astype(np.float64) + 0.5) * _TWO_M53


def standard_normal(seed: int, stream: int, count: int) -> np.ndarray:
    """Box–Muller normals: element k uses uniforms 2k and 2k+1 of the stream."""
    u = uniform01(seed, stream, 2 * count)
    u1 = u[0::2]
    u2 = u[1::2]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


# ---------------------------------------------------------------- torch twin
# The same words computed with torch int64 tensors (two's-complement wrapping
# multiply, logical shifts by masking), on any device; used to draw the edges
# of the largest graphs where they are consumed.
def _i64(c: int) -> int:
    return c - (1 << 64) if c >= (1 << 63) else c


def _shr(z, k: int):
    return (z >> k) & ((1 << (64 - k)) - 1)


def mix64_torch(z):
    z = (z ^ _shr(z, 30)) * _i64(0xBF58476D1CE4E5B9)
    z = (z ^ _shr(z, 27)) * _i64(0x94D049BB133111EB)
    return z ^ _shr(z, 31)


def words_torch(seed: int, stream: int, start: int, count: int, device="cpu"):
    import torch
    key = int(stream_key(seed, stream))
    idx = torch.arange(start + 1, start + 1 + count, dtype=torch.int64, device=device)
    return mix64_torch(idx * _i64(0x9E3779B97F4A7C15) + _i64(key))


def uniform01_torch(seed: int, stream: int, count: int, start: int = 0, device="cpu"):
    import torch
    w = words_torch(seed, stream, start, count, device)
    return (_shr(w, 11).to(torch.float64) + 0.5) * _TWO_M53
