"""Reference for the 16-bit storage of the geometric factors used by the
reduced-precision inner operator.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  The paper stores every
real in double and lists half precision and fixed point as further work
(Section V); this module states the storage format in plain numpy:

  per element e: m = max |G_e|; gscale = 2^(floor(log2 m) - 14) (1 if m = 0);
  word = round16(round32(G / gscale)), both roundings to nearest, ties to
  even, first to IEEE single, then to IEEE binary16 ("f16") or to bfloat16
  ("bf16": the upper 16 bits of the single, rounded);
  dequantised factor = value(word) * gscale.

Pins (tests/test_oracle_g16.py): exactly representable values survive;
the scale puts max |G_e| / gscale in [2^14, 2^15); ties go to even; the
relative error respects the unit round-off of each format; AX with the
dequantised factors differs from AX with G by at most that round-off in
the energy norm on positive-definite factors.
"""
from __future__ import annotations

import numpy as np

FORMATS = ("f16", "bf16")


def scales(G, N: int) -> np.ndarray:
    """gscale[e] (float32) for G [E][6][N^3]."""
    Ge = np.abs(np.asarray(G, dtype=np.float64)).reshape(-1, 6 * N ** 3)
    m = Ge.max(axis=1)
    s = np.ones_like(m)
    pos = m > 0
    # floor(log2 m) from the binary exponent: m = f 2^k with f in [0.5, 1)
    _, k = np.frexp(m[pos])
    s[pos] = np.ldexp(1.0, k - 1 - 14)
    return s.astype(np.float32)


def _bf16_word(f32: np.ndarray) -> np.ndarray:
    bits = np.ascontiguousarray(f32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    up = (bits + 0x7FFF + ((bits >> 16) & 1)) >> 16
    return (up & 0xFFFF).astype(np.uint16)


def pack(G, N: int, fmt: str):
    """(words uint16 [E][6][N^3], gscale float32 [E])."""
    if fmt not in FORMATS:
        raise ValueError(fmt)
    G = np.asarray(G, dtype=np.float64).reshape(-1, 6, N ** 3)
    gs = scales(G, N)
    v32 = (G / gs.astype(np.float64)[:, None, None]).astype(np.float32)
    if fmt == "f16":
        words = v32.astype(np.float16).view(np.uint16)
    else:
        words = _bf16_word(v32)
    return words.reshape(G.shape), gs


def unpack(words, gscale, N: int, fmt: str) -> np.ndarray:
    """Dequantised factors (float64) value(word) * gscale."""
    w = np.ascontiguousarray(words, dtype=np.uint16).reshape(-1, 6, N ** 3)
    if fmt == "f16":
        v = w.view(np.float16).astype(np.float64)
    elif fmt == "bf16":
        v = (w.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    else:
        raise ValueError(fmt)
    return v * np.asarray(gscale, dtype=np.float64)[:, None, None]


def unit_roundoff(fmt: str) -> float:
    """Half the spacing of 1.0: 2^-11 (binary16), 2^-8 (bfloat16)."""
    return {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}[fmt]
