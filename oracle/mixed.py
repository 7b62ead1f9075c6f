"""Bit-level emulation of the BF16 three-way split of an FP32 number (test infrastructure).

An FP32 value x is written as hi + mid + lo with each part a bfloat16 obtained
by round-to-nearest-even: hi = bf16(x), mid = bf16(x - hi), lo = bf16(x - hi - mid);
the two subtractions are exact in FP32.  Three 8-bit significands cover the 24
bits of an FP32 significand, so hi + mid + lo == x for every normal float32 whose
parts stay normal.
"""
from __future__ import annotations

import numpy as np


def bf16_rne(x) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even); returned as float32."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    b = x.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).copy()
    nan = np.isnan(x)
    out[nan] = x[nan]
    return out


def split_bf16x3(x):
    """(hi, mid, lo) bfloat16 parts of float32 x, each returned as float32."""
    x = np.asarray(x, dtype=np.float32)
    hi = bf16_rne(x)
    r1 = (x - hi).astype(np.float32)
    mid = bf16_rne(r1)
    r2 = (r1 - mid).astype(np.float32)
    lo = bf16_rne(r2)
    return hi, mid, lo
