"""Bit-level emulation of bf16 rounding and the three-product split.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

bf16 keeps the sign, the 8 exponent bits and the top 7 fraction bits of an
IEEE binary32 value.  Rounding to nearest, ties to even, on the bit pattern:
    bits' = bits + 0x7FFF + ((bits >> 16) & 1),  then clear the low 16 bits
(finite inputs; NaN/Inf are not produced by the method).

Split of an fp32 value a (Henry, Tang & Heinecke, ARITH 2019):
    hi = bf16(a),  lo = bf16(a - hi)          (a - hi is exact in fp32)
Product of a and b with three bf16 products accumulated in fp32:
    a*b ~= hi_a*hi_b + hi_a*lo_b + lo_a*hi_b
(each bf16 x bf16 product is exact in fp32; the lo*lo term is dropped).
The accumulation order inside a matrix-core instruction is not specified, so
bit-exact agreement of sums is "parity unpinned"; products are pinned.
"""
from __future__ import annotations

import numpy as np


def bf16_round(x) -> np.ndarray:
    """Round float32 values to the nearest bf16 (ties to even); returns float32."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    bits = x.view(np.uint32).astype(np.uint64)
    bias = np.uint64(0x7FFF) + ((bits >> np.uint64(16)) & np.uint64(1))
    rounded = ((bits + bias) & np.uint64(0xFFFF0000)).astype(np.uint32)
    return rounded.view(np.float32).reshape(x.shape)


def split(a):
    a = np.asarray(a, dtype=np.float32)
    hi = bf16_round(a)
    lo = bf16_round((a - hi).astype(np.float32))
    return hi, lo


def bf16x3_matmul(a, b) -> np.ndarray:
    """C = A B with each product formed by the three-product split, fp32 accumulation
    (accumulated term by term in k order: hi*hi, hi*lo, lo*hi)."""
    a = np.asarray(a, np.float32)
    b = np.asarray(b, np.float32)
    ah, al = split(a)
    bh, bl = split(b)
    m, k = a.shape
    n = b.shape[1]
    c = np.zeros((m, n), np.float32)
    for kk in range(k):
        for x, y in ((ah, bh), (ah, bl), (al, bh)):
            c = (c + np.outer(x[:, kk], y[kk, :]).astype(np.float32)).astype(np.float32)
    return c
