"""Philox4x32-10 on the host (numpy), written from its published definition
(Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11), and the mapping of its output to complex values in [-1, 1) that the
library's device generator (fftu_fill_uniform) uses. Counter-based: element e
of a request's input is a pure function of (key, e), so the host reproduces
device-generated inputs bit for bit without copying them back.

Holds no arithmetic of the transform.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Ten Philox rounds on the counter words (arrays of uint32 values) under the
    key (k0, k1). Returns the four output words as uint64 arrays (< 2^32)."""
    c0 = np.asarray(c0, dtype=np.uint64)
    c1 = np.asarray(c1, dtype=np.uint64)
    c2 = np.asarray(c2, dtype=np.uint64)
    c3 = np.asarray(c3, dtype=np.uint64)
    k0 = int(k0) & _MASK
    k1 = int(k1) & _MASK
    m0 = np.uint64(M0)
    m1 = np.uint64(M1)
    lo = np.uint64(_MASK)
    sh = np.uint64(32)
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & _MASK
            k1 = (k1 + W1) & _MASK
        p0 = m0 * c0                       # < 2^64: no wrap-around
        p1 = m1 * c2
        n0 = (p1 >> sh) ^ c1 ^ np.uint64(k0)
        n2 = (p0 >> sh) ^ c3 ^ np.uint64(k1)
        c1 = p1 & lo
        c3 = p0 & lo
        c0 = n0
        c2 = n2
    return c0, c1, c2, c3


def uniform_complex(count: int, key0: int, key1: int, dtype=np.complex128, counter_base: int = 0) -> np.ndarray:
    """The values fftu_fill_uniform writes: element e from the counter
    (c mod 2^32, c div 2^32, 0, 0), c = counter_base + e, mapped exactly into [-1, 1)."""
    e = np.arange(int(count), dtype=np.uint64) + np.uint64(counter_base)
    zero = np.zeros_like(e)
    x0, x1, x2, x3 = philox4x32_10(e & np.uint64(_MASK), e >> np.uint64(32), zero, zero, key0, key1)
    if np.dtype(dtype) == np.complex64:
        re = (x0 >> np.uint64(8)).astype(np.float64) * 2.0 ** -23 - 1.0
        im = (x1 >> np.uint64(8)).astype(np.float64) * 2.0 ** -23 - 1.0
        out = np.empty(int(count), dtype=np.complex64)
        out.real = re.astype(np.float32)       # exact: 24-bit values
        out.imag = im.astype(np.float32)
        return out
    re = ((x0 << np.uint64(21)) | (x1 >> np.uint64(11))).astype(np.float64) * 2.0 ** -52 - 1.0
    im = ((x2 << np.uint64(21)) | (x3 >> np.uint64(11))).astype(np.float64) * 2.0 ** -52 - 1.0
    out = np.empty(int(count), dtype=np.complex128)
    out.real = re
    out.imag = im
    return out
