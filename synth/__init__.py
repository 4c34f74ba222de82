"""Seeded synthetic inputs shaped like the workloads of arXiv 2203.11795.

This module holds random number draws and workload recipes only -- none of the
transform's arithmetic. It is the one piece shared by the test suite (and the
oracle checks there) and the GPU path's callers (tests, benchmark, smoke).

Conventions:
* Values are drawn with numpy's PCG64 (``np.random.default_rng(seed)``): all
  real parts first, then all imaginary parts, in FP64. complex64 inputs are
  those FP64 draws rounded once to FP32.
* A generated array of N entries is used as the *cyclic buffer* that the
  virtual processors hold (the input layout of the transform). Because the
  entries are iid, the natural-order array it represents has the same
  distribution.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["uniform_complex", "normal_complex", "batch_shapes", "serving_trace"]


def _finish(re: np.ndarray, im: np.ndarray, dtype) -> np.ndarray:
    z = np.empty(re.shape, dtype=np.complex128)
    z.real = re
    z.imag = im
    if np.dtype(dtype) == np.complex64:
        return z.astype(np.complex64)
    if np.dtype(dtype) != np.complex128:
        raise ValueError(f"dtype must be complex64 or complex128, got {dtype}")
    return z


def uniform_complex(count: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """``count`` complex values, real and imaginary parts iid uniform on [-1, 1)."""
    rng = np.random.default_rng(seed)
    re = rng.uniform(-1.0, 1.0, size=int(count))
    im = rng.uniform(-1.0, 1.0, size=int(count))
    return _finish(re, im, dtype)


def normal_complex(count: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """``count`` complex values, real and imaginary parts iid standard normal."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(size=int(count))
    im = rng.standard_normal(size=int(count))
    return _finish(re, im, dtype)


def batch_shapes(count: int = 256, seed: int = 4, exponents=(4, 5, 6, 7, 8), ndim: int = 3):
    """Uneven 3-D shapes: each side 2^e with e drawn uniformly from ``exponents``
    independently per dimension (log-uniform over {16, ..., 256})."""
    rng = np.random.default_rng(seed)
    ex = rng.choice(np.asarray(exponents), size=(int(count), ndim))
    return [tuple(int(1 << int(e)) for e in row) for row in ex]


def serving_trace(seed: int = 5, rate: float = 2000.0, duration: float = 30.0,
                  ranks=(2, 3, 4), exponents=(5, 6, 7, 8, 9, 10), max_points: int = 1 << 26):
    """Poisson request stream: list of dicts with arrival time (s), shape, dtype, direction.

    Rank uniform over ``ranks``; each side 2^e with e uniform over
    ``exponents``; a draw with more than ``max_points`` points is rejected and
    redrawn; dtype uniform over {complex64, complex128}; direction uniform over
    {forward (-1), inverse (+1)}.
    """
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    i = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        rank = int(rng.choice(np.asarray(ranks)))
        while True:
            shape = tuple(int(1 << int(e)) for e in rng.choice(np.asarray(exponents), size=rank))
            if math.prod(shape) <= max_points:
                break
        dtype = np.complex64 if rng.integers(0, 2) == 0 else np.complex128
        direction = -1 if rng.integers(0, 2) == 0 else 1
        out.append({"id": i, "t": t, "shape": shape, "dtype": dtype, "direction": direction})
        i += 1
    return out
