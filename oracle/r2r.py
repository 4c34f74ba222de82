"""The discrete cosine and sine transforms in the zig-zag cyclic distribution
(oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 6 names the DCT and the DST as next transforms for the method, built by
combining 1-D algorithms dimension by dimension, and suggests the zig-zag cyclic
distribution (defined only by citation) to exploit their symmetry. This module
is this package's reading:

* Definitions, per dimension of length N (the d-dimensional transforms apply
  them along every dimension; eq. (1.3)'s factorisation over dimensions):
    DCT-II   y[k] = 2 sum_n x[n] cos(pi k (2n + 1) / (2N))
    DST-II   y[k] = 2 sum_n x[n] sin(pi (k + 1) (2n + 1) / (2N))
  and their exact inverses (DCT-III and DST-III scaled by 1/N):
    x[n] = (1/N) (y[0]/2 + sum_{k >= 1} y[k] cos(pi k (2n + 1) / (2N)))
    x[n] = (1/N) (sum_{k < N-1} y[k] sin(pi (k + 1)(2n + 1) / (2N)) + (-1)^n y[N-1]/2)
* Zig-zag order: v[m(j)] = x[j] along every dimension, m(j) = j/2 for even j
  and N - 1 - (j - 1)/2 for odd j: the even samples ascending, then the odd
  samples descending. The DCT-II of x depends on the DFT of v alone, so a
  distribution that deals v out cyclically makes that reordering free: the
  zig-zag cyclic distribution, read here as the cyclic distribution of v.
* Buffers (real, N values each): the signal side holds v in the real-side
  layout of the real transform (`oracle.real`: packed pairs, cyclic over p);
  the coefficient side holds y in the cyclic distribution over p (Section 1.1).
  The forward transforms go signal -> coefficients, the inverses back.

Every n_l must be even, and p_d must divide n_d / 2 (the real transform's
packed array).
"""
from __future__ import annotations

import numpy as np

from . import FORWARD, INVERSE, from_cyclic, to_cyclic
from . import real

DCT = "dct"
DST = "dst"


def _check(n, p):
    n = tuple(int(v) for v in n)
    p = tuple(int(v) for v in p)
    if len(n) != len(p) or not n:
        raise ValueError("n and p must have the same, nonzero length")
    if any(v % 2 for v in n):
        raise ValueError(f"every side must be even, got n={n}")
    if any(nl % pl for nl, pl in zip(n, p)) or (n[-1] // 2) % p[-1]:
        raise ValueError(f"p_l must divide n_l and p_d must divide n_d / 2, got n={n} p={p}")
    return n, p


def zigzag_index(N: int) -> np.ndarray:
    """m(j) for j in [N]: the position of x[j] in the zig-zag order."""
    j = np.arange(N)
    return np.where(j % 2 == 0, j // 2, N - 1 - (j - 1) // 2)


def to_zigzag(X: np.ndarray) -> np.ndarray:
    """v with v[m(j)] = X[j] along every axis."""
    V = np.asarray(X, dtype=np.float64)
    for ax, N in enumerate(V.shape):
        out = np.empty_like(V)
        idx = [slice(None)] * V.ndim
        idx[ax] = zigzag_index(N)
        out[tuple(idx)] = V
        V = out
    return V


def from_zigzag(V: np.ndarray) -> np.ndarray:
    X = np.asarray(V, dtype=np.float64)
    for ax, N in enumerate(X.shape):
        idx = [slice(None)] * X.ndim
        idx[ax] = zigzag_index(N)
        X = X[tuple(idx)]
    return np.ascontiguousarray(X)


def _matrix(N: int, kind: str, direction: int) -> np.ndarray:
    """The 1-D transform as an N x N matrix A (y = A x), from the definitions above."""
    n = np.arange(N)[None, :]
    k = np.arange(N)[:, None]
    if direction == FORWARD:
        if kind == DCT:
            return 2.0 * np.cos(np.pi * k * (2 * n + 1) / (2 * N))
        return 2.0 * np.sin(np.pi * (k + 1) * (2 * n + 1) / (2 * N))
    # inverse: rows are the outputs x[n], columns the inputs y[k]
    nn = np.arange(N)[:, None]
    kk = np.arange(N)[None, :]
    if kind == DCT:
        A = np.cos(np.pi * kk * (2 * nn + 1) / (2 * N))
        A[:, 0] = 0.5
    else:
        A = np.sin(np.pi * (kk + 1) * (2 * nn + 1) / (2 * N))
        A[:, N - 1] = 0.5 * (-1.0) ** np.arange(N)
    return A / N


def transform(X: np.ndarray, kind: str, direction: int = FORWARD) -> np.ndarray:
    """The d-dimensional DCT-II / DST-II (FORWARD) or its inverse (INVERSE) of a
    real array in natural order: the 1-D matrix applied along every axis."""
    if kind not in (DCT, DST) or direction not in (FORWARD, INVERSE):
        raise ValueError("kind must be 'dct' or 'dst' and direction FORWARD or INVERSE")
    Y = np.asarray(X, dtype=np.float64)
    for ax, N in enumerate(Y.shape):
        Y = np.moveaxis(np.tensordot(_matrix(N, kind, direction), np.moveaxis(Y, ax, 0), axes=1), 0, ax)
    return np.ascontiguousarray(Y)


def signal_to_buffer(X: np.ndarray, p) -> np.ndarray:
    """Signal-side buffer of a real array X in natural order."""
    _check(np.shape(X), p)
    return real.to_cyclic_real(to_zigzag(X), p)


def buffer_to_signal(buf: np.ndarray, n, p) -> np.ndarray:
    n, p = _check(n, p)
    return from_zigzag(real.from_cyclic_real(buf, n, p))


def coeffs_to_buffer(Y: np.ndarray, p) -> np.ndarray:
    """Coefficient-side buffer: Y cyclic over p."""
    _check(np.shape(Y), p)
    return np.ascontiguousarray(to_cyclic(np.asarray(Y, dtype=np.float64), p))


def buffer_to_coeffs(buf: np.ndarray, n, p) -> np.ndarray:
    n, p = _check(n, p)
    return from_cyclic(np.asarray(buf, dtype=np.float64), n, p)


def r2r_cyclic(buf: np.ndarray, n, p, kind: str, direction: int = FORWARD) -> np.ndarray:
    """Expected output buffer of the transform of a buffer: FORWARD takes the
    signal side to the coefficient side, INVERSE the reverse."""
    n, p = _check(n, p)
    if direction == FORWARD:
        return coeffs_to_buffer(transform(buffer_to_signal(buf, n, p), kind, FORWARD), p)
    return signal_to_buffer(transform(buffer_to_coeffs(buf, n, p), kind, INVERSE), p)
