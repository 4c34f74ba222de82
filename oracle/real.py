"""The transform of a real array in the cyclic distribution (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 6 names the real-to-complex FFT as the next transform for the method,
built by combining 1-D algorithms dimension by dimension. For a real array X of
n_1 x ... x n_d (n_d even) eq. (1.2) gives a spectrum with Y[-k] = conj(Y[k])
(indices mod n per dimension), so the half k_d in [0, n_d/2] holds all of it.
The layout is this package's reading (the paper's zig-zag cyclic distribution
is defined only by citation):

* real side: the array is held through its packed complex view
  z[j', j'_d] = X[j', 2 j'_d] + i X[j', 2 j'_d + 1] (shape n' = n_1 x ... x n_{d-1}
  x n_d/2), in the cyclic distribution of z over the grid p (Section 1.1): the
  buffer of N reals is the cyclic buffer of z, read as (re, im) pairs. With
  p = (1, ..., 1) it is the row-major real array.
* complex side: the half spectrum Y[k', k_d], k_d < n_d/2, as an n' array in the
  same cyclic distribution over p (input and output keep one layout), followed
  by the Nyquist plane Y[k', n_d/2] (shape n_1 x ... x n_{d-1}) in the cyclic
  distribution over (p_1, ..., p_{d-1}); for d = 1 the plane is one element.

The oracle computes the plain definition: eq. (1.2) of the real array with the
full complex DFT, then selects the half and the plane; the inverse rebuilds the
full spectrum from the half by the Hermitian symmetry and applies the inverse
DFT (conjugated weights, times 1/N, Section 1.3).
"""
from __future__ import annotations

import numpy as np

from . import FORWARD, INVERSE, dft, from_cyclic, to_cyclic


def _check(n, p):
    n = tuple(int(v) for v in n)
    p = tuple(int(v) for v in p)
    if len(n) != len(p) or not n:
        raise ValueError("n and p must have the same, nonzero length")
    if n[-1] % 2:
        raise ValueError(f"the last side must be even, got n={n}")
    if (n[-1] // 2) % p[-1]:
        raise ValueError(f"p_d must divide n_d / 2, got n={n} p={p}")
    return n, p


def packed_shape(n):
    return tuple(n[:-1]) + (n[-1] // 2,)


def pack(X: np.ndarray) -> np.ndarray:
    """z[j', j'_d] = X[j', 2 j'_d] + i X[j', 2 j'_d + 1] (natural order)."""
    X = np.asarray(X, dtype=np.float64)
    return X[..., 0::2] + 1j * X[..., 1::2]


def unpack(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z)
    X = np.empty(z.shape[:-1] + (2 * z.shape[-1],), dtype=np.float64)
    X[..., 0::2] = z.real
    X[..., 1::2] = z.imag
    return X


def to_cyclic_real(X: np.ndarray, p) -> np.ndarray:
    """The buffer of N reals holding X (real side layout of the module docstring)."""
    X = np.asarray(X, dtype=np.float64)
    _check(X.shape, p)
    return np.ascontiguousarray(to_cyclic(pack(X), p)).view(np.float64)


def from_cyclic_real(buf: np.ndarray, n, p) -> np.ndarray:
    n, p = _check(n, p)
    z = np.ascontiguousarray(np.asarray(buf, dtype=np.float64)).view(np.complex128)
    return unpack(from_cyclic(z, packed_shape(n), p))


def spectrum_to_buffer(Y: np.ndarray, p) -> np.ndarray:
    """Complex side buffer of a full spectrum Y (natural order): the half
    k_d < n_d/2 cyclic over p, then the plane k_d = n_d/2 cyclic over p[:-1]."""
    Y = np.asarray(Y, dtype=np.complex128)
    n, p = _check(Y.shape, p)
    h = n[-1] // 2
    half = to_cyclic(Y[..., :h], p)
    plane = Y[..., h]
    tail = to_cyclic(plane, p[:-1]) if len(n) > 1 else np.asarray(plane).reshape(1)
    return np.concatenate([half, tail])


def buffer_to_half(buf: np.ndarray, n, p):
    """(half, plane) in natural order from a complex side buffer."""
    n, p = _check(n, p)
    Nh = int(np.prod(packed_shape(n)))
    buf = np.asarray(buf, dtype=np.complex128)
    half = from_cyclic(buf[:Nh], packed_shape(n), p)
    if len(n) > 1:
        plane = from_cyclic(buf[Nh:], n[:-1], p[:-1])
    else:
        plane = buf[Nh:].reshape(())
    return half, plane


def rfft(X: np.ndarray) -> np.ndarray:
    """eq. (1.2) of a real array (natural order, full complex spectrum)."""
    return dft(np.asarray(X, dtype=np.float64).astype(np.complex128), FORWARD)


def rfft_cyclic(buf_real: np.ndarray, n, p) -> np.ndarray:
    """Expected complex side buffer of the forward transform of a real side buffer."""
    X = from_cyclic_real(buf_real, n, p)
    return spectrum_to_buffer(rfft(X), p)


def full_from_half(half: np.ndarray, plane: np.ndarray, n) -> np.ndarray:
    """The full spectrum from the half k_d < n_d/2 and the plane k_d = n_d/2 by
    Y[k', k_d] = conj(Y[-k', n_d - k_d]) for k_d > n_d/2 (indices mod n_l)."""
    n = tuple(int(v) for v in n)
    h = n[-1] // 2
    Y = np.empty(n, dtype=np.complex128)
    Y[..., :h] = half
    Y[..., h] = plane
    for kd in range(h + 1, n[-1]):
        src = np.conj(Y[..., n[-1] - kd])
        # negate every other index: k'_l -> (-k'_l) mod n_l
        for ax in range(len(n) - 1):
            src = np.roll(np.flip(src, axis=ax), 1, axis=ax)
        Y[..., kd] = src
    return Y


def irfft_cyclic(buf_cplx: np.ndarray, n, p) -> np.ndarray:
    """Expected real side buffer of the inverse transform (times 1/N) of a
    complex side buffer whose half spectrum belongs to a real array."""
    n, p = _check(n, p)
    half, plane = buffer_to_half(buf_cplx, n, p)
    Y = full_from_half(half, plane, n)
    X = dft(Y, INVERSE).real
    return to_cyclic_real(X, p)
