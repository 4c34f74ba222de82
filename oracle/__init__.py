"""FP64 CPU oracle for the cyclic-to-cyclic multidimensional DFT.

TEST INFRASTRUCTURE ONLY. Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package. It shares no code
with the HIP library and never imports it.

What it computes (Koopman & Bisseling, arXiv 2203.11795):

* :func:`dft` -- the d-dimensional DFT of eq. (1.2) in natural row-major order,
  by 1-D DFTs along each axis (eq. (1.3)): radix-2 FFTs for power-of-two
  lengths, the 1-D definition summed term by term for other lengths; the
  inverse conjugates every weight and multiplies by 1/N (Section 1.3, last
  paragraph).
* :func:`dft_direct` / :func:`dft_points` -- eq. (1.2) summed term by term
  (all outputs of a tiny array, or chosen outputs of a large one).
* :func:`to_cyclic` / :func:`from_cyclic` -- the d-dimensional cyclic
  distribution of Section 1.1, phi(s, k) = s + k*p elementwise, with the local
  arrays of the P = p_1...p_d virtual processors stored one after the other
  (processor rank row-major over s, local arrays row-major over k).
* :func:`cyclic_dft` -- the expected output buffer of the method: the DFT of
  the array held in a cyclic buffer, returned in the same cyclic buffer layout
  (Algorithm 2.3 starts and ends in the same distribution).
* :func:`emulate` -- Algorithm 2.3 carried out literally, virtual processor by
  virtual processor, exposing the buffer after each superstep, so that each
  GPU stage can be checked on its own.
* :mod:`oracle.real`, :mod:`oracle.r2r`, :mod:`oracle.group_cyclic` -- the real-input
  transform, the DCT / DST in the zig-zag cyclic distribution and grids beyond
  p_max (Sections 6 and 2.3), each with its reading of the paper in its docstring.
* :func:`circular_convolution` -- the cyclic convolution of two arrays of one
  shape, summed from its definition (the application that motivates keeping
  input and output in the same distribution: forward transform, pointwise
  product, inverse transform, with no reordering; Sections 1 and 2.2).

Complex arrays are numpy complex128. Directions: FORWARD = -1 (omega_n =
exp(-2 pi i / n), unnormalised), INVERSE = +1.
"""
from __future__ import annotations

import ctypes
import itertools
import os

import numpy as np

FORWARD = -1
INVERSE = +1

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    i64p = ctypes.POINTER(ctypes.c_int64)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_fft_axes.argtypes = [ctypes.c_int, i64p, ctypes.c_uint32, dp, ctypes.c_int, ctypes.c_int]
    lib.oracle_fft_axes.restype = ctypes.c_int
    lib.oracle_dft_direct.argtypes = [ctypes.c_int, i64p, dp, dp, ctypes.c_int]
    lib.oracle_dft_direct.restype = ctypes.c_int
    lib.oracle_dft_points.argtypes = [ctypes.c_int, i64p, dp, ctypes.c_int64, i64p, dp, ctypes.c_int,
                                      ctypes.c_int]
    lib.oracle_dft_points.restype = ctypes.c_int
    lib.oracle_max_threads.argtypes = []
    lib.oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def max_threads() -> int:
    """Number of OpenMP threads the oracle uses by default."""
    return int(_load().oracle_max_threads())


def _shape_arr(shape):
    return (ctypes.c_int64 * len(shape))(*[int(s) for s in shape])


def _check_direction(direction):
    if direction not in (FORWARD, INVERSE):
        raise ValueError(f"direction must be FORWARD (-1) or INVERSE (+1), got {direction!r}")


def fft_axes(x: np.ndarray, axes, direction: int = FORWARD, nthreads: int = 0) -> np.ndarray:
    """Unnormalised 1-D DFTs along each axis in ``axes``: radix-2 FFTs for
    power-of-two lengths, the 1-D definition summed term by term otherwise."""
    _check_direction(direction)
    y = np.ascontiguousarray(x, dtype=np.complex128).copy()
    if y.ndim == 0:
        return y
    mask = 0
    for a in axes:
        mask |= 1 << (int(a) % y.ndim)
    rc = _load().oracle_fft_axes(y.ndim, _shape_arr(y.shape), mask,
                                 y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), direction, nthreads)
    if rc == 2:
        raise ValueError(f"oracle FFT needs power-of-two lengths, got shape {y.shape}")
    if rc != 0:
        raise RuntimeError(f"oracle_fft_axes failed with status {rc}")
    return y


def dft(x: np.ndarray, direction: int = FORWARD, nthreads: int = 0) -> np.ndarray:
    """The d-D DFT of eq. (1.2) of a natural-order array; INVERSE includes the 1/N factor."""
    y = fft_axes(x, range(np.ndim(x)), direction, nthreads)
    if direction == INVERSE:
        y *= 1.0 / y.size
    return y


def dft_direct(x: np.ndarray, direction: int = FORWARD) -> np.ndarray:
    """eq. (1.2) summed term by term in long double (N <= 16384); INVERSE includes 1/N."""
    _check_direction(direction)
    xc = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty_like(xc)
    rc = _load().oracle_dft_direct(xc.ndim, _shape_arr(xc.shape),
                                   xc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), direction)
    if rc != 0:
        raise RuntimeError(f"oracle_dft_direct failed with status {rc} (N must be <= 16384)")
    if direction == INVERSE:
        y *= 1.0 / y.size
    return y


def dft_points(x: np.ndarray, kflat, direction: int = FORWARD, nthreads: int = 0) -> np.ndarray:
    """eq. (1.2) for the outputs with flat row-major indices ``kflat`` (O(N) each)."""
    _check_direction(direction)
    xc = np.ascontiguousarray(x, dtype=np.complex128)
    k = np.ascontiguousarray(np.asarray(kflat, dtype=np.int64).reshape(-1))
    y = np.empty(k.size, dtype=np.complex128)
    rc = _load().oracle_dft_points(xc.ndim, _shape_arr(xc.shape),
                                   xc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), k.size,
                                   k.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), direction, nthreads)
    if rc != 0:
        raise RuntimeError(f"oracle_dft_points failed with status {rc}")
    if direction == INVERSE:
        y *= 1.0 / xc.size
    return y


# ----------------------------------------------------------------------------
# Cyclic distribution (Section 1.1)
# ----------------------------------------------------------------------------

def _local_shape(n, p):
    n = tuple(int(v) for v in n)
    p = tuple(int(v) for v in p)
    if len(n) != len(p):
        raise ValueError("n and p must have the same length")
    for nl, pl in zip(n, p):
        if pl < 1 or nl % pl:
            raise ValueError(f"p_l must divide n_l, got n={n} p={p}")
    return n, p, tuple(nl // pl for nl, pl in zip(n, p))


def to_cyclic(X: np.ndarray, p) -> np.ndarray:
    """Buffer D with D[rank(s)*M + lin(k)] = X[s + k*p] (s, k, p are d-tuples).

    rank(s) is row-major over s (s_d fastest); lin(k) is row-major over the
    local index k in [n_1/p_1] x ... x [n_d/p_d].
    """
    X = np.asarray(X)
    n, p, m = _local_shape(X.shape, p)
    d = len(n)
    split = []
    for l in range(d):
        split += [m[l], p[l]]           # global index g_l = k_l * p_l + s_l
    order = [2 * l + 1 for l in range(d)] + [2 * l for l in range(d)]
    return np.ascontiguousarray(X.reshape(split).transpose(order)).reshape(-1)


def from_cyclic(D: np.ndarray, n, p) -> np.ndarray:
    """Inverse of :func:`to_cyclic`: the natural-order n_1 x ... x n_d array."""
    n, p, m = _local_shape(n, p)
    d = len(n)
    blocks = np.asarray(D).reshape(tuple(p) + tuple(m))
    order = []
    for l in range(d):
        order += [d + l, l]              # back to (k_1, s_1, ..., k_d, s_d)
    return np.ascontiguousarray(blocks.transpose(order)).reshape(n)


def cyclic_dft(D: np.ndarray, n, p, direction: int = FORWARD, nthreads: int = 0) -> np.ndarray:
    """Expected output of the method: the DFT of the cyclic buffer D, in the same layout."""
    return to_cyclic(dft(from_cyclic(D, n, p), direction, nthreads), p)


# ----------------------------------------------------------------------------
# Algorithm 2.3, executed processor by processor
# ----------------------------------------------------------------------------

def _root(nl: int, e: np.ndarray, sign: int) -> np.ndarray:
    """exp(sign*2*pi*i*e/nl) with e reduced mod nl; exact at the quarter points."""
    e = np.mod(np.asarray(e, dtype=np.int64), nl)
    w = np.exp(sign * 2j * np.pi * (e.astype(np.float64) / nl))
    quarter = (4 * e) % nl == 0
    if np.any(quarter):
        qv = (4 * e[quarter]) // nl
        w[quarter] = np.array([1, 1j * sign, -1, -1j * sign])[qv]
    return w


def _grid(n, p):
    n, p, m = _local_shape(n, p)
    for nl, pl in zip(n, p):
        if nl % (pl * pl):
            raise ValueError(f"Algorithm 2.3 needs p_l^2 | n_l, got n={n} p={p}")
    q = tuple(ml // pl for ml, pl in zip(m, p))
    procs = list(itertools.product(*[range(pl) for pl in p]))   # row-major rank order
    return n, p, m, q, procs


def emulate_local_fft(D: np.ndarray, n, p, direction: int = FORWARD) -> np.ndarray:
    """Superstep 0, first line: Y^(s) = (F_{m_1} x ... x F_{m_d}) X^(s) on every processor s."""
    _check_direction(direction)
    n, p, m, q, procs = _grid(n, p)
    X = np.asarray(D, dtype=np.complex128).reshape((len(procs),) + m)
    Y = np.empty_like(X)
    for rank in range(len(procs)):
        Y[rank] = fft_axes(X[rank], range(len(n)), direction)
    return Y.reshape(-1)


def emulate_twiddle(Y: np.ndarray, n, p, direction: int = FORWARD) -> np.ndarray:
    """Superstep 0, loop: Z^(s)[k] = (prod_l omega_{n_l}^{k_l s_l}) Y^(s)[k]; the factor is
    built dimension by dimension as in Algorithm 3.1 (factor_1, factor_1*factor_2, ...)."""
    _check_direction(direction)
    n, p, m, q, procs = _grid(n, p)
    d = len(n)
    M = int(np.prod(m))
    Y = np.asarray(Y, dtype=np.complex128).reshape(len(procs), M)
    Z = np.empty_like(Y)
    kgrid = np.indices(m).reshape(d, -1)
    for rank, s in enumerate(procs):
        factor = np.ones(M, dtype=np.complex128)
        for l in range(d):
            factor = factor * _root(n[l], kgrid[l] * s[l], direction)
        Z[rank] = factor * Y[rank]
    return Z.reshape(-1)


def emulate_permute(Z: np.ndarray, n, p) -> np.ndarray:
    """Superstep 1: P(s) puts Z^(s)(r : p : m) into P(r) as W^(r)[s*q : (s+1)*q - 1].

    Pure data movement; the dtype of Z is kept so the result can be compared bit for bit.
    """
    n, p, m, q, procs = _grid(n, p)
    d = len(n)
    Z = np.asarray(Z)
    Zv = Z.reshape((len(procs),) + m)
    W = np.empty_like(Zv)
    for rank_s, s in enumerate(procs):
        for rank_r, r in enumerate(procs):
            dst = tuple(slice(s[l] * q[l], (s[l] + 1) * q[l]) for l in range(d))
            src = tuple(slice(r[l], None, p[l]) for l in range(d))
            W[(rank_r,) + dst] = Zv[(rank_s,) + src]
    return W.reshape(-1)


def emulate_remaining_fft(W: np.ndarray, n, p, direction: int = FORWARD) -> np.ndarray:
    """Superstep 2: V^(r)(t : q : m) = (F_{p_1} x ... x F_{p_d}) W^(r)(t : q : m) for every t.

    Inside a processor the local index is i_l = s'_l q_l + t_l, so the subarray
    W^(r)(t : q : m) is the (s'_1, ..., s'_d) slice of W^(r) viewed as
    (p_1, q_1, ..., p_d, q_d); all t are transformed together."""
    _check_direction(direction)
    n, p, m, q, procs = _grid(n, p)
    d = len(n)
    M = int(np.prod(m))
    W = np.asarray(W, dtype=np.complex128).reshape(len(procs), M)
    V = np.empty_like(W)
    split = []
    for l in range(d):
        split += [p[l], q[l]]
    for rank_r in range(len(procs)):
        V[rank_r] = fft_axes(W[rank_r].reshape(split), [2 * l for l in range(d)], direction).reshape(-1)
    return V.reshape(-1)


def emulate(D: np.ndarray, n, p, direction: int = FORWARD) -> dict:
    """Run Algorithm 2.3 on the cyclic buffer D and return every intermediate buffer.

    Keys (all in the processor-major buffer layout of :func:`to_cyclic`):
      "S0"      Y^(s) = (F_{m_1} x ... x F_{m_d}) X^(s)      (Superstep 0, local DFT)
      "twiddle" Z^(s)[k] = prod_l omega_{n_l}^{k_l s_l} Y^(s)[k]  (Superstep 0, twiddle)
      "S1"      W^(r)[s*q + t] = Z^(s)[r + t*p]             (Superstep 1, the Put)
      "S2"      V^(r)(t:q:m) = (F_{p_1} x ... x F_{p_d}) W^(r)(t:q:m)  (Superstep 2)
      "out"     S2, times 1/N for the inverse
    with m = n/p and q = n/p^2 elementwise. INVERSE conjugates every weight.
    """
    Y = emulate_local_fft(D, n, p, direction)
    Z = emulate_twiddle(Y, n, p, direction)
    W = emulate_permute(Z, n, p)
    V = emulate_remaining_fft(W, n, p, direction)
    out = V.copy()
    if direction == INVERSE:
        out *= 1.0 / V.size
    return {"S0": Y, "twiddle": Z, "S1": W, "S2": V, "out": out}


def circular_convolution(x: np.ndarray, h: np.ndarray) -> np.ndarray:
    """y[j] = sum_k x[k] h[(j - k) mod n], indices taken per dimension (natural
    order, complex128), summed term by term over every k: O(N^2), small arrays only."""
    x = np.asarray(x, dtype=np.complex128)
    h = np.asarray(h, dtype=np.complex128)
    if x.shape != h.shape:
        raise ValueError("x and h must have the same shape")
    axes = tuple(range(x.ndim))
    y = np.zeros_like(x)
    for k in np.ndindex(x.shape):
        if x[k] != 0:
            y += x[k] * np.roll(h, shift=k, axis=axes)     # roll(h, k)[j] = h[(j - k) mod n]
    return y


def rel_l2(y: np.ndarray, yref: np.ndarray) -> float:
    """||y - yref||_2 / ||yref||_2 over all complex entries, in FP64 (numpy pairwise sums)."""
    y = np.asarray(y).astype(np.complex128).reshape(-1)
    yref = np.asarray(yref).astype(np.complex128).reshape(-1)
    num = np.sqrt(np.sum(np.abs(y - yref) ** 2))
    den = np.sqrt(np.sum(np.abs(yref) ** 2))
    if den == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return float(num / den)
