"""Pins of the oracle's DCT and DST (types II and III) in the zig-zag cyclic
distribution.

Independent of the oracle's code path: the hand-worked layout fixture, the
library transforms (scipy.fft.dctn / dstn / idctn / idstn, type 2, unnormalised),
the definitions summed term by term on tiny arrays, closed forms (constant input,
basis vectors), the round trips, and the identity that makes the zig-zag order
the natural one for the DCT (its coefficients follow from the DFT of v alone).
Planted mistakes must each fail a pin.
"""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.fft

import oracle
from oracle import FORWARD, INVERSE
from oracle import r2r

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rreal(shape, seed):
    return np.random.default_rng(seed).uniform(-1, 1, shape)


def test_layout_matches_the_hand_worked_fixture():
    rows = 0
    for line in open(os.path.join(GOLDEN, "r2r_layout.txt")):
        if line.startswith("#") or not line.strip():
            continue
        kind, n, p, idx = [f.strip() for f in line.split("|")]
        n = tuple(int(v) for v in n.split())
        p = tuple(int(v) for v in p.split())
        idx = [int(v) for v in idx.split()]
        X = np.arange(int(np.prod(n)), dtype=float).reshape(n)
        if kind == "signal":
            assert r2r.signal_to_buffer(X, p).astype(int).tolist() == idx
            assert np.array_equal(r2r.buffer_to_signal(np.array(idx, float), n, p).reshape(-1),
                                  np.arange(X.size, dtype=float))
        else:
            assert r2r.coeffs_to_buffer(X, p).astype(int).tolist() == idx
        rows += 1
    assert rows == 4


SHAPES = [(8,), (6,), (4, 6), (8, 4), (4, 6, 8), (2, 4, 2, 6)]
LIB = {(r2r.DCT, FORWARD): lambda a: scipy.fft.dctn(a, type=2),
       (r2r.DST, FORWARD): lambda a: scipy.fft.dstn(a, type=2),
       (r2r.DCT, INVERSE): lambda a: scipy.fft.idctn(a, type=2),
       (r2r.DST, INVERSE): lambda a: scipy.fft.idstn(a, type=2)}


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("kind", [r2r.DCT, r2r.DST])
@pytest.mark.parametrize("direction", [FORWARD, INVERSE])
def test_matches_scipy(shape, kind, direction):
    X = rreal(shape, 1)
    assert np.abs(r2r.transform(X, kind, direction) - LIB[(kind, direction)](X)).max() < 1e-12


def _direct(X, kind):
    """The forward definitions summed term by term."""
    n = X.shape
    Y = np.zeros(n)
    for k in itertools.product(*[range(v) for v in n]):
        acc = 0.0
        for j in itertools.product(*[range(v) for v in n]):
            w = 1.0
            for kl, jl, N in zip(k, j, n):
                if kind == r2r.DCT:
                    w *= 2 * math.cos(math.pi * kl * (2 * jl + 1) / (2 * N))
                else:
                    w *= 2 * math.sin(math.pi * (kl + 1) * (2 * jl + 1) / (2 * N))
            acc += w * X[j]
        Y[k] = acc
    return Y


@pytest.mark.parametrize("shape", [(6,), (4, 2), (2, 4, 2)])
@pytest.mark.parametrize("kind", [r2r.DCT, r2r.DST])
def test_forward_is_the_definition_summed_by_terms(shape, kind):
    X = rreal(shape, 2)
    assert np.abs(r2r.transform(X, kind) - _direct(X, kind)).max() < 1e-12


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("kind", [r2r.DCT, r2r.DST])
def test_round_trips(shape, kind):
    X = rreal(shape, 3)
    assert np.abs(r2r.transform(r2r.transform(X, kind), kind, INVERSE) - X).max() < 1e-13
    assert np.abs(r2r.transform(r2r.transform(X, kind, INVERSE), kind) - X).max() < 1e-13


def test_closed_forms():
    N = 8
    # constant c: DCT 2^d N c at k = 0 and nothing else; DST of a constant: y[k] = 0 for odd k
    X = np.full((N, N), 0.25)
    Y = r2r.transform(X, r2r.DCT)
    want = np.zeros((N, N))
    want[0, 0] = 4 * N * N * 0.25
    assert np.abs(Y - want).max() < 1e-12
    Ys = r2r.transform(np.full(N, 1.0), r2r.DST)
    assert np.abs(Ys[1::2]).max() < 1e-12 and np.all(Ys[0::2] > 0)
    # basis vectors: cos(pi k0 (2n+1)/(2N)) gives N at k0 (k0 >= 1); sin(pi (k0+1)(2n+1)/(2N))
    # gives N at k0, or 2N at k0 = N - 1
    n = np.arange(N)
    for k0 in range(1, N):
        y = r2r.transform(np.cos(np.pi * k0 * (2 * n + 1) / (2 * N)), r2r.DCT)
        assert abs(y[k0] - N) < 1e-12 and np.abs(np.delete(y, k0)).max() < 1e-12
    for k0 in range(N):
        y = r2r.transform(np.sin(np.pi * (k0 + 1) * (2 * n + 1) / (2 * N)), r2r.DST)
        assert abs(y[k0] - (2 * N if k0 == N - 1 else N)) < 1e-12 and np.abs(np.delete(y, k0)).max() < 1e-12


@pytest.mark.parametrize("n", [(8,), (6, 4), (4, 8, 2)])
def test_dct_follows_from_the_dft_of_the_zigzag_order(n):
    """y = (tensor product over dimensions of C_l) applied to V = DFT(v), with
    (C f)[k] = w^k f[k] + w^-k f[-k], w = exp(-2 pi i / (4 N_l)): the coefficients
    need only the DFT of the zig-zag array (the reason for the layout)."""
    X = rreal(n, 4)
    V = np.fft.fftn(r2r.to_zigzag(X))
    for ax, N in enumerate(n):
        k = np.arange(N)
        w = np.exp(-2j * np.pi * k / (4 * N))
        shape = [1] * len(n)
        shape[ax] = N
        Vm = np.take(V, (-k) % N, axis=ax)
        V = w.reshape(shape) * V + np.conj(w).reshape(shape) * Vm
    assert np.abs(V.imag).max() < 1e-11
    assert np.abs(V.real - r2r.transform(X, r2r.DCT)).max() < 1e-11


@pytest.mark.parametrize("n,p", [((8,), (2,)), ((4, 4), (2, 2)), ((8, 12), (2, 3)), ((4, 6, 8), (1, 3, 2))])
@pytest.mark.parametrize("kind", [r2r.DCT, r2r.DST])
def test_buffer_transforms(n, p, kind):
    X = rreal(n, 5)
    buf = r2r.signal_to_buffer(X, p)
    out = r2r.r2r_cyclic(buf, n, p, kind, FORWARD)
    assert np.abs(r2r.buffer_to_coeffs(out, n, p) - LIB[(kind, FORWARD)](X)).max() < 1e-12
    back = r2r.r2r_cyclic(out, n, p, kind, INVERSE)
    assert np.abs(back - buf).max() < 1e-13


def test_rejects_odd_sides_and_bad_grids():
    with pytest.raises(ValueError):
        r2r.signal_to_buffer(np.zeros((5, 4)), (1, 1))
    with pytest.raises(ValueError):
        r2r.signal_to_buffer(np.zeros(12), (4,))        # 4 does not divide 6


def _pins_pass(transform, zigzag):
    try:
        for shape in [(8,), (4, 6)]:
            X = rreal(shape, 9)
            for kind in (r2r.DCT, r2r.DST):
                if np.abs(transform(X, kind, FORWARD) - LIB[(kind, FORWARD)](X)).max() > 1e-12:
                    return False
                if np.abs(transform(LIB[(kind, FORWARD)](X), kind, INVERSE) - X).max() > 1e-12:
                    return False
        got = zigzag(np.arange(8, dtype=float))
        if got.astype(int).tolist() != [0, 2, 4, 6, 7, 5, 3, 1]:
            return False
    except Exception:
        return False
    return True


def test_pins_detect_planted_mistakes():
    assert _pins_pass(r2r.transform, r2r.to_zigzag)

    def half_offset_dropped(X, kind, direction):            # (2n) instead of (2n + 1)
        if direction == INVERSE or kind == r2r.DST:
            return r2r.transform(X, kind, direction)
        Y = np.asarray(X, float)
        for ax, N in enumerate(Y.shape):
            A = 2.0 * np.cos(np.pi * np.arange(N)[:, None] * (2 * np.arange(N)[None, :]) / (2 * N))
            Y = np.moveaxis(np.tensordot(A, np.moveaxis(Y, ax, 0), axes=1), 0, ax)
        return Y

    def dst_without_shift(X, kind, direction):             # sin(pi k ...) instead of (k + 1)
        if kind == r2r.DCT or direction == INVERSE:
            return r2r.transform(X, kind, direction)
        Y = np.asarray(X, float)
        for ax, N in enumerate(Y.shape):
            A = 2.0 * np.sin(np.pi * np.arange(N)[:, None] * (2 * np.arange(N)[None, :] + 1) / (2 * N))
            Y = np.moveaxis(np.tensordot(A, np.moveaxis(Y, ax, 0), axes=1), 0, ax)
        return Y

    def inverse_without_half(X, kind, direction):          # y[0] weighted 1 instead of 1/2
        if direction == FORWARD or kind == r2r.DST:
            return r2r.transform(X, kind, direction)
        Y = np.asarray(X, float)
        for ax, N in enumerate(Y.shape):
            A = np.cos(np.pi * np.arange(N)[None, :] * (2 * np.arange(N)[:, None] + 1) / (2 * N)) / N
            Y = np.moveaxis(np.tensordot(A, np.moveaxis(Y, ax, 0), axes=1), 0, ax)
        return Y

    def odd_ascending(X):                                  # odd samples ascending, not descending
        X = np.asarray(X, float)
        return np.concatenate([X[0::2], X[1::2]])

    assert not _pins_pass(half_offset_dropped, r2r.to_zigzag)
    assert not _pins_pass(dst_without_shift, r2r.to_zigzag)
    assert not _pins_pass(inverse_without_half, r2r.to_zigzag)
    assert not _pins_pass(r2r.transform, odd_ascending)
