"""Pins of the oracle's real-input transform in the cyclic distribution.

Independent of the oracle's code path: the hand-worked layout fixture, a
library real FFT (numpy.fft.rfftn / irfftn), eq. (1.2) summed term by term on
tiny arrays, closed forms, the Hermitian symmetry and the round trip; planted
mistakes must each fail a pin.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import real

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rreal(shape, seed):
    return np.random.default_rng(seed).uniform(-1, 1, shape)


def test_layout_matches_the_hand_worked_fixture():
    rows = 0
    for line in open(os.path.join(GOLDEN, "real_layout.txt")):
        if line.startswith("#") or not line.strip():
            continue
        kind, n, p, idx = [f.strip() for f in line.split("|")]
        n = tuple(int(v) for v in n.split())
        p = tuple(int(v) for v in p.split())
        idx = [int(v) for v in idx.split()]
        N = int(np.prod(n))
        if kind == "real":
            assert real.to_cyclic_real(np.arange(N, dtype=float).reshape(n), p).astype(int).tolist() == idx
            back = real.from_cyclic_real(np.array(idx, dtype=float), n, p)
            assert (back.reshape(-1) == np.arange(N)).all()
        else:
            Y = np.arange(N).reshape(n).astype(complex)
            assert real.spectrum_to_buffer(Y, p).real.astype(int).tolist() == idx
        rows += 1
    assert rows == 6


SHAPES = [((8,), (2,)), ((16,), (4,)), ((4, 4), (2, 2)), ((8, 16), (2, 4)), ((4, 6, 8), (2, 3, 2)),
          ((2,), (1,)), ((6, 2), (1, 1)), ((16, 32), (4, 4))]


@pytest.mark.parametrize("n,p", SHAPES)
def test_forward_matches_numpy_rfftn(n, p):
    X = rreal(n, 1)
    got = real.rfft_cyclic(real.to_cyclic_real(X, p), n, p)
    R = np.fft.rfftn(X)                               # [..., : n_d/2 + 1]
    h = n[-1] // 2
    half, plane = real.buffer_to_half(got, n, p)
    assert np.abs(half - R[..., :h]).max() < 1e-12
    assert np.abs(plane - R[..., h]).max() < 1e-12


@pytest.mark.parametrize("n,p", SHAPES[:5])
def test_forward_is_eq_1_2_summed_by_terms(n, p):
    X = rreal(n, 2)
    want = real.spectrum_to_buffer(oracle.dft_direct(X.astype(complex)), p)
    assert oracle.rel_l2(real.rfft_cyclic(real.to_cyclic_real(X, p), n, p), want) < 1e-15


@pytest.mark.parametrize("n,p", SHAPES)
def test_inverse_matches_numpy_irfftn_and_round_trips(n, p):
    X = rreal(n, 3)
    buf = real.rfft_cyclic(real.to_cyclic_real(X, p), n, p)
    back = real.irfft_cyclic(buf, n, p)
    assert np.abs(back - real.to_cyclic_real(X, p)).max() < 1e-14
    R = np.fft.rfftn(X)
    Xn = np.fft.irfftn(R, s=n, axes=list(range(len(n))))
    assert np.abs(real.from_cyclic_real(back, n, p) - Xn).max() < 1e-14


def test_hermitian_extension_gives_the_full_spectrum():
    n = (6, 4, 8)
    X = rreal(n, 4)
    Y = oracle.dft(X.astype(complex))
    half, plane = Y[..., :4], Y[..., 4]
    assert np.abs(real.full_from_half(half, plane, n) - Y).max() < 1e-12


def test_closed_forms():
    n, p = (8, 16), (2, 4)
    N = 128
    # impulse at the origin: every output is exactly one
    X = np.zeros(n)
    X[0, 0] = 1.0
    assert np.array_equal(real.rfft_cyclic(real.to_cyclic_real(X, p), n, p), np.ones(N // 2 + 8, complex))
    # constant c: c N at k = 0, nothing elsewhere
    X = np.full(n, 0.5)
    half, plane = real.buffer_to_half(real.rfft_cyclic(real.to_cyclic_real(X, p), n, p), n, p)
    expect = np.zeros((8, 8), complex)
    expect[0, 0] = 0.5 * N
    assert np.abs(half - expect).max() < 1e-12 and np.abs(plane).max() < 1e-12
    # a cosine of frequency f along the last axis: N/2 at k = (0, f)
    f = 3
    X = np.cos(2 * np.pi * f * np.arange(16) / 16)[None, :].repeat(8, axis=0)
    half, plane = real.buffer_to_half(real.rfft_cyclic(real.to_cyclic_real(X, p), n, p), n, p)
    expect = np.zeros((8, 8), complex)
    expect[0, f] = N / 2
    assert np.abs(half - expect).max() < 1e-12 and np.abs(plane).max() < 1e-12
    # alternating signs along the last axis: all in the Nyquist plane, N at k' = 0
    X = np.ones(n) * (-1.0) ** np.arange(16)[None, :]
    half, plane = real.buffer_to_half(real.rfft_cyclic(real.to_cyclic_real(X, p), n, p), n, p)
    assert np.abs(half).max() < 1e-12
    assert abs(plane[0] - N) < 1e-12 and np.abs(plane[1:]).max() < 1e-12


def test_rejects_odd_last_side_and_bad_grid():
    with pytest.raises(ValueError):
        real.to_cyclic_real(np.zeros(7), (1,))
    with pytest.raises(ValueError):
        real.to_cyclic_real(np.zeros(12), (4,))     # 4 does not divide 6


def _pins_pass(forward):
    for n, p in [((8,), (2,)), ((4, 4), (2, 2)), ((8, 16), (2, 4))]:
        X = rreal(n, 9)
        R = np.fft.rfftn(X)
        h = n[-1] // 2
        want = np.concatenate([oracle.to_cyclic(R[..., :h], p),
                               oracle.to_cyclic(R[..., h], p[:-1]) if len(n) > 1 else R[..., h].reshape(1)])
        if np.abs(forward(real.to_cyclic_real(X, p), n, p) - want).max() > 1e-12:
            return False
    return True


def test_pins_detect_planted_mistakes():
    assert _pins_pass(real.rfft_cyclic)

    def upper_half(buf, n, p):
        X = real.from_cyclic_real(buf, n, p)
        Y = real.rfft(X)
        h = n[-1] // 2
        return real.spectrum_to_buffer(np.concatenate([Y[..., h:], Y[..., :h]], axis=-1), p)

    def pairs_swapped(buf, n, p):
        b = np.asarray(buf).reshape(-1, 2)[:, ::-1].reshape(-1)      # (im, re) instead of (re, im)
        return real.rfft_cyclic(b, n, p)

    def plane_from_zero(buf, n, p):
        X = real.from_cyclic_real(buf, n, p)
        Y = real.rfft(X)
        Y[..., n[-1] // 2] = Y[..., 0]
        return real.spectrum_to_buffer(Y, p)

    def conjugated(buf, n, p):
        return np.conj(real.rfft_cyclic(buf, n, p))

    for name, fn in {"upper half": upper_half, "re/im swapped": pairs_swapped,
                     "Nyquist plane from k_d = 0": plane_from_zero, "conjugated": conjugated}.items():
        assert not _pins_pass(fn), name
