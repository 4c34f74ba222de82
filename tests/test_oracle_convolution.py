"""Pins of the oracle's direct circular convolution (the definition summed term
by term), by facts the definition fixes: a worked example, deltas (identity and
exact cyclic shifts), commutativity, linearity, and the convolution theorem
through the oracle's independent FFT."""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "convolution_1d_4.txt")


def rnd(shape, seed):
    r = np.random.default_rng(seed)
    return r.uniform(-1, 1, shape) + 1j * r.uniform(-1, 1, shape)


def test_worked_example():
    rows = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        k, *vals = line.split()
        rows[k] = np.array([float(v) for v in vals])
    assert np.array_equal(oracle.circular_convolution(rows["x"], rows["h"]).real, rows["y"])


@pytest.mark.parametrize("shape", [(8,), (4, 6), (3, 4, 5)])
def test_deltas_give_identity_and_exact_shifts(shape):
    x = rnd(shape, 1)
    d0 = np.zeros(shape, complex)
    d0[(0,) * len(shape)] = 1
    assert np.array_equal(oracle.circular_convolution(x, d0), x)
    s = tuple((i + 1) % n for i, n in enumerate(shape))
    ds = np.zeros(shape, complex)
    ds[s] = 1
    assert np.array_equal(oracle.circular_convolution(x, ds), np.roll(x, s, axis=tuple(range(len(shape)))))


def test_commutative_and_linear():
    x, h, g = rnd((4, 8), 2), rnd((4, 8), 3), rnd((4, 8), 4)
    a = oracle.circular_convolution(x, h)
    assert np.abs(a - oracle.circular_convolution(h, x)).max() < 1e-13
    lhs = oracle.circular_convolution(2.5 * x - 1j * g, h)
    rhs = 2.5 * a - 1j * oracle.circular_convolution(g, h)
    assert np.abs(lhs - rhs).max() < 1e-12


@pytest.mark.parametrize("shape", [(16,), (8, 8), (4, 8, 2)])
def test_convolution_theorem_against_the_oracle_fft(shape):
    x, h = rnd(shape, 5), rnd(shape, 6)
    via_fft = oracle.dft(oracle.dft(x) * oracle.dft(h), oracle.INVERSE)     # inverse includes 1/N
    direct = oracle.circular_convolution(x, h)
    assert oracle.rel_l2(direct, via_fft) < 1e-13
