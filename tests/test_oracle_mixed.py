"""Pins of the oracle on sides that are not powers of two (the 1-D transforms
of eq. (1.3) summed from the 1-D definition), for the mixed-radix path:
brute force against the d-dimensional sum of eq. (1.2), numpy.fft, closed
forms, Parseval, Theorem 2.1 on mixed grids, and planted mistakes."""
import numpy as np
import pytest

import oracle
from oracle import FORWARD, INVERSE

SHAPES = [(3,), (5,), (6,), (7,), (12,), (3, 5), (6, 10), (7, 4, 3), (9, 25), (15, 14)]


def crand(shape, seed):
    r = np.random.default_rng(seed)
    return r.uniform(-1, 1, shape) + 1j * r.uniform(-1, 1, shape)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("direction", [FORWARD, INVERSE])
def test_axes_transform_equals_direct_sum(shape, direction):
    x = crand(shape, 1)
    assert oracle.rel_l2(oracle.dft(x, direction), oracle.dft_direct(x, direction)) < 1e-14


@pytest.mark.parametrize("shape", [(60,), (12, 18), (14, 15, 6), (98,), (45, 8)])
def test_numpy_fftn(shape):
    x = crand(shape, 2)
    assert oracle.rel_l2(oracle.dft(x), np.fft.fftn(x)) < 1e-14
    assert oracle.rel_l2(oracle.dft(x, INVERSE), np.fft.ifftn(x)) < 1e-14


@pytest.mark.parametrize("shape", [(12,), (6, 10), (7, 9, 5)])
def test_closed_forms(shape):
    N = int(np.prod(shape))
    d = np.zeros(shape, complex)
    d[(0,) * len(shape)] = 1
    assert np.array_equal(oracle.dft(d), np.ones(shape, complex))      # impulse: all ones, exactly
    c = np.full(shape, 0.75 - 0.5j)
    y = oracle.dft(c)
    assert abs(y[(0,) * len(shape)] - N * (0.75 - 0.5j)) < 1e-12
    y[(0,) * len(shape)] = 0
    assert np.abs(y).max() < 1e-12                                   # constant: only the zero frequency
    f = tuple(min(2, n - 1) for n in shape)                          # plane wave exp(+2 pi i f.j / n) -> N delta_f
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    x = np.exp(2j * np.pi * sum(fi * g / n for fi, g, n in zip(f, grids, shape)))
    z = oracle.dft(x)
    assert abs(z[f] - N) < 1e-10
    z[f] = 0
    assert np.abs(z).max() < 1e-10


@pytest.mark.parametrize("shape", [(30,), (9, 14), (5, 6, 7)])
def test_parseval_and_round_trip(shape):
    x = crand(shape, 3)
    y = oracle.dft(x)
    assert abs(np.vdot(y, y).real - x.size * np.vdot(x, x).real) < 1e-11 * x.size
    assert oracle.rel_l2(oracle.dft(y, INVERSE), x) < 1e-14


@pytest.mark.parametrize("n,p", [((12,), (2,)), ((36,), (3,)), ((60, 60), (2, 2)), ((126, 12), (3, 2)),
                                 ((49, 27), (7, 3)), ((18, 20, 12), (3, 2, 2)), ((100,), (5,))])
@pytest.mark.parametrize("direction", [FORWARD, INVERSE])
def test_algorithm_2_3_on_mixed_grids(n, p, direction):
    """Theorem 2.1 on grids with p_l not a power of two: emulating the
    supersteps gives exactly the DFT (up to rounding)."""
    N = int(np.prod(n))
    D = crand(N, 4)
    em = oracle.emulate(D, n, p, direction)
    assert oracle.rel_l2(em["out"], oracle.cyclic_dft(D, n, p, direction)) < 1e-14
    assert np.array_equal(np.sort_complex(em["S1"]), np.sort_complex(em["twiddle"]))   # S1 is a permutation


def test_pins_detect_planted_mistakes_on_mixed_sizes():
    def pins_pass(fn):
        for shape in [(6,), (12, 5), (3, 7, 2)]:
            x = crand(shape, 5)
            if oracle.rel_l2(fn(x), oracle.dft_direct(x)) > 1e-12:
                return False
            d = np.zeros(shape, complex)
            d[(0,) * len(shape)] = 1
            if np.abs(fn(d) - 1).max() > 1e-12:
                return False
        return True
    assert pins_pass(oracle.dft)
    mutants = {
        "sign flipped": lambda x: oracle.dft(x, INVERSE) * x.size,
        "axis strides swapped": lambda x: oracle.dft(x.reshape(x.shape[::-1])).reshape(x.shape),
        "last term dropped": lambda x: oracle.dft(np.where(np.arange(x.size).reshape(x.shape) == x.size - 1, 0, x)),
        "index off by one": lambda x: np.roll(oracle.dft(x), 1),
        "one axis skipped": lambda x: oracle.fft_axes(x, range(max(x.ndim - 1, 0))) if x.ndim > 1 else x,
        "conjugated output": lambda x: np.conj(oracle.dft(x)),
    }
    for name, fn in mutants.items():
        assert not pins_pass(fn), name
