"""Pins of the FP64 oracle to facts fixed by the paper and by mathematics.

Every check here is independent of the oracle's own code path: hand-worked
DFTs, closed forms, invariants, brute force on tiny inputs, a library FFT, and
the layout facts of Section 1.1 / Algorithm 2.2. The mutation tests at the end
plant plausible mistakes in a copy of the oracle and confirm that a pin fails.
"""
import itertools
import os

import numpy as np
import pytest

import oracle
from oracle import FORWARD, INVERSE

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
rng = np.random.default_rng(12345)


def crand(shape, seed=None):
    g = rng if seed is None else np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


SMALL_SHAPES = [(1,), (2,), (4,), (8,), (16,), (64,), (8, 8), (16, 4), (4, 16), (2, 32), (4, 4, 4),
                (8, 2, 4), (2, 4, 8, 2), (4, 4, 4, 4), (1, 8), (8, 1, 2), (2, 2, 2, 2, 2, 2)]


# ---------------------------------------------------------------- hand-worked DFTs (eq. 1.1)

def _read_hand():
    cases = []
    for line in open(os.path.join(GOLDEN, "dft_hand.txt")):
        if line.startswith("#") or not line.strip():
            continue
        n, xs, ys = [f.strip() for f in line.split("|")]
        x = np.array([complex(*map(float, t.split(","))) for t in xs.split()])
        y = np.array([complex(*map(float, t.split(","))) for t in ys.split()])
        assert len(x) == int(n) == len(y)
        cases.append((x, y))
    return cases


@pytest.mark.parametrize("case", range(6))
def test_hand_worked_dft(case):
    x, y = _read_hand()[case]
    np.testing.assert_allclose(oracle.dft_direct(x), y, atol=1e-15)
    np.testing.assert_allclose(oracle.dft(x), y, atol=1e-15)
    np.testing.assert_allclose(oracle.dft_points(x, range(len(x))), y, atol=1e-15)


# ---------------------------------------------------------------- brute force and library

@pytest.mark.parametrize("shape", SMALL_SHAPES)
@pytest.mark.parametrize("direction", [FORWARD, INVERSE])
def test_fft_matches_direct_sum(shape, direction):
    x = crand(shape)
    ref = oracle.dft_direct(x, direction)
    assert oracle.rel_l2(oracle.dft(x, direction), ref) < 1e-15
    assert oracle.rel_l2(oracle.dft_points(x, np.arange(x.size), direction), ref.reshape(-1)) < 1e-15


@pytest.mark.parametrize("shape", [(64, 64, 64), (32, 16, 8, 4), (256, 2), (2, 1024), (8, 8, 8, 8, 8)])
def test_fft_matches_numpy(shape):
    x = crand(shape)
    assert oracle.rel_l2(oracle.dft(x), np.fft.fftn(x)) < 1e-15
    assert oracle.rel_l2(oracle.dft(x, INVERSE), np.fft.ifftn(x)) < 1e-15


def test_direct_sum_matches_numpy():
    for shape in [(16,), (8, 4), (4, 2, 8), (3, 5), (6, 10)]:   # direct sum is not tied to powers of two
        x = crand(shape)
        assert oracle.rel_l2(oracle.dft_direct(x), np.fft.fftn(x)) < 1e-15


def test_points_on_large_array():
    x = crand((64, 32, 16))
    full = oracle.dft(x).reshape(-1)
    k = np.random.default_rng(1).integers(0, x.size, 24)
    assert oracle.rel_l2(oracle.dft_points(x, k), full[k]) < 1e-15


# ---------------------------------------------------------------- closed forms

def _omega_power(shape, j0, sign=-1):
    grids = np.indices(shape)
    phase = sum(grids[l] * j0[l] / shape[l] for l in range(len(shape)))
    return np.exp(sign * 2j * np.pi * phase)


@pytest.mark.parametrize("shape", [(8,), (16, 4), (4, 8, 2), (2, 2, 4, 8)])
def test_impulse_at_origin_gives_exact_ones(shape):
    x = np.zeros(shape, complex)
    x[(0,) * len(shape)] = 1.0
    y = oracle.dft(x)
    assert np.array_equal(y, np.ones(shape, complex))


@pytest.mark.parametrize("shape", [(8,), (16, 4), (4, 8, 2), (2, 2, 4, 8)])
def test_shifted_impulse(shape):
    j0 = tuple(int(v) for v in np.random.default_rng(len(shape)).integers(0, shape))
    x = np.zeros(shape, complex)
    x[j0] = 1.0
    assert np.abs(oracle.dft(x) - _omega_power(shape, j0)).max() < 1e-14
    assert np.abs(oracle.dft(x, INVERSE) * x.size - _omega_power(shape, j0, +1)).max() < 1e-14


@pytest.mark.parametrize("shape", [(8,), (16, 4), (4, 8, 2)])
def test_constant_and_plane_wave(shape):
    N = int(np.prod(shape))
    c = 0.75 - 0.5j
    y = oracle.dft(np.full(shape, c))
    expect = np.zeros(shape, complex)
    expect[(0,) * len(shape)] = c * N
    assert np.abs(y - expect).max() < 1e-13
    f = tuple(int(v) for v in np.random.default_rng(7).integers(0, shape))
    wave = _omega_power(shape, f, +1)      # exp(+2 pi i f.j / n) -> N delta_f
    y = oracle.dft(wave)
    expect = np.zeros(shape, complex)
    expect[f] = N
    assert np.abs(y - expect).max() < 1e-12


def test_separable_input_reduces_to_1d():
    vs = [crand((8,)), crand((4,)), crand((16,))]
    x = np.einsum("i,j,k->ijk", *vs)
    y1 = [oracle.dft(v) for v in vs]
    assert oracle.rel_l2(oracle.dft(x), np.einsum("i,j,k->ijk", *y1)) < 1e-15


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("shape", [(64,), (16, 32), (8, 4, 16), (4, 4, 4, 4, 4)])
def test_parseval_linearity_roundtrip(shape):
    x, z = crand(shape), crand(shape)
    a, b = 0.3 - 1.7j, -2.1 + 0.4j
    X, Z = oracle.dft(x), oracle.dft(z)
    N = x.size
    assert abs(np.sum(np.abs(X) ** 2) - N * np.sum(np.abs(x) ** 2)) / (N * np.sum(np.abs(x) ** 2)) < 1e-14
    assert oracle.rel_l2(oracle.dft(a * x + b * z), a * X + b * Z) < 1e-14
    assert oracle.rel_l2(oracle.dft(X, INVERSE), x) < 1e-15


@pytest.mark.parametrize("shape", [(16,), (8, 16), (4, 8, 2)])
def test_shift_theorem(shape):
    x = crand(shape)
    j0 = tuple(int(v) for v in np.random.default_rng(3).integers(0, shape))
    shifted = np.roll(x, j0, axis=tuple(range(len(shape))))   # x'[j] = x[j - j0]
    assert oracle.rel_l2(oracle.dft(shifted), oracle.dft(x) * _omega_power(shape, j0)) < 1e-14


@pytest.mark.parametrize("shape", [(16,), (8, 16), (4, 8, 2)])
def test_hermitian_symmetry_of_real_input(shape):
    x = np.random.default_rng(9).standard_normal(shape)
    Y = oracle.dft(x + 0j)
    neg = tuple((-np.indices(shape)[l]) % shape[l] for l in range(len(shape)))
    assert np.abs(Y[neg] - np.conj(Y)).max() < 1e-12


# ---------------------------------------------------------------- cyclic distribution (Section 1.1)

def _phi_buffer(X, p):
    """D[rank(s) M + lin(k)] = X[s + k p], written out with explicit loops."""
    n = X.shape
    m = tuple(a // b for a, b in zip(n, p))
    M = int(np.prod(m))
    D = np.empty(X.size, X.dtype)
    for rank, s in enumerate(itertools.product(*[range(v) for v in p])):
        for lin, k in enumerate(itertools.product(*[range(v) for v in m])):
            D[rank * M + lin] = X[tuple(s[l] + k[l] * p[l] for l in range(len(n)))]
    return D


@pytest.mark.parametrize("n,p", [((8,), (4,)), ((8, 8), (2, 2)), ((8, 8, 8), (2, 2, 2)), ((16, 4, 8), (4, 2, 1)),
                                 ((4, 4, 4, 4), (2, 1, 2, 4))])
def test_to_cyclic_matches_phi(n, p):
    X = crand(n)
    D = oracle.to_cyclic(X, p)
    assert np.array_equal(D, _phi_buffer(X, p))
    assert np.array_equal(oracle.from_cyclic(D, n, p), X)


def test_fig_1_1_ownership():
    # (a) 8 over 4
    rows = [list(map(int, l.split())) for l in open(os.path.join(GOLDEN, "cyclic_1d_8_over_4.txt"))
            if not l.startswith("#")]
    D = oracle.to_cyclic(np.arange(8), (4,))
    for j, s, k in rows:
        assert D[s * 2 + k] == j
    # (b) 8x8 over 2x2 and (c) 8x8x8 over 2x2x2: owner of element g is the block that holds it
    for fname, n, p in [("cyclic_2d_8x8_over_2x2.txt", (8, 8), (2, 2)),
                        ("cyclic_3d_8x8x8_over_2x2x2.txt", (8, 8, 8), (2, 2, 2))]:
        lines = [l.split() for l in open(os.path.join(GOLDEN, fname)) if not l.startswith("#")]
        D = oracle.to_cyclic(np.arange(int(np.prod(n))).reshape(n), p)
        M = D.size // int(np.prod(p))
        owner_of = {int(g): int(i) // M for i, g in enumerate(D)}
        grid = [list(r) for r in lines if r[0] != "plane"]
        for idx, code in enumerate(itertools.chain.from_iterable(grid)):
            s = tuple(int(c) for c in code)
            rank = int(np.ravel_multi_index(s, p))
            assert owner_of[idx] == rank


def test_alg22_worked_example():
    spec = {}
    for line in open(os.path.join(GOLDEN, "alg22_n8_p2.txt")):
        if line.startswith("#") or not line.strip():
            continue
        key, *vals = line.split()
        spec[key] = vals
    x = np.arange(8).astype(complex) + 100j    # label element j of x by its index
    D = oracle.to_cyclic(x, (2,))
    assert [int(v.real) for v in D] == [int(v) for v in spec["input"]]
    st = oracle.emulate(D, (8,), (2,))
    Z = st["twiddle"].reshape(2, 4)
    W = st["S1"].reshape(2, 4)
    for r in (0, 1):
        want = [Z[int(a), int(b)] for a, b in (t.split(":") for t in spec[f"put_to_{r}"])]
        assert np.array_equal(W[r], np.array(want))
    # output placement: the result buffer holds y in the same cyclic order
    y = oracle.dft(x)
    assert np.array_equal(np.array([int(v) for v in spec["output"]]),
                          np.array([0, 2, 4, 6, 1, 3, 5, 7]))
    assert oracle.rel_l2(st["out"], y[[int(v) for v in spec["output"]]]) < 1e-15


# ---------------------------------------------------------------- Algorithm 2.3 (Theorem 2.1)

EMU_CASES = [((8,), (2,)), ((16,), (4,)), ((64,), (8,)), ((16, 8), (2, 2)), ((16, 16, 4), (4, 2, 2)),
             ((8, 8, 8), (2, 2, 2)), ((4, 16, 8), (2, 2, 2)), ((16, 16), (1, 4)), ((4, 4, 4), (2, 2, 2)),
             ((32, 8, 4, 16), (2, 2, 1, 4)), ((4, 4, 4, 4, 4), (2, 2, 2, 2, 2)), ((8, 1, 4), (2, 1, 1)),
             ((1,), (1,)), ((64, 64), (8, 8))]


@pytest.mark.parametrize("n,p", EMU_CASES)
@pytest.mark.parametrize("direction", [FORWARD, INVERSE])
def test_algorithm_2_3_computes_the_dft(n, p, direction):
    X = crand(n)
    D = oracle.to_cyclic(X, p)
    st = oracle.emulate(D, n, p, direction)
    assert oracle.rel_l2(st["out"], oracle.to_cyclic(oracle.dft(X, direction), p)) < 1e-14
    assert oracle.rel_l2(st["out"], oracle.cyclic_dft(D, n, p, direction)) < 1e-14
    # Superstep 1 moves each element exactly once: W is a permutation of Z
    assert np.array_equal(np.sort_complex(st["S1"]), np.sort_complex(st["twiddle"]))


def test_s1_matches_element_formula():
    n, p = (16, 8, 16), (2, 2, 4)
    m = tuple(a // b for a, b in zip(n, p))
    q = tuple(a // b for a, b in zip(m, p))
    D = oracle.to_cyclic(crand(n), p)
    st = oracle.emulate(D, n, p)
    Z = st["twiddle"].reshape(p + m)
    W = st["S1"].reshape(p + m)
    for r in itertools.product(*[range(v) for v in p]):
        for s in itertools.product(*[range(v) for v in p]):
            for t in itertools.product(*[range(v) for v in q]):
                dst = tuple(s[l] * q[l] + t[l] for l in range(3))
                src = tuple(r[l] + t[l] * p[l] for l in range(3))
                assert W[r + dst] == Z[s + src]


def test_grid_of_ones_is_plain_fftn():
    X = crand((8, 16, 4))
    st = oracle.emulate(oracle.to_cyclic(X, (1, 1, 1)), X.shape, (1, 1, 1))
    assert oracle.rel_l2(st["out"], np.fft.fftn(X).reshape(-1)) < 1e-15


def test_emulate_rejects_invalid_grid():
    with pytest.raises(ValueError):
        oracle.emulate(np.zeros(8, complex), (8,), (4,))       # 4^2 does not divide 8


# ---------------------------------------------------------------- pins catch planted mistakes

def _pins_pass(dft_fn):
    """A compact version of the pins above, parameterised by the DFT under test."""
    for x, y in _read_hand():
        if np.abs(dft_fn(x) - y).max() > 1e-12:
            return False
    for shape in [(8,), (16, 4), (4, 8, 2)]:
        x = crand(shape, seed=5)
        if oracle.rel_l2(dft_fn(x), oracle.dft_direct(x)) > 1e-12:
            return False
    return True


def test_pins_detect_planted_mistakes():
    assert _pins_pass(oracle.dft)
    mutants = {
        "sign flipped": lambda x: oracle.dft(x, INVERSE) * x.size,
        "axis strides swapped": lambda x: oracle.dft(x.reshape(x.shape[::-1])).reshape(x.shape),
        "last term dropped": lambda x: oracle.dft(np.where(np.arange(x.size).reshape(x.shape) == x.size - 1,
                                                           0, x)),
        "index off by one": lambda x: np.roll(oracle.dft(x), 1),
        "one axis skipped": lambda x: oracle.fft_axes(x, range(max(x.ndim - 1, 0))) if x.ndim > 1 else x,
        "conjugated output": lambda x: np.conj(oracle.dft(x)),
    }
    for name, fn in mutants.items():
        assert not _pins_pass(fn), name


# ---------------------------------------------------------------- the error measure itself

def _read_rel_l2_cases():
    cases = []
    for line in open(os.path.join(GOLDEN, "rel_l2.txt")):
        if line.startswith("#") or not line.strip():
            continue
        _, ys, refs, expect = [f.strip() for f in line.split("|")]
        y = np.array([complex(*map(float, t.split(","))) for t in ys.split()])
        ref = np.array([complex(*map(float, t.split(","))) for t in refs.split()])
        cases.append((y, ref, float(expect)))
    return cases


def _rel_l2_pins_pass(fn):
    """Every hand-worked case of tests/golden/rel_l2.txt, to 1e-15 relative."""
    for y, ref, expect in _read_rel_l2_cases():
        got = fn(y, ref)
        if np.isinf(expect):
            if not np.isinf(got):
                return False
        elif expect == 0.0:
            if got != 0.0:
                return False
        elif not abs(got - expect) <= 1e-15 * expect:
            return False
    return True


def test_rel_l2_hand_worked_cases():
    cases = _read_rel_l2_cases()
    assert len(cases) == 9
    assert _rel_l2_pins_pass(oracle.rel_l2)
    # shape and dtype of the operands do not matter: the measure is over all entries
    y, ref, expect = cases[2]
    assert oracle.rel_l2(y.reshape(2, 1), ref) == pytest.approx(expect, rel=1e-15)
    assert oracle.rel_l2(y.astype(np.complex64), ref) == pytest.approx(expect, rel=1e-15)


def test_rel_l2_pins_detect_planted_mistakes():
    def ratio(num, den):
        return 0.0 if den == 0 and num == 0 else (float("inf") if den == 0 else num / den)

    def l2(v):
        return np.sqrt(np.sum(np.abs(v) ** 2))

    mutants = {
        "no square root": lambda y, r: ratio(np.sum(np.abs(y - r) ** 2), np.sum(np.abs(r) ** 2)),
        "max-abs ratio": lambda y, r: ratio(np.max(np.abs(y - r)), np.max(np.abs(r))),
        "no denominator": lambda y, r: ratio(l2(y - r), 1.0 if l2(r) else 0.0),
        "normalised by y": lambda y, r: ratio(l2(y - r), l2(y)) if l2(r) else ratio(l2(y), 0.0),
        "L1 norms": lambda y, r: ratio(np.sum(np.abs(y - r)), np.sum(np.abs(r))),
        "real parts only": lambda y, r: ratio(l2((y - r).real), l2(r.real)) if l2(r) else ratio(l2(y), 0.0),
        "single precision": lambda y, r: ratio(float(l2((y - r).astype(np.complex64))),
                                               float(l2(r.astype(np.complex64)))),
        "zero reference passes anything": lambda y, r: 0.0 if l2(r) == 0 else ratio(l2(y - r), l2(r)),
    }
    for name, fn in mutants.items():
        assert not _rel_l2_pins_pass(fn), name
