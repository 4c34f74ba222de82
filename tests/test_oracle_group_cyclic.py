"""Pins of the oracle's group-cyclic distribution and of its FFT with more than
one communication superstep (grids beyond p_max = sqrt(N), Section 2.3).

Independent of the emulator's own code path: the hand-dealt distribution table,
the distribution's two special cases named by the paper (cycle p = cyclic,
cycle 1 = block), eq. (1.2) summed term by term on tiny grids, a library FFT,
Algorithm 2.3's emulator where p_l^2 | n_l (one superstep), the
intermediate data placed exactly as the group-cyclic distribution says, and
planted mistakes that the pins must catch.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import FORWARD, INVERSE
from oracle import group_cyclic as gc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def crand(shape, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def _examples():
    rows = []
    for line in open(os.path.join(GOLDEN, "group_cyclic_examples.txt")):
        if line.startswith("#") or not line.strip():
            continue
        head, own, loc = [f.strip() for f in line.split("|")]
        n, p, c = (int(v) for v in head.split())
        rows.append((n, p, c, [int(v) for v in own.split()], [int(v) for v in loc.split()]))
    return rows


def test_group_cyclic_owner_matches_the_hand_dealt_tables():
    rows = _examples()
    assert len(rows) == 6
    for n, p, c, own, loc in rows:
        got_o, got_l = gc.group_cyclic_owner(np.arange(n), n, p, c)
        assert got_o.tolist() == own, (n, p, c)
        assert got_l.tolist() == loc, (n, p, c)


@pytest.mark.parametrize("n,p", [(8, 4), (16, 4), (64, 8), (36, 6), (1024, 64)])
def test_cycle_p_is_cyclic_and_cycle_1_is_block(n, p):
    j = np.arange(n)
    o, l = gc.group_cyclic_owner(j, n, p, p)
    assert (o == j % p).all() and (l == j // p).all()
    o, l = gc.group_cyclic_owner(j, n, p, 1)
    assert (o == j // (n // p)).all() and (l == j % (n // p)).all()
    # the cycle-p owner is the layout of oracle.to_cyclic (Section 1.1)
    D = oracle.to_cyclic(j, (p,))
    o, l = gc.group_cyclic_owner(D, n, p, p)
    assert (o * (n // p) + l == np.arange(n)).all()


def test_levels_and_superstep_counts():
    assert gc.levels(64, 8) == [(64, 8)]                       # p^2 | n: Algorithm 2.2
    assert gc.levels(64, 16) == [(64, 16), (16, 4)]
    assert gc.levels(16, 8) == [(16, 8), (8, 4), (4, 2)]
    assert gc.levels(1024, 64) == [(1024, 64), (64, 4)]
    assert gc.supersteps((512, 512, 512), (32, 32, 32)) == 2
    assert gc.supersteps((512, 512, 512), (4, 4, 4)) == 1
    for bad in [(8, 8), (12, 6), (12, 3)]:
        with pytest.raises(ValueError):
            gc.levels(*bad)
    # powers of two: each computation phase covers at most log2(m) of the log2(n)
    # index bits of a dimension, so ceil(log n / log m) phases and one superstep fewer
    for K in range(1, 13):
        for P in range(0, K):
            L = K - P
            if 2 * P <= K:
                assert len(gc.levels(1 << K, 1 << P)) == 1
            else:
                assert len(gc.levels(1 << K, 1 << P)) == -(-K // L) - 1, (K, P)


TINY = [((16,), (8,)), ((32,), (16,)), ((8,), (4,)), ((64,), (16,)), ((16, 16), (8, 2)), ((8, 8), (4, 4)),
        ((4, 16, 8), (2, 8, 4)), ((36,), (6,)), ((8, 27), (4, 9)), ((2, 8, 8), (1, 4, 2))]


@pytest.mark.parametrize("n,p", TINY)
@pytest.mark.parametrize("direction", [FORWARD, INVERSE])
def test_emulation_is_the_dft_on_tiny_grids(n, p, direction):
    """eq. (1.2) summed term by term: the group-cyclic algorithm computes the DFT
    and ends in the cyclic distribution it started in."""
    assert gc.supersteps(n, p) >= 1
    X = crand(n, 3)
    D = oracle.to_cyclic(X, p)
    got = gc.emulate_group_cyclic(D, n, p, direction)["out"]
    want = oracle.to_cyclic(oracle.dft_direct(X, direction), p)
    assert oracle.rel_l2(got, want) < 1e-14


@pytest.mark.parametrize("n,p", [((1024,), (64,)), ((512, 256), (32, 64)), ((64, 64, 64), (16, 16, 8)),
                                 ((4096,), (1024,)), ((100, 125), (10, 25))])
def test_emulation_matches_numpy_fftn(n, p):
    X = crand(n, 4)
    D = oracle.to_cyclic(X, p)
    assert oracle.rel_l2(gc.emulate_group_cyclic(D, n, p)["out"], oracle.to_cyclic(np.fft.fftn(X), p)) < 1e-14
    assert oracle.rel_l2(gc.emulate_group_cyclic(D, n, p, INVERSE)["out"],
                         oracle.to_cyclic(np.fft.ifftn(X), p)) < 1e-14


@pytest.mark.parametrize("n,p", [((64,), (8,)), ((16, 32), (4, 2)), ((8, 8, 8), (2, 2, 2)), ((60, 36), (2, 3))])
def test_one_superstep_is_algorithm_2_3(n, p):
    """Where every p_l^2 | n_l the multi-superstep emulator is Algorithm 2.3 stage
    for stage (the Put bit for bit)."""
    X = crand(n, 5)
    D = oracle.to_cyclic(X, p)
    a = gc.emulate_group_cyclic(D, n, p)
    b = oracle.emulate(D, n, p)
    assert a["H"] == 1
    assert np.allclose(a["fft0"], b["S0"], rtol=0, atol=1e-12)
    assert np.allclose(a["tw0"], b["twiddle"], rtol=0, atol=1e-12)
    assert np.array_equal(a["put0"], oracle.emulate_permute(a["tw0"], n, p))
    assert np.allclose(a["fft1"], b["S2"], rtol=0, atol=1e-12)


def test_first_put_lands_in_the_group_cyclic_distribution():
    """After Superstep 0 (F_m, twiddle) the m sub-transforms w^(k)_u = z^(u)_k of
    length p go to groups of c = p/m processors: the array W with W[k p + u] =
    w^(k)_u sits in the group-cyclic distribution with cycle c (Section 2.3)."""
    n, p = 1024, 64
    m, c = n // p, p // (n // p)
    D = oracle.to_cyclic(crand((n,), 6), (p,))
    st = gc.emulate_group_cyclic(D, (n,), (p,))
    Z = st["tw0"].reshape(p, m)                   # z^(u)_k on processor u, local k
    W = np.empty(n, complex)
    for k in range(m):
        for u in range(p):
            W[k * p + u] = Z[u, k]
    owner, local = gc.group_cyclic_owner(np.arange(n), n, p, c)
    put = st["put0"].reshape(p, m)
    assert np.array_equal(put[owner, local], W)


def test_every_put_is_a_permutation():
    n, p = (16, 32), (8, 16)
    D = np.arange(int(np.prod(n))).astype(complex)
    st = gc.emulate_group_cyclic(D, n, p)
    assert st["H"] == 4
    for c in range(st["H"]):
        assert np.array_equal(np.sort_complex(st[f"put{c}"]), np.sort_complex(st[f"tw{c}"]))


# ---------------------------------------------------------------- planted mistakes

def _pins_pass(emulate):
    for n, p in [((16,), (8,)), ((64,), (16,)), ((16, 16), (8, 2)), ((8, 27), (4, 9))]:
        X = crand(n, 7)
        want = oracle.to_cyclic(oracle.dft_direct(X), p)
        if oracle.rel_l2(emulate(oracle.to_cyclic(X, p), n, p), want) > 1e-12:
            return False
    return True


def test_pins_detect_planted_mistakes(monkeypatch):
    def run(D, n, p):
        return gc.emulate_group_cyclic(D, n, p)["out"]

    assert _pins_pass(run)
    real_put, real_tw, real_rev = gc._Dim.put, gc._Dim.twiddle_exponent, gc._rev

    def no_reversal(B, m, h):
        return B

    def twiddle_over_n(self, i):
        e, ni = real_tw(self, i)
        return e, self.n                            # omega_n instead of omega_{n_i}

    def blocked_inside_the_group(self, i):
        src, dst = real_put(self, i)
        if i < self.h:                               # sub-transform dealt in blocks, not cyclically
            ni, pi = self.lv[i]
            pn = pi // self.m
            r, k = src[:, 0], src[:, 1]
            u, bn = r % pi, (r // pi) * self.m + k
            dst = np.stack([bn * pn + u // self.m, u % self.m], axis=1)
        return src, dst

    def last_local_transposed(self, i):
        src, dst = real_put(self, i)
        if i == self.h and self.lv[i][1] > 1 and self.m // self.lv[i][1] > 1:
            ph, q = self.lv[i][1], self.m // self.lv[i][1]
            s_, t_ = dst[:, 1] // q, dst[:, 1] % q
            dst = np.stack([dst[:, 0], t_ * ph + s_], axis=1)
        return src, dst

    mutants = {
        "no digit reversal of the group": ("_rev", no_reversal, gc),
        "twiddle over n instead of n_i": ("twiddle_exponent", twiddle_over_n, gc._Dim),
        "blocks instead of cyclic inside a group": ("put", blocked_inside_the_group, gc._Dim),
        "last Put's local index transposed": ("put", last_local_transposed, gc._Dim),
    }
    for name, (attr, fn, owner) in mutants.items():
        with monkeypatch.context() as mp:
            mp.setattr(owner, attr, fn)
            assert not _pins_pass(run), name
