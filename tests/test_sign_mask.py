"""The DST-II's signal signs in the packed cyclic layout, on the CPU.

The DST of x is the DCT of x' = (-1)^j x stored reversed; in zig-zag order that
negates, once per dimension, the samples with m_l >= n_l / 2, and on the packed
array (last dimension paired, z[.., j] = v[.., 2j] + i v[.., 2j + 1]) the packed
samples with j >= n_d / 4. The line and exchange kernels apply these signs as the
parity of the local index under one mask, the top bit of each dimension's field,
which holds when every local side of the packed array is a power of two. This
checks that claim element by element against the definition on natural indices,
over the cyclic layout buf[rank(s) M + lin(k)].
"""
import itertools

import numpy as np
import pytest


def signs_by_definition(n, p):
    """Sign of every packed buffer element from its natural index."""
    d = len(n)
    npk = list(n[:-1]) + [n[-1] // 2]
    m = [npk[l] // p[l] for l in range(d)]
    M = int(np.prod(m))
    out = np.empty(int(np.prod(npk)), dtype=np.int8)
    for s in itertools.product(*[range(v) for v in p]):
        rank = 0
        for l in range(d):
            rank = rank * p[l] + s[l]
        for k in itertools.product(*[range(v) for v in m]):
            lin = 0
            sign = 1
            for l in range(d):
                lin = lin * m[l] + k[l]
                j = s[l] + p[l] * k[l]                      # natural packed index along l
                half = n[l] // 2 if l < d - 1 else n[l] // 4  # m_l >= n_l / 2, or 2j >= n_d / 2
                if j >= half:
                    sign = -sign
            out[rank * M + lin] = sign
    return out


def signs_by_mask(n, p):
    """Sign as the parity of the local index under the top bit of each field."""
    d = len(n)
    npk = list(n[:-1]) + [n[-1] // 2]
    m = [npk[l] // p[l] for l in range(d)]
    mask, off = 0, 0
    for l in range(d - 1, -1, -1):
        lg = int(m[l]).bit_length() - 1
        mask |= 1 << (off + lg - 1)
        off += lg
    M = int(np.prod(m))
    idx = np.arange(int(np.prod(npk)), dtype=np.int64) % M
    parity = np.array([bin(int(i) & mask).count("1") & 1 for i in idx], dtype=np.int8)
    return 1 - 2 * parity


@pytest.mark.parametrize("n,p", [((8,), (2,)), ((16, 8), (2, 2)), ((8, 16, 32), (2, 2, 4)),
                                 ((16, 16, 16), (4, 2, 2)), ((4, 8, 4, 16), (2, 1, 2, 2)),
                                 ((32, 64), (4, 8))])
def test_mask_parity_is_the_dst_sign(n, p):
    assert np.array_equal(signs_by_definition(n, p), signs_by_mask(n, p))


def test_mask_parity_fails_for_odd_local_sides():
    """With a local side that is not even the signs are no parity of index bits: the
    planner keeps the separate sign pass there (local sides of 3 and 6)."""
    n, p = (12, 24), (2, 2)
    assert not np.array_equal(signs_by_definition(n, p), signs_by_mask(n, p))
