"""Processor grids beyond p_max = sqrt(N): the group-cyclic distribution and the
FFT with more than one communication superstep (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2.3 (after eq. (2.13)) states that a grid with p_l^2 not dividing n_l
needs more than one communication superstep and the group-cyclic distribution:
with cycle c it splits an array of n elements into p/c blocks of c n / p
elements, gives each block to a group of c processors and distributes the block
cyclically inside its group, so element x_j goes to processor
P((j div (c n/p)) c + j mod c). Cycle c = p is the cyclic distribution, c = 1
the block distribution. The paper gives the assignment only; the algorithm
below is this package's reading, built from the paper's own pieces:

1-D, n = m p (m = n/p elements per processor), p^2 not dividing n.
  Superstep 0 of Algorithm 2.2 is unchanged: F_m on every processor's local
  array, then the twiddle omega_n^{u k} (u = processor, k = local index).
  Its output z^(u)_k must then go through F_p along u for every k: the m
  sub-transforms w^(k)_u = z^(u)_k of length p (eq. (2.3)'s y_{t m + k} =
  sum_u omega_p^{u t} w^(k)_u). A processor holds m elements, so each
  sub-transform is spread over a group of c = p/m processors (this needs m | p),
  cyclically inside the group: the array W with W_{k p + u} = w^(k)_u in the
  group-cyclic distribution with cycle c. That redistribution is the first Put.
  Each group now holds an instance of the same problem, n' = p on p' = c
  processors with m elements each, and runs it the same way: one Put per level
  until a level has p'^2 | n', which ends with Algorithm 2.2's own Put and its
  length-p' FFTs.
  Levels i = 0 .. h: n_0 = n, p_0 = p; n_{i+1} = p_i, p_{i+1} = p_i / m; level h
  is the first with p_h^2 | n_h. At level i the data is the group-cyclic
  distribution with cycle p_i of the level's array (blocks of n_i elements, one
  sub-transform each); the transform output of block b at index t m + k is the
  output of block b m + k of level i + 1 at index t.
  Output: the sub-transform outputs end cyclic inside their groups, which in
  the paper's processor numbering is a relabelling of the cyclic distribution:
  element e of level-h block B = k_0 m^{h-1} + ... + k_{h-1} is y_a with
  a = e m^h + k_{h-1} m^{h-1} + ... + k_0, whose cyclic owner is
  a mod p = (e mod p_h) m^h + rev(B), rev(B) = k_0 + k_1 m + ... + k_{h-1} m^{h-1},
  at local index e div p_h, the same local index as in the group. The last Put
  therefore sends each element straight to that processor, and the transform
  ends in the cyclic distribution it started in.
  h + 1 communication supersteps in all; h = 0 is Algorithm 2.2 itself.

d dimensions (Algorithm 2.3's combination, dimension by dimension): each
dimension has its own levels; communication superstep c runs, for every
dimension l at once, the Put of level c (identity for a dimension whose levels
are done), and computation phase c runs level c's local F_{m_l} and twiddle for
dimensions with c <= h_l, and level h_l's length-p FFTs for dimensions with
c = h_l + 1. The operations of different dimensions act on different index
coordinates and commute (eq. (1.3)), so a grid with every p_l^2 | n_l is
exactly Algorithm 2.3.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import FORWARD, INVERSE, _check_direction, fft_axes


# ----------------------------------------------------------------------------
# The distribution (Section 2.3, the group-cyclic paragraph)
# ----------------------------------------------------------------------------

def group_cyclic_owner(j, n: int, p: int, c: int):
    """(processor, local index) of element j of an n-array in the group-cyclic
    distribution with cycle c over p processors: P((j div (c n/p)) c + j mod c),
    at position (j mod (c n/p)) div c of its processor (cyclic inside the block)."""
    if p < 1 or n % p or c < 1 or p % c:
        raise ValueError(f"need p | n and c | p, got n={n} p={p} c={c}")
    j = np.asarray(j, dtype=np.int64)
    block = c * n // p
    return (j // block) * c + j % c, (j % block) // c


# ----------------------------------------------------------------------------
# Levels of one dimension
# ----------------------------------------------------------------------------

def levels(n: int, p: int):
    """[(n_i, p_i)] for i = 0..h as in the module docstring; raises ValueError
    when the chain does not reach a level with p_h^2 | n_h."""
    n, p = int(n), int(p)
    if p < 1 or n % p:
        raise ValueError(f"p must divide n, got n={n} p={p}")
    m = n // p
    out = []
    ni, pi = n, p
    while True:
        if ni % (pi * pi) == 0:
            out.append((ni, pi))
            return out
        if m == 1 or pi % m:
            raise ValueError(f"n={n} over p={p}: no chain of group-cyclic levels (m={m} must divide p_i={pi})")
        out.append((ni, pi))
        ni, pi = pi, pi // m


def _rev(B: int, m: int, h: int) -> int:
    """Base-m digit reversal of B over h digits."""
    r = 0
    for _ in range(h):
        B, dgt = divmod(B, m)
        r = r * m + dgt
    return r


class _Dim:
    def __init__(self, n: int, p: int):
        self.n, self.p = int(n), int(p)
        self.m = self.n // self.p
        self.lv = levels(self.n, self.p)
        self.h = len(self.lv) - 1

    # Put of level i of this dimension as a map of (processor, local) pairs:
    # returns (dst_proc, dst_local) for every (src_proc, src_local).
    def put(self, i: int):
        ni, pi = self.lv[i]
        m = self.m
        src = np.array(list(itertools.product(range(self.p), range(m))), dtype=np.int64)
        r, k = src[:, 0], src[:, 1]
        b, u = r // pi, r % pi                        # block of level i, member inside the group
        if i < self.h:
            pn = pi // m                              # p_{i+1}
            bn = b * m + k                            # sub-transform k of block b
            return src, np.stack([bn * pn + u % pn, u // pn], axis=1)
        # level h: Algorithm 2.2 inside the group (n_h over p_h, q = m / p_h), to the
        # cyclic processor numbering
        q = m // pi
        rho, t = k % pi, k // pi                      # destination member, block offset
        rev_b = np.array([_rev(int(v), m, self.h) for v in b], dtype=np.int64)
        return src, np.stack([rho * m ** self.h + rev_b, u * q + t], axis=1)

    def twiddle_exponent(self, i: int):
        """Level i's twiddle omega_{n_i}^{u k} as exponents over n_i, indexed [proc, local]."""
        ni, pi = self.lv[i]
        r = np.arange(self.p)[:, None]
        k = np.arange(self.m)[None, :]
        return ((r % pi) * k) % ni, ni


def _root(nl: int, e: np.ndarray, sign: int) -> np.ndarray:
    """exp(sign 2 pi i e / nl), exact at the quarter points."""
    e = np.mod(np.asarray(e, dtype=np.int64), nl)
    w = np.exp(sign * 2j * np.pi * (e.astype(np.float64) / nl))
    quarter = (4 * e) % nl == 0
    if np.any(quarter):
        w[quarter] = np.array([1, 1j * sign, -1, -1j * sign])[(4 * e[quarter]) // nl]
    return w


def plan_levels(n, p):
    """Per-dimension levels and the number of communication supersteps H."""
    dims = [_Dim(nl, pl) for nl, pl in zip(n, p)]
    return dims, max(dm.h + 1 for dm in dims)


def put_superstep(W: np.ndarray, n, p, c: int) -> np.ndarray:
    """The Put of communication superstep c applied to the buffer W (processor-major
    layout): every dimension with a level c moves its (processor, local) coordinates
    by that level's Put, the others keep theirs. Pure data movement: the dtype of W
    is kept, so results compare bit for bit."""
    n = tuple(int(v) for v in n)
    p = tuple(int(v) for v in p)
    d = len(n)
    dims, _ = plan_levels(n, p)
    m = tuple(dm.m for dm in dims)
    Wv = np.asarray(W).reshape(p + m)
    Y = np.empty_like(Wv)
    src_idx = [None] * (2 * d)
    dst_idx = [None] * (2 * d)
    for l, dm in enumerate(dims):
        if c > dm.h:
            ident = np.array(list(itertools.product(range(dm.p), range(dm.m))), dtype=np.int64)
            src, dst = ident, ident
        else:
            src, dst = dm.put(c)
        # broadcast the per-dimension pair lists over the other dimensions
        shape = [1] * d
        shape[l] = src.shape[0]
        src_idx[l] = src[:, 0].reshape(shape)
        src_idx[d + l] = src[:, 1].reshape(shape)
        dst_idx[l] = dst[:, 0].reshape(shape)
        dst_idx[d + l] = dst[:, 1].reshape(shape)
    Y[tuple(dst_idx)] = Wv[tuple(src_idx)]
    return Y.reshape(-1)


def emulate_group_cyclic(D: np.ndarray, n, p, direction: int = FORWARD) -> dict:
    """Carry out the multi-superstep algorithm of the module docstring on the
    cyclic buffer D (layout of ``to_cyclic``), virtual processor by virtual
    processor, and return every intermediate buffer (same layout: processor
    rank row-major over the grid, then the local array row-major):

      "fft0"            computation phase 0: F_{m_l} of every local array along every dimension
      "tw{c}", "put{c}" communication superstep c: after the twiddle, after the Put
      "fft{c+1}"        computation phase c + 1: the local FFTs of the next level
                        (dimensions with levels left) and the length-p_h FFTs
                        (dimensions whose last Put this was)
      "out"             the last phase, times 1/N for the inverse
    """
    _check_direction(direction)
    n = tuple(int(v) for v in n)
    p = tuple(int(v) for v in p)
    d = len(n)
    dims, H = plan_levels(n, p)
    m = tuple(dm.m for dm in dims)
    sign = direction
    X = np.asarray(D, dtype=np.complex128).reshape(p + m).copy()
    out = {}

    def local_fft(A, which):
        # F along local axis d + l for the dimensions in `which` (every processor's array)
        axes = [d + l for l in which]
        if not axes:
            return A
        return fft_axes(A, axes, direction)

    X = local_fft(X, range(d))
    out["fft0"] = X.reshape(-1).copy()
    for c in range(H):
        # twiddle of level c, per dimension, on the source coordinates
        W = X.copy()
        for l, dm in enumerate(dims):
            if c > dm.h:
                continue
            e, ni = dm.twiddle_exponent(c)
            shape = [1] * (2 * d)
            shape[l], shape[d + l] = dm.p, dm.m
            W = W * _root(ni, e, sign).reshape(shape)
        out[f"tw{c}"] = W.reshape(-1).copy()
        # the Put: each dimension moves its own (processor, local) coordinates
        Y = put_superstep(W, n, p, c).reshape(W.shape)
        out[f"put{c}"] = Y.reshape(-1).copy()
        # computation phase c + 1
        nxt = [l for l, dm in enumerate(dims) if c + 1 <= dm.h]
        Z = local_fft(Y, nxt)
        last = [l for l, dm in enumerate(dims) if c == dm.h]
        for l in last:
            dm = dims[l]
            ph = dm.lv[-1][1]
            q = dm.m // ph
            # local index s' q + t: F_{p_h} along s' for every t (Superstep 2 of level h)
            shp = list(Z.shape)
            shp[d + l:d + l + 1] = [ph, q]
            Zs = fft_axes(Z.reshape(shp), [d + l], direction)   # after the split, s' is axis d + l
            Z = Zs.reshape(Z.shape)
        out[f"fft{c + 1}"] = Z.reshape(-1).copy()
        X = Z
    res = X.reshape(-1).copy()
    if direction == INVERSE:
        res *= 1.0 / res.size
    out["out"] = res
    out["H"] = H
    return out


def supersteps(n, p) -> int:
    """Communication supersteps of the grid (1 when every p_l^2 | n_l)."""
    return plan_levels(n, p)[1]
