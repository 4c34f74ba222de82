"""k_ttranspose: Superstep 0's twiddle and Superstep 1 as one tiled transpose, for
grids with every q_l = n_l / p_l^2 equal to 1 (then m = p, M = P, and the
all-to-all W^(r)[s] = Z^(s)[r] transposes the P x M matrix of blocks).

Where the innermost side m_d = p_d is 2..32, the kernel also runs that
dimension's FFTs of Superstep 0 (before the twiddle) and Superstep 2 (after the
transpose). Whole transforms through the C ABI against the FP64 oracle (eq.
(1.2)), forward and inverse, in place and out of place, at sizes of one to 64
tiles of 64 x 64, with dimensions whose digits lie inside or outside a tile's
low 6 index bits, with and without the fused FFTs.
Tolerances (relative L2): 1e-12 complex128, 5e-6 complex64.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import FORWARD, INVERSE

pytestmark = pytest.mark.gpu

TOL = {"complex128": 1e-12, "complex64": 5e-6}
NP_DTYPE = {"complex128": np.complex128, "complex64": np.complex64}
TNAME = {"complex128": "double", "complex64": "float"}

CASES = [
    ((64, 64), (8, 8)),                  # P = M = 64: one tile
    ((1024, 64), (32, 8)),               # 16 tiles; dimension 1's digit straddles the low 6 bits
    ((256, 256), (16, 16)),
    ((64, 64, 64), (8, 8, 8)),           # 64 tiles, three dimensions
    ((4096, 64), (64, 8)),               # dimension 1 entirely above the low 6 bits
    ((4,) * 8, (2,) * 8),                # d = 8, one bit per dimension
    ((64, 4096), (8, 64)),               # innermost side 64: the transpose without the fused FFTs
]
IDS = [f"{'x'.join(map(str, n))}-p{'x'.join(map(str, p))}" for n, p in CASES]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2203_11795_amd as fftu
    fftu.load_library()
    return torch


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def run(torch, plan, D, dtype, inplace=False):
    x = torch.from_numpy(np.ascontiguousarray(D.astype(NP_DTYPE[dtype]))).to("cuda")
    out = x if inplace else torch.empty_like(x)
    plan(x, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("direction", [FORWARD, INVERSE])
@pytest.mark.parametrize("n,p", CASES, ids=IDS)
def test_transpose_exchange_matches_oracle(torch_dev, n, p, dtype, direction):
    import paper_2203_11795_amd as fftu
    N = int(np.prod(n))
    say(f"ttranspose n={n} p={p} {dtype} dir={direction}")
    D = synth.uniform_complex(N, 41, NP_DTYPE[dtype]).astype(np.complex128)
    with fftu.Plan(n, p, dtype, direction) as plan:
        names = plan.launch_names()
        info = plan.info()
        ld = (n[-1] // p[-1]).bit_length() - 1          # m_d = p_d = 2^ld
        fused = ld if ld <= 5 else 0                       # innermost FFTs inside the transpose
        assert info["exchange_fused"] == 0 and f"fftu::k_ttranspose<{TNAME[dtype]}, {fused}>" in names, names
        assert len(names) == info["launches"]
        assert "fftu::k_permute" not in " ".join(names)
        got = run(torch_dev, plan, D, dtype)
        again = run(torch_dev, plan, D, dtype, inplace=True)
    assert np.array_equal(got, again), "in place must equal out of place"
    assert oracle.rel_l2(got, oracle.cyclic_dft(D, n, p, direction)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_transpose_moves_a_marked_element(torch_dev, dtype):
    """An impulse at global index (1, 0) transforms to omega_{n_1}^{k_1} in every
    column: a closed form that checks dimension 1's twiddle factors and where
    every output lands."""
    import paper_2203_11795_amd as fftu
    n, p = (1024, 64), (32, 8)
    N = int(np.prod(n))
    X = np.zeros(n, dtype=np.complex128)
    X[1, 0] = 1.0
    D = oracle.to_cyclic(X, p)
    with fftu.Plan(n, p, dtype, FORWARD) as plan:
        got = oracle.from_cyclic(run(torch_dev, plan, D, dtype), n, p)
    k1 = np.arange(n[0])[:, None]
    want = np.broadcast_to(np.exp(-2j * np.pi * k1 / n[0]), n)
    assert oracle.rel_l2(got.reshape(-1), want.reshape(-1)) <= TOL[dtype]
    assert N == got.size
