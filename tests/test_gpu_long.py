"""k_long: lines of 2^11 / 2^12 points over short rows (B <= W columns), where no
per-thread split of k_line fits.

Checked against the FP64 oracle through the C ABI: the local-FFT stage alone
(against the oracle's per-block local FFT) and whole transforms, forward and
inverse, for every compiled line length, rows of B = 1..16 (several outer blocks
per tile, one, or a half, quarter or eighth of one with the pieces grouped on an
XCD), and the unfused Superstep 2 of grids with p_1 = 2048 and 4096. Tolerances (relative L2): 1e-12 complex128, 5e-6 complex64.
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

# (n, p, dtype, the k_long launch expected: (log2 L, log2 B)); W = 2 lines per tile for
# 4096-point complex64 and 2048-point complex128, 4 for 2048-point complex64
CASES = [
    ((8192, 16), (2, 2), "complex64", (12, 3)),      # lines of 4096, rows of 8 = 4 W: a quarter row per tile
    ((8, 8192, 16), (2, 2, 2), "complex64", (12, 3)),  # the same over 128 tiles, grouped by four on an XCD
    ((8192, 8), (2, 2), "complex64", (12, 2)),       # rows of 4 = 2 W
    ((8192, 4), (2, 2), "complex64", (12, 1)),       # rows of 2 = W: one block per tile
    ((4096, 16), (2, 2), "complex64", (11, 3)),      # lines of 2048, rows of 8 = 2 W
    ((4096, 32), (2, 2), "complex64", (11, 4)),      # rows of 16 = 4 W
    ((4096, 4), (2, 2), "complex64", (11, 1)),       # rows of 2 < W: two blocks per tile
    ((4096, 16), (2, 2), "complex128", (11, 3)),     # rows of 8 = 4 W
    ((8, 4096, 16), (2, 2, 2), "complex128", (11, 3)),
    ((2048, 8), (1, 2), "complex128", (11, 2)),      # p_1 = 1, rows of 4 = 2 W
    ((2048, 4), (1, 2), "complex128", (11, 1)),      # rows of 2 = W: one block per tile
    # 4096-point complex128: W = 1 line per tile, rows of up to 8 = 8 W columns
    ((8192, 16), (2, 2), "complex128", (12, 3)),     # rows of 8: an eighth of a row per tile
    ((8, 8192, 16), (2, 2, 2), "complex128", (12, 3)),  # 512 tiles, grouped by eight on an XCD
    ((8192, 8), (2, 2), "complex128", (12, 2)),      # rows of 4
    ((8192, 2), (2, 1), "complex128", (12, 1)),      # rows of 2
    ((8192,), (2,), "complex128", (12, 0)),          # one line per tile
]
IDS = [f"{'x'.join(map(str, n))}-p{'x'.join(map(str, p))}-{dt}" for n, p, dt, _ in CASES]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2203_11795_amd as fftu
    fftu.load_library()
    return torch


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def run(torch, plan, D, dtype, stage=None, inplace=False):
    x = torch.from_numpy(np.ascontiguousarray(D.astype(NP_DTYPE[dtype]))).to("cuda")
    out = x if inplace else torch.empty_like(x)
    if stage is None:
        plan(x, out)
    else:
        plan.stage(stage, x, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("direction", [FORWARD, INVERSE])
@pytest.mark.parametrize("n,p,dtype,lw", CASES, ids=IDS)
def test_long_lines_match_oracle(torch_dev, n, p, dtype, lw, direction):
    import paper_2203_11795_amd as fftu
    N = int(np.prod(n))
    say(f"long n={n} p={p} {dtype} dir={direction}")
    D = synth.uniform_complex(N, 31, NP_DTYPE[dtype]).astype(np.complex128)
    with fftu.Plan(n, p, dtype, direction) as plan:
        names = plan.launch_names()
        assert f"fftu::k_long<{TNAME[dtype]}, {lw[0]}, {lw[1]}>" in names, names
        S0 = run(torch_dev, plan, D, dtype, "local_fft")
        got = run(torch_dev, plan, D, dtype)
        again = run(torch_dev, plan, D, dtype, inplace=True)
    assert oracle.rel_l2(S0, oracle.emulate_local_fft(D, n, p, direction)) <= TOL[dtype]
    assert oracle.rel_l2(got, oracle.cyclic_dft(D, n, p, direction)) <= TOL[dtype]
    assert np.array_equal(got, again), "in place must equal out of place"


@pytest.mark.parametrize("direction", [FORWARD, INVERSE])
def test_unfused_superstep2_with_long_lines(torch_dev, direction):
    """p_1 = 2048: P = 4096 takes the unfused exchange, and Superstep 2's transforms
    along p_1 run on k_long as Superstep 0's along m_1 do; k_long is then the last
    kernel (conjugation and 1/N of the inverse on its store)."""
    import paper_2203_11795_amd as fftu
    n, p = (1 << 22, 8), (2048, 2)
    N = int(np.prod(n))
    say(f"long S2 n={n} p={p} dir={direction}")
    D = synth.uniform_complex(N, 32, np.complex64).astype(np.complex128)
    with fftu.Plan(n, p, "complex64", direction) as plan:
        names = plan.launch_names()
        assert names.count("fftu::k_long<float, 11, 2>") == 2 and names[-1] == "fftu::k_long<float, 11, 2>", names
        assert plan.info()["exchange_fused"] == 0
        got = run(torch_dev, plan, D, "complex64")
    assert oracle.rel_l2(got, oracle.cyclic_dft(D, n, p, direction)) <= TOL["complex64"]


@pytest.mark.parametrize("direction", [FORWARD, INVERSE])
def test_unfused_superstep2_with_long_complex128_lines(torch_dev, direction):
    """p_1 = 4096 in complex128 (one line per tile): Superstep 2's transforms along p_1
    on k_long<double, 12>, rows of q_1 = 1 times the local side 2 after it."""
    import paper_2203_11795_amd as fftu
    n, p = (1 << 24, 2), (4096, 1)
    N = int(np.prod(n))
    say(f"long S2 c128 n={n} p={p} dir={direction}")
    D = synth.uniform_complex(N, 33, np.complex128)
    with fftu.Plan(n, p, "complex128", direction) as plan:
        names = plan.launch_names()
        assert names.count("fftu::k_long<double, 12, 1>") == 2 and names[-1] == "fftu::k_long<double, 12, 1>", names
        got = run(torch_dev, plan, D, "complex128")
    assert oracle.rel_l2(got, oracle.cyclic_dft(D, n, p, direction)) <= TOL["complex128"]
