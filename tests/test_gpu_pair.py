"""k_pair: two adjacent strided dimensions of 8..32-point lines in one pass.

Superstep 0 factorises over dimensions (eq. (1.3)), so a pass may transform two
of them at once. Checked against the FP64 oracle through the C ABI:
  - the local-FFT stage alone (k_group2 on the two inner dimensions, then k_pair
    on the two outer ones) against the oracle's per-block local FFT, for every
    pair of line lengths and both precisions and directions;
  - whole transforms whose plan runs k_pair and then the fused innermost
    dimension (k_lastx), against eq. (1.2) summed by the oracle;
  - in place against out of place, bitwise.
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
NT = {"complex128": 8, "complex64": 9}       # log2 threads of k_pair where rows are near each other
LENS = [8, 16, 32]


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


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("direction", [FORWARD, INVERSE])
@pytest.mark.parametrize("la", LENS)
@pytest.mark.parametrize("lb", LENS)
def test_local_fft_stage_with_pair(torch_dev, la, lb, dtype, direction):
    import paper_2203_11795_amd as fftu
    n, p = (2 * la, 2 * lb, 16, 16), (2, 2, 2, 2)
    say(f"pair stage n={n} p={p} {dtype} dir={direction}")
    D = synth.uniform_complex(int(np.prod(n)), 21, NP_DTYPE[dtype]).astype(np.complex128)
    fftu.set_tuning("fuse_last", 0)
    try:
        with fftu.Plan(n, p, dtype, direction) as plan:
            names = plan.launch_names()
            lla, llb = la.bit_length() - 1, lb.bit_length() - 1
            assert names[:2] == [f"fftu::k_group2<{TNAME[dtype]}, 3, 3>",
                                 f"fftu::k_pair<{TNAME[dtype]}, {lla}, {llb}, {NT[dtype]}>"], names
            got = run(torch_dev, plan, D, dtype, "local_fft")
    finally:
        fftu.set_tuning("fuse_last", -1)
    want = oracle.emulate_local_fft(D, n, p, direction)
    assert oracle.rel_l2(got, want) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("direction", [FORWARD, INVERSE])
@pytest.mark.parametrize("la,lb", [(8, 8), (8, 32), (16, 16), (32, 8), (32, 16), (32, 32)])
def test_transform_pair_then_fused_last(torch_dev, la, lb, dtype, direction):
    import paper_2203_11795_amd as fftu
    n, p = (2 * la, 2 * lb, 128), (2, 2, 2)
    say(f"pair + lastx n={n} p={p} {dtype} dir={direction}")
    D = synth.uniform_complex(int(np.prod(n)), 22, NP_DTYPE[dtype]).astype(np.complex128)
    with fftu.Plan(n, p, dtype, direction) as plan:
        names = plan.launch_names()
        lla, llb = la.bit_length() - 1, lb.bit_length() - 1
        assert len(names) == 2 and names[0] == f"fftu::k_pair<{TNAME[dtype]}, {lla}, {llb}, {NT[dtype]}>", names
        assert names[1].startswith(f"fftu::k_lastx<{TNAME[dtype]}, 6,"), names
        got = run(torch_dev, plan, D, dtype)
        again = run(torch_dev, plan, D, dtype, inplace=True)
    assert np.array_equal(got, again), "in place must equal out of place"
    assert oracle.rel_l2(got, oracle.cyclic_dft(D, n, p, direction)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("n,p,kernels", [
    # the 64^5 benchmark's plan shape: two k_pair passes, then k_lastx
    ((16, 16, 16, 32, 64), (2,) * 5, ["k_pair", "k_pair", "k_lastx"]),
    # k_pair for (1, 2) and k_group2 for (3, 4) beat two passes before k_lastx
    ((64, 16, 64, 64), (2,) * 4, ["k_group2", "k_pair", "k_exchange"]),
    ((64, 64, 32, 64), (2,) * 4, ["k_group2", "k_pair", "k_exchange"]),
])
def test_whole_transforms_with_pairs(torch_dev, n, p, kernels, dtype):
    """Forward against eq. (1.2) summed by the oracle, and the round trip, for
    plans that run k_pair inside a whole transform."""
    import paper_2203_11795_amd as fftu
    N = int(np.prod(n))
    say(f"pairs n={n} p={p} {dtype}")
    D = synth.uniform_complex(N, 23, NP_DTYPE[dtype]).astype(np.complex128)
    with fftu.Plan(n, p, dtype, FORWARD) as fwd, fftu.Plan(n, p, dtype, INVERSE) as inv:
        names = fwd.launch_names()
        assert [s.split("<")[0] for s in names] == ["fftu::" + k for k in kernels], names
        Y = run(torch_dev, fwd, D, dtype)
        X = run(torch_dev, inv, Y, dtype)
    assert oracle.rel_l2(Y, oracle.cyclic_dft(D, n, p)) <= TOL[dtype]
    assert oracle.rel_l2(X, D) <= 2 * TOL[dtype]


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("la,lb", [(32, 32), (8, 32), (32, 16)])
def test_far_rows_take_the_wide_tile(torch_dev, la, lb, dtype):
    """Rows 64 KiB apart (B = 8192 complex64 columns): complex64 pairs with a line
    of 32 take 1024 threads and 32 columns per tile; complex128 keeps 256."""
    import paper_2203_11795_amd as fftu
    n, p = (la, lb, 64, 128), (1, 1, 1, 1)
    say(f"far rows n={n} {dtype}")
    D = synth.uniform_complex(int(np.prod(n)), 25, NP_DTYPE[dtype]).astype(np.complex128)
    lla, llb = la.bit_length() - 1, lb.bit_length() - 1
    nt = 10 if dtype == "complex64" else 8
    with fftu.Plan(n, p, dtype, FORWARD) as fwd, fftu.Plan(n, p, dtype, INVERSE) as inv:
        names = fwd.launch_names()
        assert f"fftu::k_pair<{TNAME[dtype]}, {lla}, {llb}, {nt}>" in names, names
        Y = run(torch_dev, fwd, D, dtype)
        X = run(torch_dev, inv, Y, dtype, inplace=True)
    assert oracle.rel_l2(Y, oracle.cyclic_dft(D, n, p)) <= TOL[dtype]
    assert oracle.rel_l2(X, D) <= 2 * TOL[dtype]


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_pair_off_gives_the_same_transform(torch_dev, dtype):
    """The knob that turns k_pair off changes the passes, not the result."""
    import paper_2203_11795_amd as fftu
    n, p = (64, 64, 32, 64), (2, 2, 2, 2)
    D = synth.uniform_complex(int(np.prod(n)), 24, NP_DTYPE[dtype]).astype(np.complex128)
    outs = {}
    for v in (-1, 0):
        fftu.set_tuning("pair", v)
        try:
            with fftu.Plan(n, p, dtype, FORWARD) as plan:
                names = plan.launch_names()
                assert any("k_pair" in s for s in names) == (v == -1), names
                outs[v] = run(torch_dev, plan, D, dtype)
        finally:
            fftu.set_tuning("pair", -1)
    want = oracle.cyclic_dft(D, n, p)
    for v in outs:
        assert oracle.rel_l2(outs[v], want) <= TOL[dtype]
