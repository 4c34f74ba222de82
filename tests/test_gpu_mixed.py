"""Mixed-radix path on the GPU (sides with prime factors 2, 3, 5, 7; grids with
p_l^2 | n_l): the whole transform, each superstep against the oracle's
emulation of Algorithm 2.3, external plans, convolution, and a full-size
480^3 transform on sampled outputs."""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import FORWARD, INVERSE

pytestmark = pytest.mark.gpu

TOL = {"complex128": 1e-12, "complex64": 5e-6}
NP = {"complex128": np.complex128, "complex64": np.complex64}

CASES = [((12,), (2,)), ((36,), (3,)), ((100,), (5,)), ((1000,), (10,)), ((7,), (1,)), ((60, 60), (2, 2)),
         ((126, 12), (3, 2)), ((49, 27), (7, 3)), ((18, 20, 12), (3, 2, 2)), ((96, 96), (4, 2)), ((45, 8), (3, 2)),
         ((384,), (8,)), ((30, 30, 30), (1, 1, 1)), ((3072,), (4,)),
         ((48, 48, 48), (4, 4, 4)),          # P = 64 in k_mexchange, the 480^3 benchmark's grid
         ((192, 64), (8, 8)), ((75, 98), (5, 7)), ((36, 36, 36), (6, 3, 2)),   # p = 6: unfused
         # rows of the last dimension that are not whole 128-byte lines: blocks of 2 or 4 rows per workgroup
         ((80, 200), (2, 2)), ((96, 48, 240), (4, 2, 4)),
         # d = 4 on a power-of-two grid; rows of 300 in several chunks (blocks of 2 rows in complex128)
         ((12, 20, 6, 24), (2, 2, 1, 2)), ((10, 600), (1, 2)),
         # whole output rows staged in LDS (segments of q_{d-1} elements not whole 128-byte lines):
         # one wave dimension of 2 (complex128), two wave dimensions (complex128), rows of 108 of 128 slots
         ((4, 4, 4, 4, 40), (2, 2, 2, 2, 2)), ((4, 4, 4, 4, 4, 24), (2, 2, 2, 2, 2, 2)), ((16, 16, 432), (4, 4, 4))]

# (grid, dtype) pairs whose exchange takes the row-staged k_mxexchange
STAGED = {((48, 48, 48), "complex64"), ((48, 48, 48), "complex128"), ((4, 4, 4, 4, 40), "complex128"),
          ((4, 4, 4, 4, 4, 24), "complex128"), ((16, 16, 432), "complex64"), ((16, 16, 432), "complex128")}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.mark.parametrize("n,p", CASES)
@pytest.mark.parametrize("dtype", ["complex64", "complex128"])
@pytest.mark.parametrize("direction", [FORWARD, INVERSE])
def test_mixed_transform_matches_oracle(torch, n, p, dtype, direction):
    import paper_2203_11795_amd as fftu
    N = int(np.prod(n))
    D = synth.uniform_complex(N, 5, NP[dtype])
    want = oracle.cyclic_dft(D.astype(np.complex128), n, p, direction)
    with fftu.Plan(n, p, dtype, direction) as plan:
        info, names = plan.info(), plan.launch_names()
        fused = all(v in (1, 2, 3, 4, 5, 7, 8) for v in p) and int(np.prod(p)) <= 64
        assert info["exchange_fused"] == (1 if fused else 0)
        t = "double" if dtype == "complex128" else "float"
        if fused:
            # power-of-two grids with a register split take k_mxexchange, the others k_mexchange
            assert (names[-1].startswith(f"fftu::k_mexchange<{t}, ") or names[-1].startswith(f"fftu::k_mxexchange<{t}, ")) \
                and len(names) == info["s0_kernels"] + 1, names
            if p == (4, 4, 4):
                # q_{d-1} = 3: output segments that are not whole lines take the row-staged form
                assert names[-1] == f"fftu::k_mxexchange<{t}, 2, 2, 1, 2, true>", names
            if p == (3, 2):
                assert names[-1].startswith(f"fftu::k_mexchange<{t}, "), names
            if names[-1].startswith("fftu::k_mxexchange"):
                assert names[-1].endswith(", true>" if (n, dtype) in STAGED else ", false>"), names
        else:
            assert f"fftu::k_mpermute<{t}>" in names
        assert "k_mline" in names[0] or info["s0_kernels"] == 0
        x = torch.from_numpy(D).cuda()
        y = plan(x)
        z = x.clone()
        plan(z, z)                                         # in place
        torch.cuda.synchronize()
        got = y.cpu().numpy()
        err = oracle.rel_l2(got.astype(np.complex128), want)
        assert err <= TOL[dtype], (n, p, err)
        assert torch.equal(y, z)
        assert np.array_equal(x.cpu().numpy(), D)         # input unchanged


@pytest.mark.parametrize("n,p", [((60, 60), (2, 2)), ((18, 20, 12), (3, 2, 2)), ((1000,), (10,))])
@pytest.mark.parametrize("direction", [FORWARD, INVERSE])
def test_mixed_stages_match_emulation(torch, n, p, direction):
    import paper_2203_11795_amd as fftu
    N = int(np.prod(n))
    D = synth.uniform_complex(N, 6)
    em = oracle.emulate(D, n, p, direction)
    with fftu.Plan(n, p, "complex128", direction) as plan:
        x = torch.from_numpy(D).cuda()
        s0 = plan.stage("local_fft", x)
        tw = plan.stage("twiddle", torch.from_numpy(em["S0"]).cuda())
        ex = plan.stage("exchange", torch.from_numpy(em["twiddle"]).cuda())
        s2 = plan.stage("remaining_fft", torch.from_numpy(em["S1"]).cuda())
        torch.cuda.synchronize()
        assert oracle.rel_l2(s0.cpu().numpy(), em["S0"]) <= 1e-12
        assert oracle.rel_l2(tw.cpu().numpy(), em["twiddle"]) <= 1e-12
        assert np.array_equal(ex.cpu().numpy(), em["S1"])                   # a permutation: bitwise
        assert oracle.rel_l2(s2.cpu().numpy(), em["S2"]) <= 1e-12


@pytest.mark.parametrize("dtype", ["complex64", "complex128"])
def test_mixed_external_plan_and_convolution(torch, dtype):
    import paper_2203_11795_amd as fftu
    n, p = (60, 60), (2, 2)
    N = 3600
    x = synth.uniform_complex(N, 7, NP[dtype])
    h = synth.uniform_complex(N, 8, NP[dtype])
    dx = torch.from_numpy(x).cuda()
    with fftu.Plan(n, p, dtype) as a, fftu.Plan(n, p, dtype, external=True) as b:
        ws = torch.empty_like(dx)
        assert b.device_bytes() == 0
        assert torch.equal(a(dx), b(dx, workspace=ws))
    X = oracle.from_cyclic(x.astype(np.complex128), n, p)
    H = oracle.from_cyclic(h.astype(np.complex128), n, p)
    want = oracle.circular_convolution(X, H)
    with fftu.ConvolutionPlan(n, p, dtype) as conv:
        hhat = conv(torch.from_numpy(h).cuda())
        y = conv.convolve(dx, hhat)
        got = oracle.from_cyclic(y.cpu().numpy().astype(np.complex128), n, p)
        assert oracle.rel_l2(got, want) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["complex64", "complex128"])
def test_mixed_staged_rows_convolution(torch, dtype):
    """Convolution on a grid whose exchange stages whole output rows (16 x 16 x 48
    over 4^3, q_{d-1} = 3): the product by the filter spectrum happens in the staged
    store."""
    import paper_2203_11795_amd as fftu
    n, p = (16, 16, 48), (4, 4, 4)
    N = 16 * 16 * 48
    x = synth.uniform_complex(N, 12, NP[dtype])
    h = synth.uniform_complex(N, 13, NP[dtype])
    X = oracle.from_cyclic(x.astype(np.complex128), n, p)
    H = oracle.from_cyclic(h.astype(np.complex128), n, p)
    want = oracle.circular_convolution(X, H)
    with fftu.ConvolutionPlan(n, p, dtype) as conv:
        names = conv.launch_names()
        assert names[-1].startswith("fftu::k_mxexchange") and names[-1].endswith(", true>"), names
        hhat = conv(torch.from_numpy(h).cuda())
        y = conv.convolve(torch.from_numpy(x).cuda(), hhat)
        got = oracle.from_cyclic(y.cpu().numpy().astype(np.complex128), n, p)
    assert oracle.rel_l2(got, want) <= TOL[dtype]


@pytest.mark.parametrize("n,p,dtype", [((2880,), (3,), "complex128"),      # m = 960: longest mixed line, FP64
                                       ((9600,), (5,), "complex64"),       # m = 1920: longest mixed line, FP32
                                       ((2880, 6), (3, 1), "complex128")])
def test_mixed_longest_lines(torch, n, p, dtype):
    import paper_2203_11795_amd as fftu
    N = int(np.prod(n))
    D = synth.uniform_complex(N, 10, NP[dtype])
    want = oracle.cyclic_dft(D.astype(np.complex128), n, p)
    with fftu.Plan(n, p, dtype) as plan:
        got = plan(torch.from_numpy(D).cuda()).cpu().numpy()
    assert oracle.rel_l2(got.astype(np.complex128), want) <= TOL[dtype]


def test_mixed_limits_are_rejected(torch):
    import paper_2203_11795_amd as fftu
    assert fftu.check((3 * 2048,), (2,), "complex128") == 3        # m = 3072 > 1024
    assert fftu.check((3 * 2048,), (2,), "complex64") == 3         # m = 3072 > 2048
    assert fftu.check((2 * 11 * 4,), (2,)) == 3                    # prime factor 11
    with pytest.raises(fftu.FftuError):
        fftu.BatchPlan([(48, 16, 16)], [(2, 2, 2)], "complex64")     # batches: powers of two only


def test_mixed_full_size_sampled(torch):
    """480^3 complex128 on a 4^3 grid (m = 120, q = 30; T = 480): outputs at
    sampled indices against eq. (1.2) summed directly, and the round trip."""
    import paper_2203_11795_amd as fftu
    n, p = (480, 480, 480), (4, 4, 4)
    N = 480 ** 3
    say("480^3: generating input")
    D = synth.uniform_complex(N, 9)
    x = torch.from_numpy(D).cuda()
    with fftu.Plan(n, p, "complex128") as fwd, fftu.Plan(n, p, "complex128", INVERSE) as inv:
        y = fwd(x)
        back = inv(y)
        torch.cuda.synchronize()
        err_rt = float(torch.linalg.vector_norm(back - x) / torch.linalg.vector_norm(x))
        say(f"480^3 round trip rel-L2 {err_rt:.2e}")
        assert err_rt <= 1e-12
        X = oracle.from_cyclic(D, n, p)
        rng = np.random.default_rng(3)
        ks = [tuple(int(v) for v in rng.integers(0, 480, 3)) for _ in range(4)] + [(0, 0, 0), (479, 1, 240)]
        flat = [np.ravel_multi_index(k, n) for k in ks]
        want = oracle.dft_points(X, flat)
        Y = oracle.from_cyclic(y.cpu().numpy(), n, p).reshape(-1)
        got = Y[flat]
        err = np.abs(got - want).max() / np.abs(want).max()
        say(f"480^3 sampled max rel error {err:.2e}")
        assert err <= 1e-12


@pytest.mark.parametrize("dtype", ["complex64", "complex128"])
def test_mixed_graph_replays(torch, dtype):
    """A captured HIP graph of a mixed-radix transform (persistent line passes whose
    grid comes from an occupancy query, the fused exchange), replayed three times
    with eager work of the same plan in between, each replay against the eager
    result bitwise."""
    import paper_2203_11795_amd as fftu
    n, p = (36, 343, 28), (2, 1, 2)          # 343 = 7^3: lines of three radix-7 stages
    N = int(np.prod(n))
    D = synth.uniform_complex(N, 11, NP[dtype])
    x = torch.from_numpy(D).cuda()
    with fftu.Plan(n, p, dtype) as plan:
        assert any("k_mline" in k for k in plan.launch_names())
        out = plan(x)
        torch.cuda.synchronize()
        want = out.clone()
        assert oracle.rel_l2(want.cpu().numpy().astype(np.complex128),
                             oracle.cyclic_dft(D.astype(np.complex128), n, p)) <= TOL[dtype]
        g = fftu.Graph(plan, x, out)
        try:
            for rep in range(3):
                out.zero_()
                scratch = plan(x.flip(0).contiguous())
                torch.cuda.synchronize()
                g.launch()
                torch.cuda.synchronize()
                assert torch.equal(out, want), rep
                del scratch
        finally:
            g.close()
