"""Grids beyond p_max = sqrt(N) on the GPU: several communication supersteps
through the group-cyclic distribution (Section 2.3, the paragraph after
eq. (2.13)), through the C ABI.

End to end the result is checked against the oracle's DFT (eq. (1.2) in the
cyclic layout, which does not go through the group-cyclic emulator); each step
of each superstep is checked against the oracle's group-cyclic emulator, the
Puts bit for bit.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import FORWARD, INVERSE
from oracle import group_cyclic as gc

pytestmark = pytest.mark.gpu

TOL = {"complex128": 1e-12, "complex64": 5e-6}
NP = {"complex128": np.complex128, "complex64": np.complex64}


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


GRIDS = [
    ((8,), (4,)),                   # 2 supersteps, p_h = 2
    ((16,), (8,)),                  # 3 supersteps
    ((1024,), (64,)),
    ((32,), (16,)),                 # 4 supersteps
    ((16, 16), (8, 2)),             # one dimension beyond p_max, one within
    ((64, 64), (16, 16)),
    ((64, 32, 16), (16, 8, 8)),     # levels per dimension: 2, 2 and 3 (3 supersteps)
    ((4, 16, 8), (2, 8, 4)),
    ((256, 64), (32, 16)),
    ((27, 8), (9, 4)),              # mixed radix: 27 over 9 (m = 3), then 9 over 3
    ((125,), (25,)),
    ((2, 8, 8, 4), (1, 4, 4, 2)),
    ((1 << 20, 8), (2048, 2)),      # lines of 512 and length-4 FFTs 128 apart, over 4096 blocks
]


@pytest.mark.parametrize("n,p", GRIDS)
@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("direction", [FORWARD, INVERSE])
def test_group_cyclic_transform_matches_the_dft(torch, n, p, dtype, direction):
    import paper_2203_11795_amd as fftu
    N = int(np.prod(n))
    say(f"group-cyclic n={n} p={p} {dtype} dir={direction}")
    D = synth.uniform_complex(N, 300 + N % 101, NP[dtype])
    want = oracle.cyclic_dft(D.astype(np.complex128), n, p, direction)
    x = torch.from_numpy(D).cuda()
    with fftu.Plan(n, p, dtype, direction) as plan:
        info = plan.info()
        assert info["supersteps"] == gc.supersteps(n, p) >= 2
        y = plan(x)
        z = x.clone()
        plan(z, z)                                   # in place
        torch.cuda.synchronize()
        got = y.cpu().numpy()
        assert np.array_equal(z.cpu().numpy(), got)
        assert np.array_equal(x.cpu().numpy(), D)    # the input is left alone
    assert oracle.rel_l2(got, want) <= TOL[dtype]
    with fftu.Plan(n, p, dtype, direction, external=True) as ext:
        ws = torch.empty_like(x)
        e = ext(x, workspace=ws)
        torch.cuda.synchronize()
        assert np.array_equal(e.cpu().numpy(), got)


@pytest.mark.parametrize("n,p", [((1024,), (64,)), ((16, 16), (8, 2)), ((64, 32, 16), (16, 8, 8)), ((27, 8), (9, 4)),
                                 ((32,), (16,))])
@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("direction", [FORWARD, INVERSE])
def test_each_step_matches_the_emulator(torch, n, p, dtype, direction):
    """Each computation phase, twiddle and Put on the GPU, fed the emulator's
    buffer before it, against the emulator's buffer after it; the Puts move data
    only and must agree bit for bit."""
    import paper_2203_11795_amd as fftu
    N = int(np.prod(n))
    D = synth.uniform_complex(N, 77, NP[dtype]).astype(np.complex128)
    ref = gc.emulate_group_cyclic(D, n, p, direction)
    H = ref["H"]
    tol = TOL[dtype]

    def run(phase, part, host):
        x = torch.from_numpy(host.astype(NP[dtype])).cuda()
        out = torch.full_like(x, float("nan"))
        plan.superstep(phase, part, x, out)
        torch.cuda.synchronize()
        return out.cpu().numpy()

    with fftu.Plan(n, p, dtype, direction) as plan:
        assert plan.info()["supersteps"] == H
        assert oracle.rel_l2(run(0, 0, D), ref["fft0"]) <= tol
        for c in range(H):
            assert oracle.rel_l2(run(c, 1, ref[f"fft{c}"]), ref[f"tw{c}"]) <= tol, f"twiddle {c}"
            tw = ref[f"tw{c}"].astype(NP[dtype])
            moved = run(c, 2, tw)
            assert np.array_equal(moved, gc.put_superstep(tw, n, p, c)), f"Put {c}"
            assert oracle.rel_l2(moved, ref[f"put{c}"]) <= tol, f"Put {c}"
            assert oracle.rel_l2(run(c + 1, 0, ref[f"put{c}"]), ref[f"fft{c + 1}"]) <= tol, f"phase {c + 1}"
        with pytest.raises(fftu.FftuError):
            plan.superstep(H, 1, torch.zeros(N, dtype=plan.torch_dtype, device="cuda"))
        with pytest.raises(fftu.FftuError):
            plan.stage("exchange", torch.zeros(N, dtype=plan.torch_dtype, device="cuda"))


@pytest.mark.parametrize("n,p", [((1024,), (64,)), ((16, 16), (8, 2)), ((64, 32, 16), (16, 8, 8)), ((32,), (16,))])
def test_puts_move_exactly_the_emulators_elements(torch, n, p):
    """Every Put bit for bit on distinct values (element numbers, exact in
    complex128): a lost, duplicated or misplaced element shows at once."""
    import paper_2203_11795_amd as fftu
    N = int(np.prod(n))
    idx = np.arange(N, dtype=np.float64) + 1j * np.arange(N, dtype=np.float64)[::-1]
    with fftu.Plan(n, p, "complex128", FORWARD) as plan:
        for c in range(gc.supersteps(n, p)):
            x = torch.from_numpy(idx).cuda()
            y = plan.superstep(c, 2, x)
            torch.cuda.synchronize()
            assert np.array_equal(y.cpu().numpy(), gc.put_superstep(idx, n, p, c)), f"Put {c}"


def test_kernels_of_each_phase(torch):
    """Power-of-two sides run the phases on the power-of-two pass kernels (the
    passes of the cyclic path's Superstep 0), other sides on k_mline."""
    import paper_2203_11795_amd as fftu
    with fftu.Plan((512, 512, 512), (32, 32, 32), "complex128") as plan:
        names = plan.launch_names()
    # 16^3 blocks: the two inner sides in one k_group2 pass, the outer side in a k_line
    # pass; the last Put with the 2 x 2 x 2 FFTs of length p_h = 2 in one k_gplast
    assert len(names) == 6 and names[2] == "fftu::k_gputt<double, 4>", names
    assert names[0] == names[3] == "fftu::k_group2<double, 4, 4>", names
    assert all(k.startswith("fftu::k_line<double, 4,") for k in (names[1], names[4])), names
    assert names[5] == "fftu::k_gplast<double, 3>", names
    with fftu.Plan((16, 16), (8, 2), "complex128") as plan:
        names = plan.launch_names()
    # N = 256: the first two Puts move one tile of 256 elements; the last is k_gplast
    assert names.count("fftu::k_gputt<double, 1>") == 2 and names[-1] == "fftu::k_gplast<double, 1>", names
    with fftu.Plan((16,), (8,), "complex128") as plan:
        names = plan.launch_names()
    assert names.count("fftu::k_gput<double>") == 2, names   # N = 16: below one tile, the gather
    with fftu.Plan((27, 8), (9, 4), "complex64") as plan:
        names = plan.launch_names()
    assert names.count("fftu::k_gput<float>") == 2 and all(k in ("fftu::k_gput<float>", "fftu::k_mline<float>")
                                                            for k in names), names


def _cyclic_position(j, n, p):
    """Buffer position of natural index j in the cyclic layout (Section 1.1)."""
    rank, lin = 0, 0
    for jl, nl, pl in zip(j, n, p):
        rank = rank * pl + jl % pl
        lin = lin * (nl // pl) + jl // pl
    m = [nl // pl for nl, pl in zip(n, p)]
    return rank * int(np.prod(m)) + lin


def test_512cube_on_32cube_grid_full_size(torch):
    """512^3 complex128 over 32^3 virtual processors (P = 32768 > sqrt(N) = 11585):
    two supersteps. Sparse input (40 nonzeros): 2000 sampled outputs against eq.
    (1.2) over the nonzeros in FP64; dense input: Parseval and the round trip."""
    import paper_2203_11795_amd as fftu
    n, p = (512, 512, 512), (32, 32, 32)
    N = 512 ** 3
    rng = np.random.default_rng(61)
    js = np.unique(rng.integers(0, 512, size=(40, 3)), axis=0)
    vals = rng.uniform(-1, 1, len(js)) + 1j * rng.uniform(-1, 1, len(js))
    x = torch.zeros(N, dtype=torch.complex128, device="cuda")
    pos = torch.tensor([_cyclic_position(tuple(j), n, p) for j in js], device="cuda")
    x[pos] = torch.from_numpy(vals).to("cuda")
    with fftu.Plan(n, p, "complex128", FORWARD) as plan, fftu.Plan(n, p, "complex128", INVERSE) as inv:
        assert plan.info()["supersteps"] == 2
        y = plan(x)
        torch.cuda.synchronize()
        ks = rng.integers(0, 512, size=(2000, 3))
        kpos = torch.tensor([_cyclic_position(tuple(k), n, p) for k in ks], device="cuda")
        got = y[kpos].cpu().numpy()
        phase = (ks @ js.T) % 512
        want = (np.exp(-2j * np.pi * phase / 512.0) * vals[None, :]).sum(axis=1)
        err = np.abs(got - want).max() / np.abs(want).max()
        say(f"512^3 over 32^3 sparse input: max rel error {err:.2e} over 2000 outputs")
        assert err <= 1e-12
        xd = torch.empty(N, dtype=torch.complex128, device="cuda")
        fftu.fill_uniform(xd, 11, 0)
        yd = plan(xd)
        zd = inv(yd)
        torch.cuda.synchronize()
        nx = torch.linalg.vector_norm(xd).item()
        ny = torch.linalg.vector_norm(yd).item()
        assert abs(ny * ny / (N * nx * nx) - 1.0) <= 1e-12
        rt = (torch.linalg.vector_norm(zd - xd) / nx).item()
        say(f"512^3 over 32^3 dense input: round trip {rt:.2e}")
        assert rt <= 1e-12


def test_convolution_on_a_group_cyclic_grid(torch):
    """Forward, pointwise product, inverse on a grid beyond p_max, against the
    oracle's circular convolution summed from its definition."""
    import paper_2203_11795_amd as fftu
    n, p = (16, 16), (8, 2)
    X = synth.uniform_complex(256, 5).reshape(n)
    Hh = synth.uniform_complex(256, 6).reshape(n)
    want = oracle.to_cyclic(oracle.circular_convolution(X, Hh), p)
    with fftu.ConvolutionPlan(n, p, "complex128") as cp:
        h = torch.from_numpy(oracle.to_cyclic(Hh, p)).cuda()
        h_hat = cp(h)
        x = torch.from_numpy(oracle.to_cyclic(X, p)).cuda()
        y = cp.convolve(x, h_hat)
        torch.cuda.synchronize()
    assert oracle.rel_l2(y.cpu().numpy(), want) <= 1e-12
