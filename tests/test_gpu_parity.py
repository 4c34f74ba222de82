"""Parity of the HIP path with the FP64 oracle, element by element, through the C ABI.

Tolerances (relative L2 over all outputs): 1e-12 for complex128, 5e-6 for
complex64. The permutation of Superstep 1 moves data only and must match the
emulator of Algorithm 2.3 bit for bit.
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


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2203_11795_amd as fftu
    fftu.load_library()
    return torch


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def run_plan(torch, n, p, dtype, direction, D, entry=None, out_init=None, inplace=False):
    import paper_2203_11795_amd as fftu
    plan = fftu.Plan(n, p, dtype, direction)
    x = torch.from_numpy(np.ascontiguousarray(D.astype(NP_DTYPE[dtype]))).to("cuda")
    if inplace:
        out = x
    elif out_init is not None:
        out = torch.from_numpy(out_init.astype(NP_DTYPE[dtype])).to("cuda")
    else:
        out = torch.empty_like(x)
    if entry is None:
        plan(x, out)
    else:
        plan.stage(entry, x, out)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    plan.close()
    return res


CASES = [
    ((64, 64, 64), (2, 2, 2)),        # the 64^3 configuration
    ((8,), (2,)),                     # Algorithm 2.2, n = 8, p = 2
    ((16,), (4,)),                    # q = 1
    ((4,), (2,)),
    ((1,), (1,)),                     # N = 1
    ((2,), (1,)),
    ((256,), (1,)),                   # plain 1-D FFT
    ((1024,), (32,)),
    ((16, 8), (2, 2)),
    ((64, 64), (8, 8)),               # P = 64, q = 1
    ((16, 16, 4), (4, 2, 2)),
    ((4, 16, 8), (2, 2, 2)),          # uneven sides
    ((8, 1, 4), (2, 1, 1)),           # a side of 1
    ((32, 8, 4, 16), (2, 2, 1, 4)),
    ((4, 4, 4, 4, 4), (2, 2, 2, 2, 2)),
    ((16, 16, 16), (4, 4, 4)),        # P = 64 in registers
    ((64, 64, 64), (8, 8, 2)),        # P = 128: unfused twiddle / permute / F_p passes
    ((4,) * 8, (2,) * 8),             # d = 8, P = 256, unfused
    ((128, 128, 32), (1, 1, 1)),      # ordinary row-major fftn
    ((2048,), (1,)),                  # longest complex128 line in one tile
    ((32, 2048), (2, 4)),
]


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("direction", [FORWARD, INVERSE])
@pytest.mark.parametrize("n,p", CASES, ids=[f"{'x'.join(map(str, n))}-p{'x'.join(map(str, p))}" for n, p in CASES])
def test_end_to_end_matches_oracle(torch_dev, n, p, dtype, direction):
    N = int(np.prod(n))
    seed = 1 + N % 1000 + 7 * len(n)
    say(f"e2e n={n} p={p} {dtype} dir={direction} seed={seed}")
    D = synth.uniform_complex(N, seed, NP_DTYPE[dtype])
    got = run_plan(torch_dev, n, p, dtype, direction, D)
    want = oracle.cyclic_dft(D.astype(np.complex128), n, p, direction)
    err = oracle.rel_l2(got, want)
    assert err <= TOL[dtype], f"rel-L2 {err:.3e}"


def test_complex64_longest_line(torch_dev):
    n, p = (4096,), (1,)
    D = synth.uniform_complex(4096, 11, np.complex64)
    got = run_plan(torch_dev, n, p, "complex64", FORWARD, D)
    assert oracle.rel_l2(got, oracle.cyclic_dft(D.astype(np.complex128), n, p)) <= TOL["complex64"]


def test_forward_inverse_64cubed(torch_dev):
    """The 64^3 / 2x2x2 configuration: forward checked against the oracle, then the
    inverse of the GPU result checked against the original input."""
    n, p = (64, 64, 64), (2, 2, 2)
    D = synth.uniform_complex(64 ** 3, 1)
    Y = run_plan(torch_dev, n, p, "complex128", FORWARD, D)
    assert oracle.rel_l2(Y, oracle.cyclic_dft(D, n, p)) <= 1e-12
    X = run_plan(torch_dev, n, p, "complex128", INVERSE, Y)
    assert oracle.rel_l2(X, D) <= 1e-12


STAGE_CASES = [((64, 64, 64), (2, 2, 2)), ((16, 16, 4), (4, 2, 2)), ((32, 8, 4, 16), (2, 2, 1, 4)),
               ((64, 64, 64), (8, 8, 2)), ((16,), (4,))]


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("direction", [FORWARD, INVERSE])
@pytest.mark.parametrize("n,p", STAGE_CASES)
def test_each_superstep_matches_emulator(torch_dev, n, p, dtype, direction):
    N = int(np.prod(n))
    say(f"stages n={n} p={p} {dtype} dir={direction}")
    D = synth.uniform_complex(N, 3, NP_DTYPE[dtype]).astype(np.complex128)
    st = oracle.emulate(D, n, p, direction)
    tol = TOL[dtype]
    got = run_plan(torch_dev, n, p, dtype, direction, D, "local_fft")
    assert oracle.rel_l2(got, st["S0"]) <= tol
    Yin = st["S0"].astype(NP_DTYPE[dtype]).astype(np.complex128)
    got = run_plan(torch_dev, n, p, dtype, direction, Yin, "twiddle")
    assert oracle.rel_l2(got, oracle.emulate_twiddle(Yin, n, p, direction)) <= (1e-15 if dtype == "complex128"
                                                                                 else 1e-6)
    Z = st["twiddle"].astype(NP_DTYPE[dtype])
    got = run_plan(torch_dev, n, p, dtype, direction, Z, "exchange")
    assert np.array_equal(got, oracle.emulate_permute(Z, n, p)), "Superstep 1 must be an exact permutation"
    got = run_plan(torch_dev, n, p, dtype, direction, st["S1"], "remaining_fft")
    assert oracle.rel_l2(got, st["S2"]) <= tol


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("n,p", [((64, 64, 64), (2, 2, 2)), ((16, 16, 16), (4, 4, 4)), ((64, 64, 64), (8, 8, 2)),
                                 ((4, 4, 4, 4, 4), (2, 2, 2, 2, 2))])
def test_impulse_at_origin_gives_exact_ones(torch_dev, n, p, dtype):
    N = int(np.prod(n))
    D = np.zeros(N, np.complex128)
    D[0] = 1.0               # global element 0 is local element 0 of processor 0
    got = run_plan(torch_dev, n, p, dtype, FORWARD, D)
    assert np.array_equal(got, np.ones(N, NP_DTYPE[dtype]))


@pytest.mark.parametrize("n,p", [((64, 64, 64), (2, 2, 2)), ((64, 64, 64), (8, 8, 2)), ((1,), (1,))])
def test_in_place_equals_out_of_place_and_is_deterministic(torch_dev, n, p):
    N = int(np.prod(n))
    D = synth.uniform_complex(N, 21)
    a = run_plan(torch_dev, n, p, "complex128", FORWARD, D)
    b = run_plan(torch_dev, n, p, "complex128", FORWARD, D, inplace=True)
    c = run_plan(torch_dev, n, p, "complex128", FORWARD, D)
    assert np.array_equal(a, b)
    assert np.array_equal(a, c)


@pytest.mark.parametrize("n,p", [((64, 64, 64), (2, 2, 2)), ((32, 8, 4, 16), (2, 2, 1, 4)), ((16,), (4,))])
def test_exchange_writes_every_output_once(torch_dev, n, p):
    """NaN sentinels in the output must all be overwritten, and W is a permutation of Z."""
    N = int(np.prod(n))
    Z = synth.uniform_complex(N, 5)
    sentinel = np.full(N, np.nan + 1j * np.nan)
    got = run_plan(torch_dev, n, p, "complex128", FORWARD, Z, "exchange", out_init=sentinel)
    assert not np.isnan(got).any()
    assert np.array_equal(np.sort_complex(got), np.sort_complex(Z))


def test_input_left_unchanged(torch_dev):
    import paper_2203_11795_amd as fftu
    torch = torch_dev
    n, p = (64, 64, 64), (2, 2, 2)
    D = synth.uniform_complex(64 ** 3, 8)
    x = torch.from_numpy(D).to("cuda")
    with fftu.Plan(n, p, "complex128", FORWARD) as plan:
        plan(x)
        torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), D)


def test_execute_rejects_partial_overlap(torch_dev):
    import paper_2203_11795_amd as fftu
    torch = torch_dev
    x = torch.zeros(2 * 4096, dtype=torch.complex128, device="cuda")
    with fftu.Plan((4096,), (8,), "complex128", FORWARD) as plan:
        with pytest.raises(fftu.FftuError):
            plan.execute_ptr(x.data_ptr(), x.data_ptr() + 16 * 7, 0)
        with pytest.raises(fftu.FftuError):
            plan.stage("exchange", x[:4096], x[:4096])


def test_512_cubed_full_size(torch_dev):
    """The 512^3 complex128 configuration on the 4x4x4 grid, in the launch
    configuration the benchmark times, checked over all 2^27 outputs."""
    n, p = (512, 512, 512), (4, 4, 4)
    N = 512 ** 3
    say("512^3 full size: generating input")
    D = synth.uniform_complex(N, 2)
    got = run_plan(torch_dev, n, p, "complex128", FORWARD, D)
    say("512^3 full size: oracle")
    want = oracle.cyclic_dft(D, n, p)
    err = oracle.rel_l2(got, want)
    say(f"512^3 rel-L2 {err:.3e}")
    assert err <= 1e-12


def test_launch_names(torch_dev):
    import paper_2203_11795_amd as fftu
    with fftu.Plan((512, 512, 512), (4, 4, 4), "complex128", FORWARD) as plan:
        assert plan.launch_names() == ["fftu::k_line<double, 7, 1>", "fftu::k_line<double, 7, 1>",
                                       "fftu::k_lastx<double, 7, 2, 2, 1, 2, false, true, 9>"]
    fftu.set_tuning("fuse_last", 0)
    try:
        with fftu.Plan((512, 512, 512), (4, 4, 4), "complex128", FORWARD) as plan:
            assert plan.launch_names() == ["fftu::k_line<double, 7, 2>", "fftu::k_line<double, 7, 1>",
                                           "fftu::k_line<double, 7, 1>", "fftu::k_exchange<double, 2, 2, 1, 2>"]
    finally:
        fftu.set_tuning("fuse_last", -1)
    with fftu.Plan((64,) * 5, (2,) * 5, "complex64", FORWARD) as plan:
        # dimensions (1, 2) and (3, 4) in k_pair passes, dimension 5 fused with the exchange
        # (rows 256 KiB apart in the first pair: 1024 threads; 256 bytes apart in the second: 512)
        assert plan.launch_names() == ["fftu::k_pair<float, 5, 5, 10>", "fftu::k_pair<float, 5, 5, 9>",
                                       "fftu::k_lastx<float, 5, 3, 1, 2, 1, false, true, 9>"]
    fftu.set_tuning("fuse_last", 0)
    fftu.set_tuning("pair", 0)
    try:
        with fftu.Plan((64,) * 5, (2,) * 5, "complex64", FORWARD) as plan:
            names = plan.launch_names()
            assert names[0] == "fftu::k_group2<float, 5, 5>" and names[-1] == "fftu::k_exchange<float, 5, 1, 0, 0>"
            assert len(names) == 5
    finally:
        fftu.set_tuning("fuse_last", -1)
        fftu.set_tuning("pair", -1)
    with fftu.Plan((64, 64, 64), (8, 8, 2), "complex128", FORWARD) as plan:
        # unfused exchange: Superstep 0 passes, twiddle, permutation, then Superstep 2 passes
        names = plan.launch_names()
        info = plan.info()
        assert len(names) == info["launches"] and info["exchange_fused"] == 0
        i = names.index("fftu::k_twiddle<double>")
        assert i == info["s0_kernels"] and names[i + 1] == "fftu::k_permute<double>"
        assert len(names) - i == info["s2_kernels"] > 2     # twiddle, permutation and the F_p passes


@pytest.mark.parametrize("knob,values", [("line_strided_logw", [2, 3, 4, 5]), ("line_contig_logw", [0, 1, 3, 5]),
                                         ("line_pad", [0, 2, 4]), ("max_lds_kb", [16, 160])])
def test_tuning_changes_tiling_not_results(torch_dev, knob, values):
    """Tiling knobs move work between workgroups; every element sees the same arithmetic."""
    import paper_2203_11795_amd as fftu
    n, p = (64, 128, 256), (2, 2, 4)
    D = synth.uniform_complex(int(np.prod(n)), 31)
    base = run_plan(torch_dev, n, p, "complex128", FORWARD, D)
    assert oracle.rel_l2(base, oracle.cyclic_dft(D, n, p)) <= 1e-12
    try:
        for v in values:
            fftu.set_tuning(knob, v)
            got = run_plan(torch_dev, n, p, "complex128", FORWARD, D)
            assert oracle.rel_l2(got, base) <= 1e-15, (knob, v)
    finally:
        fftu.set_tuning(knob, -1)


def test_misaligned_buffers_are_rejected(torch_dev):
    """Buffers hold whole complex elements: a pointer off the element size is refused
    before any launch."""
    import paper_2203_11795_amd as fftu
    torch = torch_dev
    with fftu.Plan((64, 64), (2, 2), "complex128") as plan:
        x = torch.zeros(64 * 64 + 1, dtype=torch.complex128, device="cuda")
        base = x.data_ptr()
        with pytest.raises(fftu.FftuError):
            plan.execute_ptr(base + 8, base + 8)           # in place, 8 bytes off
        with pytest.raises(fftu.FftuError):
            plan.execute_ptr(base, base + 8)
        plan.execute_ptr(base, base)                       # aligned, in place: accepted
        torch.cuda.synchronize()
    lib = fftu.load_library()
    y = torch.zeros(16, dtype=torch.complex64, device="cuda")
    assert lib.fftu_fill_uniform(y.data_ptr() + 4, 4, 1, 0, 0, 0, None) == 1
    assert lib.fftu_pointwise_mul(y.data_ptr() + 4, y.data_ptr(), y.data_ptr(), 4, 1, 1.0, None) == 1


def _cyclic_position(j, n, p):
    """Buffer position of natural index j (a d-tuple) in the cyclic layout
    (Section 1.1): processor s = j mod p, local index k = j div p, position
    rank(s) M + lin(k), both row-major."""
    m = [a // b for a, b in zip(n, p)]
    rank = lin = 0
    for l in range(len(n)):
        rank = rank * p[l] + j[l] % p[l]
        lin = lin * m[l] + j[l] // p[l]
    return rank * int(np.prod(m)) + lin


def test_64pow5_full_size_sparse_and_properties(torch_dev):
    """The 64^5 complex64 configuration on the 2^5 grid at full size, in the launch
    configuration the benchmark times. (1) A sparse input (40 nonzeros) has a dense
    transform whose every output is a 40-term sum of eq. (1.2): 2000 sampled outputs
    are checked against it in FP64. (2) Parseval and the round trip on a dense input
    from the device generator hold at any size."""
    import paper_2203_11795_amd as fftu
    torch = torch_dev
    n, p = (64,) * 5, (2,) * 5
    N = 64 ** 5
    rng = np.random.default_rng(53)
    js = np.unique(rng.integers(0, 64, size=(40, 5)), axis=0)      # distinct positions
    vals = (rng.uniform(-1, 1, len(js)) + 1j * rng.uniform(-1, 1, len(js))).astype(np.complex64)
    x = torch.zeros(N, dtype=torch.complex64, device="cuda")
    pos = torch.tensor([_cyclic_position(tuple(j), n, p) for j in js], device="cuda")
    x[pos] = torch.from_numpy(vals).to("cuda")
    with fftu.Plan(n, p, "complex64", FORWARD) as plan:
        y = plan(x)
        torch.cuda.synchronize()
        ks = rng.integers(0, 64, size=(2000, 5))
        kpos = torch.tensor([_cyclic_position(tuple(k), n, p) for k in ks], device="cuda")
        got = y[kpos].cpu().numpy().astype(np.complex128)
        # eq. (1.2) over the nonzeros, in FP64, with exact integer phases mod 64
        phase = (ks @ js.T) % 64
        want = (np.exp(-2j * np.pi * phase / 64.0) * vals.astype(np.complex128)[None, :]).sum(axis=1)
        err = np.abs(got - want).max() / np.abs(want).max()
        say(f"64^5 sparse input: max rel error {err:.2e} over 2000 sampled outputs")
        assert err <= 5e-6
        # dense input: Parseval (||F x||^2 = N ||x||^2) and the round trip
        xd = torch.empty(N, dtype=torch.complex64, device="cuda")
        fftu.fill_uniform(xd, 3, 0)
        yd = plan(xd)
        with fftu.Plan(n, p, "complex64", INVERSE) as inv:
            zd = inv(yd)
        torch.cuda.synchronize()
        nx = torch.linalg.vector_norm(xd.to(torch.complex128)).item()
        ny = torch.linalg.vector_norm(yd.to(torch.complex128)).item()
        assert abs(ny * ny / (N * nx * nx) - 1.0) <= 1e-5
        rt = (torch.linalg.vector_norm((zd - xd).to(torch.complex128)) / nx).item()
        say(f"64^5 dense input: Parseval ratio {ny * ny / (N * nx * nx):.8f}, round trip {rt:.2e}")
        assert rt <= 5e-6
