"""Parity of k_lastx (the innermost dimension's local FFTs fused with the twiddle,
the exchange and the length-p FFTs) with the FP64 oracle, through the C ABI.

Superstep 0 factorises over dimensions (eq. (1.3)), so running the innermost
dimension last and inside the exchange kernel must give the DFT of eq. (1.2)
within the same tolerances as the unfused path: 1e-12 (complex128) and 5e-6
(complex64) relative L2. Every compiled register/wave split of k_lastx is
reached by one shape below (the split is checked by kernel name).
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

# (n, p, template arguments after the type: log2 m_d, nr, lpr, nh, lph)
CASES = [
    ((16, 32, 512), (4, 4, 4), (7, 2, 2, 1, 2)),           # the 512^3 / 4x4x4 kernel, few rows
    ((64, 64, 512), (4, 4, 4), (7, 2, 2, 1, 2)),           # the same kernel over 16384 tiles... of 2^21 points
    ((4, 256, 64), (2, 2, 2), (5, 3, 1, 0, 0)),
    ((4, 256, 128), (2, 2, 2), (6, 3, 1, 0, 0)),
    ((4, 4, 4, 4, 64), (2, 2, 2, 2, 2), (5, 3, 1, 2, 1)),
    ((16, 4, 4, 64), (4, 2, 2, 2), (5, 3, 1, 1, 2)),
    ((8, 4, 4, 4, 128), (2, 2, 2, 2, 2), (6, 3, 1, 2, 1)),
    ((4, 4, 4, 256), (2, 2, 2, 2), (7, 4, 1, 0, 0)),
    ((4, 4, 4, 4, 4, 256), (2, 2, 2, 2, 2, 2), (7, 4, 1, 2, 1)),
    ((16, 4, 4, 4, 256), (4, 2, 2, 2, 2), (7, 4, 1, 1, 2)),
    ((4, 16, 512), (2, 4, 4), (7, 2, 2, 1, 1)),
    ((64, 512), (4, 4), (7, 2, 2, 0, 0)),
    ((4, 4, 4, 512), (2, 2, 2, 2), (8, 4, 1, 0, 0)),
    ((4, 4, 4, 4, 512), (2, 2, 2, 2, 2), (8, 4, 1, 1, 1)),
    ((16, 1024), (4, 4), (8, 2, 2, 0, 0)),
    ((8, 16, 1024), (2, 4, 4), (8, 2, 2, 1, 1)),
    # 1024-thread tiles: a row of 256 in each of 64 blocks (the 1024^3 / 4x4x4 kernel)
    ((16, 16, 1024), (4, 4, 4), (8, 2, 2, 1, 2)),
    ((4, 4, 16, 1024), (2, 2, 4, 4), (8, 2, 2, 2, 1)),
    ((16, 4, 4, 4, 512), (4, 2, 2, 2, 2), (8, 4, 1, 1, 2)),
    ((4, 4, 4, 4, 4, 512), (2, 2, 2, 2, 2, 2), (8, 4, 1, 2, 1)),
    # lines of 64 held as 16 elements per thread (stages of 16 and 4) for splits of 16
    # register sources: the packed 512 x 512 x 256 array of the real transforms over 4^3
    ((32, 64, 256), (4, 4, 4), (6, 2, 2, 1, 2)),
    ((32, 32, 256), (2, 4, 4), (6, 2, 2, 1, 1)),
    ((256, 256), (4, 4), (6, 2, 2, 0, 0)),
    # lines of 32 the same way (stages of 16 and 2)
    ((32, 64, 128), (4, 4, 4), (5, 2, 2, 1, 2)),
    ((64, 128, 128), (4, 4, 4), (5, 2, 2, 1, 2)),
]
IDS = [f"{'x'.join(map(str, n))}-p{'x'.join(map(str, p))}" for n, p, _ in CASES]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2203_11795_amd as fftu
    fftu.load_library()
    return torch


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def run(torch, n, p, dtype, direction, D, inplace=False, fuse=-1):
    import paper_2203_11795_amd as fftu
    fftu.set_tuning("fuse_last", fuse)
    try:
        plan = fftu.Plan(n, p, dtype, direction)
    finally:
        fftu.set_tuning("fuse_last", -1)
    with plan:
        x = torch.from_numpy(np.ascontiguousarray(D.astype(NP_DTYPE[dtype]))).to("cuda")
        out = x if inplace else torch.empty_like(x)
        plan(x, out)
        torch.cuda.synchronize()
        return out.cpu().numpy(), plan.info(), plan.launch_names()


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("direction", [FORWARD, INVERSE])
@pytest.mark.parametrize("n,p,split", CASES, ids=IDS)
def test_lastx_matches_oracle(torch_dev, n, p, split, dtype, direction):
    N = int(np.prod(n))
    seed = 100 + N % 997 + len(n)
    say(f"lastx n={n} p={p} {dtype} dir={direction} seed={seed}")
    D = synth.uniform_complex(N, seed, NP_DTYPE[dtype])
    got, info, names = run(torch_dev, n, p, dtype, direction, D)
    t = "double" if dtype == "complex128" else "float"
    assert info["exchange_fused"] == 2 and info["launches"] == info["s0_kernels"] + 1
    assert names[-1].startswith(f"fftu::k_lastx<{t}, {', '.join(map(str, split))}, false, ")
    lognt = 10 if (split[0], split[3] * split[4]) == (8, 2) else 9     # rows of 256 over 2 wave bits: 1024
    assert names[-1].endswith(f", {lognt}>")
    want = oracle.cyclic_dft(D.astype(np.complex128), n, p, direction)
    err = oracle.rel_l2(got, want)
    assert err <= TOL[dtype], f"rel-L2 {err:.3e}"


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("n,p,split", CASES[:3] + CASES[4:5], ids=IDS[:3] + IDS[4:5])
def test_lastx_agrees_with_unfused_path(torch_dev, n, p, split, dtype):
    """The same transform with the fusion switched off (innermost dimension first,
    separate exchange): only the order of the dimensions' roundings differs."""
    N = int(np.prod(n))
    D = synth.uniform_complex(N, 77, NP_DTYPE[dtype])
    a, ia, _ = run(torch_dev, n, p, dtype, FORWARD, D)
    b, ib, _ = run(torch_dev, n, p, dtype, FORWARD, D, fuse=0)
    assert ia["exchange_fused"] == 2 and ib["exchange_fused"] != 2
    assert ia["launches"] == ib["launches"] - 1     # one pass over HBM fewer
    assert oracle.rel_l2(a, b) <= (1e-14 if dtype == "complex128" else 1e-6)


@pytest.mark.parametrize("n,p,split", CASES[:3], ids=IDS[:3])
def test_lastx_in_place_impulse_and_round_trip(torch_dev, n, p, split):
    N = int(np.prod(n))
    D = synth.uniform_complex(N, 5)
    a, _, _ = run(torch_dev, n, p, "complex128", FORWARD, D)
    b, _, _ = run(torch_dev, n, p, "complex128", FORWARD, D, inplace=True)
    assert np.array_equal(a, b)
    back, _, _ = run(torch_dev, n, p, "complex128", INVERSE, a, inplace=True)
    assert oracle.rel_l2(back, D) <= 1e-12
    delta = np.zeros(N, np.complex128)
    delta[0] = 1.0
    ones, _, _ = run(torch_dev, n, p, "complex128", FORWARD, delta)
    assert np.array_equal(ones, np.ones(N))        # omega^0 = 1 and the DFT of a delta are exact


def test_lastx_writes_every_output(torch_dev):
    """NaN sentinels in the output buffer are all overwritten."""
    import paper_2203_11795_amd as fftu
    torch = torch_dev
    n, p = (64, 64, 512), (4, 4, 4)
    N = int(np.prod(n))
    x = torch.from_numpy(synth.uniform_complex(N, 9)).to("cuda")
    out = torch.full((N,), complex(float("nan"), float("nan")), dtype=torch.complex128, device="cuda")
    with fftu.Plan(n, p, "complex128", FORWARD) as plan:
        assert plan.info()["exchange_fused"] == 2
        plan(x, out)
    torch.cuda.synchronize()
    assert not torch.isnan(out).any().item()


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_lastx_external_plan_with_workspace(torch_dev, dtype):
    """An external plan (shared table, workspace given per call) runs k_lastx with the
    same results as a plan that owns its workspace, bit for bit, in place as well."""
    import paper_2203_11795_amd as fftu
    torch = torch_dev
    n, p = (16, 32, 512), (4, 4, 4)
    N = int(np.prod(n))
    D = synth.uniform_complex(N, 12, NP_DTYPE[dtype])
    x = torch.from_numpy(D).to("cuda")
    with fftu.Plan(n, p, dtype) as own, fftu.Plan(n, p, dtype, external=True) as ext:
        assert ext.info()["exchange_fused"] == 2 and ext.device_bytes() == 0
        ws = torch.empty_like(x)
        a = own(x)
        b = ext(x, workspace=ws)
        c = x.clone()
        ext(c, c, workspace=ws)
        torch.cuda.synchronize()
        assert torch.equal(a, b) and torch.equal(a, c)


def test_lastx_graph_replays(torch_dev):
    """A captured k_lastx plan replays correctly several times, with eager work and
    synchronisation between the replays (no memset nodes are recorded)."""
    import paper_2203_11795_amd as fftu
    torch = torch_dev
    n, p = (64, 64, 512), (4, 4, 4)
    N = int(np.prod(n))
    x = torch.from_numpy(synth.uniform_complex(N, 13)).to("cuda")
    y = torch.empty_like(x)
    with fftu.Plan(n, p, "complex128") as plan:
        want = plan(x)
        torch.cuda.synchronize()
        g = fftu.Graph(plan, x, y)
        try:
            for _ in range(3):
                y.zero_()
                g.launch()
                torch.cuda.synchronize()
                assert torch.equal(y, want)
                plan(x, torch.empty_like(x))          # eager work between replays
                torch.cuda.synchronize()
        finally:
            g.close()
