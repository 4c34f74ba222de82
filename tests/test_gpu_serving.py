"""Serving on the GPU: the device input generator against its host twin, plans
without device memory of their own, and the request loop (results alone equal
results in the mix; the oracle, fed by the host twin, agrees)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from synth import philox
from oracle import FORWARD, INVERSE

pytestmark = pytest.mark.gpu

TOL = {"complex128": 1e-12, "complex64": 5e-6}
NP = {"complex128": np.complex128, "complex64": np.complex64}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.mark.parametrize("dtype", ["complex64", "complex128"])
@pytest.mark.parametrize("count,base", [(1, 0), (1_000_003, 0), (4097, (1 << 32) - 2000), (0, 0)])
def test_fill_matches_host_twin_bitwise(torch, dtype, count, base):
    import paper_2203_11795_amd as fftu
    say(f"fill {dtype} count={count} base={base}")
    t = torch.full((max(count, 1),), complex(7.0, 7.0), dtype=getattr(torch, dtype), device="cuda")
    fftu.fill_uniform(t[:count], 5, 123, base)
    torch.cuda.synchronize()
    got = t[:count].cpu().numpy()
    want = philox.uniform_complex(count, 5, 123, NP[dtype], counter_base=base)
    assert got.dtype == want.dtype and np.array_equal(got.view(np.uint8), want.view(np.uint8))
    if count == 0:
        assert t[0].item() == complex(7.0, 7.0)        # nothing written


def test_fill_rejects_bad_arguments(torch):
    import paper_2203_11795_amd as fftu
    lib = fftu.load_library()
    assert lib.fftu_fill_uniform(None, 10, 1, 0, 0, 0, None) == 1
    assert lib.fftu_fill_uniform(None, 0, 1, 0, 0, 0, None) == 0
    x = torch.empty(4, dtype=torch.complex64, device="cuda")
    assert lib.fftu_fill_uniform(x.data_ptr(), -1, 1, 0, 0, 0, None) == 1
    assert lib.fftu_fill_uniform(x.data_ptr(), 4, 7, 0, 0, 0, None) == 1


@pytest.mark.parametrize("n,p", [((64, 64, 64), (2, 2, 2)), ((512, 512), (4, 4)), ((64, 64, 64), (8, 8, 2)),
                                 ((32, 1024), (2, 2)), ((16,) * 4, (2,) * 4)])
@pytest.mark.parametrize("dtype", ["complex64", "complex128"])
@pytest.mark.parametrize("direction", [FORWARD, INVERSE])
def test_external_plan_equals_plan_bitwise(torch, n, p, dtype, direction):
    import paper_2203_11795_amd as fftu
    N = int(np.prod(n))
    x = torch.from_numpy(synth.uniform_complex(N, 77, NP[dtype])).cuda()
    with fftu.Plan(n, p, dtype, direction) as a, fftu.Plan(n, p, dtype, direction, external=True) as b:
        assert b.device_bytes() == 0 and a.device_bytes() > 0
        ws = torch.empty(N, dtype=x.dtype, device="cuda")
        ya = a(x)
        yb = b(x, workspace=ws)
        yc = x.clone()
        b(yc, yc, workspace=ws)                              # in place
        torch.cuda.synchronize()
        assert torch.equal(ya, yb) and torch.equal(ya, yc)
        with pytest.raises(fftu.FftuError):
            b(x)                                             # an external plan needs a workspace
        with pytest.raises(fftu.FftuError):
            b.execute_ws_ptr(x.data_ptr(), yb.data_ptr(), x.data_ptr())   # workspace overlaps the input


def serving_requests(duration, exps=(5, 6), rate=400.0):
    from paper_2203_11795_amd import serving
    return serving.requests_from_trace(synth.serving_trace(seed=5, rate=rate, duration=duration, exponents=exps))


def test_serving_alone_equals_mix_and_oracle(torch):
    from paper_2203_11795_amd import serving
    reqs = serving_requests(0.1)
    say(f"serving {len(reqs)} requests, largest {max(r.N for r in reqs)} points")
    srv = serving.Server(arena_bytes=2 << 30, streams=4)
    try:
        mix = srv.serve(reqs, "continuous", keep=[r.rid for r in reqs])
        assert mix.completed == len(reqs) and mix.unfinished == 0
        assert all(v > 0 for v in mix.latencies.values())
        rng = np.random.default_rng(2)
        sample = [reqs[i] for i in sorted(rng.choice(len(reqs), size=6, replace=False))]
        for r in sample:
            alone = srv.serve([serving.Request(r.rid, 0.0, r.shape, r.dtype, r.direction)], "fifo", keep=[r.rid])
            assert np.array_equal(alone.outputs[r.rid], mix.outputs[r.rid]), r
        for r in sorted(reqs, key=lambda q: q.N)[:4]:
            x = philox.uniform_complex(r.N, 5, r.rid, NP[r.dtype]).astype(np.complex128)
            want = oracle.cyclic_dft(x, r.shape, r.grid, r.direction)
            err = oracle.rel_l2(mix.outputs[r.rid], want)
            say(f"request {r.rid} {r.shape} {r.dtype} dir={r.direction}: rel-L2 {err:.2e}")
            assert err <= TOL[r.dtype]
    finally:
        srv.close()


def test_serving_admission_with_a_small_arena(torch):
    from paper_2203_11795_amd import serving
    reqs = serving_requests(0.05)
    need = max(2 * r.N * r.esize for r in reqs)
    cap = 3 * need + 4096
    srv = serving.Server(arena_bytes=cap, streams=4)
    try:
        for policy in ("continuous", "fifo"):
            res = srv.serve(reqs, policy)
            s = serving.summarize(res, reqs)
            say(f"{policy}: {s}")
            assert res.completed == len(reqs) and res.peak_arena_bytes <= cap
    finally:
        srv.close()
