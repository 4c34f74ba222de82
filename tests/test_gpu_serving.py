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


def test_serving_large_lanes_alone_equals_mix(torch):
    """The first 0.1 s of the serving trace itself (2000 requests/s, sides up to
    1024, up to 2^26 points): 104 of its 235 requests are 64 MiB or more and run
    on the large lanes. Large requests of both dtypes, and two small ones, give
    bitwise the same result alone as in the mix."""
    from paper_2203_11795_amd import serving
    reqs = serving.requests_from_trace(synth.serving_trace(seed=5, rate=2000.0, duration=30.0), limit_seconds=0.1)
    big = [r for r in reqs if r.N * r.esize >= 64 << 20]
    pick = ([r for r in big if r.dtype == "complex64"][:2] + [r for r in big if r.dtype == "complex128"][:2]
            + [r for r in reqs if r.N * r.esize < 1 << 20][:2])
    assert len(pick) == 6
    say(f"serving {len(reqs)} requests ({len(big)} large); checking {[(r.rid, r.shape, r.dtype) for r in pick]}")
    srv = serving.Server(arena_bytes=16 << 30, streams=4)
    try:
        mix = srv.serve(reqs, "continuous", keep=[r.rid for r in pick], time_limit=60)
        assert mix.completed == len(reqs) and mix.unfinished == 0
        for r in pick:
            alone = srv.serve([serving.Request(r.rid, 0.0, r.shape, r.dtype, r.direction)], "fifo", keep=[r.rid],
                              time_limit=20)
            assert np.array_equal(alone.outputs[r.rid], mix.outputs[r.rid]), r
    finally:
        srv.close()


def test_coalesced_batches_alone_equal_mix_and_oracle(torch):
    """Small requests that wait together run as one persistent batch launch. Each
    coalesced result is bitwise the result of the same request in a batch of one
    (same kernels), within tolerance of the request served alone (the
    per-request path, which a request that waits alone takes), and the smallest
    match the oracle fed by the host Philox twin."""
    import paper_2203_11795_amd as fftu
    from paper_2203_11795_amd import serving
    base = serving_requests(0.2, exps=(5, 6, 7), rate=1000.0)
    # a burst of the requests of at most 4 MiB: everything arrives at once, so requests wait together
    reqs = [serving.Request(r.rid, 0.0, r.shape, r.dtype, r.direction) for r in base if r.N * r.esize <= 4 << 20]
    assert len(reqs) >= 40
    srv = serving.Server(arena_bytes=2 << 30, streams=4, coalesce_max=32)
    try:
        assert all(srv.batchable(r) for r in reqs)
        mix = srv.serve(reqs, "coalesced", keep=[r.rid for r in reqs], time_limit=60)
        say(f"coalesced: {mix.coalesced_requests} of {len(reqs)} requests in {mix.batches} batches "
            f"(largest {mix.max_batch})")
        assert mix.completed == len(reqs) and mix.max_batch > 1 and mix.coalesced_requests > mix.batches
        rng = np.random.default_rng(4)
        together = [r for r in reqs if r.rid in mix.coalesced_rids]
        apart = [r for r in reqs if r.rid not in mix.coalesced_rids]
        assert len(together) >= 2
        sample = [together[i] for i in sorted(rng.choice(len(together), size=min(6, len(together)), replace=False))]
        for r in sample + apart[:2]:
            alone = srv.serve([r], "coalesced", keep=[r.rid], time_limit=20)
            assert alone.batches == 0                    # alone: the per-request path
            if r in apart:
                assert np.array_equal(alone.outputs[r.rid], mix.outputs[r.rid]), r
                continue
            assert oracle.rel_l2(alone.outputs[r.rid], mix.outputs[r.rid]) <= 2 * TOL[r.dtype], r
            x = torch.empty(r.N, dtype=getattr(torch, r.dtype), device="cuda")
            fftu.fill_uniform(x, 5, r.rid, 0)
            with fftu.BatchPlan([r.shape], [r.grid], r.dtype, r.direction) as one:
                y = one([x])[0]
                torch.cuda.synchronize()
            assert np.array_equal(y.cpu().numpy(), mix.outputs[r.rid]), r   # a batch of one, bit for bit
        plain = srv.serve(reqs, "continuous", keep=[r.rid for r in reqs], time_limit=60)
        for r in reqs:
            assert oracle.rel_l2(mix.outputs[r.rid], plain.outputs[r.rid]) <= 2 * TOL[r.dtype], r
        for r in sorted(reqs, key=lambda q: q.N)[:4]:
            x = philox.uniform_complex(r.N, 5, r.rid, NP[r.dtype]).astype(np.complex128)
            want = oracle.cyclic_dft(x, r.shape, r.grid, r.direction)
            assert oracle.rel_l2(mix.outputs[r.rid], want) <= TOL[r.dtype], r
    finally:
        srv.close()


def test_precision_error_is_stated_per_result(torch):
    """Every complex64 request's error against the complex128 transform of its own
    input, within the FP32 tolerance; the complex128 transform of the smallest
    against the oracle."""
    from paper_2203_11795_amd import serving
    reqs = serving_requests(0.05, exps=(5, 6, 7))
    srv = serving.Server(arena_bytes=1 << 30, streams=2)
    try:
        errs = serving.precision_errors(srv, reqs)
        c64 = [r for r in reqs if r.dtype == "complex64"]
        assert set(errs) == {r.rid for r in c64} and c64
        say(f"FP32 errors over {len(errs)} results: max {max(errs.values()):.2e}")
        assert all(0 < e <= 5e-6 for e in errs.values())
        r = min(c64, key=lambda q: q.N)
        x = philox.uniform_complex(r.N, 5, r.rid, np.complex64).astype(np.complex128)
        want = oracle.cyclic_dft(x, r.shape, r.grid, r.direction)
        y = torch.from_numpy(x).cuda()
        with __import__("paper_2203_11795_amd").Plan(r.shape, r.grid, "complex128", r.direction) as pl:
            got = pl(y).cpu().numpy()
        assert oracle.rel_l2(got, want) <= 1e-12
    finally:
        srv.close()


def test_external_batch_equals_batch_bitwise(torch):
    """fftu_plan_batch_external with a caller workspace and pinned staging gives
    bitwise the results of fftu_plan_batch; a second call on other buffers reuses
    nothing stale."""
    import paper_2203_11795_amd as fftu
    shapes = synth.batch_shapes(9, 21, exponents=(4, 5, 6))
    grids = [(2, 2, 2)] * 9
    xs = [torch.from_numpy(synth.uniform_complex(int(np.prod(s)), 500 + i, np.complex64)).cuda()
          for i, s in enumerate(shapes)]
    with fftu.BatchPlan(shapes, grids, "complex64", FORWARD) as a, \
            fftu.BatchPlan(shapes, grids, "complex64", FORWARD, external=True) as b:
        want = a(xs)
        ws = torch.empty(b.workspace_bytes, dtype=torch.uint8, device="cuda")
        stage = torch.empty(b.staging_bytes, dtype=torch.uint8, pin_memory=True)
        outs = [torch.empty_like(x) for x in xs]
        b.execute_ws(xs, outs, ws, stage)
        torch.cuda.synchronize()
        assert b.error_flag() == 0
        for o, w in zip(outs, want):
            assert torch.equal(o, w)
        xs2 = [x.clone() for x in xs]
        b.execute_ws(xs2, xs2, ws, stage)              # in place, new buffers
        torch.cuda.synchronize()
        for o, w in zip(xs2, want):
            assert torch.equal(o, w)
        with pytest.raises(fftu.FftuError):
            b(xs)                                      # needs execute_ws
        with pytest.raises(ValueError):
            b.execute_ws(xs, outs, ws, torch.empty(b.staging_bytes, dtype=torch.uint8))   # not pinned
        with pytest.raises(fftu.FftuError):
            b.execute_ws_ptrs([x.data_ptr() for x in xs], [ws.data_ptr()] + [o.data_ptr() for o in outs[1:]],
                              ws.data_ptr(), stage.data_ptr())    # an output inside the workspace
