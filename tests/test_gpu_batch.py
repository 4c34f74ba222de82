"""Batches of uneven transforms in one persistent launch, and HIP graph replays.

Each member of a batch is its own instance of Algorithm 2.3; it is checked
against the FP64 oracle, and against the same transform run alone (same
kernels, so bit for bit).
"""
import sys

import numpy as np
import pytest

import oracle
import synth
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


def members(count, seed, exps=(4, 5, 6)):
    shapes = synth.batch_shapes(count, seed, exponents=exps)
    return shapes, [(2, 2, 2)] * count


def to_dev(torch, arrays, dtype):
    return [torch.from_numpy(np.ascontiguousarray(a.astype(NP[dtype]))).cuda() for a in arrays]


@pytest.mark.parametrize("dtype", ["complex64", "complex128"])
@pytest.mark.parametrize("direction", [FORWARD, INVERSE])
def test_batch_matches_oracle_and_alone(torch, dtype, direction):
    import paper_2203_11795_amd as fftu
    shapes, grids = members(12, 40 + direction)
    say(f"batch {dtype} dir={direction} shapes={shapes}")
    xs_h = [synth.uniform_complex(int(np.prod(s)), 1000 + i, NP[dtype]) for i, s in enumerate(shapes)]
    xs = to_dev(torch, xs_h, dtype)
    with fftu.BatchPlan(shapes, grids, dtype, direction) as bp:
        outs = bp(xs)
        torch.cuda.synchronize()
        assert bp.error_flag() == 0
        got = [o.cpu().numpy() for o in outs]
    for i, (s, g) in enumerate(zip(shapes, grids)):
        want = oracle.cyclic_dft(xs_h[i].astype(np.complex128), s, g, direction)
        assert oracle.rel_l2(got[i], want) <= TOL[dtype], (i, s)
        with fftu.BatchPlan([s], [g], dtype, direction) as one:
            alone = one([xs[i]])[0]
            torch.cuda.synchronize()
        assert np.array_equal(alone.cpu().numpy(), got[i]), f"member {i} differs alone"


def test_batch_rebinds_buffers_and_allows_in_place(torch):
    import paper_2203_11795_amd as fftu
    shapes, grids = members(6, 7)
    xs_h = [synth.uniform_complex(int(np.prod(s)), 50 + i, np.complex64) for i, s in enumerate(shapes)]
    with fftu.BatchPlan(shapes, grids, "complex64", FORWARD) as bp:
        a = bp(to_dev(torch, xs_h, "complex64"))
        b_in = to_dev(torch, xs_h, "complex64")
        bp(b_in, b_in)                      # new buffers, in place
        torch.cuda.synchronize()
        for x, y in zip(a, b_in):
            assert torch.equal(x, y)


def test_batch_graph_replays(torch):
    import paper_2203_11795_amd as fftu
    shapes, grids = members(8, 9)
    xs_h = [synth.uniform_complex(int(np.prod(s)), 70 + i, np.complex64) for i, s in enumerate(shapes)]
    xs = to_dev(torch, xs_h, "complex64")
    outs = [torch.empty_like(x) for x in xs]
    with fftu.BatchPlan(shapes, grids, "complex64", FORWARD) as bp:
        eager = [o.clone() for o in bp(xs)]
        g = fftu.Graph(bp, xs, outs)
        for rep in range(3):
            for o in outs:
                o.zero_()                   # eager work between replays
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            for o, e in zip(outs, eager):
                assert torch.equal(o, e), f"replay {rep}"
            xs[0].mul_(2.0)                 # inputs change between replays; the graph reads them afresh
            eager[0] = eager[0] * 2.0
        g.close()


def test_single_plan_graph_replays(torch):
    import paper_2203_11795_amd as fftu
    n, p = (64, 64, 64), (2, 2, 2)
    D = synth.uniform_complex(64 ** 3, 3)
    x = torch.from_numpy(D).cuda()
    y = torch.empty_like(x)
    with fftu.Plan(n, p, "complex128", FORWARD) as plan:
        g = fftu.Graph(plan, x, y)
        want = oracle.cyclic_dft(D, n, p)
        for rep in range(3):
            y.fill_(float("nan"))
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            assert oracle.rel_l2(y.cpu().numpy(), want) <= 1e-12, rep
        g.close()


def test_batch_rejects_unsupported_members(torch):
    import paper_2203_11795_amd as fftu
    with pytest.raises(fftu.FftuError):
        fftu.BatchPlan([(1024, 16, 16)], [(2, 2, 2)], "complex64")     # local length 512
    with pytest.raises(fftu.FftuError):
        fftu.BatchPlan([(64, 64)], [(8, 8)], "complex64")              # 64 points per exchange
    with pytest.raises(fftu.FftuError):
        fftu.BatchPlan([(16, 16)], [(8, 2)], "complex64")              # 8^2 does not divide 16


def test_uneven_batch_of_256(torch):
    """The batch configuration: 256 3-D complex64 transforms, sides log-uniform in
    {16..256} per dimension, 2x2x2 grids, in one persistent launch. Eight members
    (the largest, the smallest and six more) are checked against the oracle."""
    import paper_2203_11795_amd as fftu
    shapes = synth.batch_shapes(256, 4)
    grids = [(2, 2, 2)] * 256
    sizes = [int(np.prod(s)) for s in shapes]
    say(f"batch of 256: {sum(sizes)} elements")
    xs = [torch.from_numpy(synth.uniform_complex(n, 4_000_000 + i, np.complex64)).cuda() for i, n in enumerate(sizes)]
    with fftu.BatchPlan(shapes, grids, "complex64", FORWARD) as bp:
        outs = bp(xs)
        torch.cuda.synchronize()
        assert bp.error_flag() == 0
    order = np.argsort(sizes)
    pick = sorted({int(order[0]), int(order[-1])} | set(np.random.default_rng(1).integers(0, 256, 6).tolist()))
    for i in pick:
        want = oracle.cyclic_dft(xs[i].cpu().numpy().astype(np.complex128), shapes[i], grids[i])
        assert oracle.rel_l2(outs[i].cpu().numpy(), want) <= 5e-6, (i, shapes[i])


def test_autotune_batch_keeps_results_and_caches(torch, tmp_path, monkeypatch):
    import paper_2203_11795_amd as fftu
    from paper_2203_11795_amd import autotune
    monkeypatch.setenv("FFTU_WISDOM", str(tmp_path / "wisdom.json"))
    shapes, grids = members(5, 11)
    xs_h = [synth.uniform_complex(int(np.prod(s)), 90 + i, np.complex64) for i, s in enumerate(shapes)]
    xs = to_dev(torch, xs_h, "complex64")
    outs = [torch.empty_like(x) for x in xs]
    res = autotune.tune_batch(shapes, grids, "complex64", FORWARD, xs, outs, reps=2)
    say(f"autotune: {res['knobs']} {res['ms']} ms over {len(res['candidates'])} candidates")
    assert not res["cached"] and len(res["candidates"]) >= 5
    assert all(fftu.get_tuning(k) == -1 for k in autotune.KNOB_NAMES)     # defaults restored
    again = autotune.tune_batch(shapes, grids, "complex64", FORWARD, xs, outs)
    assert again["cached"] and again["knobs"] == res["knobs"]
    with fftu.BatchPlan(shapes, grids, "complex64", FORWARD) as bp:
        base = [o.clone() for o in bp(xs)]
    autotune.apply(res["knobs"])
    try:
        with fftu.BatchPlan(shapes, grids, "complex64", FORWARD) as bp:
            tuned = bp(xs)
            torch.cuda.synchronize()
            assert bp.error_flag() == 0
    finally:
        autotune.apply({})
    for a, b in zip(base, tuned):
        assert torch.equal(a, b)


def test_batch_graph_keeps_its_buffers(torch):
    """A graph captured on (xs, outs) replays on them even after the plan ran
    eagerly on other buffers; those other outputs are left alone."""
    import paper_2203_11795_amd as fftu
    shapes, grids = members(7, 13)
    xs_h = [synth.uniform_complex(int(np.prod(s)), 110 + i, np.complex64) for i, s in enumerate(shapes)]
    xs = to_dev(torch, xs_h, "complex64")
    xs2 = [x * 0.5 for x in xs]
    outs = [torch.empty_like(x) for x in xs]
    outs2 = [torch.empty_like(x) for x in xs]
    with fftu.BatchPlan(shapes, grids, "complex64", FORWARD) as bp:
        want = [o.clone() for o in bp(xs)]
        g = fftu.Graph(bp, xs, outs)
        for rep in range(3):
            bp(xs2, outs2)                       # rebinds the plan to other buffers
            torch.cuda.synchronize()
            snap = [o.clone() for o in outs2]
            for o in outs:
                o.fill_(float("nan"))
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            for i, (o, w) in enumerate(zip(outs, want)):
                assert torch.equal(o, w), f"replay {rep}, member {i}"
            for i, (o, s) in enumerate(zip(outs2, snap)):
                assert torch.equal(o, s), f"replay {rep} wrote the eager outputs (member {i})"
            again = bp(xs2, outs2)               # and eager calls after a replay rebind again
            torch.cuda.synchronize()
            for o, s in zip(again, snap):
                assert torch.equal(o, s)
        g.close()


def test_batch_rebind_does_not_wait(torch):
    """New buffers are bound in stream order: the call returns while earlier work
    on the stream is still running."""
    import paper_2203_11795_amd as fftu
    shapes, grids = members(5, 17)
    xs = [torch.ones(int(np.prod(s)), dtype=torch.complex64, device="cuda") for s in shapes]
    outs = [torch.empty_like(x) for x in xs]
    big = torch.zeros(512 ** 3, dtype=torch.complex128, device="cuda")
    with fftu.BatchPlan(shapes, grids, "complex64", FORWARD) as bp, \
            fftu.Plan((512, 512, 512), (4, 4, 4), "complex128", FORWARD) as slow:
        bp(xs, outs)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        for _ in range(10):                      # about 20 ms of queued work
            slow(big, big)
        xs2 = [x.clone() for x in xs]            # enqueued after the transforms too
        outs2 = [torch.empty_like(x) for x in xs]
        bp(xs2, outs2)
        busy = not stream.query()
        torch.cuda.synchronize()
        assert busy, "fftu_execute_batch waited for the stream"
        for a, b in zip(outs, outs2):
            assert torch.equal(a, b)


def test_batch_rejects_bad_buffers(torch):
    """Overlaps that would race inside the persistent kernel, and misaligned or
    NULL pointers, are refused before anything is enqueued."""
    import paper_2203_11795_amd as fftu
    shapes, grids = [(16, 16, 16), (16, 32, 16)], [(2, 2, 2)] * 2
    sizes = [int(np.prod(s)) for s in shapes]
    pool = torch.zeros(4 * sum(sizes) + 16, dtype=torch.complex64, device="cuda")
    base = pool.data_ptr()
    es = 8
    a0, a1 = base, base + sizes[0] * es
    b0, b1 = a1 + sizes[1] * es, a1 + sizes[1] * es + sizes[0] * es
    with fftu.BatchPlan(shapes, grids, "complex64", FORWARD) as bp:
        bp.execute_ptrs([a0, a1], [b0, b1])             # disjoint: fine
        bp.execute_ptrs([a0, a1], [a0, a1])             # in place: fine
        torch.cuda.synchronize()
        bad = {
            "outputs overlap": ([a0, a1], [b0, b0 + 8 * es]),
            "output over another input": ([a0, a1], [a1, b1]),
            "partial in/out overlap": ([a0, a1], [a0 + es, b1]),
            "misaligned": ([a0 + 4, a1], [b0, b1]),
            "null": ([0, a1], [b0, b1]),
        }
        for name, (ins, outs) in bad.items():
            with pytest.raises(fftu.FftuError) as err:
                bp.execute_ptrs(ins, outs)
            assert err.value.status == 1, name
        with pytest.raises(ValueError):
            bp([pool[:sizes[0]], pool[sizes[0]:sizes[0] + sizes[1]]], [pool[:sizes[0]], pool[:7]])
        # a batch plan runs only through fftu_execute_batch
        lib = fftu.load_library()
        import ctypes
        h = bp._h
        for entry in ["fftu_execute", "fftu_stage_local_fft", "fftu_stage_twiddle", "fftu_stage_exchange",
                      "fftu_stage_remaining_fft"]:
            assert getattr(lib, entry)(h, ctypes.c_void_p(a0), ctypes.c_void_p(b0), None) == 1, entry
        assert lib.fftu_execute_ws(h, ctypes.c_void_p(a0), ctypes.c_void_p(b0), ctypes.c_void_p(b1), None) == 1
        torch.cuda.synchronize()
