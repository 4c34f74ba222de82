"""Host logic of the serving layer (no GPU): the HBM arena's first-fit allocator
and the request list built from the seeded trace."""
import math
import random

import numpy as np

import synth
from paper_2203_11795_amd import serving


def test_arena_first_fit_coalesces_and_never_overlaps():
    a = serving.Arena(1 << 20)
    rng = random.Random(3)
    live = []
    for step in range(3000):
        if live and (rng.random() < 0.45 or a.used > (1 << 20) - 65536):
            blk = live.pop(rng.randrange(len(live)))
            a.release(*blk)
        else:
            got = a.alloc(rng.randint(1, 40000))
            if got is not None:
                live.append(got)
        spans = sorted(live)
        for (o1, s1), (o2, _) in zip(spans, spans[1:]):
            assert o1 + s1 <= o2                            # no overlap
        assert all(o % serving.ALIGN == 0 for o, _ in spans)
        assert a.used == sum(s for _, s in live)
        assert a.used + sum(s for _, s in a.free) == a.capacity
        frees = a.free
        assert all(f1[0] + f1[1] < f2[0] for f1, f2 in zip(frees, frees[1:]))   # coalesced
    for blk in live:
        a.release(*blk)
    assert a.free == [(0, 1 << 20)] and a.used == 0


def test_arena_refuses_what_does_not_fit():
    a = serving.Arena(4096)
    x = a.alloc(3000)
    assert x is not None and a.alloc(2000) is None
    a.release(*x)
    assert a.alloc(4096) == (0, 4096)


def test_requests_from_trace():
    trace = synth.serving_trace(seed=5, rate=2000.0, duration=0.5)
    reqs = serving.requests_from_trace(trace)
    assert len(reqs) == len(trace) and 700 < len(reqs) < 1300
    assert all(r.arrival < 0.5 for r in reqs)
    assert sorted(r.arrival for r in reqs) == [r.arrival for r in reqs]
    for r, t in zip(reqs, trace):
        assert r.N == math.prod(t["shape"]) <= 1 << 26
        assert r.dtype == ("complex128" if np.dtype(t["dtype"]) == np.complex128 else "complex64")
        assert all(n % 4 == 0 for n in r.shape) and r.grid == (2,) * len(r.shape)
    assert {r.dtype for r in reqs} == {"complex64", "complex128"} and {r.direction for r in reqs} == {-1, 1}
    head = serving.requests_from_trace(trace, limit_seconds=0.1)
    assert head == reqs[:len(head)] and all(r.arrival < 0.1 for r in head)


def test_size_classes_and_lane_queues():
    import collections
    small_req = serving.Request(0, 0.0, (64, 64), "complex64", -1)           # 32 KiB
    big_req = serving.Request(1, 0.0, (1024, 1024, 64), "complex128", 1)    # 1 GiB
    assert serving.request_class(small_req, 2, 64 << 20) == "small"
    assert serving.request_class(big_req, 2, 64 << 20) == "large"
    assert serving.request_class(big_req, 0, 64 << 20) == "small"         # FIFO: one class
    large, small = collections.deque([big_req]), collections.deque([small_req])
    assert serving.next_queue(0, 2, large, small) is large                 # a large lane prefers large
    assert serving.next_queue(1, 2, large, small) is large
    assert serving.next_queue(2, 2, large, small) is small                 # small lanes never take large
    assert serving.next_queue(2, 2, large, collections.deque()) is None
    assert serving.next_queue(0, 2, collections.deque(), small) is small   # an idle large lane takes small
    assert serving.next_queue(0, 0, large, small) is small                 # FIFO: no lanes


def test_requests_larger_than_the_arena_are_refused_not_queued():
    r = serving.Request(0, 0.0, (64, 64), "complex128", -1)      # 64 KiB per block
    assert serving.fits_arena(r, 2 * 65536)
    assert not serving.fits_arena(r, 2 * 65536 - 1)
    odd = serving.Request(1, 0.0, (3, 5), "complex64", -1)        # 120 B, rounded up to one 256-byte block
    assert serving.fits_arena(odd, 512) and not serving.fits_arena(odd, 511)
