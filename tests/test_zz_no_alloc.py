"""fftu_execute_noalloc (the entry point that allocates nothing) against
fftu_execute_ws, the entry point whose workspace it replaces, through the C ABI."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import FORWARD, INVERSE

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _noalloc(lib, plan, x, out, stream):
    return lib.fftu_execute_noalloc(plan.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                    ctypes.c_void_p(int(stream.cuda_stream)))


CASES = [  # (n, p, dtype, direction): the second of each pair is smaller than the first
    ((64, 64, 128), (4, 4, 4), "complex128", FORWARD),      # 8 MiB: k_lastx form
    ((32, 32, 32), (2, 2, 2), "complex128", FORWARD),
    ((256, 256, 64), (4, 4, 2), "complex64", INVERSE),      # 32 MiB
    ((60, 100), (2, 5), "complex64", INVERSE),              # mixed radix, far smaller
    ((2048, 2048), (32, 32), "complex128", FORWARD),        # exactly the maximum: 2^22 complex128 = 64 MiB
    ((64,), (8,), "complex128", INVERSE),
]


@pytest.mark.parametrize("pair", [0, 2, 4])
@pytest.mark.parametrize("external", [False, True])
def test_noalloc_matches_execute_ws_on_two_calls(torch, pair, external):
    import paper_2203_11795_amd as fftu
    lib = fftu.load_library()
    stream = torch.cuda.current_stream()
    for n, p, dtype, direction in CASES[pair:pair + 2]:
        say(f"noalloc: n={n} p={p} {dtype} dir={direction} external={external}")
        N = int(np.prod(n))
        npdt = np.complex128 if dtype == "complex128" else np.complex64
        D = synth.uniform_complex(N, 7 + N % 97, npdt)
        x = torch.from_numpy(D).cuda()
        with fftu.Plan(n, p, dtype, direction, external=external) as plan:
            ws = torch.empty(N, dtype=x.dtype, device="cuda")
            want = plan(x, workspace=ws)
            got = torch.full_like(x, float("nan"))
            assert _noalloc(lib, plan, x, got, stream) == 0
            inplace = x.clone()
            assert _noalloc(lib, plan, inplace, inplace, stream) == 0
            torch.cuda.synchronize()
            assert torch.equal(got, want), "differs from fftu_execute_ws"
            assert torch.equal(inplace, want), "in place differs"
        tol = 1e-12 if dtype == "complex128" else 5e-6
        ref = oracle.cyclic_dft(D.astype(np.complex128), n, p, direction)
        assert oracle.rel_l2(got.cpu().numpy(), ref) <= tol


def test_noalloc_refuses_what_does_not_fit_and_allocates_nothing(torch):
    import paper_2203_11795_amd as fftu
    lib = fftu.load_library()
    stream = torch.cuda.current_stream()
    assert fftu.NOALLOC_MAX_BYTES == 64 << 20
    n, p = (512, 512, 64), (4, 4, 2)                          # 2^24 complex64 = 128 MiB: too large
    with fftu.Plan(n, p, "complex64", FORWARD, external=True) as big:
        x = torch.zeros(big.N, dtype=torch.complex64, device="cuda")
        assert _noalloc(lib, big, x, x, stream) == 4          # FFTU_ERROR_OUT_OF_MEMORY
        assert lib.fftu_last_error() == 4
    n, p = (64, 64, 64), (2, 2, 2)
    D = synth.uniform_complex(64 ** 3, 3)
    x = torch.from_numpy(D).cuda()
    y = torch.empty_like(x)
    with fftu.Plan(n, p, "complex128", FORWARD, external=True) as plan:
        assert _noalloc(lib, plan, x, y, stream) == 0         # first call on the device: symbol lookup
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        for _ in range(5):
            assert _noalloc(lib, plan, x, y, stream) == 0
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        assert free1 == free0
        assert oracle.rel_l2(y.cpu().numpy(), oracle.cyclic_dft(D, n, p)) <= 1e-12
        # the scratch array must not overlap the caller's buffers: a NULL buffer is refused
        assert lib.fftu_execute_noalloc(plan.handle, None, ctypes.c_void_p(y.data_ptr()), None) == 1
