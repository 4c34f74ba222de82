"""The DCT-II / DST-II and their inverses on the GPU (fftu_plan_r2r) against the
oracle's transforms in the zig-zag cyclic distribution: the signal as the zig-zag
order of x in the real transform's packed layout, the coefficients cyclic."""
import sys

import numpy as np
import pytest

import oracle
from oracle import FORWARD, INVERSE
from oracle import r2r

pytestmark = pytest.mark.gpu

TOL = {"complex128": 1e-12, "complex64": 5e-6}
RDT = {"complex128": np.float64, "complex64": np.float32}


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


SHAPES = [
    ((8,), (2,)), ((12,), (1,)), ((2,), (1,)), ((2, 4), (1, 1)), ((16, 16), (2, 2)), ((8, 24), (2, 2)),
    ((4, 18, 8), (1, 3, 2)),               # mixed radix: the packed 4 x 18 x 4 over 1 x 3 x 2
    ((32, 64), (8, 4)),                    # packed 32 x 32 over 8 x 4: group-cyclic levels
    ((64, 64, 64), (2, 2, 2)),
    ((8, 16, 8, 32), (2, 2, 2, 2)),        # d = 4: groups of 16 mirror images
    # whole coefficient rows staged in LDS (n_d / 2 a multiple of 64, at least 1024 rows)
    ((2048, 128), (4, 2)), ((64, 64, 128), (2, 2, 2)), ((32, 16, 16, 128), (2, 2, 2, 2)),
    ((96, 40, 128), (2, 2, 2)),            # mixed radix below, rows staged in the last pass
]


def pre_rows(n):
    """Whether the inverse's first pass takes k_r2rpre's row form: n_d / 2 a multiple
    of 64, at least 1024 rows of representatives."""
    return len(n) >= 2 and (n[-1] // 2) % 64 == 0 and int(np.prod([v // 2 + 1 for v in n[:-1]])) >= 1024


def pre_merge(n, dtype):
    """Whether the inverse's first pass is k_r2rpre_merge (the spectrum and the real
    transform's merge in one pass): the row form, with 2^(d-1) (n_d / 2 + 1) spectrum
    values of a row within 32 KiB."""
    es = 16 if dtype == "complex128" else 8
    return pre_rows(n) and 2 ** (len(n) - 1) * (n[-1] // 2 + 1) * es <= 32768


def post_rows(n, p, dtype):
    """Whether the forward pass takes k_r2rpost_rows: n_d / 2 a multiple of 64, the
    2^(d-1) staged rows within 32 KiB, at least 1024 rows of representatives."""
    d = len(n)
    if d < 2 or (n[-1] // 2) % 64:
        return False
    es = 8 if dtype == "complex128" else 4
    rows = int(np.prod([v // 2 + 1 for v in n[:-1]]))
    return 2 ** (d - 1) * p[-1] * (n[-1] // p[-1] + 1) * es <= 32768 and rows >= 1024


@pytest.mark.parametrize("n,p", SHAPES)
@pytest.mark.parametrize("kind", ["dct", "dst"])
@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_forward_and_inverse_match_the_oracle(torch, n, p, kind, dtype):
    import paper_2203_11795_amd as fftu
    say(f"r2r n={n} p={p} {kind} {dtype}")
    X = np.random.default_rng(int(np.prod(n)) % 977).uniform(-1, 1, n)
    sig = r2r.signal_to_buffer(X, p).astype(RDT[dtype])
    want = r2r.r2r_cyclic(sig.astype(np.float64), n, p, kind, FORWARD)
    x = torch.from_numpy(sig).cuda()
    with fftu.R2RPlan(n, p, kind, dtype, FORWARD) as fwd, fftu.R2RPlan(n, p, kind, dtype, INVERSE) as inv:
        names = fwd.launch_names()
        post = "k_r2rpost_rows" if post_rows(n, p, dtype) else "k_r2rpost"
        assert names[-1] == f"fftu::{post}<{'double' if dtype == 'complex128' else 'float'}, {len(n)}>", names
        # the DST's signs: a pass of their own, or folded into the first line pass
        fused = any(k.startswith("fftu::k_line_sign<") for k in names)
        assert (names[0].startswith("fftu::k_r2rsign") or fused) == (kind == "dst"), names
        assert not (fused and names[0].startswith("fftu::k_r2rsign")), names
        t = "double" if dtype == "complex128" else "float"
        inames = inv.launch_names()
        if pre_merge(n, dtype):
            assert inames[0] == f"fftu::k_r2rpre_merge<{t}, {len(n)}>" and not any("rmerge" in k for k in inames)
        else:
            assert inames[0] == f"fftu::k_r2rpre<{t}, {len(n)}, {'true' if pre_rows(n) else 'false'}>"
        # the inverse DST's signs: a pass of their own, or in the last exchange's stores
        ifused = any(k.startswith(("fftu::k_exchange_sign<", "fftu::k_lastx_sign<")) for k in inames)
        assert (inames[-1].startswith("fftu::k_r2rsign") or ifused) == (kind == "dst"), inames
        assert not (ifused and inames[-1].startswith("fftu::k_r2rsign")), inames
        assert inv.info()["launches"] == len(inames)
        y = fwd(x)
        z = x.clone()
        fwd(z, z)                                        # in place
        torch.cuda.synchronize()
        got = y.cpu().numpy()
        assert np.array_equal(z.cpu().numpy(), got)
        assert np.array_equal(x.cpu().numpy(), sig)      # the input is left alone
        assert oracle.rel_l2(got, want) <= TOL[dtype]
        # inverse of the exact coefficients, and the round trip
        yc = torch.from_numpy(want.astype(RDT[dtype])).cuda()
        xb = inv(yc)
        rt = inv(y)
        torch.cuda.synchronize()
        assert oracle.rel_l2(xb.cpu().numpy(), r2r.r2r_cyclic(want, n, p, kind, INVERSE)) <= TOL[dtype]
        assert oracle.rel_l2(rt.cpu().numpy(), sig.astype(np.float64)) <= TOL[dtype]
        yi = yc.clone()
        inv(yi, yi)                                      # the inverse in place
        torch.cuda.synchronize()
        assert np.array_equal(yi.cpu().numpy(), xb.cpu().numpy())
        assert fwd.info()["launches"] == len(names)


def test_r2r_plan_checks(torch):
    import ctypes
    import paper_2203_11795_amd as fftu
    lib = fftu.load_library()
    n5 = (ctypes.c_int64 * 5)(2, 2, 2, 2, 2)
    assert not lib.fftu_plan_r2r(5, n5, (ctypes.c_int64 * 5)(1, 1, 1, 1, 1), 1, 0, -1)
    assert lib.fftu_last_error() == 3                    # d > 4
    with pytest.raises(fftu.FftuError) as e:
        fftu.R2RPlan((6, 5), (1, 1))
    assert e.value.status == 1                           # an odd side
    with pytest.raises(fftu.FftuError) as e:
        fftu.R2RPlan((24,), (8,))                        # 8 does not divide 12
    assert e.value.status == 2
    with fftu.R2RPlan((16, 16), (2, 2), "dst") as pl:
        x = torch.zeros(256, dtype=torch.float64, device="cuda")
        with pytest.raises(ValueError):
            pl(x.to(torch.float32))
        # the plain-buffer entry points refuse an r2r plan; partial overlap is refused
        assert lib.fftu_execute_ws(pl.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                   ctypes.c_void_p(x.data_ptr()), None) == 1
        assert lib.fftu_stage_local_fft(pl.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                        None) == 1
        assert lib.fftu_execute(pl.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr() + 8),
                                None) == 1
        assert fftu.load_library().fftu_plan_device_bytes(pl.handle) >= 128 * 16


def test_dct_512cube_full_size(torch):
    """512^3 FP64 DCT-II over 4^3 at full size: a sparse signal (40 nonzeros) gives
    2000 sampled coefficients against the definition summed over its nonzeros; a
    dense signal round-trips."""
    import paper_2203_11795_amd as fftu
    n, p = (512, 512, 512), (4, 4, 4)
    N = 512 ** 3
    rng = np.random.default_rng(81)
    js = np.unique(rng.integers(0, 512, size=(40, 3)), axis=0)
    vals = rng.uniform(-1, 1, len(js))
    X = np.zeros(n)
    X[tuple(js.T)] = vals
    sig = r2r.signal_to_buffer(X, p)
    del X
    x = torch.from_numpy(sig).cuda()
    with fftu.R2RPlan(n, p, "dct", "complex128", FORWARD) as fwd, \
            fftu.R2RPlan(n, p, "dct", "complex128", INVERSE) as inv:
        y = fwd(x)
        torch.cuda.synchronize()
        ks = rng.integers(0, 512, size=(2000, 3))
        rank = ((ks[:, 0] % 4) * 4 + ks[:, 1] % 4) * 4 + ks[:, 2] % 4
        pos = rank * (128 ** 3) + ((ks[:, 0] // 4) * 128 + ks[:, 1] // 4) * 128 + ks[:, 2] // 4
        got = y.cpu().numpy()[pos]
        w = np.ones((len(ks), len(js)))
        for l in range(3):
            e = (ks[:, l][:, None] * (2 * js[:, l][None, :] + 1)) % 2048     # the angle reduced exactly
            w *= 2 * np.cos(np.pi * e / 1024)
        want = w @ vals
        err = np.abs(got - want).max() / np.abs(want).max()
        say(f"512^3 DCT sparse signal: max rel error {err:.2e} over 2000 coefficients")
        assert err <= 1e-13
        xd = torch.empty(N, dtype=torch.float64, device="cuda")
        xd.uniform_(-1, 1)
        rt = inv(fwd(xd))
        torch.cuda.synchronize()
        e = (torch.linalg.vector_norm(rt - xd) / torch.linalg.vector_norm(xd)).item()
        say(f"512^3 DCT round trip {e:.2e}")
        assert e <= 1e-12


def test_dst_512cube_signs_in_first_pass(torch):
    """512^3 FP64 DST-II over 4^3 at full size, whose signal signs are applied by the
    complex transform's first line pass (forward) and its last kernel, k_lastx (inverse): 2000
    sampled coefficients of a sparse signal against the definition summed over its
    nonzeros, and the round trip."""
    import paper_2203_11795_amd as fftu
    n, p = (512, 512, 512), (4, 4, 4)
    N = 512 ** 3
    rng = np.random.default_rng(83)
    js = np.unique(rng.integers(0, 512, size=(40, 3)), axis=0)
    vals = rng.uniform(-1, 1, len(js))
    X = np.zeros(n)
    X[tuple(js.T)] = vals
    sig = r2r.signal_to_buffer(X, p)
    del X
    x = torch.from_numpy(sig).cuda()
    with fftu.R2RPlan(n, p, "dst", "complex128", FORWARD) as fwd, \
            fftu.R2RPlan(n, p, "dst", "complex128", INVERSE) as inv:
        names = fwd.launch_names()
        assert names[0].startswith("fftu::k_line_sign<double, ") and not any("r2rsign" in k for k in names), names
        inames = inv.launch_names()
        assert inames[-1].startswith("fftu::k_lastx_sign<double, 6, ") and not any("r2rsign" in k for k in inames), inames
        y = fwd(x)
        torch.cuda.synchronize()
        ks = rng.integers(0, 512, size=(2000, 3))
        rank = ((ks[:, 0] % 4) * 4 + ks[:, 1] % 4) * 4 + ks[:, 2] % 4
        pos = rank * (128 ** 3) + ((ks[:, 0] // 4) * 128 + ks[:, 1] // 4) * 128 + ks[:, 2] // 4
        got = y.cpu().numpy()[pos]
        w = np.ones((len(ks), len(js)))
        for l in range(3):
            e = ((ks[:, l][:, None] + 1) * (2 * js[:, l][None, :] + 1)) % 2048     # the angle reduced exactly
            w *= 2 * np.sin(np.pi * e / 1024)
        want = w @ vals
        err = np.abs(got - want).max() / np.abs(want).max()
        say(f"512^3 DST sparse signal: max rel error {err:.2e} over 2000 coefficients")
        assert err <= 1e-13
        xd = torch.empty(N, dtype=torch.float64, device="cuda")
        xd.uniform_(-1, 1)
        xin = xd.clone()
        rt = inv(fwd(xd))
        torch.cuda.synchronize()
        assert torch.equal(xd, xin)                      # the signs do not touch the input
        e = (torch.linalg.vector_norm(rt - xd) / torch.linalg.vector_norm(xd)).item()
        say(f"512^3 DST round trip {e:.2e}")
        assert e <= 1e-12


@pytest.mark.parametrize("kind", ["real", "dct", "dst"])
def test_graph_replays_match_eager(torch, kind):
    """A captured HIP graph of a real or DCT / DST transform, replayed three times with
    eager work and host synchronisation in between, each replay against the eager
    result bitwise (the buffers are the ones given at capture)."""
    import paper_2203_11795_amd as fftu
    n, p = (32, 64, 16), (2, 4, 2)
    N = int(np.prod(n))
    plan = fftu.RealPlan(n, p, "complex128", FORWARD) if kind == "real" else fftu.R2RPlan(n, p, kind, "complex128", FORWARD)
    with plan:
        x = torch.empty(N, dtype=torch.float64, device="cuda")
        x.uniform_(-1, 1)
        out = plan(x)
        torch.cuda.synchronize()
        want = out.clone()
        g = fftu.Graph(plan, x, out)
        try:
            for rep in range(3):
                out.zero_()
                scratch = plan(x.flip(0).contiguous())   # eager work of the same plan between replays
                torch.cuda.synchronize()
                g.launch()
                torch.cuda.synchronize()
                assert torch.equal(out, want), (kind, rep)
                del scratch
        finally:
            g.close()
