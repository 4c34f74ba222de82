"""Host-side checks of the C-ABI library: it loads, exports every entry point that
include/fftu.h declares, and validates plans (Algorithm 2.3's precondition
p_l^2 | n_l and this build's limits) without touching a device."""
import ctypes
import os
import re

import pytest

import paper_2203_11795_amd as fftu
from paper_2203_11795_amd import fftu as binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fftu.h")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fftu_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = fftu.load_library()
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(binding.EXPORTS) == names


def test_version_and_status_strings():
    lib = fftu.load_library()
    assert lib.fftu_version().startswith(b"fftu ")
    for code, name in binding.STATUS.items():
        assert lib.fftu_status_string(code).decode() == name
    assert lib.fftu_status_string(99) == b"FFTU_UNKNOWN_STATUS"


@pytest.mark.parametrize("n,p,expect", [
    ((512, 512, 512), (4, 4, 4), 0),
    ((64, 64, 64), (2, 2, 2), 0),
    ((64,) * 5, (2,) * 5, 0),
    ((8,), (2,), 0),
    ((1,), (1,), 0),
    ((16,), (4,), 0),            # p^2 = n: q = 1
    ((8,), (4,), 0),             # 16 does not divide 8: group-cyclic levels (8 over 4, then 4 over 2)
    ((32, 32), (2, 8), 0),       # 32 over 8, then 8 over 2
    ((8,), (8,), 2),             # one element per processor: no group-cyclic chain
    ((12,), (6,), 2),            # 12 over 6 (m = 2), then 6 over 3: 2 does not divide 3
    ((16,), (3,), 2),            # 3 does not divide 16
    ((12,), (2,), 0),            # mixed radix: 12 = 4 * 3
    ((60, 36), (2, 3), 0),
    ((44,), (2,), 3),            # p^2 | n holds, but 11 is not a radix of the mixed path
    ((3 * 2048,), (1,), 3),      # mixed-radix line longer than one LDS tile (complex128)
    ((12,), (3,), 2),
    ((64,) * 9, (2,) * 9, 3),    # d > 8
    ((0,), (1,), 1),
    ((8,), (0,), 1),
    ((1 << 24, 64), (1, 1), 3),  # local length above one LDS tile
])
def test_check_status(n, p, expect):
    assert fftu.check(n, p) == expect
    assert fftu.load_library().fftu_last_error() == expect


def test_check_rejects_bad_enums_and_null():
    lib = fftu.load_library()
    n = binding._arr([8])
    p = binding._arr([2])
    assert lib.fftu_check(1, n, p, 3, -1) == 1
    assert lib.fftu_check(1, n, p, 2, 0) == 1
    assert lib.fftu_check(0, n, p, 2, -1) == 1
    assert lib.fftu_check(1, None, p, 2, -1) == 1
    assert lib.fftu_execute(None, None, None, None) == 1
    assert lib.fftu_get_plan_info(None, None) == 1
    lib.fftu_destroy(None)


def test_p_max_examples():
    """eq. (2.13) and the examples after it: the largest grid with one all-to-all is
    planned with one superstep, and doubling any side of it needs more than one
    (the group-cyclic levels) or is refused."""
    for line in open(os.path.join(GOLDEN, "pmax_examples.txt")):
        if line.startswith("#") or not line.strip():
            continue
        shape_s, pmax_s = line.split()
        n = tuple(int(v) for v in shape_s.split("x"))
        grid = []
        for nl in n:
            e = nl.bit_length() - 1
            grid.append(1 << (e // 2))
        prod = 1
        for g in grid:
            prod *= g
        assert prod == int(pmax_s)
        st = fftu.check(n, grid)
        assert st in (0, 3)     # 3 only where a local length exceeds one tile (2^24 x 64)
        if st == 0:
            assert fftu.describe(n, grid)["supersteps"] == 1
        for l in range(len(n)):
            bigger = list(grid)
            bigger[l] *= 2
            st = fftu.check(n, bigger)
            assert st in (0, 3)     # 3: group-cyclic lines beyond the mixed-radix tile (2^24 x 64)
            if st == 0:
                assert fftu.describe(n, bigger)["supersteps"] == 2


@pytest.mark.parametrize("n,p,dtype,s0,fused,launches", [
    ((512, 512, 512), (4, 4, 4), "complex128", 2, 2, 3),    # dims 2, 1 as passes; dim 3 fused with the exchange
    ((64, 64, 64), (2, 2, 2), "complex128", 1, 2, 2),      # dims 1, 2 in one k_pair pass; dim 3 fused
    ((64,) * 5, (2,) * 5, "complex64", 2, 2, 3),            # k_pair (1, 2), k_pair (3, 4); dim 5 fused
    ((32,) * 4, (2,) * 4, "complex64", 2, 1, 3),            # k_pair (1, 2), k_group2 (3, 4), k_exchange
    ((1024,) * 3, (16, 16, 16), "complex128", 3, 0, 8),
    ((1,), (1,), "complex128", 0, 1, 1),
    ((60, 60), (2, 2), "complex128", 2, 1, 3),            # mixed radix: 2 passes, then k_mexchange
    ((49, 27, 8), (7, 3, 2), "complex64", 3, 1, 4),
    ((1000, 60), (10, 2), "complex128", 2, 0, 5),         # p = 10: twiddle + permutation, then 2 passes
    # the paper's sizes: 1024^3 takes the 1024-thread k_lastx; 2^24 x 64 (every q_l = 1) takes
    # k_long, k_ttranspose with the 8-point FFTs of Supersteps 0 and 2, k_long
    ((1024,) * 3, (4, 4, 4), "complex128", 2, 2, 3),
    ((1 << 24, 64), (4096, 8), "complex64", 1, 0, 3),
    ((64, 4096), (8, 64), "complex64", 1, 0, 4),            # every q_l = 1, innermost side 64: plain transpose
    ((64, 64, 64), (8, 8, 8), "complex128", 2, 0, 5),       # P = 512: k_ttranspose with the 8-point FFTs
    ((8192, 16), (2, 2), "complex64", 2, 1, 3),             # k_long for the lines of 4096
    ((16, 16, 16, 32, 64), (2,) * 5, "complex64", 2, 2, 3),  # two k_pair passes, then k_lastx
    # lines of 64 over a 4 x 4 x 4 split: k_lastx with 16 elements per thread (the packed
    # array of the 512^3 real transforms)
    ((512, 512, 256), (4, 4, 4), "complex128", 2, 2, 3),
])
def test_describe(n, p, dtype, s0, fused, launches):
    info = fftu.describe(n, p, dtype)
    N = 1
    for v in n:
        N *= v
    P = 1
    for v in p:
        P *= v
    assert info["N"] == N and info["P"] == P and info["M"] == N // P
    assert info["s0_kernels"] == s0 and info["exchange_fused"] == fused and info["launches"] == launches
    assert info["workspace_bytes"] == N * (16 if dtype == "complex128" else 8)
    assert info["supersteps"] == 1
    with pytest.raises(fftu.FftuError):
        fftu.describe((8,), (8,))


@pytest.mark.parametrize("n,p,supersteps,launches", [
    ((8,), (4,), 2, 4),                       # F_2, Put, F_2, the last Put with its F_2 (k_gplast)
    # 16^3 local blocks: a k_group2 pass of the two inner sides and a k_line pass, Put, the
    # same two passes, then the last Put with the 2 x 2 x 2 FFTs of length p_h = 2
    ((512, 512, 512), (32, 32, 32), 2, 6),
    ((16, 16), (8, 2), 3, 8),
    ((1024,), (64,), 2, 4),
    ((27, 8), (9, 4), 2, 8),                  # mixed radix: the phases on k_mline, no fused last Put
])
def test_describe_group_cyclic(n, p, supersteps, launches):
    info = fftu.describe(n, p, "complex128")
    assert info["supersteps"] == supersteps and info["exchange_fused"] == 0 and info["launches"] == launches


def test_info_struct_layout_matches_header():
    # int32 d, int64 N, P, M, 4 x int32, 2 x uint64, int32 supersteps (+ tail padding to 8)
    assert ctypes.sizeof(binding.PlanInfo) == 4 + 4 + 8 * 3 + 4 * 4 + 8 * 2 + 8
    assert binding.PlanInfo.supersteps.offset == 4 + 4 + 8 * 3 + 4 * 4 + 8 * 2


def test_tuning_knobs_roundtrip_and_ranges():
    names = ["line_strided_logw", "line_contig_logw", "line_pad", "max_lds_kb", "fuse_last", "pair"]
    try:
        for name in names:
            assert fftu.get_tuning(name) == -1
        fftu.set_tuning("line_strided_logw", 4)
        assert fftu.get_tuning("line_strided_logw") == 4
        for name, bad in [("line_strided_logw", 1), ("line_strided_logw", 7), ("line_pad", 5), ("max_lds_kb", 8),
                          ("max_lds_kb", 161), ("line_contig_logw", 9), ("fuse_last", 2), ("pair", 2), ("pair", -2)]:
            with pytest.raises(fftu.FftuError):
                fftu.set_tuning(name, bad)
        lib = fftu.load_library()
        assert lib.fftu_set_tuning(99, 1) == 1
        assert lib.fftu_get_tuning(-1) == -1 and lib.fftu_last_error() == 1
        # planning is unchanged in what it computes; only tiling moves
        base = fftu.describe((512, 512, 512), (4, 4, 4))
        fftu.set_tuning("line_strided_logw", 3)
        assert fftu.describe((512, 512, 512), (4, 4, 4)) == base
    finally:
        for name in names:
            fftu.set_tuning(name, -1)


def test_benchmark_ideal_pass_counts():
    """The roofline's ideal pass count (local dimensions grouped greedily under
    the LDS budget, plus one exchange pass) for the benchmarked shapes."""
    import bench
    assert bench.ideal_passes((512, 512, 512), (4, 4, 4), 16) == 4
    assert bench.ideal_passes((64,) * 5, (2,) * 5, 8) == 4
    assert bench.ideal_passes((64, 64, 64), (2, 2, 2), 16) == 3
    assert bench.ideal_passes((16, 16, 16), (2, 2, 2), 8) == 1          # fits one workgroup's LDS
    assert bench.ideal_passes((256, 256, 256), (2, 2, 2), 8) == 3
