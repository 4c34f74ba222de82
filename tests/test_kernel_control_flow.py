"""Control flow of the compiled gfx950 kernels (host-side, no GPU).

A barrier is executed per wave: if a loop that contains one exits lane by lane
(its latch clears finished lanes from the exec mask), the waves of a workgroup
can execute different numbers of barriers, and a workgroup whose lanes leave the
loop at different trips never finishes. Every loop of every kernel that holds an
s_barrier must therefore branch on wave-uniform values. This test compiles each
kernel source to AMDGPU assembly with the library's own flags and checks that,
using the loop annotations the compiler writes into the assembly.

The persistent batch kernel once failed exactly this way: its loop exit was
decided on a copy of the item index read from LDS into vector registers, and
the compiler let thread 0 leave the loop after each item while the other lanes
went straight back to the first barrier.
"""
import os
import re
import subprocess
from collections import defaultdict
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2203_11795_amd import build as fbuild

SOURCES = [s for s in fbuild.SOURCES if s.endswith(".hip")]


def compile_to_asm(src, tmpdir):
    out = os.path.join(tmpdir, os.path.splitext(src)[0] + ".s")
    flags = [f for f in fbuild.COMMON if f != "-fPIC"]
    cmd = [fbuild.HIPCC, *flags, "-x", "hip", "--cuda-device-only", "-S", os.path.join(fbuild.CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out


def loops_with_divergent_barrier(asm_text):
    """Loops (by header) whose own blocks hold an s_barrier and a per-lane exit."""
    blocks = []
    cur = None
    for line in asm_text.split("\n"):
        m = re.match(r"^(\.LBB\d+_\d+|; %bb\.\d+):\s*(;.*)?$", line)
        if m:
            hm = re.search(r"Header=(BB\d+_\d+)", m.group(2) or "")
            cur = {"name": m.group(1).lstrip(".").replace("; %bb.", "bb"), "loop": hm.group(1) if hm else None,
                   "lines": [], "header": "Loop Header" in (m.group(2) or "")}
            blocks.append(cur)
            continue
        if cur is not None:
            cur["lines"].append(line)
            if "Loop Header" in line:
                cur["header"] = True
    loops = defaultdict(list)
    for b in blocks:
        key = b["name"].replace("LBB", "BB") if b["header"] else b["loop"]
        if key:
            loops[key].append(b)
    bad = []
    for header, bs in loops.items():
        text = [l for b in bs for l in b["lines"]]
        has_barrier = any("s_barrier" in l for l in text)
        lane_exit = any(re.search(r"s_andn2_b64\s+exec, exec, s\[", l) for l in text)
        if has_barrier and lane_exit:
            bad.append(header)
    return bad, len(loops)


def test_detector_flags_a_lane_exit_loop_with_a_barrier():
    good = """
.LBB0_1:                                ; =>This Inner Loop Header: Depth=1
	s_barrier
	s_add_u32 s0, s0, 1
	s_cmp_lt_u32 s0, s1
	s_cbranch_scc1 .LBB0_1
"""
    bad = """
.LBB0_1:                                ; =>This Inner Loop Header: Depth=1
	s_barrier
	ds_read_b64 v[6:7], v1
	s_cbranch_vccnz .LBB0_2
.LBB0_2:                                ;   in Loop: Header=BB0_1 Depth=1
	s_or_b64 s[90:91], s[8:9], s[90:91]
	s_andn2_b64 exec, exec, s[90:91]
	s_cbranch_execnz .LBB0_1
"""
    assert loops_with_divergent_barrier(good) == ([], 1)
    assert loops_with_divergent_barrier(bad) == (["BB0_1"], 1)


@pytest.mark.slow
def test_no_kernel_loop_with_a_barrier_exits_per_lane(tmp_path):
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as pool:
        outs = list(pool.map(lambda s: compile_to_asm(s, str(tmp_path)), SOURCES))
    total = 0
    for src, path in zip(SOURCES, outs):
        bad, nloops = loops_with_divergent_barrier(open(path).read())
        total += nloops
        assert not bad, f"{src}: loops {bad} hold a barrier and exit lane by lane"
    assert total > 100   # the annotations were found
