"""Benchmark of the cyclic-to-cyclic multidimensional FFT on one MI355X.

Default workload: the 512 x 512 x 512 complex128 forward DFT on a 4 x 4 x 4
virtual processor grid (cyclic in, cyclic out), iid uniform[-1, 1) input from
seed 2. One step is one full transform (Superstep 0 local FFTs, twiddle, the
one permutation, Superstep 2 length-p FFTs) with the input already in HBM.

Prints one JSON line: GFLOP/s under the 5 N log2 N convention, the roofline of
the dominant kernel (HIP events on the execution stream, algorithmic bytes =
one read and one write of the N-element array per launch), the oracle timed on
the host cores, and the error of the timed output against the oracle.

With the default workload the line also carries a "batch" object: 256 uneven
3-D complex64 transforms (sides 2^4..2^8 per dimension, 2x2x2 grids) in one
persistent launch, its HIP-graph replay, and the same 256 transforms as plain
per-transform executions, after a measured tuning of the tiling knobs; and a
"serving" object: p50/p99 latency of the 30 s real-time request stream served
with four streams, with small waiting requests coalesced into persistent batch
launches, and with a plain one-at-a-time FIFO, and the FP32 error of every
complex64 result.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 512cube|64cube|64pow5]
                    [--no-batch] [--retune] [--no-serving] [--serving-seconds S]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GFLOP/s (5N log2N) + %HBM roofline, 512^3 c2c FP64; served p50/p99 latency"

WORKLOADS = {
    "512cube": dict(n=(512, 512, 512), p=(4, 4, 4), dtype="complex128", dist="uniform", seed=2,
                    name="512x512x512 complex128 forward DFT, 4x4x4 cyclic grid"),
    "64cube": dict(n=(64, 64, 64), p=(2, 2, 2), dtype="complex128", dist="uniform", seed=1,
                   name="64x64x64 complex128 forward DFT, 2x2x2 cyclic grid"),
    "64pow5": dict(n=(64,) * 5, p=(2,) * 5, dtype="complex64", dist="normal", seed=3,
                   name="64^5 complex64 forward DFT, 2x2x2x2x2 cyclic grid (FP32 butterflies, FP64-generated twiddles)"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_digest():
    """Digest of every source the kernels are built from (counter summaries record it)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2203_11795_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp", ".cpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode())
                h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was
    taken from the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"pmc_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != source_digest():
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None
    return float(k["hbm_bytes_per_launch"])


def ideal_passes(n, p, esize, lds=160 * 1024):
    """Fewest HBM passes a transform of this shape needs: local dimensions grouped
    greedily from the innermost outwards, the innermost group holding at most
    `lds` bytes and every strided group at most lds/8 (so that at least 8
    contiguous columns can be staged), plus one pass for the exchange (twiddle,
    permutation and the length-p transforms fused). A transform whose N elements
    fit in `lds` needs one pass."""
    m = [a // b for a, b in zip(n, p)]
    if math.prod(n) * esize <= lds:
        return 1
    groups, l = 0, len(m) - 1
    while l >= 0:
        cap = lds if groups == 0 else lds // 8
        prod = m[l]
        l -= 1
        while l >= 0 and prod * m[l] * esize <= cap:
            prod *= m[l]
            l -= 1
        groups += 1
    return groups + 1


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_single_thread(np, oracle, synth, X, flops):
    """The oracle on one host thread: the headline array once, and the 64^3 small
    case (median of 3) on one thread and on all. (The oracle's thread count is
    process-wide state: the last call restores the full count.)"""
    nt_all = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.fft_axes(X, range(X.ndim), oracle.FORWARD, nthreads=1)
    t1 = time.perf_counter() - t0
    Xs = oracle.from_cyclic(synth.uniform_complex(64 ** 3, 1), (64, 64, 64), (2, 2, 2))
    fs = 5.0 * 64 ** 3 * math.log2(64 ** 3)
    small = {}
    for label, nt in (("1_thread", 1), ("all_threads", nt_all)):
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            oracle.fft_axes(Xs, range(3), oracle.FORWARD, nthreads=nt)
            ts.append(time.perf_counter() - t0)
        small[label] = {"median_s": round(float(np.median(ts)), 5), "GFLOPs": round(fs / float(np.median(ts)) / 1e9, 3),
                        "threads": nt}
    return {"single_thread": {"value": round(flops / t1 / 1e9, 3), "unit": "GFLOP/s", "cores": 1,
                              "sample": f"the same transform on one thread: {t1:.2f} s"},
            "small_64cube": small}


def run_batch(args, torch, np, fftu, synth, with_oracle):
    """The batch workload: 256 uneven 3-D complex64 transforms on 2x2x2 grids."""
    from paper_2203_11795_amd import autotune
    count, seed = 256, 4
    shapes = synth.batch_shapes(count, seed)
    grids = [(2, 2, 2)] * count
    sizes = [math.prod(s) for s in shapes]
    dev = torch.device("cuda:0")
    log(f"[bench] batch: {count} transforms, {sum(sizes)} elements; generating input")
    xs = [torch.from_numpy(synth.uniform_complex(n, 4_000_000 + i, np.complex64)).to(dev) for i, n in enumerate(sizes)]
    outs = [torch.empty_like(x) for x in xs]
    flops = sum(5.0 * n * math.log2(n) for n in sizes)
    esize = 8

    tune = autotune.tune_batch(shapes, grids, "complex64", fftu.FORWARD, xs, outs, reps=3, use_cache=not args.retune)
    log(f"[bench] batch knobs {tune['knobs']} (cached={tune['cached']})")
    autotune.apply(tune["knobs"])
    try:
        bp = fftu.BatchPlan(shapes, grids, "complex64", fftu.FORWARD)
    finally:
        autotune.apply({})
    stream = torch.cuda.current_stream(dev)
    steps = max(3, args.steps // 2)

    def timed(run, k, begin=None):
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        if begin:
            begin()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(k):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    ms_persistent = timed(lambda: bp(xs, outs, stream=stream), steps, begin=lambda: bp.timing_begin(steps))
    per_launch, _ = bp.timing_end()          # [reset kernel, persistent kernel]
    assert bp.error_flag() == 0, "a dependency wait of the persistent kernel gave up"
    g = fftu.Graph(bp, xs, outs)
    ms_graph = timed(lambda: g.launch(stream), steps)
    g.close()
    log(f"[bench] batch persistent {ms_persistent:.3f} ms, graph {ms_graph:.3f} ms")

    plans = {}
    for s in shapes:
        if s not in plans:
            plans[s] = fftu.Plan(s, (2, 2, 2), "complex64", fftu.FORWARD)
    outs_plain = [torch.empty_like(x) for x in xs]

    def plain():
        for x, o, s in zip(xs, outs_plain, shapes):
            plans[s](x, o, stream=stream)
    ms_plain = timed(plain, steps)
    log(f"[bench] batch as {count} plain executions {ms_plain:.3f} ms")
    # different pass structures (the plain plans fuse the two inner dimensions), so not bitwise
    diff = max(float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)) for a, b in zip(outs, outs_plain))

    # passes each member runs in the batch: its Superstep-0 passes plus the exchange. The
    # batch groups the two inner dimensions under the single-plan rule but has neither
    # k_pair passes nor the fused innermost dimension, so those are off while counting.
    saved = {k: fftu.get_tuning(k) for k in ("fuse_last", "pair")}
    try:
        for k in saved:
            fftu.set_tuning(k, 0)
        exec_passes = [fftu.describe(s, (2, 2, 2), "complex64")["s0_kernels"] + 1 for s in shapes]
    finally:
        for k, v in saved.items():
            fftu.set_tuning(k, v)
    bytes_exec = sum(2.0 * esize * n * k for n, k in zip(sizes, exec_passes))
    bytes_ideal = sum(2.0 * esize * n * ideal_passes(s, (2, 2, 2), esize) for n, s in zip(sizes, shapes))
    k_ms = per_launch[1] if len(per_launch) > 1 else ms_persistent
    traffic = measured_traffic("512cube", "fftu::k_batch<float>")
    res = {
        "workload": f"{count} uneven 3-D complex64 forward DFTs, sides 2^4..2^8 per dimension (shapes seed {seed}), "
                    "2x2x2 cyclic grids, one persistent launch",
        "elements": sum(sizes), "gflop": round(flops / 1e9, 3),
        "ms_persistent": round(ms_persistent, 4), "ms_graph": round(ms_graph, 4), "ms_plain": round(ms_plain, 4),
        "GFLOPs_persistent": round(flops / (ms_persistent * 1e-3) / 1e9, 1),
        "GFLOPs_graph": round(flops / (ms_graph * 1e-3) / 1e9, 1),
        "GFLOPs_plain": round(flops / (ms_plain * 1e-3) / 1e9, 1),
        "speedup_vs_plain": round(ms_plain / ms_graph, 3),
        "roofline": {"bound": "hbm", "kernel": "fftu::k_batch<float>", "avg_launch_ms": round(k_ms, 4),
                     "bytes_executed_passes": bytes_exec, "bytes_ideal_passes": bytes_ideal,
                     "achieved": round(bytes_exec / (k_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(bytes_exec / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "frac_vs_ideal_passes": round(bytes_ideal / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": traffic},
        "tuning": {"knobs": tune["knobs"], "cached": tune["cached"], "candidates": len(tune.get("candidates", []))},
        "rel_l2_persistent_vs_plain_max": diff,
    }
    if with_oracle:
        import oracle
        order = np.argsort(sizes)
        pick = sorted({int(order[0]), int(order[-1]), int(order[count // 2])})
        errs = []
        for i in pick:
            want = oracle.cyclic_dft(xs[i].cpu().numpy().astype(np.complex128), shapes[i], grids[i])
            errs.append(oracle.rel_l2(outs[i].cpu().numpy(), want))
        res["rel_l2_vs_oracle_max"] = max(errs)
        res["checked_members"] = pick
    for pl in plans.values():
        pl.close()
    bp.close()
    return res


def run_convolution(args, torch, np, fftu, synth, info):
    """Circular convolution at the headline shape (512^3 complex128, 4x4x4 grid):
    forward transform with the product by the filter spectrum fused into its
    exchange, then the inverse transform; against the same three steps unfused
    (forward, a pointwise pass, inverse)."""
    n, p = (512, 512, 512), (4, 4, 4)
    N = math.prod(n)
    esize = 16
    dev = torch.device("cuda:0")
    log("[bench] convolution: generating input and filter")
    x = torch.from_numpy(synth.uniform_complex(N, 41, np.complex128)).to(dev)
    hh = torch.from_numpy(synth.uniform_complex(N, 42, np.complex128)).to(dev)
    conv = fftu.ConvolutionPlan(n, p, "complex128")
    hhat = conv(hh)
    del hh
    y = torch.empty_like(x)
    inv = fftu.Plan(n, p, "complex128", fftu.INVERSE)
    stream = torch.cuda.current_stream(dev)
    steps = max(3, args.steps // 2)

    def timed(run):
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms_fused = timed(lambda: conv.convolve(x, hhat, out=y, stream=stream))
    fused_out = y.clone()

    def unfused():
        conv(x, y, stream=stream)
        fftu.pointwise_mul(y, hhat, out=y, stream=stream)
        inv(y, y, stream=stream)
    ms_unfused = timed(unfused)
    diff = float(torch.linalg.vector_norm(fused_out - y) / torch.linalg.vector_norm(y))
    passes = 2 * info["launches"]
    bytes_fused = passes * 2.0 * N * esize + N * esize
    flops = 2 * 5.0 * N * math.log2(N) + 6.0 * N
    conv.close()
    inv.close()
    log(f"[bench] convolution fused {ms_fused:.3f} ms, unfused {ms_unfused:.3f} ms")
    return {"workload": "circular convolution of 512x512x512 complex128 arrays in the 4x4x4 cyclic layout: "
                        "forward transform x pointwise filter spectrum, inverse transform",
            "ms_fused": round(ms_fused, 4), "ms_unfused": round(ms_unfused, 4),
            "speedup_fused": round(ms_unfused / ms_fused, 3),
            "GFLOPs_fused": round(flops / (ms_fused * 1e-3) / 1e9, 1),
            "roofline": {"bound": "hbm", "algorithmic_bytes": bytes_fused,
                         "achieved": round(bytes_fused / (ms_fused * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(bytes_fused / (ms_fused * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
            "rel_l2_fused_vs_unfused": diff}


def run_mixed(args, torch, np, fftu, synth, with_oracle):
    """The mixed-radix path at full size: 480^3 complex128 (480 = 2^5 3 5) on a 4^3
    grid (m = 120, q = 30), forward; per-kernel times from HIP events."""
    n, p = (480, 480, 480), (4, 4, 4)
    N = math.prod(n)
    esize = 16
    dev = torch.device("cuda:0")
    log("[bench] mixed radix 480^3: generating input")
    D = synth.uniform_complex(N, 6, np.complex128)
    x = torch.from_numpy(D).to(dev)
    out = torch.empty_like(x)
    plan = fftu.Plan(n, p, "complex128", fftu.FORWARD)
    info = plan.info()
    stream = torch.cuda.current_stream(dev)
    steps = max(3, args.steps // 2)
    for _ in range(args.warmup):
        plan(x, out, stream=stream)
    torch.cuda.synchronize()
    plan.timing_begin(steps)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        plan(x, out, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    per_launch, _ = plan.timing_end()
    names = plan.launch_names()
    alg = 2.0 * N * esize
    flops = 5.0 * N * math.log2(N)
    res = {"workload": "480x480x480 complex128 forward DFT (480 = 2^5 3 5), 4x4x4 cyclic grid, mixed-radix path",
           "ms_per_transform": round(ms, 4), "GFLOPs": round(flops / (ms * 1e-3) / 1e9, 1),
           "launches": info["launches"],
           "roofline": {"bound": "hbm", "algorithmic_bytes": info["launches"] * alg,
                        "achieved": round(info["launches"] * alg / (ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(info["launches"] * alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
           "kernels": [{"kernel": k, "avg_ms": round(t, 4), "GBps_alg": round(alg / (t * 1e-3) / 1e9, 1)}
                       for k, t in zip(names, per_launch)]}
    if with_oracle:
        import oracle
        X = oracle.from_cyclic(D, n, p)
        ks = [(0, 0, 0), (1, 2, 3), (479, 240, 17), (100, 333, 451)]
        flat = [int(np.ravel_multi_index(k, n)) for k in ks]
        want = oracle.dft_points(X, flat)
        got = oracle.from_cyclic(out.cpu().numpy(), n, p).reshape(-1)[flat]
        res["sampled_max_rel_error_vs_oracle"] = float(np.abs(got - want).max() / np.abs(want).max())
    plan.close()
    log(f"[bench] mixed 480^3: {ms:.3f} ms, {res['GFLOPs']} GFLOP/s")
    return res


def run_group_cyclic(args, torch, np, fftu, synth, with_oracle):
    """A grid beyond p_max = sqrt(N): 512^3 complex128 over 32^3 virtual processors
    (P = 32768 > 11585), where p_l^2 does not divide n_l, so the transform takes two
    communication supersteps through the group-cyclic distribution; per-kernel
    times from HIP events, beside the one-superstep 4^3 plan of the same array."""
    n, p = (512, 512, 512), (32, 32, 32)
    N = math.prod(n)
    esize = 16
    dev = torch.device("cuda:0")
    log("[bench] group-cyclic 512^3 over 32^3: generating input")
    D = synth.uniform_complex(N, 8, np.complex128)
    x = torch.from_numpy(D).to(dev)
    out = torch.empty_like(x)
    plan = fftu.Plan(n, p, "complex128", fftu.FORWARD)
    info = plan.info()
    stream = torch.cuda.current_stream(dev)
    steps = max(3, args.steps // 2)
    for _ in range(args.warmup):
        plan(x, out, stream=stream)
    torch.cuda.synchronize()
    plan.timing_begin(steps)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        plan(x, out, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    per_launch, _ = plan.timing_end()
    names = plan.launch_names()
    alg = 2.0 * N * esize
    flops = 5.0 * N * math.log2(N)
    per_sym = {}
    for k, t in zip(names, per_launch):
        tot, cnt = per_sym.get(k, (0.0, 0))
        per_sym[k] = (tot + t, cnt + 1)
    dom = max(per_sym, key=lambda k: per_sym[k][0])
    dom_ms = per_sym[dom][0] / per_sym[dom][1]
    res = {"workload": "512x512x512 complex128 forward DFT, 32x32x32 virtual grid (P = 32768 > sqrt(N)): "
                       "group-cyclic levels, two communication supersteps",
           "ms_per_transform": round(ms, 4), "GFLOPs": round(flops / (ms * 1e-3) / 1e9, 1),
           "supersteps": info["supersteps"], "launches": info["launches"],
           "roofline": {"bound": "hbm", "kernel": dom, "avg_launch_ms": round(dom_ms, 4),
                        "algorithmic_bytes_per_launch": alg,
                        "achieved": round(alg / (dom_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(alg / (dom_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                        "traffic": measured_traffic("512cube_gc", dom)},
           "hbm_roofline_frac_transform": round(info["launches"] * alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "kernels": [{"kernel": k, "avg_ms": round(t, 4), "GBps_alg": round(alg / (t * 1e-3) / 1e9, 1)}
                       for k, t in zip(names, per_launch)]}
    if with_oracle:
        import oracle
        X = oracle.from_cyclic(D, n, p)
        ks = [(0, 0, 0), (1, 2, 3), (511, 256, 17), (100, 333, 451)]
        flat = [int(np.ravel_multi_index(k, n)) for k in ks]
        want = oracle.dft_points(X, flat)
        got = oracle.from_cyclic(out.cpu().numpy(), n, p).reshape(-1)[flat]
        res["sampled_max_rel_error_vs_oracle"] = float(np.abs(got - want).max() / np.abs(want).max())
    plan.close()
    log(f"[bench] group-cyclic 512^3 over 32^3: {ms:.3f} ms, {res['GFLOPs']} GFLOP/s")
    return res


def cyclic_positions(np, idx, n, p):
    """Buffer positions of natural multi-indices idx[:, l] in the cyclic layout
    (processor rank row-major over s = j mod p, then the local index j div p)."""
    idx = np.asarray(idx, dtype=np.int64)
    rank = np.zeros(len(idx), dtype=np.int64)
    lin = np.zeros(len(idx), dtype=np.int64)
    for l, (nl, pl) in enumerate(zip(n, p)):
        rank = rank * pl + idx[:, l] % pl
        lin = lin * (nl // pl) + idx[:, l] // pl
    return rank * (math.prod(n) // math.prod(p)) + lin


def sparse_forward_check(np, torch, plan, n, p, tdt, seed, nonzeros=40, samples=500):
    """Forward transform of a sparse input: each output is a sum of `nonzeros` terms
    of eq. (1.2), evaluated in FP64 with exact integer phases per dimension, at
    `samples` random outputs. Returns the max error relative to the largest output."""
    rng = np.random.default_rng(seed)
    N = math.prod(n)
    js = np.unique(np.stack([rng.integers(0, nl, nonzeros) for nl in n], axis=1), axis=0)
    vals = rng.uniform(-1, 1, len(js)) + 1j * rng.uniform(-1, 1, len(js))
    x = torch.zeros(N, dtype=tdt, device="cuda:0")
    x[torch.from_numpy(cyclic_positions(np, js, n, p)).cuda()] = torch.from_numpy(vals).to(tdt).cuda()
    vals = x[torch.from_numpy(cyclic_positions(np, js, n, p)).cuda()].cpu().numpy().astype(np.complex128)
    y = plan(x)
    torch.cuda.synchronize()
    ks = np.stack([rng.integers(0, nl, samples) for nl in n], axis=1)
    got = y[torch.from_numpy(cyclic_positions(np, ks, n, p)).cuda()].cpu().numpy().astype(np.complex128)
    turns = np.zeros((samples, len(js)))
    for l, nl in enumerate(n):
        turns += ((ks[:, l:l + 1] * js[None, :, l]) % nl) / float(nl)
    want = (np.exp(-2j * np.pi * turns) * vals[None, :]).sum(axis=1)
    del x, y
    return float(np.abs(got - want).max() / np.abs(want).max())


def run_real(args, torch, np, fftu, synth, with_oracle):
    """The real-input transform at the headline shape: a real 512^3 FP64 array on
    the 4x4x4 grid (its packed 512 x 512 x 256 complex view), forward to the half
    spectrum and the Nyquist plane; per-kernel times from HIP events, beside the
    complex transform of the same shape."""
    n, p = (512, 512, 512), (4, 4, 4)
    N = math.prod(n)
    dev = torch.device("cuda:0")
    log("[bench] real 512^3: generating input")
    X = np.random.default_rng(9).uniform(-1.0, 1.0, N)            # used directly as the real-side buffer
    x = torch.from_numpy(X).to(dev)
    plan = fftu.RealPlan(n, p, "complex128", fftu.FORWARD)
    out = torch.empty(plan.complex_elems, dtype=torch.complex128, device=dev)
    stream = torch.cuda.current_stream(dev)
    steps = max(3, args.steps // 2)
    for _ in range(args.warmup):
        plan(x, out, stream=stream)
    torch.cuda.synchronize()
    plan.timing_begin(steps)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        plan(x, out, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    per_launch, _ = plan.timing_end()
    names = plan.launch_names()
    # algorithmic bytes: read N reals once and write the N/2 + N/n_d complex outputs once
    alg = N * 8 + plan.complex_elems * 16
    half_pass = 2.0 * (N // 2) * 16                     # a pass over the packed array
    res = {"workload": "512x512x512 real FP64 forward DFT (half spectrum and Nyquist plane), 4x4x4 cyclic grid "
                       "of its packed 512x512x256 complex view",
           "ms_per_transform": round(ms, 4),
           "GFLOPs_real_convention": round(2.5 * N * math.log2(N) / (ms * 1e-3) / 1e9, 1),
           "launches": len(names),
           "roofline": {"bound": "hbm", "algorithmic_bytes_one_pass": alg,
                        "bytes_executed_passes": half_pass * len(names),
                        "achieved": round(half_pass * len(names) / (ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(half_pass * len(names) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
           "kernels": [{"kernel": k, "avg_ms": round(t, 4), "GBps_alg": round(half_pass / (t * 1e-3) / 1e9, 1)}
                       for k, t in zip(names, per_launch)]}
    if with_oracle:
        import oracle
        from oracle import real
        got = out.cpu().numpy()
        want = real.rfft_cyclic(X, n, p)
        res["rel_l2_vs_oracle"] = oracle.rel_l2(got, want)
    plan.close()
    log(f"[bench] real 512^3: {ms:.3f} ms")
    return res


def run_r2r(args, torch, np, fftu, with_oracle):
    """The DCT-II and DST-II at the headline shape: a real 512^3 FP64 signal in the
    zig-zag cyclic layout over 4x4x4, forward to the coefficients (cyclic) and back;
    per-kernel times from HIP events. Checked on 1000 sampled coefficients of a sparse signal
    against the definitions summed over its nonzeros, and by the dense round trip."""
    n, p = (512, 512, 512), (4, 4, 4)
    N = math.prod(n)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    steps = max(3, args.steps // 2)
    out = {}
    for kind in ("dct", "dst"):
        log(f"[bench] {kind} 512^3")
        fwd = fftu.R2RPlan(n, p, kind, "complex128", fftu.FORWARD)
        x = torch.empty(N, dtype=torch.float64, device=dev)
        x.uniform_(-1.0, 1.0)
        y = torch.empty_like(x)
        for _ in range(args.warmup):
            fwd(x, y, stream=stream)
        torch.cuda.synchronize()
        fwd.timing_begin(steps)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fwd(x, y, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        per_launch, _ = fwd.timing_end()
        names = fwd.launch_names()
        # a pass over the signal's packed array (N/2 complex128 in and out)
        half_pass = 2.0 * (N // 2) * 16
        res = {"workload": f"512x512x512 real FP64 {kind.upper()}-II, signal in the zig-zag cyclic layout over 4x4x4, "
                           "coefficients cyclic",
               "ms_per_transform": round(ms, 4), "launches": len(names),
               "roofline": {"bound": "hbm", "bytes_executed_passes": half_pass * len(names),
                            "achieved": round(half_pass * len(names) / (ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                            "unit": "GB/s",
                            "frac": round(half_pass * len(names) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
               "kernels": [{"kernel": k, "avg_ms": round(t, 4), "GBps_alg": round(half_pass / (t * 1e-3) / 1e9, 1)}
                           for k, t in zip(names, per_launch)]}
        inv = fftu.R2RPlan(n, p, kind, "complex128", fftu.INVERSE)
        rt = inv(y)
        torch.cuda.synchronize()
        res["rel_l2_roundtrip"] = (torch.linalg.vector_norm(rt - x) / torch.linalg.vector_norm(x)).item()
        # the inverse (coefficients to signal), timed the same way
        for _ in range(args.warmup):
            inv(y, rt, stream=stream)
        torch.cuda.synchronize()
        inv.timing_begin(steps)
        e0.record(stream)
        for _ in range(steps):
            inv(y, rt, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ims = e0.elapsed_time(e1) / steps
        iper, _ = inv.timing_end()
        inames = inv.launch_names()
        res["inverse"] = {"ms_per_transform": round(ims, 4), "launches": len(inames),
                          "kernels": [{"kernel": k, "avg_ms": round(t, 4)} for k, t in zip(inames, iper)]}
        del rt
        if with_oracle:
            from oracle import r2r
            rng = np.random.default_rng(83)
            js = np.unique(rng.integers(0, 512, size=(40, 3)), axis=0)
            vals = rng.uniform(-1, 1, len(js))
            X = np.zeros(n)
            X[tuple(js.T)] = vals
            xs = torch.from_numpy(r2r.signal_to_buffer(X, p)).to(dev)
            del X
            ys = fwd(xs)
            torch.cuda.synchronize()
            ks = rng.integers(0, 512, size=(1000, 3))
            pos = cyclic_positions(np, ks, n, p)
            got = ys.cpu().numpy()[pos]
            w = np.ones((len(ks), len(js)))
            for l in range(3):
                # the angle pi e / 1024 with e = k (2j + 1) reduced mod 2048 in integers first
                if kind == "dct":
                    e = (ks[:, l][:, None] * (2 * js[:, l][None, :] + 1)) % 2048
                    w *= 2 * np.cos(np.pi * e / 1024)
                else:
                    e = ((ks[:, l][:, None] + 1) * (2 * js[:, l][None, :] + 1)) % 2048
                    w *= 2 * np.sin(np.pi * e / 1024)
            want = w @ vals
            res["sampled_max_rel_error_vs_definition"] = float(np.abs(got - want).max() / np.abs(want).max())
            del xs, ys
        fwd.close()
        inv.close()
        del x, y
        torch.cuda.empty_cache()
        log(f"[bench] {kind} 512^3: {ms:.3f} ms, inverse {ims:.3f} ms")
        out[kind] = res
    return out


def run_paper_workloads(args, torch, fftu):
    """The paper's own test sizes on one GPU: 1024^3 complex128 (4^3 grid, the fused
    exchange) and the very rectangular 16,777,216 x 64 (complex64 and complex128 on a
    4096 x 8 grid: the only grids for it have a local line of 4096, and P = 32768 takes
    the unfused exchange). Input from the device generator; checked by the round trip (forward,
    then inverse, against the input) on the device, and the forward transform of a
    sparse input at 500 sampled outputs against eq. (1.2)."""
    import numpy as np
    res = []
    for n, p, dt in [((1024, 1024, 1024), (4, 4, 4), "complex128"), ((1 << 24, 64), (4096, 8), "complex64"),
                     ((1 << 24, 64), (4096, 8), "complex128")]:
        N = math.prod(n)
        tdt = torch.complex128 if dt == "complex128" else torch.complex64
        log(f"[bench] paper workload {'x'.join(map(str, n))} {dt}")
        x = torch.empty(N, dtype=tdt, device="cuda:0")
        fftu.fill_uniform(x, 7, 0)
        y = torch.empty_like(x)
        fwd = fftu.Plan(n, p, dt, fftu.FORWARD)
        stream = torch.cuda.current_stream()
        fwd(x, y, stream=stream)
        torch.cuda.synchronize()
        steps = 3
        fwd.timing_begin(steps)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fwd(x, y, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        per_launch, _ = fwd.timing_end()
        names = fwd.launch_names()
        info = fwd.info()
        fwd_err = sparse_forward_check(np, torch, fwd, n, p, tdt, seed=17)
        fwd.close()
        inv = fftu.Plan(n, p, dt, fftu.INVERSE)
        inv(y, y, stream=stream)                 # in place: y becomes the round trip
        torch.cuda.synchronize()
        inv.close()
        rt = (torch.linalg.vector_norm(y - x) / torch.linalg.vector_norm(x)).item()
        esize = 16 if dt == "complex128" else 8
        alg = info["launches"] * 2.0 * N * esize
        res.append({"workload": f"{'x'.join(map(str, n))} {dt} forward DFT, {'x'.join(map(str, p))} cyclic grid",
                    "ms_per_transform": round(ms, 3), "GFLOPs": round(5.0 * N * math.log2(N) / (ms * 1e-3) / 1e9, 1),
                    "launches": info["launches"], "exchange_fused": info["exchange_fused"],
                    "roofline": {"bound": "hbm", "algorithmic_bytes": alg, "unit": "GB/s", "peak": HBM_PEAK_GBS,
                                 "achieved": round(alg / (ms * 1e-3) / 1e9, 1),
                                 "frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
                    "rel_l2_roundtrip": rt, "sparse_forward_max_rel_error": fwd_err,
                    # traffic: HBM bytes per launch from the committed counter summary (None when
                    # it was taken from other kernel sources)
                    "kernels": [{"kernel": k, "avg_ms": round(t, 3),
                                 "GBps_alg": round(2.0 * N * esize / (t * 1e-3) / 1e9, 1) if t > 0 else None,
                                 "algorithmic_bytes": 2.0 * N * esize, "traffic": measured_traffic("paper", k)}
                                for k, t in zip(names, per_launch)]})
        del x, y
        torch.cuda.empty_cache()
        log(f"[bench] paper workload {'x'.join(map(str, n))}: {ms:.2f} ms, {res[-1]['GFLOPs']} GFLOP/s")
    return res


def run_precision(args, torch, np, fftu, synth, with_oracle):
    """The precision pattern at 64^5 (2^30 points, 2^5 grid): the complex64 path
    (FP32 butterflies, FP64-generated tables rounded once) timed, and its error
    against the FP64 oracle with the complex128 path's error on the same input
    (the N(0,1) draw rounded once to complex64, promoted exactly) beside it."""
    n, p = (64,) * 5, (2,) * 5
    N = math.prod(n)
    dev = torch.device("cuda:0")
    log("[bench] precision 64^5: generating input")
    D32 = synth.normal_complex(N, 3, np.complex64)
    x32 = torch.from_numpy(D32).to(dev)
    y32 = torch.empty_like(x32)
    plan32 = fftu.Plan(n, p, "complex64", fftu.FORWARD)
    info = plan32.info()
    stream = torch.cuda.current_stream(dev)
    steps = max(3, args.steps // 4)
    for _ in range(args.warmup):
        plan32(x32, y32, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        plan32(x32, y32, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    plan32.close()
    alg = info["launches"] * 2.0 * N * 8
    res = {"workload": "64^5 complex64 forward DFT, 2^5 cyclic grid, N(0,1) input (seed 3)",
           "ms_per_transform": round(ms, 4), "GFLOPs": round(5.0 * N * math.log2(N) / (ms * 1e-3) / 1e9, 1),
           "roofline": {"bound": "hbm", "algorithmic_bytes": alg, "achieved": round(alg / (ms * 1e-3) / 1e9, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}
    if with_oracle:
        import oracle
        got32 = y32.cpu().numpy()
        del x32, y32
        torch.cuda.empty_cache()
        D64 = D32.astype(np.complex128)
        del D32
        x64 = torch.from_numpy(D64).to(dev)
        with fftu.Plan(n, p, "complex128", fftu.FORWARD) as plan64:
            got64 = plan64(x64).cpu().numpy()
        del x64
        torch.cuda.empty_cache()
        log("[bench] precision 64^5: FP64 oracle on the host")
        want = oracle.to_cyclic(oracle.fft_axes(oracle.from_cyclic(D64, n, p), range(5), oracle.FORWARD), p)
        res["rel_l2_complex64_vs_fp64_oracle"] = oracle.rel_l2(got32, want)
        res["rel_l2_complex128_vs_fp64_oracle"] = oracle.rel_l2(got64, want)
        res["tolerance_complex64"] = 5e-6
    log(f"[bench] precision 64^5 complex64: {ms:.3f} ms")
    return res


def run_small(args, torch, np, fftu, synth, with_oracle):
    """The small case: 64^3 complex128 on a 2^3 grid, forward then inverse. 4 MiB
    fits in the caches, so latency (HIP-graph replays, and plain calls) is the
    measure here, not the HBM roofline."""
    n, p = (64, 64, 64), (2, 2, 2)
    N = math.prod(n)
    dev = torch.device("cuda:0")
    D = synth.uniform_complex(N, 1, np.complex128)
    x = torch.from_numpy(D).to(dev)
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    fwd = fftu.Plan(n, p, "complex128", fftu.FORWARD)
    inv = fftu.Plan(n, p, "complex128", fftu.INVERSE)
    stream = torch.cuda.current_stream(dev)
    gf = fftu.Graph(fwd, x, y)
    gi = fftu.Graph(inv, y, z)
    reps = 200

    def timed(run):
        for _ in range(10):
            run()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3

    us_graph = timed(lambda: (gf.launch(stream), gi.launch(stream)))
    us_plain = timed(lambda: (fwd(x, y, stream=stream), inv(y, z, stream=stream)))
    res = {"workload": "64x64x64 complex128 forward then inverse DFT, 2x2x2 cyclic grid",
           "us_fwd_inv_graph": round(us_graph, 2), "us_fwd_inv_plain": round(us_plain, 2),
           "launches_fwd": fwd.info()["launches"]}
    if with_oracle:
        import oracle
        want = oracle.cyclic_dft(D, n, p)
        res["rel_l2_forward_vs_oracle"] = oracle.rel_l2(y.cpu().numpy(), want)
        res["rel_l2_roundtrip"] = oracle.rel_l2(z.cpu().numpy(), D)
    gf.close()
    gi.close()
    fwd.close()
    inv.close()
    log(f"[bench] small 64^3 fwd+inv: {us_graph:.1f} us (graphs), {us_plain:.1f} us (plain calls)")
    return res


def run_serving(args, torch, synth):
    """The serving workload: a Poisson stream of 2-D/3-D/4-D requests (2000/s,
    sides 2^5..2^10, at most 2^26 points, complex64/complex128, forward/inverse,
    trace seed 5), served in real time with the continuous policy (4 streams),
    the coalesced policy (continuous, and small requests that wait together run
    as one persistent batch launch) and the plain one-at-a-time FIFO, on the same
    arena, plan cache and kernels. Then every complex64 result's error against
    the complex128 transform of its own input."""
    from paper_2203_11795_amd import serving
    secs = float(args.serving_seconds)
    reqs = serving.requests_from_trace(synth.serving_trace(seed=5, rate=2000.0, duration=30.0), limit_seconds=secs)
    log(f"[bench] serving: {len(reqs)} requests in the first {secs:g} s of the trace")
    srv = serving.Server(arena_bytes=16 << 30, streams=4, seed=5)
    try:
        srv.warmup(reqs)
        out = {"workload": f"first {secs:g} s of a Poisson trace at 2000 requests/s (seed 5): rank 2-4, sides "
                           "2^5..2^10, <= 2^26 points, complex64/complex128, forward/inverse, p_l = 2; "
                           "input generated on the device (Philox4x32-10, key (5, request id))",
               "streams": srv.nstreams, "large_lanes": srv.large_lanes, "large_MiB": srv.large_bytes >> 20,
               "arena_GiB": srv.arena_bytes / 2 ** 30}
        out["coalesce_MiB"] = srv.coalesce_bytes >> 20
        out["coalesce_max"] = srv.coalesce_max
        for policy in ("continuous", "coalesced", "fifo"):
            res = srv.serve(reqs, policy, time_limit=3 * secs + 5)
            out[policy] = serving.summarize(res, reqs)
            log(f"[bench] serving {policy}: {out[policy]}")
        f = out["fifo"]
        for policy in ("continuous", "coalesced"):
            c = out[policy]
            c["p99_speedup_vs_fifo"] = round(f["p99_ms"] / c["p99_ms"], 3) if c["p99_ms"] > 0 else None
            c["p50_speedup_vs_fifo"] = round(f["p50_ms"] / c["p50_ms"], 3) if c["p50_ms"] > 0 else None
        # a burst: the trace's first 2000 requests of at most 4 MiB, all arriving at once, where
        # requests wait together and coalescing has something to gather
        burst = [serving.Request(r.rid, 0.0, r.shape, r.dtype, r.direction) for r in reqs
                 if r.N * r.esize <= srv.coalesce_bytes][:2000]
        out["burst"] = {"workload": f"{len(burst)} requests of at most {srv.coalesce_bytes >> 20} MiB from the "
                                    "trace, all arriving at t = 0"}
        for policy in ("continuous", "coalesced"):
            res = srv.serve(burst, policy, time_limit=60)
            out["burst"][policy] = {k: v for k, v in serving.summarize(res, burst).items()
                                    if k in ("completed", "p50_ms", "p99_ms", "mean_ms", "max_ms", "wall_s", "batches",
                                             "coalesced_requests", "max_batch")}
            log(f"[bench] serving burst {policy}: {out['burst'][policy]}")
        if not args.no_check:
            import numpy as np
            log("[bench] serving: FP32 error of every complex64 result against complex128")
            t0 = time.perf_counter()
            errs = {}
            for k in range(0, len(reqs), 5000):
                errs.update(serving.precision_errors(srv, reqs[k:k + 5000]))
                log(f"[bench] serving: FP32 errors of {len(errs)} results so far")
            ev = np.array(list(errs.values())) if errs else np.array([float("nan")])
            out["precision_complex64_vs_complex128"] = {
                "results": len(errs), "max": float(ev.max()), "median": float(np.median(ev)),
                "p99": float(np.percentile(ev, 99)), "tolerance": 5e-6,
                "within_tolerance": int((ev <= 5e-6).sum()), "seconds": round(time.perf_counter() - t0, 1)}
    finally:
        srv.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="512cube", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batch workload")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving workload")
    ap.add_argument("--no-convolution", action="store_true", help="skip the convolution workload")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-radix workload")
    ap.add_argument("--no-real", action="store_true", help="skip the real-input 512^3 transform")
    ap.add_argument("--no-r2r", action="store_true", help="skip the 512^3 DCT-II / DST-II")
    ap.add_argument("--no-group-cyclic", action="store_true",
                    help="skip the grid beyond p_max (512^3 over 32^3, two supersteps)")
    ap.add_argument("--no-paper", action="store_true",
                    help="skip the paper's own sizes (1024^3 complex128, 16777216 x 64 complex64 and complex128)")
    ap.add_argument("--no-small", action="store_true", help="skip the 64^3 latency workload")
    ap.add_argument("--no-precision", action="store_true", help="skip the 64^5 complex64 precision workload")
    ap.add_argument("--serving-seconds", type=float, default=30.0,
                    help="seconds of the 30 s request trace to serve (each policy runs it in real time)")
    ap.add_argument("--retune", action="store_true", help="measure the tiling knobs again instead of the cached ones")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="time a plain device copy of the workload's N elements instead (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): this build has no multi-GPU path; "
              "the exchange is an on-device permutation.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2203_11795_amd as fftu
    import synth

    wl = WORKLOADS[args.workload]
    n, p, dtype = wl["n"], wl["p"], wl["dtype"]
    N = math.prod(n)
    esize = 16 if dtype == "complex128" else 8
    npdt = np.complex128 if dtype == "complex128" else np.complex64

    if args.copy_calibration:
        # A plain copy of N elements: its HBM counters read N*b fetched and N*b written.
        src = torch.empty(N, dtype=torch.complex128 if esize == 16 else torch.complex64, device="cuda:0")
        src.zero_()
        dst = torch.empty_like(src)
        for _ in range(args.warmup):
            dst.copy_(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        print(json.dumps({"copy_bytes_each_way": N * esize, "ms": round(dt * 1e3, 4),
                          "GBps": round(2 * N * esize / dt / 1e9, 1)}), flush=True)
        return

    log(f"[bench] workload {args.workload}: generating input")
    gen = synth.uniform_complex if wl["dist"] == "uniform" else synth.normal_complex
    D = gen(N, wl["seed"], npdt)
    dev = torch.device("cuda:0")
    x = torch.from_numpy(D).to(dev)
    out = torch.empty_like(x)
    plan = fftu.Plan(n, p, dtype, fftu.FORWARD)
    info = plan.info()
    stream = torch.cuda.current_stream(dev)

    log(f"[bench] plan: {info}; warmup {args.warmup}")
    for _ in range(args.warmup):
        plan(x, out)
    torch.cuda.synchronize()

    plan.timing_begin(args.steps)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    evs[0].record(stream)
    for i in range(args.steps):
        plan(x, out, stream=stream)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    total_ms = evs[0].elapsed_time(evs[-1])
    step_ms = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    per_launch, ncalls = plan.timing_end()
    ms = total_ms / args.steps
    flops = 5.0 * N * math.log2(N)
    gflops = flops / (ms * 1e-3) / 1e9
    log(f"[bench] {args.steps} steps: {ms:.3f} ms/step, {gflops:.1f} GFLOP/s; per launch ms {per_launch}")

    # Roofline of the dominant kernel: every launch reads and writes the N-element array once.
    alg_bytes = 2.0 * N * esize
    syms = plan.launch_names()
    per_sym = {}
    for s, t in zip(syms, per_launch):
        tot, cnt = per_sym.get(s, (0.0, 0))
        per_sym[s] = (tot + t, cnt + 1)
    dom = max(per_sym, key=lambda s: per_sym[s][0])
    dom_avg_ms = per_sym[dom][0] / per_sym[dom][1]
    achieved = alg_bytes / (dom_avg_ms * 1e-3) / 1e9
    kname = dom
    traffic = measured_traffic(args.workload, kname)
    roofline = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "algorithmic_bytes_per_launch": alg_bytes,
                "avg_launch_ms": round(dom_avg_ms, 4), "launches_per_step": per_sym[dom][1]}
    kernels = [{"launch": i, "kernel": s, "avg_ms": round(t, 4),
                "GBps_alg": round(alg_bytes / (t * 1e-3) / 1e9, 1) if t > 0 else None}
               for i, (s, t) in enumerate(zip(syms, per_launch))]
    # a practical reference beside the peak: a device-to-device copy of the same array
    # (torch's copy_, the runtime's copy), timed with HIP events on the same stream
    scratch = torch.empty_like(x)          # `out` keeps the transform for the check below
    for _ in range(3):
        scratch.copy_(x)
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(10):
        scratch.copy_(x)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbps = alg_bytes / (c0.elapsed_time(c1) / 10 * 1e-3) / 1e9
    del scratch
    roofline["copy_reference"] = {"what": "device-to-device copy of the same array (torch copy_)",
                                  "GBps": round(copy_gbps, 1), "frac": round(copy_gbps / HBM_PEAK_GBS, 4),
                                  "dominant_kernel_vs_copy": round(achieved / copy_gbps, 3)}
    transform_bytes = info["launches"] * alg_bytes
    frac_transform = transform_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS
    # the scope's algorithmic bytes: the fewest passes this shape needs (local dimensions
    # grouped under the LDS budget, plus the exchange), each one read and one write
    b_alg = ideal_passes(n, p, esize) * alg_bytes

    result = {
        "metric": METRIC, "value": round(gflops, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": "f64" if esize == 16 else "f32", "data": "synthetic",
        "config": {"workload": wl["name"], "n": list(n), "p": list(p), "direction": "forward",
                   "input": f"iid {wl['dist']} real/imag, seed {wl['seed']}"},
        "roofline": roofline,
        "timing": {"ms_mean": round(ms, 4), "ms_median": round(float(np.median(step_ms)), 4),
                   "ms_p10": round(float(np.percentile(step_ms, 10)), 4),
                   "ms_p90": round(float(np.percentile(step_ms, 90)), 4), "steps": args.steps},
        "hbm_roofline_frac_transform": round(frac_transform, 4),
        "transform_algorithmic_bytes": transform_bytes,
        "hbm_roofline_frac_ideal_passes": round(b_alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "ideal_passes": ideal_passes(n, p, esize), "launches": info["launches"],
        "kernels": kernels,
    }

    need_oracle = not (args.no_cpu_baseline and args.no_check)
    if need_oracle:
        import oracle
        log("[bench] oracle: layout + FP64 transform on the host")
        X = oracle.from_cyclic(D.astype(np.complex128), n, p)
        t0 = time.perf_counter()
        Y = oracle.fft_axes(X, range(len(n)), oracle.FORWARD)
        t_oracle = time.perf_counter() - t0
        if not args.no_cpu_baseline:
            result["cpu_baseline"] = {
                "value": round(flops / t_oracle / 1e9, 3), "unit": "GFLOP/s", "cores": oracle.max_threads(),
                "kind": "oracle",
                "sample": f"one full {'x'.join(map(str, n))} forward DFT (FP64 separable radix-2, natural order) "
                          f"of the same seeded input: {t_oracle:.2f} s",
                "cpu_model": cpu_model()}
            result["cpu_baseline"].update(oracle_single_thread(np, oracle, synth, X, flops))
        if not args.no_check:
            got = out.cpu().numpy()
            result["rel_l2_vs_oracle"] = oracle.rel_l2(got, oracle.to_cyclic(Y, p))
    plan.close()
    if args.workload == "512cube":
        del x, out
        torch.cuda.empty_cache()
    if args.workload == "512cube" and not args.no_precision:
        result["precision"] = run_precision(args, torch, np, fftu, synth, not args.no_check)
        torch.cuda.empty_cache()
    if args.workload == "512cube" and not args.no_small:
        result["small"] = run_small(args, torch, np, fftu, synth, not args.no_check)
    if args.workload == "512cube" and not args.no_convolution:
        result["convolution"] = run_convolution(args, torch, np, fftu, synth, info)
        torch.cuda.empty_cache()
    if args.workload == "512cube" and not args.no_paper:
        result["paper_workloads"] = run_paper_workloads(args, torch, fftu)
        torch.cuda.empty_cache()
    if args.workload == "512cube" and not args.no_mixed:
        result["mixed_radix"] = run_mixed(args, torch, np, fftu, synth, not args.no_check)
        torch.cuda.empty_cache()
    if args.workload == "512cube" and not args.no_real:
        result["real"] = run_real(args, torch, np, fftu, synth, not args.no_check)
    if args.workload == "512cube" and not args.no_r2r:
        result["r2r"] = run_r2r(args, torch, np, fftu, not args.no_check)
        torch.cuda.empty_cache()
    if args.workload == "512cube" and not args.no_group_cyclic:
        result["group_cyclic"] = run_group_cyclic(args, torch, np, fftu, synth, not args.no_check)
        torch.cuda.empty_cache()
    if args.workload == "512cube" and not args.no_batch:
        result["batch"] = run_batch(args, torch, np, fftu, synth, not args.no_check)
    if args.workload == "512cube" and not args.no_serving:
        torch.cuda.empty_cache()
        result["serving"] = run_serving(args, torch, synth)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
