"""Measured tuning of the tiling knobs (fftu_set_tuning) for a plan or a batch.

The knobs change how the local-FFT passes are tiled (lines per workgroup, LDS
padding, the LDS budget per workgroup, the mixed-radix tile), whether the
innermost dimension's lines share a kernel with the exchange, and the radix
split of mixed-radix lines (the largest power-of-two radix: 8, 4 or 2). Only
the radix split changes what is computed, within rounding. A plan reads
them when it is created, so tuning builds one plan per candidate setting, times
its executions with HIP events on the current stream, and keeps the fastest.
The search is coordinate descent: each knob in turn is swept with the others
held at the best values found so far, starting from the library defaults (-1).

Results are cached in a JSON file (``FFTU_WISDOM``, default
``~/.cache/fftu/wisdom.json``) keyed by GPU architecture and CU count, kind, dtype, direction and
the shapes and grids, so a later process can apply them without measuring.
"""
from __future__ import annotations

import hashlib
import json
import os
import statistics

from . import fftu as _b

KNOB_NAMES = ("line_strided_logw", "line_contig_logw", "line_pad", "max_lds_kb", "fuse_last", "pair", "mixed_radix",
              "mixed_tile_log")
CANDIDATES = {
    "line_strided_logw": (-1, 2, 3, 4, 5, 6),
    "line_contig_logw": (-1, 0, 1, 2, 3, 4),
    "line_pad": (-1, 0, 2),
    "max_lds_kb": (-1, 32, 96, 160),
    "fuse_last": (-1, 0),
    "pair": (-1, 0),
    "mixed_radix": (-1, 4, 2),
    "mixed_tile_log": (-1, 9, 11, 12),
}
# knobs that change the arithmetic (the radix split): a candidate with one of them off
# its default is checked against the default knobs' output within the dtype's
# tolerance instead of bit for bit
ARITHMETIC_KNOBS = ("mixed_radix",)
TOL = {"complex128": 1e-12, "complex64": 5e-6}


def wisdom_path() -> str:
    return os.environ.get("FFTU_WISDOM", os.path.join(os.path.expanduser("~"), ".cache", "fftu", "wisdom.json"))


def _load_wisdom() -> dict:
    try:
        with open(wisdom_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store_wisdom(key: str, value: dict) -> None:
    w = _load_wisdom()
    w[key] = value
    path = wisdom_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(w, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass   # a read-only home only loses the cache


def _key(kind, shapes, grids, dtype, direction) -> str:
    import torch
    if torch.cuda.is_available():
        props = torch.cuda.get_device_properties(0)   # the architecture and CU count, not the marketing name
        dev = f"{getattr(props, 'gcnArchName', props.name)}/{props.multi_processor_count}cu"
    else:
        dev = "cpu"
    h = hashlib.sha1(repr((list(map(tuple, shapes)), list(map(tuple, grids)))).encode()).hexdigest()[:16]
    return f"{dev}|{kind}|{dtype}|{int(direction)}|{h}"


def current() -> dict:
    return {k: _b.get_tuning(k) for k in KNOB_NAMES}


def apply(knobs: dict) -> None:
    for k in KNOB_NAMES:
        _b.set_tuning(k, int(knobs.get(k, -1)))


def _time_ms(run, reps: int) -> float:
    import torch
    run()                                   # warm-up (and first-touch of the plan's buffers)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        run()
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return statistics.median(times)


def _search(make_runner, reps: int):
    """Coordinate descent over the knobs. make_runner() builds a plan under the
    current knobs and returns (run, close) or (run, close, valid), or raises
    FftuError if the setting is not plannable. valid(), called after the timed
    runs, says whether the candidate's last output is right; a candidate that
    fails it is recorded as rejected and never kept, however fast it ran."""
    saved = current()
    table = []
    best = {k: -1 for k in KNOB_NAMES}
    best_ms = None
    tried = {}
    try:
        for knob in KNOB_NAMES:
            for v in CANDIDATES[knob]:
                cand = dict(best)
                cand[knob] = v
                key = tuple(cand[k] for k in KNOB_NAMES)
                if key in tried:
                    continue
                try:
                    apply(cand)
                    runner = make_runner()
                except _b.FftuError:
                    tried[key] = None
                    continue
                run, close = runner[0], runner[1]
                try:
                    ms = _time_ms(run, reps)
                    ok = runner[2]() if len(runner) > 2 else True
                finally:
                    close()
                if not ok:
                    tried[key] = None
                    table.append({**cand, "ms": round(ms, 4), "rejected": True})
                    continue
                tried[key] = ms
                table.append({**cand, "ms": round(ms, 4)})
                if best_ms is None or ms < best_ms:
                    best_ms, best = ms, cand
    finally:
        apply(saved)
    return best, best_ms, table


def tune_batch(shapes, grids, dtype, direction, xs, outs, reps: int = 5, use_cache: bool = True) -> dict:
    """Best knobs for a BatchPlan over these members (xs/outs: device tensors)."""
    key = _key("batch", shapes, grids, dtype, direction)
    if use_cache:
        hit = _load_wisdom().get(key)
        if hit:
            return {**hit, "cached": True}

    import torch
    saved = current()
    try:
        apply({})                          # the reference output: library defaults
        with _b.BatchPlan(shapes, grids, dtype, direction) as bp:
            ref = [o.clone() for o in bp(xs, [torch.empty_like(x) for x in xs])]
            torch.cuda.synchronize()
            if bp.error_flag() != 0:
                raise RuntimeError("the batch with default knobs hit its dependency wait limit")
    finally:
        apply(saved)

    def make_runner():
        bp = _b.BatchPlan(shapes, grids, dtype, direction)

        def valid():
            # the bounded dependency wait gives up by skipping work (and so runs faster);
            # tiling never changes arithmetic, so outputs must equal the defaults' bit for bit
            torch.cuda.synchronize()
            return bp.error_flag() == 0 and all(torch.equal(o, r) for o, r in zip(outs, ref))
        return (lambda: bp(xs, outs)), bp.close, valid

    best, best_ms, table = _search(make_runner, reps)
    res = {"knobs": best, "ms": round(best_ms, 4) if best_ms is not None else None, "candidates": table}
    _store_wisdom(key, {"knobs": best, "ms": res["ms"]})
    return {**res, "cached": False}


def tune_plan(n, p, dtype, direction, x, out, reps: int = 5, use_cache: bool = True) -> dict:
    """Best knobs for a single Plan (x/out: device tensors of N elements)."""
    key = _key("plan", [n], [p], dtype, direction)
    if use_cache:
        hit = _load_wisdom().get(key)
        if hit:
            return {**hit, "cached": True}

    import torch
    saved = current()
    try:
        apply({})
        with _b.Plan(n, p, dtype, direction) as pl:
            ref = pl(x, torch.empty_like(out)).clone()
            torch.cuda.synchronize()
    finally:
        apply(saved)

    def make_runner():
        pl = _b.Plan(n, p, dtype, direction)

        exact = all(current().get(k, -1) == -1 for k in ARITHMETIC_KNOBS)

        def valid():
            torch.cuda.synchronize()
            if exact:
                return torch.equal(out, ref)
            err = (torch.linalg.vector_norm(out - ref) / torch.linalg.vector_norm(ref)).item()
            return err <= TOL[str(dtype).replace("torch.", "")]
        return (lambda: pl(x, out)), pl.close, valid

    best, best_ms, table = _search(make_runner, reps)
    res = {"knobs": best, "ms": round(best_ms, 4) if best_ms is not None else None, "candidates": table}
    _store_wisdom(key, {"knobs": best, "ms": res["ms"]})
    return {**res, "cached": False}
