"""Coordinate-descent search of the tiling knobs (host logic, no GPU): the
timing and plan construction are replaced by a synthetic cost."""
import pytest

from paper_2203_11795_amd import autotune
from paper_2203_11795_amd import fftu as binding


def test_search_finds_the_separable_minimum_and_restores_knobs(monkeypatch):
    state = {k: -1 for k in autotune.KNOB_NAMES}
    monkeypatch.setattr(autotune, "current", lambda: dict(state))
    monkeypatch.setattr(autotune, "apply", lambda knobs: state.update({k: int(knobs.get(k, -1)) for k in state}))
    target = {"line_strided_logw": 4, "line_contig_logw": 2, "line_pad": 0, "max_lds_kb": 96, "fuse_last": -1, "pair": -1,
              "mixed_radix": 4, "mixed_tile_log": -1}

    def cost():
        return 1.0 + sum(abs(state[k] - v) for k, v in target.items())

    def make_runner():
        if state["line_strided_logw"] == 6:
            raise binding.FftuError(3, "fftu_plan_batch")     # a setting the planner refuses
        c = cost()
        return (lambda: c), (lambda: None)

    monkeypatch.setattr(autotune, "_time_ms", lambda run, reps: run())
    state["line_pad"] = 2                                   # knobs in force before the search
    before = dict(state)
    best, best_ms, table = autotune._search(make_runner, reps=1)
    assert best == target and best_ms == 1.0
    assert state == before                                   # restored afterwards
    assert all(row["line_strided_logw"] != 6 for row in table)
    assert len(table) == len({tuple(r[k] for k in autotune.KNOB_NAMES) for r in table})   # no repeats


def test_wisdom_roundtrip(tmp_path, monkeypatch):
    monkeypatch.setenv("FFTU_WISDOM", str(tmp_path / "w.json"))
    autotune._store_wisdom("k1", {"knobs": {"line_pad": 0}, "ms": 1.5})
    autotune._store_wisdom("k2", {"knobs": {"line_pad": 2}, "ms": 2.5})
    w = autotune._load_wisdom()
    assert w["k1"]["ms"] == 1.5 and w["k2"]["knobs"]["line_pad"] == 2
    (tmp_path / "w.json").write_text("not json")
    assert autotune._load_wisdom() == {}


def test_candidates_are_in_the_knob_ranges():
    lo_hi = {"line_strided_logw": (2, 6), "line_contig_logw": (0, 8), "line_pad": (0, 4), "max_lds_kb": (16, 160),
             "fuse_last": (0, 1), "pair": (0, 1), "mixed_radix": (2, 8), "mixed_tile_log": (9, 12)}
    for k, vals in autotune.CANDIDATES.items():
        assert vals[0] == -1
        for v in vals[1:]:
            assert lo_hi[k][0] <= v <= lo_hi[k][1]
    try:
        for k, vals in autotune.CANDIDATES.items():
            for v in vals:
                binding.set_tuning(k, v)
    finally:
        for k in autotune.KNOB_NAMES:
            binding.set_tuning(k, -1)


def test_search_never_keeps_a_candidate_with_a_wrong_output(monkeypatch):
    """A setting that runs fastest because it skipped work (a batch whose bounded
    wait gave up) must lose to every valid one."""
    state = {k: -1 for k in autotune.KNOB_NAMES}
    monkeypatch.setattr(autotune, "current", lambda: dict(state))
    monkeypatch.setattr(autotune, "apply", lambda knobs: state.update({k: int(knobs.get(k, -1)) for k in state}))
    monkeypatch.setattr(autotune, "_time_ms", lambda run, reps: run())

    def make_runner():
        broken = state["line_pad"] == 0
        c = 0.1 if broken else 1.0 + abs(state["max_lds_kb"] - 96) / 100.0
        return (lambda: c), (lambda: None), (lambda: not broken)

    best, best_ms, table = autotune._search(make_runner, reps=1)
    assert best["line_pad"] != 0 and best["max_lds_kb"] == 96 and best_ms == 1.0
    assert any(r.get("rejected") for r in table)
