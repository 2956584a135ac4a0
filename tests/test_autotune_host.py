"""CPU tests of the autotuner's selection logic (its timer replaced by a scripted one)."""
import pytest
import torch

from paper_1901_03088_amd import autotune


def scripted(times):
    """A timer returning the scripted time of the candidate currently applied, call after call."""
    state = {"cur": None, "calls": {}}

    def apply(c):
        state["cur"] = c

    def timer(run, reps):
        run()
        c = state["cur"]
        k = state["calls"].get(c, 0)
        state["calls"][c] = k + 1
        seq = times[c]
        return seq[min(k, len(seq) - 1)]
    return apply, timer, state


def test_finalists_are_retimed_and_the_best_median_wins():
    # first sweep: 'a' looks fastest by a fluke; its re-timings are slow, 'b' is steady and wins
    times = {"a": [1.0, 3.0, 3.0, 3.0], "b": [1.5, 1.5, 1.6, 1.4], "c": [1.8, 1.8], "d": [5.0]}
    apply, timer, state = scripted(times)
    out = torch.zeros(4)
    best, rows = autotune._sweep(["a", "b", "c", "d"], apply, lambda: None, lambda: [out], reps=5, timer=timer)
    assert best == "b"
    assert [r["candidate"] for r in rows] == ["a", "b", "c", "d"]
    assert sum("final_ms" in r for r in rows) == 3 and "final_ms" not in rows[3]
    assert state["calls"] == {"a": 4, "b": 4, "c": 4, "d": 1}     # one sweep + three rounds for finalists


def test_a_variant_with_different_results_is_refused():
    vals = {"x": torch.tensor([1.0]), "y": torch.tensor([2.0])}
    state = {}

    def apply(c):
        state["c"] = c
    with pytest.raises(RuntimeError, match="changed the results"):
        autotune._sweep(["x", "y"], apply, lambda: None, lambda: [vals[state["c"]]], reps=1,
                        timer=lambda run, reps: 1.0)


def test_fewer_candidates_than_finalists():
    apply, timer, _ = scripted({7: [2.0], 9: [1.0]})
    best, rows = autotune._sweep([7, 9], apply, lambda: None, lambda: [torch.zeros(1)], reps=1, timer=timer)
    assert best == 9 and all("final_ms" in r for r in rows)
