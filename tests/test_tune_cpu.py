"""Host logic of the launch-shape autotuner (no GPU): the fastest candidate
wins, ties go to the earlier candidate, and a candidate whose counts differ
from the others is an error."""
import numpy as np
import pytest

from paper_2310_15668_amd.tune import CANDIDATES, tune_batch


def fake(times, counts=None):
    calls = []

    def run(launch, blocks):
        calls.append((launch, blocks))
        c = counts.get((launch, blocks), np.arange(457)) if counts else np.arange(457)
        t = times[(launch, blocks)]
        return c, (t.pop(0) if isinstance(t, list) else t)
    return run, calls


def test_fastest_candidate_wins():
    times = {c: 10.0 + i for i, c in enumerate(CANDIDATES)}
    times[(2, 4)] = 3.0
    run, calls = fake(times)
    res = tune_batch(None, None, run=run)
    assert (res["launch"], res["blocks"]) == (2, 4)
    assert calls == list(CANDIDATES)
    assert res["times"][(2, 4)] == 3.0


def test_tie_goes_to_the_earlier_candidate():
    run, _ = fake({c: 5.0 for c in CANDIDATES})
    res = tune_batch(None, None, run=run)
    assert (res["launch"], res["blocks"]) == CANDIDATES[0]


def test_repeats_keep_the_best_time():
    times = {(1, 8): [9.0, 4.0, 7.0], (2, 8): [5.0, 6.0, 5.5]}
    run, calls = fake(times)
    res = tune_batch(None, None, candidates=[(1, 8), (2, 8)], repeats=3, run=run)
    assert (res["launch"], res["blocks"]) == (1, 8) and res["times"] == {(1, 8): 4.0, (2, 8): 5.0}
    assert len(calls) == 6


def test_differing_counts_are_an_error():
    bad = np.arange(457)
    bad[100] += 1
    run, _ = fake({c: 1.0 for c in CANDIDATES}, counts={(1, 4): bad})
    with pytest.raises(RuntimeError, match=r"\(1, 4\)"):
        tune_batch(None, None, run=run)
    with pytest.raises(ValueError):
        tune_batch(None, None, candidates=(), run=run)
