"""Launch-shape autotuner for the batched exact pass (``mochy_profile``).

Two launch choices of the group-pair kernel change its speed and never its
counts:

* ``MOCHY_OPT_BATCH_LAUNCH``: one launch over the whole batch (1), whose
  waves carry two histogram copies each and overlap the graphs' tails, or
  one launch per graph (2), whose blocks share four copies;
* ``MOCHY_OPT_PAIR_BLOCKS``: blocks launched per compute unit.

Which is faster depends on how the batch's work is spread over its graphs.
``tune_batch`` counts a representative batch once per candidate, checks that
every candidate returns the same counts, and leaves the context set to the one
whose pair phase (the pair kernel's own event-timed span) was shortest.  The
choice holds for later batches of the same shape: a server tunes on its first
request and applies the result to every slot (``CPServer.apply_options``).
"""
from __future__ import annotations

import numpy as np

from . import _lib

# (batch launch, blocks per CU); the first is the library's default
CANDIDATES = ((0, 8), (1, 8), (2, 8), (1, 4), (2, 4))


def _run_profile(ctx, graphs, launch: int, blocks: int):
    ctx.set_option(_lib.MOCHY_OPT_BATCH_LAUNCH, launch)
    ctx.set_option(_lib.MOCHY_OPT_PAIR_BLOCKS, blocks)
    counts = _lib.mochy_profile(ctx, graphs)[0]
    return counts, _lib.mochy_phase_ms(ctx)["exact_pairs"]


def tune_batch(ctx, graphs, candidates=CANDIDATES, repeats: int = 1, run=None) -> dict:
    """Time each (launch, blocks) candidate on ``graphs`` and keep the fastest.

    ``run(launch, blocks) -> (counts, pair_ms)`` replaces the library call
    (tests).  Raises RuntimeError if two candidates disagree on a count (a
    launch shape must never change a result).  Returns
    ``{"launch", "blocks", "times": {(launch, blocks): best ms}}``.
    """
    if not candidates:
        raise ValueError("no candidates")
    if run is None:
        def run(launch, blocks):
            return _run_profile(ctx, graphs, launch, blocks)
    times, ref = {}, None
    for cand in candidates:
        best = None
        for _ in range(max(1, repeats)):
            counts, ms = run(*cand)
            counts = np.asarray(counts)
            if ref is None:
                ref = counts
            elif counts.shape != ref.shape or not np.array_equal(counts, ref):
                raise RuntimeError(f"launch shape {cand} changed the counts")
            best = ms if best is None else min(best, ms)
        times[tuple(cand)] = float(best)
    launch, blocks = min(times, key=lambda c: (times[c], list(times).index(c)))
    if ctx is not None:
        ctx.set_option(_lib.MOCHY_OPT_BATCH_LAUNCH, launch)
        ctx.set_option(_lib.MOCHY_OPT_PAIR_BLOCKS, blocks)
    return {"launch": launch, "blocks": blocks, "times": times}
