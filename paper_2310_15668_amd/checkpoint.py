"""Resumable exact counting over centre ranges.

Algorithm 2 attributes every instance to exactly one centre (section 4.2),
so the counts of a hypergraph are the sum of the counts of any partition of
its centres into ranges.  A long exact count can therefore be cut into
ranges, each counted by ``mochy_count_exact_range``, with the running sums
saved after every range: a count interrupted at any point (a killed process,
a lost device) resumes from the first range not yet saved and ends with the
same integers.

The checkpoint is a small JSON file written atomically (a temporary file,
then ``os.replace``): the key of the hypergraph it belongs to, the next
centre, and the 26 + 431 running sums.  A checkpoint whose key differs from
the hypergraph being counted is refused, never merged.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from . import _lib

VERSION = 1


def csr_key(edge_ptr, edge_nodes, num_nodes) -> str:
    """sha256 of a host CSR: what a checkpoint belongs to."""
    d = hashlib.sha256()
    d.update(np.ascontiguousarray(edge_ptr, dtype=np.int64).tobytes())
    d.update(np.ascontiguousarray(edge_nodes, dtype=np.int32).tobytes())
    d.update(str(int(num_nodes)).encode())
    return d.hexdigest()


def ranges(num_edges: int, chunk: int):
    """Consecutive centre ranges [a, b) of at most ``chunk`` centres."""
    if chunk <= 0:
        raise ValueError("chunk must be positive")
    return [(a, min(num_edges, a + chunk)) for a in range(0, num_edges, chunk)]


def load(path: str, key: str):
    """(next centre, counts26, counts431) saved for ``key``, or None if there is
    no checkpoint; ValueError if the file belongs to another hypergraph."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        state = json.load(f)
    if state.get("version") != VERSION or state.get("key") != key:
        raise ValueError(f"checkpoint {path} belongs to another hypergraph or format")
    c26 = np.array(state["counts26"], dtype=np.int64)
    c431 = np.array(state["counts431"], dtype=np.int64)
    if c26.shape != (_lib.NUM_H,) or c431.shape != (_lib.NUM_3H,):
        raise ValueError(f"checkpoint {path} has malformed counts")
    return int(state["next_centre"]), c26, c431


def save(path: str, key: str, next_centre: int, c26, c431) -> None:
    state = {"version": VERSION, "key": key, "next_centre": int(next_centre),
             "counts26": [int(x) for x in c26], "counts431": [int(x) for x in c431]}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(state, f)
        f.flush()
        os.fsync(f.fileno())
    os.replace(tmp, path)


def count_exact_resumable(count_range, num_edges: int, key: str, path: str, chunk: int,
                          stop_after: int | None = None):
    """Exact counts of centres [0, num_edges) in ranges of ``chunk`` centres,
    resuming from the checkpoint at ``path`` when one exists for ``key``.

    ``count_range(c0, c1) -> (counts26, counts431)`` counts one range (for
    the library: ``lambda a, b: mochy_count_exact_range(ctx, g, a, b)``).
    ``stop_after`` stops after that many ranges of this call (an interruption,
    for tests) and returns None.  Returns (counts26, counts431) when every
    centre is counted; the checkpoint then records num_edges as the next
    centre."""
    got = load(path, key)
    if got is None:
        start, c26, c431 = 0, np.zeros(_lib.NUM_H, np.int64), np.zeros(_lib.NUM_3H, np.int64)
    else:
        start, c26, c431 = got
    done = 0
    for a, b in ranges(num_edges, chunk):
        if b <= start:
            continue
        if a < start:  # a checkpoint from another chunk size: continue from where it stopped
            a = start
        if stop_after is not None and done == stop_after:
            return None
        r26, r431 = count_range(a, b)
        c26 = c26 + np.asarray(r26, dtype=np.int64)
        c431 = c431 + np.asarray(r431, dtype=np.int64)
        save(path, key, b, c26, c431)
        start = b
        done += 1
    if got is None and num_edges == 0:
        save(path, key, 0, c26, c431)
    return c26, c431
