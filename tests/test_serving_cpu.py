"""Admission policy of the CP server (host logic only)."""
import numpy as np

from paper_2310_15668_amd.serving import Admission, request_bytes
from workloads import from_edge_lists


def ids(started):
    return [rid for rid, _ in started]


def test_fits_and_backfill():
    a = Admission(budget=100, aging_s=1.0, exclusive_frac=1.0)
    a.add("A", 60, 0.0)
    a.add("B", 50, 0.0)
    a.add("C", 30, 0.0)
    assert ids(a.take(free_slots=2, now=0.0)) == ["A", "C"]  # B waits, C backfills
    assert a.in_use == 90 and a.running == 2
    assert a.take(free_slots=0, now=0.1) == []
    a.release(60)
    assert ids(a.take(free_slots=1, now=0.5)) == ["B"]
    assert a.in_use == 80


def test_aged_request_blocks_backfill():
    a = Admission(budget=100, aging_s=1.0, exclusive_frac=1.0)
    a.add("X", 70, 0.0)
    assert ids(a.take(4, 0.0)) == ["X"]
    a.add("D", 50, 0.0)
    a.add("E", 10, 0.0)
    assert ids(a.take(3, 0.5)) == ["E"]   # D young: E may pass it
    a.release(10)
    a.add("F", 10, 0.6)
    assert a.take(3, 2.0) == []            # D has waited 2 s: nothing passes it
    a.release(70)
    assert ids(a.take(3, 2.1)) == ["D", "F"]


def test_oversized_request_runs_alone():
    a = Admission(budget=100)
    a.add("big", 500, 0.0)
    a.add("small", 10, 0.0)
    assert ids(a.take(2, 0.0)) == ["big"]  # nothing else runs, so it starts...
    assert ids(a.take(1, 0.1)) == []       # ...and the budget stays exhausted
    a.release(500)
    assert ids(a.take(1, 0.2)) == ["small"]


def test_large_request_runs_exclusively():
    # a request above a quarter of the budget starts only when nothing runs,
    # and nothing starts beside it; small ones share the device as before
    a = Admission(budget=100, aging_s=1.0)
    a.add("s1", 10, 0.0)
    a.add("L", 40, 0.0)
    a.add("s2", 10, 0.0)
    assert ids(a.take(4, 0.0)) == ["s1", "s2"]  # L waits for s1 to finish
    a.release(10)
    assert a.take(3, 0.1) == []                 # s2 still runs
    a.add("s3", 10, 0.2)
    assert ids(a.take(3, 0.2)) == ["s3"]        # young L: small ones pass it
    a.release(10)
    a.release(10)
    a.add("s4", 10, 0.3)
    assert ids(a.take(3, 0.3)) == ["L"]         # nothing runs: L starts, alone
    assert a.exclusive and a.take(3, 0.4) == []
    a.release(40)
    assert not a.exclusive and ids(a.take(3, 0.5)) == ["s4"]


def test_request_bytes_bounds_the_line_graph():
    h = from_edge_lists([[0, 1], [1, 2], [1, 3]], 4)
    g = (h.edge_ptr, h.edge_nodes, h.num_nodes)
    # node 1 is in 3 hyperedges: at most 3 hyperwedges, 2 row entries each
    per = 16 * 4 + 8 * 6 + 9 * 5 + 40 * 3 + 2 * 3 * 50
    assert request_bytes([g]) == per
    assert request_bytes([g, g]) == 2 * per
    assert isinstance(request_bytes([g]), int) and np.int64(request_bytes([g])) > 0
