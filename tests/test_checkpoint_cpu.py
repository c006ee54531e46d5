"""Resumable exact counting over centre ranges (paper_2310_15668_amd/checkpoint.py),
with the oracle's plain MoCHy-E as the range counter: an interrupted count
resumes to the same integers, from any chunk size, and a checkpoint of
another hypergraph is refused."""
import json

import numpy as np
import pytest

from oracle import native
from paper_2310_15668_amd import checkpoint as ck
from workloads import make_config


def counter(h, log):
    def count(a, b):
        log.append((a, b))
        c26, c431, inv = native.mochy_e(h, a, b, nthreads=2)
        assert inv == 0
        return c26, c431
    return count


def test_interrupted_count_resumes_to_the_same_integers(tmp_path):
    h = make_config("tiny")
    key = ck.csr_key(h.edge_ptr, h.edge_nodes, h.num_nodes)
    path = str(tmp_path / "tiny.ckpt")
    full26, full431, _ = native.mochy_e(h, nthreads=2)
    log = []
    assert ck.count_exact_resumable(counter(h, log), h.num_edges, key, path, 50, stop_after=3) is None
    assert log == [(0, 50), (50, 100), (100, 150)]
    state = json.load(open(path))
    assert state["next_centre"] == 150
    # resumed with another chunk size: continues at centre 150
    log2 = []
    c26, c431 = ck.count_exact_resumable(counter(h, log2), h.num_edges, key, path, 64)
    assert log2[0] == (150, 192) and log2[-1][1] == h.num_edges
    assert (c26 == full26).all() and (c431 == full431).all()
    # a finished checkpoint counts nothing more
    log3 = []
    c26b, c431b = ck.count_exact_resumable(counter(h, log3), h.num_edges, key, path, 64)
    assert log3 == [] and (c431b == full431).all()


def test_checkpoint_of_another_hypergraph_is_refused(tmp_path):
    h = make_config("tiny")
    other = make_config("medium", scale=0.01)
    path = str(tmp_path / "x.ckpt")
    key = ck.csr_key(h.edge_ptr, h.edge_nodes, h.num_nodes)
    ck.count_exact_resumable(counter(h, []), h.num_edges, key, path, 100, stop_after=1)
    with pytest.raises(ValueError):
        ck.count_exact_resumable(counter(other, []), other.num_edges,
                                 ck.csr_key(other.edge_ptr, other.edge_nodes, other.num_nodes), path, 100)
    with pytest.raises(ValueError):
        ck.ranges(10, 0)
    assert ck.ranges(5, 2) == [(0, 2), (2, 4), (4, 5)]

