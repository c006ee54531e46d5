"""Pins of the oracle's MoCHy-A+ (Algorithm 5) and of its Philox4x32-10."""
import itertools
import math

import numpy as np
import pytest

from conftest import golden
from oracle import cp, native, patterns as P
from workloads import from_edge_lists, make_config


@pytest.mark.parametrize("row", golden("philox4x32_10_kat.txt"))
def test_philox_known_answers(row):
    vals = [int(x, 16) for x in row]
    assert native.philox4x32_10(vals[0:4], vals[4:6]) == vals[6:10]


def w_of():
    opened = set(P.open_ids())
    return np.array([2 if t in opened else 3 for t in range(1, 27)], dtype=np.int64)


def test_exhaustive_visit_equals_w_times_exact():
    # Visiting every hyperwedge once counts every instance once per hyperwedge
    # it contains: 2 for open, 3 for closed motifs (Eq. defining w[t]).
    h = make_config("tiny")
    _, wedges = native.line_graph_degrees(h, 4)
    raw26, raw431, inv, W = native.aplus_raw(h, indices=np.arange(wedges), nthreads=4)
    assert W == wedges and inv == 0
    m26, m431, _ = native.mochy_e(h, nthreads=4)
    assert (raw26 == w_of() * m26).all()
    parent = P.id3_to_id26()[1:]
    assert (raw431 == w_of()[parent - 1] * m431).all()


def _small():
    rng = np.random.default_rng(21)
    edges = set()
    while len(edges) < 11:
        s = int(rng.integers(2, 5))
        edges.add(tuple(sorted(rng.choice(9, size=s, replace=False).tolist())))
    return from_edge_lists(sorted(edges), 9)


def _instances(h):
    """(motif id, set of its hyperwedges) for every connected triple."""
    out = []
    for i, j, k in itertools.combinations(range(h.num_edges), 3):
        card = native.region_cards(h, i, j, k)
        c = P.classify_counts(card)
        if c is None:
            continue
        ij, jk, ki = card[3] + card[6] > 0, card[4] + card[6] > 0, card[5] + card[6] > 0
        if not ((ij and ki) or (ij and jk) or (jk and ki)):
            continue
        wedges = {p for p, ok in (((i, j), ij), ((j, k), jk), ((i, k), ki)) if ok}
        out.append((c[0], wedges))
    return out


def test_single_sample_distribution_matches_theorem5():
    # One sample: X = number of motif-t instances containing the hyperwedge.
    # E[X] = w M / |wedges| (unbiasedness), and r * Var of the rescaled
    # estimate equals Theorem 5's variance with q_n counted over ordered pairs
    # of distinct instances (the covariance sum in the proof runs over j != j').
    h = _small()
    _, W = native.line_graph_degrees(h, 1)
    per = np.array([native.aplus_raw(h, indices=[x], nthreads=1)[0] for x in range(W)])
    m26 = native.mochy_e(h, nthreads=1)[0]
    inst = _instances(h)
    w = w_of()
    for t in range(26):
        X = per[:, t].astype(float)
        assert X.sum() == w[t] * m26[t]
        if m26[t] == 0:
            continue
        scaled = X * W / w[t]
        var_single = scaled.var()
        mine = [s for (tid, s) in inst if tid == t + 1]
        assert len(mine) == m26[t]
        q = [0, 0]
        for a in range(len(mine)):
            for b in range(len(mine)):
                if a != b:
                    q[len(mine[a] & mine[b])] += 1
        wt = w[t]
        thm = (1 / wt) * m26[t] * (W - wt) + (1 / wt ** 2) * sum(q[n] * (n * W - wt ** 2) for n in range(2))
        assert math.isclose(var_single, thm, rel_tol=1e-9, abs_tol=1e-9), t


def test_philox_estimates_unbiased():
    h = _small()
    _, W = native.line_graph_degrees(h, 1)
    m26 = native.mochy_e(h, nthreads=1)[0]
    per = np.array([native.aplus_raw(h, indices=[x], nthreads=1)[0] for x in range(W)], dtype=float)
    r, seeds = 400, range(40)
    est = np.array([cp.aplus_estimate(native.aplus_raw(h, r=r, seed=s, nthreads=2)[0], W, r) for s in seeds])
    w = w_of()
    for t in range(26):
        if m26[t] == 0:
            assert (est[:, t] == 0).all()
            continue
        sd = (per[:, t] * W / w[t]).std() / math.sqrt(r * len(seeds))
        assert abs(est[:, t].mean() - m26[t]) <= 5 * sd + 1e-9, t


def test_index_mapping_uses_all_wedges_uniformly():
    # floor(u * W / 2^64) over many Philox draws hits every hyperwedge with
    # frequency close to 1/W
    h = _small()
    _, W = native.line_graph_degrees(h, 1)
    n = 20000
    key = [12345, 0]
    hits = np.zeros(W, dtype=np.int64)
    for c in range(n):
        x = native.philox4x32_10([c, 0, 0, 0], key)
        u = (x[1] << 32) | x[0]
        hits[(u * W) >> 64] += 1
    expected = n / W
    assert hits.min() > 0
    chi2 = float(((hits - expected) ** 2 / expected).sum())
    assert chi2 < W + 6 * math.sqrt(2 * W)


def test_prefix_additivity():
    h = make_config("tiny")
    full = native.aplus_raw(h, r=3000, seed=7, nthreads=4)[1]
    a = native.aplus_raw(h, r=1234, seed=7, n0=0, nthreads=4)[1]
    b = native.aplus_raw(h, r=3000 - 1234, seed=7, n0=1234, nthreads=4)[1]
    assert (a + b == full).all()


def test_wedge_prefix_by_brute_force():
    # up_ptr[i+1] - up_ptr[i] = |{j > i : e_i ∩ e_j non-empty}| (Algorithm 1's
    # hyperwedges, listed by their smaller hyperedge)
    rng = np.random.default_rng(5)
    for trial in range(20):
        V = int(rng.integers(3, 12))
        edges = sorted({tuple(sorted(rng.choice(V, size=int(rng.integers(1, min(V, 5) + 1)),
                                                replace=False).tolist())) for _ in range(15)})
        h = from_edge_lists(edges, V)
        up, W = native.wedge_prefix(h, 2)
        sets = [set(e) for e in edges]
        brute = [sum(1 for j in range(i + 1, len(sets)) if sets[i] & sets[j]) for i in range(len(sets))]
        assert up.tolist() == [0] + np.cumsum(brute).tolist()
        assert W == native.line_graph_degrees(h, 2)[1]


def test_sampling_with_given_order_is_unchanged():
    h = make_config("tiny")
    up, _ = native.wedge_prefix(h, 4)
    a = native.aplus_raw(h, r=3000, seed=11, n0=5, nthreads=4)
    b = native.aplus_raw(h, r=3000, seed=11, n0=5, nthreads=4, up_ptr=up)
    assert (a[1] == b[1]).all() and a[3] == b[3]
