"""Pins of the oracle's exact counters: brute force, closed forms, identities."""
import numpy as np
import pytest

from oracle import native, patterns as P
from workloads import from_edge_lists, make_config
from workloads.generators import Hypergraph


def hid(regions):
    """h-motif id of a region pattern given as a set of region numbers 1..7."""
    card = [1 if (r + 1) in regions else 0 for r in range(7)]
    return P.classify_counts(card)[0]


def both(h):
    b = native.bruteforce(h, nthreads=2)
    e = native.mochy_e(h, nthreads=2)
    assert (b[1] == e[1]).all() and b[2] == e[2] == 0
    return b[0], b[1]


def only(counts26, motif, n):
    expect = np.zeros(26, dtype=np.int64)
    if n:
        expect[motif - 1] = n
    assert counts26.tolist() == expect.tolist()


@pytest.mark.parametrize("n", [3, 4, 7])
def test_sunflower(n):
    # e_a = {centre, petal_a}: every triple has R1, R2, R3, R7 non-empty
    h = from_edge_lists([[0, a] for a in range(1, n + 1)])
    c26, _ = both(h)
    assert hid({1, 2, 3, 7}) == 9
    only(c26, 9, n * (n - 1) * (n - 2) // 6)


@pytest.mark.parametrize("m", [2, 3, 5])
def test_hyperedge_covering_disjoint_pairs(m):
    edges = [list(range(1, 2 * m + 1))] + [[2 * a - 1, 2 * a] for a in range(1, m + 1)]
    c26, _ = both(from_edge_lists(edges))
    if m == 2:
        only(c26, 17, 1)  # the big hyperedge is exactly the union of the two
    else:
        only(c26, 18, m * (m - 1) // 2)  # ... plus private nodes of the big one
    assert hid({5, 6}) == 17 and hid({3, 5, 6}) == 18


@pytest.mark.parametrize("n", [3, 5, 8])
def test_strict_chain(n):
    c26, _ = both(from_edge_lists([list(range(a)) for a in range(1, n + 1)]))
    assert hid({3, 6, 7}) == 2
    only(c26, 2, n * (n - 1) * (n - 2) // 6)


def test_pairwise_triangle():
    c26, _ = both(from_edge_lists([[0, 1], [1, 2], [2, 0]]))
    assert hid({4, 5, 6}) == 23
    only(c26, 23, 1)


def test_full_venn():
    # one node in each of the seven regions
    c26, c431 = both(from_edge_lists([[1, 4, 6, 7], [2, 4, 5, 7], [3, 5, 6, 7]]))
    only(c26, 16, 1)
    # all states are "singleton": 3h id of the all-ones tuple
    assert c431[P.classify_counts([1] * 7)[1] - 1] == 1


def test_cardinality_states_of_full_venn():
    # two nodes in R7 moves the instance to another 3h-motif of the same h-motif
    h1 = from_edge_lists([[1, 4, 6, 7], [2, 4, 5, 7], [3, 5, 6, 7]])
    h2 = from_edge_lists([[1, 4, 6, 7, 8], [2, 4, 5, 7, 8], [3, 5, 6, 7, 8]])
    a, b = both(h1)[1], both(h2)[1]
    assert a.sum() == b.sum() == 1 and (a != b).any()
    assert b[P.classify_counts([1, 1, 1, 1, 1, 1, 2])[1] - 1] == 1


def test_worked_example_text_facts():
    # A hypergraph whose hyperwedges are exactly {1,2}, {1,3}, {2,3}, {1,4}
    # (section 2.1's example): {e1,e2,e3} is closed, {e1,e2,e4} and
    # {e1,e3,e4} are open and, although their pairwise overlaps agree, they
    # are different h-motifs (section 2.2).  The figure's node sets are not in
    # the text; this instance is built to have exactly those hyperwedges.
    h = from_edge_lists([[1, 2, 3, 4], [1, 2], [2, 3, 6], [4, 7]])
    deg, w = native.line_graph_degrees(h, 1)
    assert w == 4 and deg.tolist() == [3, 2, 2, 1]
    c26, _ = both(h)
    assert c26.sum() == 3
    opened = set(P.open_ids())
    got = [t + 1 for t in range(26) for _ in range(c26[t])]
    assert sum(1 for t in got if t in opened) == 2
    assert len({t for t in got if t in opened}) == 2


def random_small(rng, V=10, E=12, smax=5, smin=1):
    edges = set()
    for _ in range(50 * E):
        if len(edges) == E:
            break
        s = min(int(rng.integers(smin, smax + 1)), V)
        edges.add(tuple(sorted(rng.choice(V, size=s, replace=False).tolist())))
    edges = list(edges)
    rng.shuffle(edges)
    return from_edge_lists(edges, V)


def test_bruteforce_equals_mochy_e_on_random_small():
    rng = np.random.default_rng(11)
    for _ in range(150):
        h = random_small(rng, V=int(rng.integers(4, 12)), E=int(rng.integers(3, 14)))
        both(h)


def test_relabel_invariance():
    rng = np.random.default_rng(3)
    h = random_small(rng, V=12, E=16)
    base = both(h)[1]
    for _ in range(5):
        perm_e = rng.permutation(h.num_edges)
        perm_v = rng.permutation(h.num_nodes)
        edges = [[int(perm_v[v]) for v in h.edge(e)] for e in perm_e]
        assert (both(from_edge_lists(edges, h.num_nodes))[1] == base).all()


def test_disjoint_union_additive_and_isolated_edge_neutral():
    rng = np.random.default_rng(4)
    a = random_small(rng, V=9, E=10)
    b = random_small(rng, V=9, E=10)
    ca, cb = both(a)[1], both(b)[1]
    union = a.edges() + [[v + 9 for v in e] for e in b.edges()] + [[100, 101]]
    cu = both(from_edge_lists(union))[1]
    assert (cu == ca + cb).all()


def _identity_check(h, nthreads=4):
    c26, c431, inv = native.mochy_e(h, nthreads=nthreads)
    assert inv == 0
    deg, _ = native.line_graph_degrees(h, nthreads)
    opened = [t - 1 for t in P.open_ids()]
    so = int(c26[opened].sum())
    sc = int(c26.sum()) - so
    # Algorithm 2 visits an open instance once and a closed one three times
    assert so + 3 * sc == int((deg * (deg - 1) // 2).sum())
    # closed instances are exactly the triangles of the line graph
    assert sc == native.line_graph_triangles(h, nthreads)
    # 3h-motif counts refine h-motif counts
    assert (native.fold26(np.concatenate([[0], c431])) == c26).all()


def test_identities_on_tiny_config():
    h = make_config("tiny")
    _identity_check(h)
    b = native.bruteforce(h, nthreads=4)
    assert (b[1] == native.mochy_e(h, nthreads=4)[1]).all()


def test_identities_on_random_graphs():
    rng = np.random.default_rng(8)
    for _ in range(20):
        _identity_check(random_small(rng, V=15, E=30, smax=6), nthreads=2)


def test_centre_slices_add_up():
    h = make_config("tiny")
    full = native.mochy_e(h, nthreads=4)[1]
    cuts = [0, 37, 38, 200, 401, h.num_edges]
    parts = sum(native.mochy_e(h, c0, c1, nthreads=4)[1] for c0, c1 in zip(cuts[:-1], cuts[1:]))
    assert (parts == full).all()


def test_size_one_hyperedges_counted():
    # a size-1 hyperedge inside two others: closed triple with an empty private region
    h = from_edge_lists([[0], [0, 1], [0, 2]])
    c26, _ = both(h)
    assert c26.sum() == 1
    assert c26[hid({2, 3, 7}) - 1] == 1


def test_invalid_slot_only_for_duplicates():
    # duplicates violate the input contract; the oracle reports them in slot 0
    h = Hypergraph(np.array([0, 2, 4, 6], dtype=np.int64), np.array([0, 1, 0, 1, 1, 2], dtype=np.int32), 3)
    _, _, inv = native.bruteforce(h, nthreads=1)
    assert inv == 1
