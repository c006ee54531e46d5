"""GPU parity of hyperedge profiles (section 3.2: for each hyperedge, the
instances of every motif that contain it) against the oracle, bit-exact, and
the identity that each motif's column sums to 3 times its exact count.

Every case prints what it runs before it touches the GPU.
"""
import numpy as np
import pytest

from oracle import native
from workloads import chung_lu_copy, from_edge_lists, make_config, powerlaw_hypergraph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2310_15668_amd as M
    c = M.Context(0)
    yield c
    c.close()


def gpu_profiles(ctx, h, c0=0, c1=None, with_431=True):
    import paper_2310_15668_amd as M
    print(f"[gpu] profiles |E|={h.num_edges} nnz={h.nnz} rows [{c0}, {c1})", flush=True)
    g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes)
    try:
        return M.mochy_hyperedge_profiles(ctx, g, c0, c1, with_431)
    finally:
        g.close()


def check(ctx, h, c0=0, c1=None, nthreads=8):
    c1 = h.num_edges if c1 is None else c1
    p26, p431 = gpu_profiles(ctx, h, c0, c1)
    o26, o431, inv = native.hyperedge_profiles(h, c0, c1, nthreads=nthreads)
    assert (inv == 0).all()
    assert p26.shape == (c1 - c0, 26) and p431.shape == (c1 - c0, 431)
    assert (p431 == o431).all(), np.argwhere(p431 != o431)[:5]
    assert (p26 == o26).all()
    return p26, p431


def exact(ctx, h):
    import paper_2310_15668_amd as M
    g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes)
    try:
        return M.mochy_count_exact(ctx, g)
    finally:
        g.close()


def test_tiny_and_column_sums(ctx):
    h = make_config("tiny")
    p26, p431 = check(ctx, h)
    c26, c431 = exact(ctx, h)
    assert (p26.sum(axis=0) == 3 * c26).all()
    assert (p431.sum(axis=0) == 3 * c431).all()


def test_hand_example(ctx):
    # three hyperedges sharing node 0 only pairwise otherwise: one instance,
    # containing each of them once
    h = from_edge_lists([[0, 1], [0, 2], [0, 3]], 4)
    p26, _ = check(ctx, h)
    assert (p26.sum(axis=1) == 1).all()
    assert (p26 == p26[0]).all()


def test_random_small_graphs(ctx):
    rng = np.random.default_rng(123)
    for trial in range(30):
        V = int(rng.integers(3, 14))
        edges = set()
        for _ in range(400):
            if len(edges) == 25:
                break
            sz = min(int(rng.integers(1, 6)), V)
            edges.add(tuple(sorted(rng.choice(V, size=sz, replace=False).tolist())))
        h = from_edge_lists(sorted(edges), V)
        p26, p431 = check(ctx, h, nthreads=2)
        c26, _ = exact(ctx, h)
        assert (p26.sum(axis=0) == 3 * c26).all()


@pytest.mark.parametrize("seed,V,E,smax,alpha", [
    (31, 60, 500, 8, 1.2),     # dense: long rows
    (32, 400, 1200, 12, 1.0),  # ragged rows
    (33, 150, 800, 25, 0.9),   # hyperedges up to 25 nodes
])
def test_powerlaw_graphs(ctx, seed, V, E, smax, alpha):
    h = powerlaw_hypergraph(V, E, 2, smax, 2.5, alpha, seed=seed)
    p26, p431 = check(ctx, h)
    c26, c431 = exact(ctx, h)
    assert (p431.sum(axis=0) == 3 * c431).all()


def test_ranges_and_empty(ctx):
    h = powerlaw_hypergraph(300, 1500, 2, 10, 2.5, 1.0, seed=34)
    full26, full431 = gpu_profiles(ctx, h)
    a26, a431 = check(ctx, h, 0, 700)
    b26, b431 = check(ctx, h, 700, h.num_edges)
    assert (np.vstack([a431, b431]) == full431).all() and (np.vstack([a26, b26]) == full26).all()
    e26, e431 = gpu_profiles(ctx, h, 5, 5)
    assert e26.shape == (0, 26) and e431.shape == (0, 431)
    only26, none431 = gpu_profiles(ctx, h, 100, 200, with_431=False)
    assert none431 is None and (only26 == full26[100:200]).all()


def test_chung_lu_copy(ctx):
    h = chung_lu_copy(make_config("tiny"), seed=5)
    check(ctx, h)


def test_more_rows_than_one_chunk(ctx):
    # 2^16 rows per device chunk: a range across the chunk edge, sampled rows
    # checked against the oracle one by one
    h = powerlaw_hypergraph(200000, 72000, 2, 6, 2.5, 0.5, seed=35)  # no hubs: cheap rows
    assert h.num_edges > 70000
    p26, _ = gpu_profiles(ctx, h, 0, 70000, with_431=False)
    rng = np.random.default_rng(7)
    for x in sorted(rng.choice(70000, size=6, replace=False).tolist()) + [65535, 65536]:
        o26, _, inv = native.hyperedge_profiles(h, x, x + 1, nthreads=16)
        assert inv[0] == 0 and (o26[0] == p26[x]).all(), x


def test_errors(ctx):
    import paper_2310_15668_amd as M
    h = make_config("tiny")
    g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes, M.MOCHY_LG_FREE)
    with pytest.raises(M.MochyError) as e:
        M.mochy_hyperedge_profiles(ctx, g)
    assert e.value.status == -6
    g.close()
    g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes)
    for c0, c1 in ((-1, 3), (4, 3), (0, h.num_edges + 1)):
        with pytest.raises(M.MochyError) as e:
            M.mochy_hyperedge_profiles(ctx, g, c0, c1)
        assert e.value.status == -1
    g.close()
