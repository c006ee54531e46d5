"""The seeded generators: determinism, the input contract, the null model."""
import numpy as np

from workloads import make_config, powerlaw_hypergraph, stub_matching_copy
from workloads import generators as G


def _check_contract(h, smin=1, smax=None):
    sizes = h.sizes()
    assert (sizes >= smin).all()
    if smax:
        assert sizes.max() <= smax
    for e in range(h.num_edges):
        nodes = h.edge(e)
        assert (np.diff(nodes) > 0).all()
    assert h.edge_nodes.min() >= 0 and h.edge_nodes.max() < h.num_nodes
    mat = G._to_padded(h)
    assert G._first_unique_rows(mat).size == h.num_edges  # no duplicate hyperedges


def test_deterministic_and_contract():
    a = make_config("tiny")
    b = make_config("tiny")
    assert (a.edge_ptr == b.edge_ptr).all() and (a.edge_nodes == b.edge_nodes).all()
    _check_contract(a, 2, 8)
    assert 400 < a.num_edges <= 500


def test_zipf_popularity_and_size_law():
    h = powerlaw_hypergraph(2000, 20000, 2, 10, 2.5, 1.0, seed=9, dedup=False)
    deg = np.bincount(h.edge_nodes, minlength=2000)
    assert deg[0] > deg[10] > deg[1000]
    sizes = np.bincount(h.sizes(), minlength=11)
    # P(2)/P(3) = (3/2)^2.5 for the truncated power law
    assert abs(sizes[2] / sizes[3] - 1.5 ** 2.5) < 0.2


def test_stub_matching_preserves_degrees_before_collapse():
    h = make_config("tiny")
    g = stub_matching_copy(h, seed=100)
    _check_contract(g, 1)
    d0 = np.bincount(h.edge_nodes, minlength=h.num_nodes)
    d1 = np.bincount(g.edge_nodes, minlength=h.num_nodes)
    # collapse and dedup can only remove incidences
    assert (d1 <= d0).all() and d1.sum() >= 0.9 * d0.sum()
    assert g.num_edges <= h.num_edges
    # different seeds give different copies; same seed the same one
    g2 = stub_matching_copy(h, seed=101)
    g3 = stub_matching_copy(h, seed=100)
    assert not (g.edge_nodes.size == g2.edge_nodes.size and (g.edge_nodes == g2.edge_nodes).all())
    assert (g.edge_nodes == g3.edge_nodes).all()


def test_chung_lu_preserves_degrees_in_expectation():
    # E[degree of v in the incidence multiset] = d_v and E[size of e] = |e|
    from workloads import chung_lu_incidences
    h = make_config("tiny")
    deg = np.bincount(h.edge_nodes, minlength=h.num_nodes).astype(float)
    size = h.sizes().astype(float)
    R = 400
    dsum = np.zeros_like(deg)
    ssum = np.zeros_like(size)
    for seed in range(R):
        e, v = chung_lu_incidences(h, seed)
        assert e.size == v.size == h.nnz
        dsum += np.bincount(v, minlength=h.num_nodes)
        ssum += np.bincount(e, minlength=h.num_edges)
    # binomial counts: the mean over R copies has sd sqrt(d (1 - d/L) / R)
    L = h.nnz
    zd = (dsum / R - deg) / np.sqrt(np.maximum(deg * (1 - deg / L), 1e-9) / R)
    zs = (ssum / R - size) / np.sqrt(size * (1 - size / L) / R)
    assert np.abs(zd).max() < 5 and np.abs(zs).max() < 5
    assert abs(zd.mean()) < 0.3 and abs(zs.mean()) < 0.3


def test_chung_lu_copy_is_a_hypergraph():
    from workloads import chung_lu_copy
    h = make_config("tiny")
    for seed in range(5):
        g = chung_lu_copy(h, seed)
        sz = g.sizes()
        assert (sz >= 1).all() and g.num_nodes == h.num_nodes
        assert g.nnz <= h.nnz and g.num_edges <= h.num_edges
        rows = [tuple(g.edge_nodes[g.edge_ptr[x]:g.edge_ptr[x + 1]]) for x in range(g.num_edges)]
        assert all(all(a < b for a, b in zip(r, r[1:])) for r in rows)
        assert len(set(rows)) == len(rows)
