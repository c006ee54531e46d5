"""GPU parity of MoCHy-A (Algorithm 4, hyperedge sampling) against the oracle:
hits bit-exact for the same Philox stream, estimates = hits * |E| / (3 s)."""
import numpy as np
import pytest

from oracle import cp, native
from workloads import from_edge_lists, make_config, powerlaw_hypergraph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2310_15668_amd as M
    c = M.Context(0)
    yield c
    c.close()


def gpu_a(ctx, h, s, seed, n0=0, flags=0):
    import paper_2310_15668_amd as M
    print(f"[gpu] MoCHy-A |E|={h.num_edges} s={s} seed={seed} n0={n0}", flush=True)
    g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes, flags)
    try:
        return M.mochy_count_sampled_edges(ctx, g, s, seed, n0)
    finally:
        g.close()


def check(ctx, h, s, seed, n0=0, nthreads=8):
    raw26, est26, raw431, est431 = gpu_a(ctx, h, s, seed, n0)
    o26, o431, inv, E = native.mochy_a_raw(h, s=s, seed=seed, n0=n0, nthreads=nthreads)
    assert inv == 0
    assert (raw431 == o431).all(), np.nonzero(raw431 != o431)
    assert (raw26 == o26).all()
    np.testing.assert_allclose(est26, cp.mochy_a_estimate(o26, E, s), rtol=1e-12, atol=0)
    return raw26


def test_tiny(ctx):
    h = make_config("tiny")
    for seed in (1, 2):
        check(ctx, h, 3000, seed)
    check(ctx, h, 500, 3, n0=(1 << 33) + 11)


def test_random_small_graphs(ctx):
    rng = np.random.default_rng(99)
    for trial in range(30):
        V = int(rng.integers(3, 14))
        edges = set()
        for _ in range(400):
            if len(edges) == 25:
                break
            sz = min(int(rng.integers(1, 6)), V)
            edges.add(tuple(sorted(rng.choice(V, size=sz, replace=False).tolist())))
        check(ctx, from_edge_lists(sorted(edges), V), 200, seed=trial, nthreads=2)


@pytest.mark.parametrize("seed,V,E,smax,alpha", [
    (21, 60, 800, 8, 1.2),     # long rows: N_i spans many bitmap words, many bins
    (22, 300, 2000, 20, 0.9),  # large hyperedges
    (23, 3000, 4000, 4, 1.1),  # sparse
])
def test_powerlaw_graphs(ctx, seed, V, E, smax, alpha):
    check(ctx, powerlaw_hypergraph(V, E, 1 if seed == 23 else 2, smax, 2.5, alpha, seed=seed), 2000,
          seed=seed)


def sampled_edge(n, seed, E):
    x = native.philox4x32_10([n & 0xffffffff, n >> 32, 1, 0], [seed & 0xffffffff, seed >> 32])
    return ((x[1] << 32 | x[0]) * E) >> 64


def test_scaled_and_full_medium(ctx):
    check(ctx, make_config("medium", scale=0.03), 400, 5)
    # full size: a window of 3 samples whose hyperedges have at most 3000
    # neighbours (the oracle's pair loop is quadratic in the degree)
    h = make_config("medium")
    deg, _ = native.line_graph_degrees(h, 16)
    n0 = next(n for n in range(100000)
              if all(2 <= deg[sampled_edge(n + t, 7, h.num_edges)] <= 3000 for t in range(3)))
    check(ctx, h, 3, 7, n0=n0, nthreads=16)


def test_unbiased_against_exact(ctx):
    import paper_2310_15668_amd as M
    h = make_config("medium", scale=0.03)
    g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes)
    m26, _ = M.mochy_count_exact(ctx, g)
    est = np.mean([M.mochy_count_sampled_edges(ctx, g, 4000, seed)[1] for seed in range(10)], axis=0)
    g.close()
    big = m26 > 0.01 * m26.sum()
    assert (np.abs(est[big] - m26[big]) / m26[big]).max() < 0.1


def test_errors(ctx):
    import paper_2310_15668_amd as M
    h = make_config("tiny")
    with pytest.raises(M.MochyError) as e:
        gpu_a(ctx, h, 10, 1, flags=4)  # no stored line graph
    assert e.value.status == -6
    with pytest.raises(M.MochyError) as e:
        gpu_a(ctx, h, 0, 1)
    assert e.value.status == -1
    raw26, est26, _, _ = gpu_a(ctx, from_edge_lists([[0, 1], [2, 3]], 4), 50, 1)
    assert raw26.sum() == 0 and est26.sum() == 0
