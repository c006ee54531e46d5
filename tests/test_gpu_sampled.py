"""GPU parity of MoCHy-A+ (Algorithm 5) against the oracle under the same Philox seed.

Raw hit counts must be bit-exact (int64); the float64 estimates are compared
against the oracle's rescaling of the oracle's hits within 1e-12 relative.
Both enumerations of N_i ∪ N_j are checked: on the fly from the node lists
(default) and by merging the stored rows (MOCHY_OPT_APLUS_ROWS).
"""
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


def gpu_sampled(ctx, h, r, seed, n0=0, rows=False):
    import paper_2310_15668_amd as M
    print(f"[gpu] A+ |E|={h.num_edges} r={r} seed={seed} n0={n0} rows={rows}", flush=True)
    g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes)
    ctx.set_option(M.MOCHY_OPT_APLUS_ROWS, int(rows))
    try:
        out = M.mochy_count_sampled(ctx, g, r, seed, n0)
    finally:
        ctx.set_option(M.MOCHY_OPT_APLUS_ROWS, 0)
    w = g.num_hyperwedges
    g.close()
    return out, w


def check(ctx, h, r, seed, n0=0, nthreads=8, rows=False):
    (raw26, est26, raw431, est431), w = gpu_sampled(ctx, h, r, seed, n0, rows)
    o26, o431, inv, ow = native.aplus_raw(h, r=r, seed=seed, n0=n0, nthreads=nthreads)
    assert inv == 0 and ow == w
    assert (raw431 == o431).all(), np.nonzero(raw431 != o431)
    assert (raw26 == o26).all()
    ref26 = np.array(cp.aplus_estimate(o26, ow, r))
    ref431 = np.array(cp.aplus_estimate3(o431, ow, r))
    np.testing.assert_allclose(est26, ref26, rtol=1e-12, atol=0)
    np.testing.assert_allclose(est431, ref431, rtol=1e-12, atol=0)
    return raw431


def test_tiny_same_seed(ctx):
    h = make_config("tiny")
    for seed in (0, 7, 2 ** 40 + 123):
        check(ctx, h, 5000, seed)
        check(ctx, h, 5000, seed, rows=True)


def test_prefix_offsets_add_up(ctx):
    h = make_config("tiny")
    full = check(ctx, h, 4000, 11)
    a = check(ctx, h, 1500, 11, n0=0)
    b = check(ctx, h, 2500, 11, n0=1500)
    assert (a + b == full).all()
    # counters above 2^32 use both counter words
    check(ctx, h, 700, 11, n0=2 ** 33 + 5)


def test_random_and_powerlaw(ctx):
    rng = np.random.default_rng(99)
    for _ in range(15):
        V = int(rng.integers(5, 15))
        E = int(rng.integers(3, 25))
        edges = set()
        for _ in range(40 * E):
            if len(edges) == E:
                break
            s = min(int(rng.integers(1, 6)), V)
            edges.add(tuple(sorted(rng.choice(V, size=s, replace=False).tolist())))
        check(ctx, from_edge_lists(list(edges), V), 300, int(rng.integers(0, 2 ** 63)), nthreads=2)
    check(ctx, powerlaw_hypergraph(300, 1500, 2, 12, 2.5, 0.8, seed=6), 3000, 5)
    check(ctx, make_config("medium", scale=0.03), 20000, 3)


def test_no_hyperwedges(ctx):
    h = from_edge_lists([[0, 1], [2, 3]], 4)
    (raw26, est26, raw431, est431), w = gpu_sampled(ctx, h, 100, 1)
    assert w == 0 and raw26.sum() == 0 and est26.sum() == 0.0


def test_unbiased_against_exact(ctx):
    # mean of A+ estimates over seeds vs MoCHy-E counts of the same graph
    import paper_2310_15668_amd as M
    h = powerlaw_hypergraph(200, 800, 2, 8, 2.5, 1.0, seed=12)
    g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes)
    exact26, _ = M.mochy_count_exact(ctx, g)
    r = g.num_hyperwedges // 10
    ests = np.array([M.mochy_count_sampled(ctx, g, r, s)[1] for s in range(30)])
    g.close()
    big = exact26 > 1000
    rel = np.abs(ests.mean(axis=0)[big] - exact26[big]) / exact26[big]
    assert rel.max() < 0.05, rel
    # relative error as defined in section 6.7, per seed
    err = np.abs(ests - exact26).sum(axis=1) / exact26.sum()
    assert err.mean() < 0.1


@pytest.mark.slow
def test_medium_full_size_prefix(ctx):
    # full-size medium hypergraph: a prefix of samples checked hit by hit
    check(ctx, make_config("medium"), 300, 2, nthreads=16)
