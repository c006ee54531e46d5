"""GPU parity of the line-graph-free mode (neighbourhoods formed on demand,
section 4.4) against the oracle: hyperwedge count and MoCHy-A+ raw hits must
be bit-exact for the same Philox stream.

Every case prints what it runs before it touches the GPU.
"""
import numpy as np
import pytest

from oracle import native
from workloads import from_edge_lists, induced_prefix, make_config, powerlaw_hypergraph
from workloads.generators import Hypergraph

pytestmark = pytest.mark.gpu

LG_FREE = 4


@pytest.fixture(scope="module")
def ctx():
    import paper_2310_15668_amd as M
    c = M.Context(0)
    yield c
    c.close()


def gpu_sampled(ctx, h, r, seed, n0=0, flags=LG_FREE):
    import paper_2310_15668_amd as M
    print(f"[gpu] project flags={flags} |E|={h.num_edges} |V|={h.num_nodes} nnz={h.nnz}; "
          f"A+ r={r} seed={seed} n0={n0}", flush=True)
    g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes, flags)
    raw26, est26, raw431, est431 = M.mochy_count_sampled(ctx, g, r, seed, n0)
    w = g.num_hyperwedges
    g.close()
    return raw26, raw431, est26, w


def check(ctx, h, r, seed, n0=0, nthreads=8, up_ptr=None):
    raw26, raw431, _, w = gpu_sampled(ctx, h, r, seed, n0)
    o26, o431, inv, ow = native.aplus_raw(h, r=r, seed=seed, n0=n0, nthreads=nthreads, up_ptr=up_ptr)
    assert inv == 0
    assert w == ow
    assert (raw431 == o431).all(), np.nonzero(raw431 != o431)
    assert (raw26 == o26).all()
    return raw431


def random_graph(rng, V, E, smax):
    edges = set()
    for _ in range(40 * E):
        if len(edges) == E:
            break
        s = min(int(rng.integers(1, smax + 1)), V)
        edges.add(tuple(sorted(rng.choice(V, size=s, replace=False).tolist())))
    return from_edge_lists(list(edges), V)


def test_tiny_config(ctx):
    h = make_config("tiny")
    for seed in (1, 2):
        check(ctx, h, 20000, seed)


def test_random_small_graphs(ctx):
    # every node shared by two hyperedges is one of the 64 heavy nodes here,
    # so the bulk counts of the two skipped lists are exercised in every form
    rng = np.random.default_rng(77)
    for trial in range(40):
        h = random_graph(rng, int(rng.integers(3, 14)), int(rng.integers(2, 30)), 6)
        check(ctx, h, 500, seed=trial, nthreads=2)


@pytest.mark.parametrize("seed,V,E,smax,alpha", [
    (11, 40, 600, 8, 1.2),     # few nodes: long lists, many heavy pairs
    (12, 400, 2500, 12, 1.0),  # more than 64 shared nodes: walked lists of all lengths
    (13, 150, 1200, 25, 0.9),  # large hyperedges (up to 25 nodes)
    (14, 3000, 4000, 4, 1.1),  # sparse, ragged rows
])
def test_powerlaw_graphs(ctx, seed, V, E, smax, alpha):
    check(ctx, powerlaw_hypergraph(V, E, 1 if seed == 14 else 2, smax, 2.5, alpha, seed=seed), 20000,
          seed=seed)


def test_matches_line_graph_path(ctx):
    # the same samples through the stored rows (merged) and without them
    import paper_2310_15668_amd as M
    h = make_config("medium", scale=0.03)
    ctx.set_option(M.MOCHY_OPT_APLUS_ROWS, 1)
    try:
        a26, a431, _, wa = gpu_sampled(ctx, h, 300000, 5, flags=0)
    finally:
        ctx.set_option(M.MOCHY_OPT_APLUS_ROWS, 0)
    b26, b431, _, wb = gpu_sampled(ctx, h, 300000, 5)
    c26, c431, _, wc = gpu_sampled(ctx, h, 300000, 5, flags=0)  # rows stored, walked on the fly
    assert wa == wb == wc and (a431 == b431).all() and (c431 == b431).all()
    check(ctx, h, 4000, 5)


def test_chunks_and_offsets_add_up(ctx):
    # more samples than one chunk (2^27 with key memos, 2^25 without), and
    # split ranges summing to the whole
    h = make_config("tiny")
    r = (1 << 27) + 12345
    import paper_2310_15668_amd as M
    _, full, _, _ = gpu_sampled(ctx, h, r, 9)
    ctx.set_option(M.MOCHY_OPT_APLUS_ROWS, 1)
    try:
        _, ref, _, _ = gpu_sampled(ctx, h, r, 9, flags=0)
    finally:
        ctx.set_option(M.MOCHY_OPT_APLUS_ROWS, 0)
    assert (full == ref).all()
    _, p1, _, _ = gpu_sampled(ctx, h, 1000, 9)
    _, p2, _, _ = gpu_sampled(ctx, h, r - 1000, 9, n0=1000)
    assert (p1 + p2 == full).all()
    check(ctx, h, 3000, 9, n0=(1 << 33) + 7)


def test_degenerate_and_errors(ctx):
    import paper_2310_15668_amd as M
    for edges in ([[0]], [[0, 1], [2, 3]], [[0], [1], [2]]):
        raw26, raw431, est, w = gpu_sampled(ctx, from_edge_lists(edges, 4), 100, 1)
        assert w == 0 and raw431.sum() == 0 and est.sum() == 0
    h = make_config("tiny")
    g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes, LG_FREE)
    with pytest.raises(M.MochyError) as e:
        M.mochy_count_exact(ctx, g)
    assert e.value.status == -6
    st = M.mochy_graph_stats(ctx, g)
    deg, w = native.line_graph_degrees(h, 4)
    assert st["hyperwedges"] == w == g.num_hyperwedges
    assert st["max_line_degree"] == deg.max()
    assert st["candidates"] == int((deg * (deg - 1) // 2).sum())
    assert st["sum_deg_sq"] == int((deg * deg).sum()) and st["candidate_min_size_sum"] == -1
    g.close()
    dup = Hypergraph(np.array([0, 2, 3, 5], dtype=np.int64), np.array([0, 1, 2, 0, 1], dtype=np.int32), 3)
    with pytest.raises(M.MochyError) as e:
        gpu_sampled(ctx, dup, 10, 1)
    assert e.value.status == -2


MEMO_MODES = {  # (arena bytes, memoize every key that fits, always the skip pool)
    "none": (0, 0, 0),        # every sample enumerated on its own
    "all": (1 << 30, 1, 0),   # every key memoized
    "pool": (1 << 30, 1, 1),  # every key memoized, other sides skipping only the pool
    "tight": (2048, 1, 0),    # the first few keys (by degree) memoized, the rest enumerated
    "auto": (16 << 30, 0, 0),  # the default: keys with enough samples
}


def set_memo(ctx, mode):
    import paper_2310_15668_amd as M
    budget, every, pool = MEMO_MODES[mode]
    ctx.set_option(M.MOCHY_OPT_MEMO_BUDGET, budget)
    ctx.set_option(M.MOCHY_OPT_MEMO_ALL, every)
    ctx.set_option(M.MOCHY_OPT_MEMO_POOL, pool)


@pytest.mark.parametrize("mode", list(MEMO_MODES))
def test_memo_modes(ctx, mode):
    # key-grouped samples with memoized key counts give the same hits as the
    # oracle's per-sample enumeration, whichever keys are memoized
    set_memo(ctx, mode)
    try:
        print(f"[gpu] memo mode {mode}", flush=True)
        check(ctx, make_config("tiny"), 30000, 3)
        rng = np.random.default_rng(5)
        for trial in range(12):
            h = random_graph(rng, int(rng.integers(3, 14)), int(rng.integers(2, 30)), 6)
            check(ctx, h, 800, seed=100 + trial, nthreads=2)
        check(ctx, powerlaw_hypergraph(40, 600, 2, 8, 2.5, 1.2, seed=11), 20000, seed=4)
        check(ctx, powerlaw_hypergraph(400, 2500, 2, 12, 2.5, 1.0, seed=12), 20000, seed=5)
        check(ctx, powerlaw_hypergraph(150, 1200, 2, 25, 2.5, 0.9, seed=13), 20000, seed=6)
        h = make_config("medium", scale=0.03)
        _, via_rows, _, _ = gpu_sampled(ctx, h, 60000, 7, flags=0)  # rows stored, walked on the fly
        assert (via_rows == check(ctx, h, 60000, 7)).all()
    finally:
        set_memo(ctx, "auto")


def test_medium_full_size_prefix(ctx):
    h = make_config("medium")
    up, _ = native.wedge_prefix(h, 16)
    check(ctx, h, 3000, 1, nthreads=16, up_ptr=up)
    check(ctx, h, 1000, 1, n0=123456789, nthreads=16, up_ptr=up)


@pytest.fixture(scope="module")
def large():
    return make_config("large")


@pytest.fixture(scope="module")
def large_order(large):
    print("[oracle] hyperwedge order of the large hypergraph", flush=True)
    return native.wedge_prefix(large, 16)


def test_large_full_size_prefix(ctx, large, large_order):
    # 1.9M hyperedges: projected without a line graph automatically
    up, W = large_order
    raw431 = check(ctx, large, 400, 2, nthreads=16, up_ptr=up)
    assert raw431.sum() > 0
    check(ctx, large, 200, 2, n0=(1 << 34) + 3, nthreads=16, up_ptr=up)


def test_large_subset_exact_vs_sampled(ctx):
    # the first 200k hyperedges (with the nodes they use): exact counts through
    # the line graph, and A+ at 5% of the hyperwedges, both on the device
    import paper_2310_15668_amd as M
    h = induced_prefix(make_config("large"), 200000)
    print(f"[gpu] large subset |E|={h.num_edges} exact + A+ 5%", flush=True)
    g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes)
    W = g.num_hyperwedges
    c26, _ = M.mochy_count_exact(ctx, g)
    g.close()
    r = W * 5 // 100
    _, _, est26, w2 = gpu_sampled(ctx, h, r, 2)
    assert w2 == W
    big = c26 > 1e-3 * c26.sum()
    rel = np.abs(est26[big] - c26[big]) / c26[big]
    print("relative errors of the frequent h-motifs:", np.round(rel, 4).tolist(), flush=True)
    assert rel.max() < 0.05
