"""GPU parity of the exact counter (projection + MoCHy-E) against the oracle.

Integer counts must be bit-exact.  Every case prints what it runs before it
touches the GPU.
"""
import numpy as np
import pytest

from oracle import native
from workloads import from_edge_lists, make_config, powerlaw_hypergraph
from workloads.generators import Hypergraph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2310_15668_amd as M
    c = M.Context(0)
    yield c
    c.close()


def gpu_counts(ctx, h, flags=0):
    import paper_2310_15668_amd as M
    print(f"[gpu] project+exact |E|={h.num_edges} |V|={h.num_nodes} nnz={h.nnz}", flush=True)
    g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes, flags)
    c26, c431 = M.mochy_count_exact(ctx, g)
    w = g.num_hyperwedges
    g.close()
    return c26, c431, w


def check(ctx, h, nthreads=8):
    c26, c431, w = gpu_counts(ctx, h)
    r26, r431, inv = native.mochy_e(h, nthreads=nthreads)
    _, rw = native.line_graph_degrees(h, nthreads)
    assert inv == 0
    assert w == rw
    assert (c431 == r431).all(), np.nonzero(c431 != r431)
    assert (c26 == r26).all()
    return c26


def test_tiny_config(ctx):
    h = make_config("tiny")
    c26 = check(ctx, h)
    b26, b431, _ = native.bruteforce(h, nthreads=8)
    assert (c26 == b26).all()


def test_closed_forms(ctx):
    cases = [
        ([[0, a] for a in range(1, 9)], 9, 56),                             # sunflower
        ([list(range(a)) for a in range(1, 7)], 2, 20),                     # strict chain
        ([[0, 1], [1, 2], [2, 0]], 23, 1),                                  # pairwise triangle
        ([[1, 4, 6, 7], [2, 4, 5, 7], [3, 5, 6, 7]], 16, 1),                # full Venn
        ([list(range(1, 11))] + [[2 * a - 1, 2 * a] for a in range(1, 6)], 18, 10),
    ]
    for edges, motif, n in cases:
        c26, _, _ = gpu_counts(ctx, from_edge_lists(edges))
        expect = np.zeros(26, dtype=np.int64)
        expect[motif - 1] = n
        assert (c26 == expect).all(), (edges, c26)


def test_random_small_graphs(ctx):
    rng = np.random.default_rng(2024)
    for trial in range(40):
        V = int(rng.integers(4, 16))
        E = int(rng.integers(2, 30))
        edges = set()
        for _ in range(40 * E):
            if len(edges) == E:
                break
            s = min(int(rng.integers(1, 7)), V)
            edges.add(tuple(sorted(rng.choice(V, size=s, replace=False).tolist())))
        check(ctx, from_edge_lists(list(edges), V), nthreads=2)


@pytest.mark.parametrize("seed,V,E,smax,alpha", [
    (5, 60, 400, 6, 1.0),     # hub rows span several 64-blocks
    (6, 300, 1500, 12, 0.8),  # many light nodes shared outside the centre
    (7, 120, 900, 25, 1.2),   # large hyperedges, masks up to 25 bits
    (8, 2000, 3000, 4, 1.0),  # sparse, ragged rows
])
def test_powerlaw_graphs(ctx, seed, V, E, smax, alpha):
    check(ctx, powerlaw_hypergraph(V, E, 1 if seed == 8 else 2, smax, 2.5, alpha, seed=seed))


def test_scaled_medium(ctx):
    check(ctx, make_config("medium", scale=0.03))


def test_degenerate_inputs(ctx):
    for edges in ([], [[0]], [[0, 1]], [[0, 1], [2, 3]], [[0, 1], [1, 2]]):
        h = from_edge_lists(edges, 4)
        c26, c431, w = gpu_counts(ctx, h)
        assert c26.sum() == 0 and c431.sum() == 0


def test_errors(ctx):
    import paper_2310_15668_amd as M
    dup = Hypergraph(np.array([0, 2, 4], dtype=np.int64), np.array([0, 1, 0, 1], dtype=np.int32), 3)
    with pytest.raises(M.MochyError) as e:
        gpu_counts(ctx, dup)
    assert e.value.status == -2
    # with MOCHY_DEDUP the repeat is dropped
    c26, _, w = gpu_counts(ctx, Hypergraph(np.array([0, 2, 4, 6], dtype=np.int64),
                                           np.array([0, 1, 0, 1, 1, 2], dtype=np.int32), 3), flags=1)
    assert w == 1 and c26.sum() == 0
    unsorted = Hypergraph(np.array([0, 2], dtype=np.int64), np.array([1, 0], dtype=np.int32), 3)
    with pytest.raises(M.MochyError) as e:
        gpu_counts(ctx, unsorted)
    assert e.value.status == -1
    big = from_edge_lists([list(range(40))])
    with pytest.raises(M.MochyError) as e:
        gpu_counts(ctx, big)
    assert e.value.status == -3


def test_device_input_matches_host_input(ctx):
    import torch
    import paper_2310_15668_amd as M
    h = make_config("tiny")
    p = torch.from_numpy(h.edge_ptr).cuda()
    n = torch.from_numpy(h.edge_nodes).cuda()
    torch.cuda.synchronize()
    print("[gpu] device-resident CSR", flush=True)
    g = M.mochy_project(ctx, p, n, h.num_nodes)
    d26, d431 = M.mochy_count_exact(ctx, g)
    g.close()
    c26, c431, _ = gpu_counts(ctx, h)
    assert (d431 == c431).all()
    # device-side validation rejects a duplicate
    n2 = n.clone()
    bad_p = torch.tensor([0, 2, 4], dtype=torch.int64, device="cuda")
    bad_n = torch.tensor([0, 1, 0, 1], dtype=torch.int32, device="cuda")
    with pytest.raises(M.MochyError) as e:
        M.mochy_project(ctx, bad_p, bad_n, 2)
    assert e.value.status == -2
    del n2


def test_centre_ranges_add_up(ctx):
    import paper_2310_15668_amd as M
    h = make_config("tiny")
    g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes)
    full = M.mochy_count_exact(ctx, g)[1]
    cuts = [0, 1, 63, 64, 200, h.num_edges]
    parts = [M.mochy_count_exact_range(ctx, g, a, b)[1] for a, b in zip(cuts[:-1], cuts[1:])]
    for (a, b), part in zip(zip(cuts[:-1], cuts[1:]), parts):
        assert (part == native.mochy_e(h, a, b, nthreads=4)[1]).all()
    assert (sum(parts) == full).all()
    again = M.mochy_count_exact(ctx, g)[1]
    assert (again == full).all()  # deterministic
    g.close()


@pytest.fixture(scope="module")
def medium():
    return make_config("medium")


@pytest.fixture(scope="module")
def medium_graph(ctx, medium):
    import paper_2310_15668_amd as M
    print("[gpu] project full medium hypergraph", flush=True)
    g = M.mochy_project(ctx, medium.edge_ptr, medium.edge_nodes, medium.num_nodes)
    yield g
    g.close()


def test_medium_full_size_centre_slices(ctx, medium, medium_graph):
    # Algorithm 2 attributes each instance to one centre, so any centre range
    # of the full-size graph can be checked against the oracle exactly.
    import paper_2310_15668_amd as M
    deg, w = native.line_graph_degrees(medium, 16)
    assert w == medium_graph.num_hyperwedges
    cand = deg * (deg - 1) // 2
    hubby = int(np.argmin(np.abs(deg - 8000)))  # a centre with ~3e7 pairs, many 64-blocks
    ranges = [(hubby, hubby + 1)]
    csum = np.concatenate([[0], np.cumsum(cand)])
    for a in range(0, medium.num_edges - 8, 997):  # 8-centre windows of moderate size
        if 2e7 <= csum[a + 8] - csum[a] <= 2.5e8:
            ranges.append((a, a + 8))
        if len(ranges) == 3:
            break
    for a, b in ranges:
        print(f"[gpu] medium centres [{a},{b}) candidates={int(cand[a:b].sum())}", flush=True)
        g26, g431 = M.mochy_count_exact_range(ctx, medium_graph, a, b)
        r26, r431, inv = native.mochy_e(medium, a, b, nthreads=16)
        assert inv == 0 and (g431 == r431).all() and (g26 == r26).all(), (a, b)


def test_medium_full_size_identity(ctx, medium, medium_graph):
    # each open instance is one candidate of Algorithm 2, each closed one three
    import paper_2310_15668_amd as M
    deg, _ = native.line_graph_degrees(medium, 16)
    print("[gpu] full medium exact count", flush=True)
    c26, c431 = M.mochy_count_exact(ctx, medium_graph)
    opened = [t - 1 for t in range(17, 23)]
    so = int(c26[opened].sum())
    sc = int(c26.sum()) - so
    assert so + 3 * sc == int((deg * (deg - 1) // 2).sum())
    assert (native.fold26(np.concatenate([[0], c431])) == c26).all()


def test_grouped_equals_every_pair(ctx):
    # neighbour groups (default) and pairing every record give the same counts
    import paper_2310_15668_amd as M
    star = [[0, a] for a in range(1, 3000)] + [[a, a + 1] for a in range(1, 2999, 2)]
    cases = [make_config("tiny"), make_config("medium", scale=0.03),
             powerlaw_hypergraph(60, 3000, 2, 6, 2.5, 1.0, seed=9),  # long rows, few distinct records
             from_edge_lists(star, 3000)]                               # one hub row of 2999 neighbours
    for h in cases:
        print(f"[gpu] grouped vs every pair |E|={h.num_edges}", flush=True)
        g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes)
        try:
            ctx.set_option(M.MOCHY_OPT_GROUPS, 0)
            a26, a431 = M.mochy_count_exact(ctx, g)
            ctx.set_option(M.MOCHY_OPT_GROUPS, 1)
            b26, b431 = M.mochy_count_exact(ctx, g)
            cuts = [0, h.num_edges // 3, h.num_edges]
            parts = [M.mochy_count_exact_range(ctx, g, x, y)[1] for x, y in zip(cuts[:-1], cuts[1:])]
            # groups counted first and allocated exactly (the layout of large batches)
            ctx.set_option(M.MOCHY_OPT_GROUP_CAPACITY, 0)
            c26, c431 = M.mochy_count_exact(ctx, g)
            cparts = [M.mochy_count_exact_range(ctx, g, x, y)[1] for x, y in zip(cuts[:-1], cuts[1:])]
        finally:
            ctx.set_option(M.MOCHY_OPT_GROUPS, 1)
            ctx.set_option(M.MOCHY_OPT_GROUP_CAPACITY, 24 << 30)
            g.close()
        assert (a431 == b431).all() and (a26 == b26).all()
        assert (c431 == b431).all() and (c26 == b26).all()
        assert (sum(parts) == b431).all() and (sum(cparts) == b431).all()
        r26, r431, _ = native.mochy_e(h, nthreads=8)
        assert (b431 == r431).all()
    with pytest.raises(M.MochyError) as e:
        ctx.set_option(M.MOCHY_OPT_GROUPS, 2)
    assert e.value.status == -1


def test_grouping_parts_double(ctx):
    # a centre e_0 (nodes 0..24) whose 7,080 neighbours all have distinct
    # signatures: each neighbour holds one of the centre nodes 0..3 and a
    # distinct pair of the 60 nodes 100..159 (with nodes 0..3 the 64
    # highest-degree nodes, so every pair is a distinct heavy mask); the row's
    # one hash part passes the per-part group limit and is regrouped with two,
    # in the one-pass layout and in the counted-first one
    import itertools
    import paper_2310_15668_amd as M
    heavy = list(range(100, 160))
    edges = [list(range(25))] + [[a, h1, h2] for a in range(4) for h1, h2 in itertools.combinations(heavy, 2)]
    h = from_edge_lists(edges, 160)
    print(f"[gpu] distinct-signature hub row |E|={h.num_edges}", flush=True)
    o26, o431, inv = native.mochy_e_centers(h, [0], nthreads=1)
    assert inv == 0 and o26.sum() > 0
    g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes)
    try:
        a26, a431 = M.mochy_count_exact_range(ctx, g, 0, 1)
        st = M.mochy_exact_stats(ctx)
        assert st["rows_regrouped"] == 1 and st["max_hash_parts"] == 2, st
        full_a = M.mochy_count_exact(ctx, g)[1]
        ctx.set_option(M.MOCHY_OPT_GROUP_CAPACITY, 0)
        b26, b431 = M.mochy_count_exact_range(ctx, g, 0, 1)
        assert M.mochy_exact_stats(ctx)["rows_regrouped"] == 1
        full_b = M.mochy_count_exact(ctx, g)[1]
        ctx.set_option(M.MOCHY_OPT_GROUPS, 0)
        c26, c431 = M.mochy_count_exact_range(ctx, g, 0, 1)
        full_c = M.mochy_count_exact(ctx, g)[1]
    finally:
        ctx.set_option(M.MOCHY_OPT_GROUPS, 1)
        ctx.set_option(M.MOCHY_OPT_GROUP_CAPACITY, 24 << 30)
        g.close()
    for x26, x431 in ((a26, a431), (b26, b431), (c26, c431)):
        assert (x431 == o431).all() and (x26 == o26).all()
    assert (full_a == full_c).all() and (full_b == full_c).all()


def test_which_selector(ctx):
    # `which` selects outputs only: every selection gives the same numbers
    import paper_2310_15668_amd as M
    h = make_config("tiny")
    g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes)
    try:
        a26, a431 = M.mochy_count_exact(ctx, g)
        b26, b431 = M.mochy_count_exact(ctx, g, M.MOCHY_H26)
        c26, c431 = M.mochy_count_exact_range(ctx, g, 0, h.num_edges, M.MOCHY_H431)
        assert b431 is None and c26 is None
        assert (b26 == a26).all() and (c431 == a431).all()
        s26, e26, s431, e431 = M.mochy_count_sampled(ctx, g, 500, 3, which=M.MOCHY_H431)
        assert s26 is None and e26 is None
        f26, _, f431, _ = M.mochy_count_sampled(ctx, g, 500, 3)
        assert (s431 == f431).all()
        for bad in (0, 4, 7):
            with pytest.raises(M.MochyError) as e:
                M.mochy_count_exact(ctx, g, bad)
            assert e.value.status == -1
    finally:
        g.close()


def test_canonicalize_flag(ctx):
    # unsorted node lists with repeated members are read as node sets
    import paper_2310_15668_amd as M
    h = make_config("tiny")
    rng = np.random.default_rng(11)
    ptr, nodes = [0], []
    for e in range(h.num_edges):
        row = h.edge(e).tolist()
        row = row + row[:int(rng.integers(0, len(row) + 1))]  # repeats
        rng.shuffle(row)
        nodes.extend(row)
        ptr.append(len(nodes))
    messy = Hypergraph(np.array(ptr, dtype=np.int64), np.array(nodes, dtype=np.int32), h.num_nodes)
    with pytest.raises(M.MochyError) as e:
        gpu_counts(ctx, messy)
    assert e.value.status == -1
    c26, c431, w = gpu_counts(ctx, messy, flags=M.MOCHY_CANONICALIZE)
    r26, r431, rw = gpu_counts(ctx, h)
    assert w == rw and (c431 == r431).all()
    # 40 distinct nodes stay too many after canonicalization; 33 repeats of 30 do not
    with pytest.raises(M.MochyError) as e:
        gpu_counts(ctx, from_edge_lists([list(range(40))]), flags=M.MOCHY_CANONICALIZE)
    assert e.value.status == -3
    rep = Hypergraph(np.array([0, 33, 35], dtype=np.int64),
                     np.array(list(range(30)) + [0, 1, 2] + [0, 40], dtype=np.int32), 41)
    c26, _, w = gpu_counts(ctx, rep, flags=M.MOCHY_CANONICALIZE)
    assert w == 1 and c26.sum() == 0


def test_size_limit(ctx):
    # hyperedges of up to 32 nodes are accepted, 33 are MOCHY_ERANGE
    import paper_2310_15668_amd as M
    edges = [list(range(32)), list(range(16, 48)), [0, 47], list(range(100, 132))]
    h = from_edge_lists(edges, 140)
    c26, c431, w = gpu_counts(ctx, h)
    r26, r431, _ = native.mochy_e(h, nthreads=2)
    assert (c431 == r431).all() and w == 3
    with pytest.raises(M.MochyError) as e:
        gpu_counts(ctx, from_edge_lists([list(range(33)), [0, 1]], 40))
    assert e.value.status == -3


def test_row_capacity_fallback(ctx):
    # the one-pass grouping's row-capacity allocation made to fail: the
    # counted-first layout gives the same counts
    import paper_2310_15668_amd as M
    h = make_config("medium", scale=0.03)
    print(f"[gpu] forced counted-first fallback |E|={h.num_edges}", flush=True)
    g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes)
    try:
        a26, a431 = M.mochy_count_exact(ctx, g)
        ctx.set_option(M.MOCHY_OPT_TEST_FAULTS, 1)
        b26, b431 = M.mochy_count_exact(ctx, g)
    finally:
        ctx.set_option(M.MOCHY_OPT_TEST_FAULTS, 0)
        g.close()
    assert (a431 == b431).all() and (a26 == b26).all()
    with pytest.raises(M.MochyError):
        ctx.set_option(M.MOCHY_OPT_TEST_FAULTS, 32)


def test_wide_pair_weights(ctx):
    # the pair kernel's 48-bit weights from unpacked group counts (taken
    # when a row reaches 2^16 neighbours) forced on graphs whose counts fit
    # 16 bits: same counts
    import paper_2310_15668_amd as M
    for h in (make_config("medium", scale=0.03), powerlaw_hypergraph(300, 2000, 2, 20, 2.5, 0.9, seed=23)):
        print(f"[gpu] 64-bit pair weights |E|={h.num_edges}", flush=True)
        g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes)
        try:
            a26, a431 = M.mochy_count_exact(ctx, g)
            ctx.set_option(M.MOCHY_OPT_TEST_FAULTS, 16)
            b26, b431 = M.mochy_count_exact(ctx, g)
        finally:
            ctx.set_option(M.MOCHY_OPT_TEST_FAULTS, 0)
            g.close()
        assert int(b431.sum()) > 0
        assert (a431 == b431).all() and (a26 == b26).all()


def test_light_pairs_two_passes(ctx):
    # the correction's light pairs listed by a counting and a filling pass
    # instead of the flat candidate list: same pairs, same counts
    import paper_2310_15668_amd as M
    for h in (make_config("medium", scale=0.03), powerlaw_hypergraph(300, 2000, 2, 20, 2.5, 0.9, seed=22)):
        print(f"[gpu] light pairs in two passes |E|={h.num_edges}", flush=True)
        g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes)
        try:
            a26, a431 = M.mochy_count_exact(ctx, g)
            sa = M.mochy_exact_stats(ctx)
            ctx.set_option(M.MOCHY_OPT_TEST_FAULTS, 8)
            b26, b431 = M.mochy_count_exact(ctx, g)
            sb = M.mochy_exact_stats(ctx)
        finally:
            ctx.set_option(M.MOCHY_OPT_TEST_FAULTS, 0)
            g.close()
        assert sa["light_pairs"] > 0 and sa["light_pairs"] == sb["light_pairs"]
        assert sa["fix_centres"] == sb["fix_centres"] and sa["fix_changed"] == sb["fix_changed"]
        assert (a431 == b431).all() and (a26 == b26).all()


def test_exact_stats(ctx):
    # the work counters of the last exact call are consistent with the graph
    import paper_2310_15668_amd as M
    h = make_config("medium", scale=0.03)
    g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes)
    try:
        M.mochy_count_exact(ctx, g)
        st = M.mochy_exact_stats(ctx)
        gs = M.mochy_graph_stats(ctx, g)
        ctx.set_option(M.MOCHY_OPT_GROUPS, 0)
        M.mochy_count_exact(ctx, g)
        st0 = M.mochy_exact_stats(ctx)
    finally:
        ctx.set_option(M.MOCHY_OPT_GROUPS, 1)
        g.close()
    deg, _ = native.line_graph_degrees(h, 4)
    assert st["rows_grouped"] == h.num_edges
    assert 0 < st["groups_above"] <= st["groups"] <= 2 * gs["hyperwedges"]
    assert st["group_pairs_full"] + st["group_pairs_open"] <= int((deg * (deg - 1) // 2).sum())
    assert st["max_hash_parts"] >= 1
    assert st["light_pairs"] > 0 and 0 < st["fix_changed"] <= st["fix_centres"] <= st["fix_scanned"]
    # without groups only the correction's counters are set, to the same values
    assert st0["groups"] == 0 and st0["group_pairs_full"] == 0
    for k in ("light_pairs", "fix_scanned", "fix_centres", "fix_changed"):
        assert st0[k] == st[k], k


def test_valu_calibration(ctx):
    # the integer VALU calibration launch: its instruction count is the
    # written-out one and its rate a plausible one; bad arguments are refused
    import torch
    import paper_2310_15668_amd as M
    print("[gpu] VALU calibration, 256 rounds", flush=True)
    ms, ops = M.mochy_calibrate_valu(ctx, 256)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert ops == cus * 8 * 256 * 256 * 32  # 8 blocks of 256 threads per CU, 32 per round
    assert ms > 0.0
    assert ops / (ms * 1e-3) < 2.0 * cus * 64 * 2.4e9  # below twice the one-per-cycle rate
    for bad in (0, -1, (1 << 32) + 1):
        with pytest.raises(M.MochyError):
            M.mochy_calibrate_valu(ctx, bad)
