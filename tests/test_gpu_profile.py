"""GPU parity of significance / characteristic profile (Eq. 1, Eq. 2) and of the
batched count of a hypergraph with its randomized copies.

Counts: bit-exact (int64) against the oracle and against one-graph-at-a-time
launches.  Significance and CP: within 1e-12 relative of the float64 oracle.
"""
import numpy as np
import pytest

from oracle import cp, native
from workloads import from_edge_lists, make_config, powerlaw_hypergraph, stub_matching_copy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2310_15668_amd as M
    c = M.Context(0)
    yield c
    c.close()


def run_profile(ctx, graphs, eps=1.0):
    import paper_2310_15668_amd as M
    print(f"[gpu] profile of {len(graphs)} graphs, |E| = {[h.num_edges for h in graphs][:6]}...", flush=True)
    return M.mochy_profile(ctx, [(h.edge_ptr, h.edge_nodes, h.num_nodes) for h in graphs], eps)


def sequential(ctx, graphs):
    import paper_2310_15668_amd as M
    out = []
    for h in graphs:
        g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes)
        c26, c431 = M.mochy_count_exact(ctx, g)
        g.close()
        out.append(np.concatenate([c26, c431]))
    return np.array(out)


def check_cp(counts, sig26, cp26, sig431, cp431, eps=1.0):
    for lo, hi, sig, prof in ((0, 26, sig26, cp26), (26, 457, sig431, cp431)):
        M = counts[0, lo:hi].tolist()
        rand = [row[lo:hi].tolist() for row in counts[1:]]
        d = cp.significance(M, rand, eps)
        c = cp.characteristic_profile(d)
        np.testing.assert_allclose(sig, d, rtol=1e-12, atol=1e-300)
        np.testing.assert_allclose(prof, c, rtol=1e-12, atol=1e-300)


def test_tiny_with_copies_matches_oracle(ctx):
    base = make_config("tiny")
    graphs = [base] + [stub_matching_copy(base, s) for s in range(100, 108)]
    counts, sig26, cp26, sig431, cp431 = run_profile(ctx, graphs)
    for k, h in enumerate(graphs):
        r26, r431, _ = native.mochy_e(h, nthreads=8)
        assert (counts[k, :26] == r26).all() and (counts[k, 26:] == r431).all(), k
    check_cp(counts, sig26, cp26, sig431, cp431)
    assert abs(float(np.sum(cp26 ** 2)) - 1.0) < 1e-12


def test_batched_equals_sequential(ctx):
    base = powerlaw_hypergraph(1500, 6000, 2, 12, 2.5, 1.1, seed=3)
    graphs = [base] + [stub_matching_copy(base, s) for s in range(100, 116)]
    counts, *_ = run_profile(ctx, graphs)
    seq = sequential(ctx, graphs)
    assert (counts == seq).all()
    sizes = {h.num_edges for h in graphs}
    assert len(sizes) > 1  # uneven sizes after collapsing repeated members


def test_batch_of_large_graphs(ctx):
    # graphs of 12k hyperedges have more work items than one launch has waves:
    # the pair kernel runs once per graph (small graphs share one launch)
    base = make_config("batched_base", scale=0.1)
    assert base.num_edges > 8192
    graphs = [base] + [stub_matching_copy(base, s) for s in range(100, 103)]
    counts, *_ = run_profile(ctx, graphs)
    assert (counts == sequential(ctx, graphs)).all()


def test_batch_above_per_graph_launch_limit(ctx):
    # more than 256 graphs: the pair kernel counts the whole batch in one
    # launch with per-wave histograms flushed at every change of graph
    base = powerlaw_hypergraph(120, 300, 2, 8, 2.5, 1.0, seed=5)
    graphs = [base] + [stub_matching_copy(base, s) for s in range(200, 499)]
    counts, *_ = run_profile(ctx, graphs)
    assert counts.shape[0] == 300
    assert (counts == sequential(ctx, graphs)).all()
    for k in (0, 1, 150, 299):
        r26, r431, _ = native.mochy_e(graphs[k], nthreads=8)
        assert (counts[k, :26] == r26).all() and (counts[k, 26:] == r431).all(), k


def test_uneven_and_degenerate_members(ctx):
    graphs = [make_config("tiny"), from_edge_lists([[0, 1], [2, 3]], 4),
              from_edge_lists([[0, 1], [1, 2], [2, 0]], 3), make_config("tiny", scale=0.5)]
    counts, sig26, cp26, sig431, cp431 = run_profile(ctx, graphs, eps=0.5)
    assert (counts == sequential(ctx, graphs)).all()
    check_cp(counts, sig26, cp26, sig431, cp431, eps=0.5)


def test_device_inputs(ctx):
    import torch
    import paper_2310_15668_amd as M
    base = make_config("tiny")
    graphs = [base] + [stub_matching_copy(base, s) for s in range(100, 104)]
    dev = [(torch.from_numpy(h.edge_ptr).cuda(), torch.from_numpy(h.edge_nodes).cuda(), h.num_nodes)
           for h in graphs]
    torch.cuda.synchronize()
    print("[gpu] profile from device-resident CSRs", flush=True)
    a = M.mochy_profile(ctx, dev)
    b = run_profile(ctx, graphs)
    for x, y in zip(a, b):
        assert (x == y).all()
    # a node id outside its own graph's range is rejected even though the
    # shifted id would land inside the union
    bad_p = torch.tensor([0, 2], dtype=torch.int64, device="cuda")
    bad_n = torch.tensor([0, 7], dtype=torch.int32, device="cuda")
    with pytest.raises(M.MochyError) as e:
        M.mochy_profile(ctx, [dev[0], (bad_p, bad_n, 3), dev[1]])
    assert e.value.status == -1


def test_scaled_batched_config(ctx):
    # the batched CP workload at 5% scale: base + 64 copies in one batch
    base = make_config("batched_base", scale=0.05)
    graphs = [base] + [stub_matching_copy(base, s) for s in range(100, 164)]
    counts, sig26, cp26, sig431, cp431 = run_profile(ctx, graphs)
    assert (counts == sequential(ctx, graphs)).all()
    check_cp(counts, sig26, cp26, sig431, cp431)


def test_small_batched_config_against_oracle(ctx):
    base = make_config("batched_base", scale=0.02)
    graphs = [base] + [stub_matching_copy(base, s) for s in (100, 101)]
    counts, *_ = run_profile(ctx, graphs)
    for k, h in enumerate(graphs):
        r26, r431, _ = native.mochy_e(h, nthreads=16)
        assert (counts[k, 26:] == r431).all(), k


def test_chung_lu_copies_match_oracle(ctx):
    # the paper's own null model (Chung-Lu on the incidence graph) as the copies
    from workloads import chung_lu_copy
    base = powerlaw_hypergraph(200, 600, 2, 10, 2.5, 1.0, seed=31)
    graphs = [base] + [chung_lu_copy(base, s) for s in range(5)]
    counts, sig26, cp26, sig431, cp431 = run_profile(ctx, graphs)
    for k, h in enumerate(graphs):
        r26, r431, _ = native.mochy_e(h, nthreads=8)
        assert (counts[k, :26] == r26).all() and (counts[k, 26:] == r431).all(), k
    check_cp(counts, sig26, cp26, sig431, cp431)


def test_launch_shapes_and_tuner(ctx):
    # every launch shape of the pair kernel over a batch gives the same counts
    # (one launch or one per graph, 1 to 16 blocks per CU); the tuner keeps one
    # of them, and a server tuned on the first request answers as before
    import paper_2310_15668_amd as M
    from paper_2310_15668_amd.serving import CPServer
    from paper_2310_15668_amd.tune import CANDIDATES, tune_batch
    base = make_config("batched_base", scale=0.05)
    graphs = [base] + [stub_matching_copy(base, s) for s in range(100, 104)]
    ref = sequential(ctx, graphs)
    try:
        for launch, blocks in list(CANDIDATES) + [(1, 1), (2, 16), (0, 3)]:
            ctx.set_option(M.MOCHY_OPT_BATCH_LAUNCH, launch)
            ctx.set_option(M.MOCHY_OPT_PAIR_BLOCKS, blocks)
            print(f"[gpu] launch={launch} blocks={blocks}", flush=True)
            counts, *_ = run_profile(ctx, graphs)
            assert (counts == ref).all(), (launch, blocks)
        for opt, val in ((M.MOCHY_OPT_BATCH_LAUNCH, 3), (M.MOCHY_OPT_PAIR_BLOCKS, 0),
                         (M.MOCHY_OPT_PAIR_BLOCKS, 17)):
            with pytest.raises(M.MochyError) as e:
                ctx.set_option(opt, val)
            assert e.value.status == -1
        req = [(h.edge_ptr, h.edge_nodes, h.num_nodes) for h in graphs]
        res = tune_batch(ctx, req)
        print(f"[gpu] tuned: {res}", flush=True)
        assert (res["launch"], res["blocks"]) in CANDIDATES
        assert all(t > 0 for t in res["times"].values())
        with CPServer(0, slots=2) as srv:
            srv.tune(req)
            out = [t.wait(timeout=120) for t in [srv.submit(req), srv.submit(req[:3])]]
        assert (out[0]["counts"] == ref).all() and (out[1]["counts"] == ref[:3]).all()
    finally:
        ctx.set_option(M.MOCHY_OPT_BATCH_LAUNCH, 0)
        ctx.set_option(M.MOCHY_OPT_PAIR_BLOCKS, 8)


def test_buffer_cache_reuse_and_release(ctx):
    # freed buffers of 64 MiB or more stay with the context and serve the next
    # call of the same shape (no growth in device memory held), setting the
    # limit to 0 gives them back, and the counts never change
    import torch
    import paper_2310_15668_amd as M
    base = make_config("batched_base", scale=0.05)
    graphs = [base] + [stub_matching_copy(base, s) for s in range(100, 104)]
    with M.Context(0) as c:
        print("[gpu] cache: first call", flush=True)
        a = run_profile(c, graphs)[0]
        torch.cuda.synchronize()
        f1 = torch.cuda.mem_get_info(0)[0]
        for k in range(2):
            print(f"[gpu] cache: repeat {k}", flush=True)
            assert (run_profile(c, graphs)[0] == a).all()
        torch.cuda.synchronize()
        f2 = torch.cuda.mem_get_info(0)[0]
        assert abs(f2 - f1) < (256 << 20), (f1, f2)
        c.set_option(M.MOCHY_OPT_CACHE_BYTES, 0)
        torch.cuda.synchronize()
        f3 = torch.cuda.mem_get_info(0)[0]
        assert f3 - f2 >= (64 << 20), (f2, f3)
        assert (run_profile(c, graphs)[0] == a).all()
        c.set_option(M.MOCHY_OPT_CACHE_BYTES, 1 << 30)  # a limit below what a call frees
        assert (run_profile(c, graphs)[0] == a).all()
        assert (run_profile(c, graphs)[0] == a).all()
        with pytest.raises(M.MochyError):
            c.set_option(M.MOCHY_OPT_CACHE_BYTES, -1)
    assert (a == sequential(ctx, graphs)).all()


@pytest.mark.parametrize("capacity", [0, 1 << 40])
def test_batch_group_layouts(ctx, capacity):
    # a batch grouped in the counted-first layout (capacity 0) and in one pass
    # into row capacity gives the counts of each graph alone
    import paper_2310_15668_amd as M
    base = make_config("batched_base", scale=0.05)
    graphs = [base] + [stub_matching_copy(base, s) for s in range(100, 104)]
    small = [make_config("tiny")] + [stub_matching_copy(make_config("tiny"), s) for s in range(7)]
    ctx.set_option(M.MOCHY_OPT_GROUP_CAPACITY, capacity)
    try:
        print(f"[gpu] group capacity {capacity}", flush=True)
        a = run_profile(ctx, graphs)[0]
        b = run_profile(ctx, small)[0]
    finally:
        ctx.set_option(M.MOCHY_OPT_GROUP_CAPACITY, 24 << 30)
    assert (a == sequential(ctx, graphs)).all()
    assert (b == sequential(ctx, small)).all()


def test_batch_split_when_memory_runs_out(ctx):
    # grouping of a batch made to report MOCHY_ENOMEM above two graphs: the
    # batch is counted in sub-batches of two (halved until it fits, the size
    # kept), with the same counts, significance and CP
    import paper_2310_15668_amd as M
    base = make_config("batched_base", scale=0.02)
    graphs = [base] + [stub_matching_copy(base, s) for s in range(100, 106)]
    print(f"[gpu] forced batch split, {len(graphs)} graphs", flush=True)
    ref = run_profile(ctx, graphs)
    assert M.mochy_exact_stats(ctx)["profile_batches"] == 1  # 7 graphs of ~2,300 hyperedges fit one
    ctx.set_option(M.MOCHY_OPT_TEST_FAULTS, 4)
    try:
        got = run_profile(ctx, graphs)
        st = M.mochy_exact_stats(ctx)
    finally:
        ctx.set_option(M.MOCHY_OPT_TEST_FAULTS, 0)
    # 7 graphs: 7 fails, 4 fails, then 2 + 2 + 2 + 1
    assert st["profile_batches"] == 4, st
    assert (got[0] == ref[0]).all()
    for x, y in zip(got[1:], ref[1:]):
        assert np.array_equal(x, y)
    assert (got[0] == sequential(ctx, graphs)).all()
