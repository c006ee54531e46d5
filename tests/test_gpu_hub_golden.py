"""GPU parity where the medium workload's exact work concentrates: single hub
centres of the full-size graph against oracle counts stored in
tests/golden/medium_hub_centres.txt (written by oracle/make_medium_hub_golden.py
from oracle/ and workloads/ only).

Algorithm 2 attributes each instance to one centre (section 4.2), so the
counts of one centre are checked exactly with mochy_count_exact_range.  The
stored centres are the ten rows of largest line-graph degree and rows at
spread ranks of every degree band above 8,192: these rows hold almost all of
the medium workload's candidates and the largest are grouped in several hash
parts by the pair kernel's grouping.  Both group layouts are checked (one pass into
row capacity, and groups counted first).  Two hyperedge-profile rows of hub
degree check the profile kernel on rows of thousands of neighbours, and MoCHy-A
samples that draw those hyperedges check the sampler on them.
"""
import numpy as np
import pytest

from conftest import golden
from oracle import cp, native
from oracle.make_medium_hub_golden import csr_digest
from workloads import make_config

pytestmark = pytest.mark.gpu

GOLDEN = "medium_hub_centres.txt"


@pytest.fixture(scope="module")
def stored():
    rows = golden(GOLDEN)
    head = {r[0]: r[1] for r in rows if r[0] in ("csr_sha256", "hyperwedges")}
    exact = [(int(r[1]), int(r[2]), np.array(r[3:], dtype=np.int64)) for r in rows if r[0] == "exact"]
    prof = [(int(r[1]), int(r[2]), np.array(r[3:], dtype=np.int64)) for r in rows if r[0] == "profile"]
    assert all(v.size == 431 for _, _, v in exact + prof)
    return head, exact, prof


@pytest.fixture(scope="module")
def medium(stored):
    h = make_config("medium")
    assert csr_digest(h) == stored[0]["csr_sha256"], "the medium generator changed since the golden was written"
    return h


@pytest.fixture(scope="module")
def ctx():
    import paper_2310_15668_amd as M
    c = M.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def graph(ctx, medium, stored):
    import paper_2310_15668_amd as M
    print("[gpu] project full medium hypergraph", flush=True)
    g = M.mochy_project(ctx, medium.edge_ptr, medium.edge_nodes, medium.num_nodes)
    assert g.num_hyperwedges == int(stored[0]["hyperwedges"])
    yield g
    g.close()


def test_golden_covers_the_hub_rows(stored):
    _, exact, _ = stored
    deg = [d for _, d, _ in exact]
    assert max(deg) == 49249  # the maximum-degree row of the medium workload
    assert sum(d > 8192 for d in deg) == len(deg)
    assert min(deg) < 12288 and sum(d >= 32768 for d in deg) >= 10
    # each stored centre's counts are non-trivial and open/closed consistent:
    # an open instance has its middle at the centre, so a row of d neighbours
    # holds at most C(d, 2) of them
    for _, d, v in exact:
        assert 0 < v.sum() <= d * (d - 1) // 2


@pytest.mark.parametrize("layout", ["one-pass", "counted-first"])
def test_hub_centres_match_oracle(ctx, graph, stored, layout):
    import paper_2310_15668_amd as M
    _, exact, _ = stored
    parts, regrouped = 0, 0
    try:
        if layout == "counted-first":
            ctx.set_option(M.MOCHY_OPT_GROUP_CAPACITY, 0)
        for c, d, want in exact:
            print(f"[gpu] medium centre {c} (degree {d}), {layout} groups", flush=True)
            g26, g431 = M.mochy_count_exact_range(ctx, graph, c, c + 1)
            st = M.mochy_exact_stats(ctx)
            parts = max(parts, st["max_hash_parts"])
            regrouped += st["rows_regrouped"]
            assert st["rows_grouped"] == 1
            assert (g431 == want).all(), (c, np.nonzero(g431 != want)[0][:8])
            assert (g26 == native.fold26(np.concatenate([[0], want]))).all(), c
    finally:
        ctx.set_option(M.MOCHY_OPT_GROUP_CAPACITY, 24 << 30)
    # the largest rows are grouped in several hash parts (16,000 records
    # per part at first): the 49,249-neighbour row in at least four
    assert parts >= 4, (parts, regrouped)


def test_hub_centres_every_pair(ctx, graph, stored):
    # pairing every record (no groups) on the largest rows
    import paper_2310_15668_amd as M
    _, exact, _ = stored
    try:
        ctx.set_option(M.MOCHY_OPT_GROUPS, 0)
        for c, d, want in sorted(exact, key=lambda x: -x[1])[:3]:
            print(f"[gpu] medium centre {c} (degree {d}), every pair", flush=True)
            _, g431 = M.mochy_count_exact_range(ctx, graph, c, c + 1)
            assert (g431 == want).all(), c
    finally:
        ctx.set_option(M.MOCHY_OPT_GROUPS, 1)


def test_hub_hyperedge_profiles_match_oracle(ctx, graph, stored):
    import paper_2310_15668_amd as M
    _, _, prof = stored
    assert prof and min(d for _, d, _ in prof) > 8000
    for e, d, want in prof:
        print(f"[gpu] medium hyperedge profile {e} (degree {d})", flush=True)
        p26, p431 = M.mochy_hyperedge_profiles(ctx, graph, e, e + 1)
        assert (p431[0] == want).all(), (e, np.nonzero(p431[0] != want)[0][:8])
        assert (p26[0] == native.fold26(np.concatenate([[0], want]))).all()


def test_hub_mochy_a_samples(ctx, graph, stored, medium):
    # MoCHy-A (Algorithm 4) hits, for one sampled hyperedge, every instance
    # that contains it once: a one-sample window whose Philox draw is a stored
    # hub hyperedge returns that hyperedge's profile row
    import paper_2310_15668_amd as M
    _, _, prof = stored
    E, seed = medium.num_edges, 7

    def drawn(n):
        x = native.philox4x32_10([n & 0xffffffff, n >> 32, 1, 0], [seed, 0])
        return ((x[1] << 32 | x[0]) * E) >> 64

    for e, d, want in prof:
        n0 = next(n for n in range(4_000_000) if drawn(n) == e)
        print(f"[gpu] medium MoCHy-A sample {n0} draws hyperedge {e} (degree {d})", flush=True)
        raw26, est26, raw431, est431 = M.mochy_count_sampled_edges(ctx, graph, 1, seed, n0)
        assert (raw431 == want).all(), (e, np.nonzero(raw431 != want)[0][:8])
        assert (raw26 == native.fold26(np.concatenate([[0], want]))).all()
        np.testing.assert_allclose(est431, cp.mochy_a_estimate(want, E, 1), rtol=1e-12, atol=0)
