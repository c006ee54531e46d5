"""The CP server: every request's answer is the same alone and in the mix of
concurrently running requests, and matches the oracle."""
import numpy as np
import pytest

from oracle import cp, native
from workloads import powerlaw_hypergraph, serving_copies

pytestmark = pytest.mark.gpu


def requests():
    out = []
    for n, E in enumerate((200, 900, 2500, 400, 1500, 3000, 700)):
        h = powerlaw_hypergraph(max(25, int(0.4 * E)), E, 2, 12, 2.5, 1.0, seed=500 + n)
        gs = [h] + serving_copies(n, h, copies=3)
        out.append([(g.edge_ptr, g.edge_nodes, g.num_nodes) for g in gs])
    return out


def test_same_alone_and_in_the_mix():
    import paper_2310_15668_amd as M
    from paper_2310_15668_amd.serving import CPServer
    reqs = requests()
    print(f"[gpu] {len(reqs)} requests alone", flush=True)
    with M.Context(0) as ctx:
        alone = [M.mochy_profile(ctx, r) for r in reqs]
    print("[gpu] the same requests through a 4-slot server", flush=True)
    with CPServer(0, slots=4) as srv:
        tickets = [srv.submit(r) for r in reqs]
        mixed = [t.wait(timeout=120) for t in tickets]
        assert all(t.start is not None and t.done >= t.start for t in tickets)
    for a, m in zip(alone, mixed):
        assert (a[0] == m["counts"]).all()
        for x, key in zip(a[1:], ("sig26", "cp26", "sig431", "cp431")):
            assert np.array_equal(x, m[key])
    # request 2 against the oracle
    r = reqs[2]
    rows = []
    for ptr, nodes, V in r:
        from workloads.generators import Hypergraph
        c26, c431, _ = native.mochy_e(Hypergraph(ptr, nodes, V), nthreads=8)
        rows.append(np.concatenate([c26, c431]))
    rows = np.array(rows)
    assert (rows == mixed[2]["counts"]).all()
    sig = cp.significance(rows[0, :26], rows[1:, :26], 1.0)
    np.testing.assert_allclose(mixed[2]["sig26"], sig, rtol=1e-12, atol=0)


def test_tight_budget_serializes_but_answers():
    import paper_2310_15668_amd as M
    from paper_2310_15668_amd.serving import CPServer
    reqs = requests()[:4]
    with M.Context(0) as ctx:
        alone = [M.mochy_profile(ctx, r)[0] for r in reqs]
    print("[gpu] 4 requests, 1-byte budget (one at a time)", flush=True)
    with CPServer(0, slots=3, budget_bytes=1) as srv:
        tickets = [srv.submit(r) for r in reqs]
        got = [t.wait(timeout=120)["counts"] for t in tickets]
    for a, g in zip(alone, got):
        assert (a == g).all()
    spans = sorted((t.start, t.done) for t in tickets)
    assert all(spans[k][1] <= spans[k + 1][0] for k in range(len(spans) - 1))  # never overlapped
