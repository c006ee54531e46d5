"""Resumable exact counting on the device: a count of the scaled medium
hypergraph interrupted after three centre ranges and resumed on a new
context gives the counts of one mochy_count_exact call."""
import pytest

from paper_2310_15668_amd import checkpoint as ck
from workloads import make_config

pytestmark = pytest.mark.gpu


def test_resume_on_a_new_context(tmp_path):
    import paper_2310_15668_amd as M
    h = make_config("medium", scale=0.05)
    key = ck.csr_key(h.edge_ptr, h.edge_nodes, h.num_nodes)
    path = str(tmp_path / "medium.ckpt")
    print(f"[gpu] resumable count |E|={h.num_edges}", flush=True)
    with M.Context(0) as ctx:
        g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes)
        full26, full431 = M.mochy_count_exact(ctx, g)
        out = ck.count_exact_resumable(lambda a, b: M.mochy_count_exact_range(ctx, g, a, b), h.num_edges,
                                       key, path, 1000, stop_after=3)
        assert out is None
        g.close()
    with M.Context(0) as ctx:  # as a new process would
        g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes)
        c26, c431 = ck.count_exact_resumable(lambda a, b: M.mochy_count_exact_range(ctx, g, a, b),
                                             h.num_edges, key, path, 1000)
        g.close()
    assert (c26 == full26).all() and (c431 == full431).all()
