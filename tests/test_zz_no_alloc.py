"""The allocation-free exact counting call (mochy_count_exact_range_noalloc)
against mochy_count_exact_range through the C ABI: the same counts, bit for
bit, on two calls in a row (the second on a smaller graph, so stale scratch
contents from the first would show), on a centre sub-range, and a clear
MOCHY_ERANGE when a call needs more scratch than the array holds.
"""
import pytest

from workloads import make_config

pytestmark = pytest.mark.gpu


def _both(ctx, M, h, c0=0, c1=None):
    c1 = h.num_edges if c1 is None else c1
    print(f"[gpu] noalloc vs range |E|={h.num_edges} centres [{c0}, {c1})", flush=True)
    g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes)
    try:
        a26, a431 = M.mochy_count_exact_range(ctx, g, c0, c1)
        b26, b431 = M.mochy_count_exact_range_noalloc(ctx, g, c0, c1)
        st = M.mochy_exact_stats(ctx)
    finally:
        g.close()
    return (a26, a431), (b26, b431), st


def test_noalloc_matches_range_call():
    import paper_2310_15668_amd as M
    with M.Context(0) as ctx:
        big = make_config("medium", scale=0.1)
        small = make_config("tiny")
        (a26, a431), (b26, b431), st = _both(ctx, M, big)
        assert (a431 == b431).all() and (a26 == b26).all()
        assert a26.sum() > 0 and st["groups"] == 0 and st["light_pairs"] > 0
        # second call, smaller input: the scratch array keeps the first call's
        # contents, which must not leak into this one
        (a26, a431), (b26, b431), _ = _both(ctx, M, small)
        assert (a431 == b431).all() and (a26 == b26).all() and a26.sum() > 0
        (a26, a431), (b26, b431), _ = _both(ctx, M, small, 17, 301)
        assert (a431 == b431).all()
        # the ordinary entry points still work after the allocation-free ones
        (a26, a431), (b26, b431), _ = _both(ctx, M, big, 100, 4000)
        assert (a431 == b431).all()


def test_noalloc_rejects_oversized_calls():
    import paper_2310_15668_amd as M
    with M.Context(0) as ctx:
        h = make_config("medium", scale=0.1)
        g = M.mochy_project(ctx, h.edge_ptr, h.edge_nodes, h.num_nodes)
        try:
            ctx.set_option(M.MOCHY_OPT_TEST_FAULTS, 2)  # scratch capped at 64 KiB
            with pytest.raises(M.MochyError) as e:
                M.mochy_count_exact_range_noalloc(ctx, g, 0, h.num_edges)
            assert e.value.status == -3 and "scratch" in str(e.value)
            ctx.set_option(M.MOCHY_OPT_TEST_FAULTS, 0)
            ref = M.mochy_count_exact(ctx, g)[1]
            again = M.mochy_count_exact_range_noalloc(ctx, g, 0, h.num_edges)[1]
            assert (ref == again).all()
            with pytest.raises(M.MochyError) as e:
                M.mochy_count_exact_range_noalloc(ctx, g, 5, 2)
            assert e.value.status == -1
        finally:
            ctx.set_option(M.MOCHY_OPT_TEST_FAULTS, 0)
            g.close()
