"""MI355X-native hypergraph-motif counter (MoCHy, arXiv 2310.15668).

The computation lives in ``libmochy.so`` (hand-written HIP for gfx950) behind
the C ABI of ``include/mochy.h``; ``paper_2310_15668_amd._lib`` is its ctypes
binding with the same names.  Importing this package loads nothing; the
library is loaded on first use and raises if it has not been built.
"""
from ._lib import (  # noqa: F401
    Context, Graph, MochyError, mochy_project, mochy_count_exact, mochy_count_exact_range,
    mochy_count_sampled, mochy_count_sampled_edges, mochy_hyperedge_profiles, mochy_profile, motif_pattern, parent_motif, NUM_H, NUM_3H, MOCHY_DEDUP,
    MOCHY_LG_FREE, MOCHY_OPT_GROUPS, MOCHY_OPT_APLUS_ROWS, MOCHY_OPT_MEMO_BUDGET, MOCHY_OPT_MEMO_ALL,
    MOCHY_OPT_MEMO_POOL, MOCHY_OPT_GROUP_CAPACITY, MOCHY_OPT_BATCH_LAUNCH, MOCHY_OPT_PAIR_BLOCKS,
    MOCHY_OPT_CACHE_BYTES, MOCHY_OPT_TEST_FAULTS, MOCHY_CANONICALIZE, MOCHY_H26, MOCHY_H431,
    MOCHY_WHICH_ALL,
    mochy_graph_stats, mochy_phase_ms, mochy_memo_stats, mochy_exact_stats,
    mochy_calibrate_valu, mochy_count_exact_range_noalloc,
)
