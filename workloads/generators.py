"""Seeded generators for the synthetic hypergraphs the counters are measured on.

Recipe (stated once here and in the design notes):

* hyperedge sizes: discrete truncated power law, P(s) proportional to
  s**-gamma for s in [smin, smax], drawn by inverse CDF (float64 CDF);
* members: node v (0-based) carries the Zipf weight (v+1)**-alpha; the members
  of one hyperedge are drawn one after another by inverse CDF over these
  weights, a draw that repeats a member already taken is drawn again
  (successive sampling, i.e. weighted sampling without replacement);
* node lists are sorted; duplicate hyperedges are removed keeping the first
  occurrence (a hypergraph's hyperedges form a set, section 2.1);
* randomized copies for the significance null model use configuration-model
  stub matching: every incidence (v, e) is a stub pair, node stubs are shuffled
  and dealt back into the hyperedge slots in edge order, repeated members of a
  hyperedge collapse (a hyperedge is a set, as in the paper's transformation
  from incidence graphs to hypergraphs, Appendix "Randomized Hypergraphs"),
  and duplicate hyperedges are dropped keeping the first.

All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64), so the
same seed gives the same hypergraph on every machine with this numpy.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Hypergraph:
    edge_ptr: np.ndarray   # int64[|E|+1]
    edge_nodes: np.ndarray  # int32[sum |e|], strictly ascending per hyperedge
    num_nodes: int

    @property
    def num_edges(self) -> int:
        return int(self.edge_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.edge_ptr[-1])

    def edge(self, e: int) -> np.ndarray:
        return self.edge_nodes[self.edge_ptr[e]:self.edge_ptr[e + 1]]

    def edges(self) -> list:
        return [self.edge(e).tolist() for e in range(self.num_edges)]

    def sizes(self) -> np.ndarray:
        return np.diff(self.edge_ptr)


def _csr_from_padded(mat: np.ndarray, num_nodes: int) -> Hypergraph:
    """Rows of ``mat`` are sorted node lists padded with -1 at the end."""
    sizes = (mat >= 0).sum(axis=1).astype(np.int64)
    ptr = np.zeros(mat.shape[0] + 1, dtype=np.int64)
    np.cumsum(sizes, out=ptr[1:])
    nodes = mat[mat >= 0].astype(np.int32)
    return Hypergraph(ptr, nodes, int(num_nodes))


def _sort_rows_padded(mat: np.ndarray) -> np.ndarray:
    big = np.iinfo(np.int64).max
    m = np.where(mat < 0, big, mat.astype(np.int64))
    m.sort(axis=1)
    return np.where(m == big, -1, m)


def _first_unique_rows(mat: np.ndarray) -> np.ndarray:
    """Indices (ascending) of the first occurrence of every distinct row."""
    if mat.shape[0] == 0:
        return np.zeros(0, dtype=np.int64)
    m = np.ascontiguousarray(mat.astype(np.int64))
    view = m.view(np.dtype((np.void, m.dtype.itemsize * m.shape[1]))).ravel()
    _, first = np.unique(view, return_index=True)
    first.sort()
    return first


def _to_padded(h: Hypergraph) -> np.ndarray:
    sizes = h.sizes()
    width = int(sizes.max()) if sizes.size else 1
    mat = np.full((h.num_edges, max(width, 1)), -1, dtype=np.int64)
    rows = np.repeat(np.arange(h.num_edges), sizes)
    cols = np.arange(h.nnz) - np.repeat(h.edge_ptr[:-1], sizes)
    mat[rows, cols] = h.edge_nodes
    return mat


def powerlaw_hypergraph(num_nodes: int, num_edges: int, smin: int, smax: int,
                        gamma: float, alpha: float, seed: int,
                        dedup: bool = True) -> Hypergraph:
    """Power-law sizes, Zipf node popularity, members without replacement."""
    if smax > num_nodes:
        raise ValueError("smax exceeds the number of nodes")
    rng = np.random.default_rng(seed)
    svals = np.arange(smin, smax + 1, dtype=np.float64)
    pmf = svals ** (-gamma)
    cdf = np.cumsum(pmf) / pmf.sum()
    u = rng.random(num_edges)
    sizes = smin + np.minimum(np.searchsorted(cdf, u, side="right"), smax - smin)

    w = np.arange(1, num_nodes + 1, dtype=np.float64) ** (-alpha)
    cw = np.cumsum(w)
    cw /= cw[-1]
    mat = np.full((num_edges, smax), -1, dtype=np.int64)
    for p in range(smax):
        pending = np.nonzero(sizes > p)[0]
        while pending.size:
            cand = np.minimum(np.searchsorted(cw, rng.random(pending.size), side="right"),
                              num_nodes - 1)
            if p:
                dup = (mat[pending, :p] == cand[:, None]).any(axis=1)
            else:
                dup = np.zeros(pending.size, dtype=bool)
            ok = ~dup
            mat[pending[ok], p] = cand[ok]
            pending = pending[dup]
    mat = _sort_rows_padded(mat)
    if dedup:
        mat = mat[_first_unique_rows(mat)]
    return _csr_from_padded(mat, num_nodes)


def from_edge_lists(edges, num_nodes: int | None = None) -> Hypergraph:
    """CSR from Python lists; each list is sorted and made a set."""
    rows = [sorted(set(int(v) for v in e)) for e in edges]
    if num_nodes is None:
        num_nodes = 1 + max((max(r) for r in rows if r), default=-1)
    ptr = np.zeros(len(rows) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(r) for r in rows])
    nodes = np.array([v for r in rows for v in r], dtype=np.int32)
    return Hypergraph(ptr, nodes, int(num_nodes))


def dedup_hypergraph(h: Hypergraph) -> Hypergraph:
    mat = _to_padded(h)
    return _csr_from_padded(mat[_first_unique_rows(mat)], h.num_nodes)


def stub_matching_copy(h: Hypergraph, seed: int) -> Hypergraph:
    """Degree- and size-preserving randomized copy (configuration model)."""
    rng = np.random.default_rng(seed)
    deg = np.bincount(h.edge_nodes, minlength=h.num_nodes)
    stubs = np.repeat(np.arange(h.num_nodes, dtype=np.int64), deg)
    stubs = stubs[rng.permutation(stubs.size)]
    sizes = h.sizes()
    owner = np.repeat(np.arange(h.num_edges, dtype=np.int64), sizes)
    # collapse repeated members: unique (edge, node) pairs, sorted by edge then node
    key = owner * np.int64(h.num_nodes) + stubs
    key = np.unique(key)
    e_of = key // h.num_nodes
    v_of = (key % h.num_nodes).astype(np.int32)
    new_sizes = np.bincount(e_of, minlength=h.num_edges).astype(np.int64)
    keep_nonempty = new_sizes > 0
    ptr = np.zeros(h.num_edges + 1, dtype=np.int64)
    np.cumsum(new_sizes, out=ptr[1:])
    g = Hypergraph(ptr, v_of, h.num_nodes)
    if not keep_nonempty.all():  # cannot happen for sizes >= 1, kept for safety
        mat = _to_padded(g)[keep_nonempty]
        g = _csr_from_padded(mat, h.num_nodes)
    return dedup_hypergraph(g)


def chung_lu_incidences(h: Hypergraph, seed: int):
    """The random incidence multiset of the Chung-Lu model on the incidence
    graph (Appendix, randomized hypergraphs): |incidences| draws, each a node
    picked with probability proportional to its degree and, independently, a
    hyperedge picked with probability proportional to its size.  A uniformly
    drawn incidence's node (hyperedge) has exactly that distribution.
    Returns (hyperedge ids, node ids), int64 arrays of length nnz."""
    rng = np.random.default_rng(seed)
    L = h.nnz
    owner = np.repeat(np.arange(h.num_edges, dtype=np.int64), h.sizes())
    nodes = h.edge_nodes.astype(np.int64)[rng.integers(0, L, size=L)]
    edges = owner[rng.integers(0, L, size=L)]
    return edges, nodes


def chung_lu_copy(h: Hypergraph, seed: int) -> Hypergraph:
    """Randomized copy by the Chung-Lu model: the incidence multiset of
    :func:`chung_lu_incidences` turned into a hypergraph whose hyperedges are
    sets (repeated members collapse); hyperedges that drew no member are
    dropped and repeated hyperedges removed, keeping the first."""
    edges, nodes = chung_lu_incidences(h, seed)
    key = np.unique(edges * np.int64(max(h.num_nodes, 1)) + nodes)
    e_of = key // max(h.num_nodes, 1)
    v_of = (key % max(h.num_nodes, 1)).astype(np.int32)
    sizes = np.bincount(e_of, minlength=h.num_edges).astype(np.int64)
    sizes = sizes[sizes > 0]
    ptr = np.zeros(sizes.size + 1, dtype=np.int64)
    np.cumsum(sizes, out=ptr[1:])
    return dedup_hypergraph(Hypergraph(ptr, v_of, h.num_nodes))


def induced_prefix(h: Hypergraph, n_edges: int) -> Hypergraph:
    """First ``n_edges`` hyperedges; nodes are renumbered compactly in order."""
    n_edges = min(n_edges, h.num_edges)
    ptr = h.edge_ptr[:n_edges + 1].copy()
    nodes = h.edge_nodes[:ptr[-1]]
    uniq, inv = np.unique(nodes, return_inverse=True)
    return Hypergraph(ptr, inv.astype(np.int32), int(uniq.size))


# ---------------------------------------------------------------------------
# Named workloads.  Sizes are counts *drawn*; duplicates are removed after.
CONFIGS = {
    "tiny": dict(num_nodes=300, num_edges=500, smin=2, smax=8, gamma=2.5, alpha=1.0, seed=0),
    "medium": dict(num_nodes=20_000, num_edges=100_000, smin=2, smax=25, gamma=2.5, alpha=1.0, seed=1),
    "large": dict(num_nodes=1_000_000, num_edges=2_000_000, smin=2, smax=25, gamma=2.8, alpha=0.9, seed=2),
    "batched_base": dict(num_nodes=50_000, num_edges=150_000, smin=2, smax=20, gamma=2.5, alpha=1.1, seed=3),
}
BATCHED_COPY_SEEDS = tuple(range(100, 164))
LARGE_SUBSET_EDGES = 200_000


def make_config(name: str, scale: float = 1.0) -> Hypergraph:
    """Named workload; ``scale`` < 1 shrinks nodes and hyperedges together."""
    if name == "large_subset":
        return induced_prefix(make_config("large", scale), int(LARGE_SUBSET_EDGES * scale))
    cfg = dict(CONFIGS[name])
    if scale != 1.0:
        cfg["num_nodes"] = max(cfg["smax"], int(round(cfg["num_nodes"] * scale)))
        cfg["num_edges"] = max(1, int(round(cfg["num_edges"] * scale)))
    return powerlaw_hypergraph(**cfg)


def serving_request(n: int, lo: int = 1_000, hi: int = 200_000) -> Hypergraph:
    """Request ``n`` of the serving stream: |E| log-uniform in [lo, hi]."""
    rng = np.random.default_rng(4 + 1_000_003 * n)
    num_edges = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
    num_nodes = max(25, int(round(0.4 * num_edges)))
    return powerlaw_hypergraph(num_nodes, num_edges, 2, 25, 2.5, 1.0, seed=1000 + n)


def serving_copies(n: int, h: Hypergraph, copies: int = 8) -> list:
    """The randomized copies of request ``n``: stub matching with seeds (1000 + n) * 64 + c."""
    return [stub_matching_copy(h, (1000 + n) * 64 + c) for c in range(copies)]


def poisson_arrivals(count: int, rate: float, seed: int = 4) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson stream of ``rate`` requests/s."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
