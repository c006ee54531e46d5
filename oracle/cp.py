"""Significance, characteristic profile and A+ rescaling in float64 (oracle side).

Test infrastructure: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may use it.
"""
from __future__ import annotations

import math

from . import patterns


def mean_random(rand_counts):
    """M_rand[t]: the average over randomized hypergraphs (integer sum, one division)."""
    R = len(rand_counts)
    T = len(rand_counts[0])
    return [float(sum(int(c[t]) for c in rand_counts)) / R for t in range(T)]


def significance(counts, rand_counts, eps=1.0):
    """Delta_t = (M[t] - M_rand[t]) / (M[t] + M_rand[t] + eps)   (Eq. 1)."""
    mr = mean_random(rand_counts)
    out = []
    for t in range(len(counts)):
        m = float(int(counts[t]))
        out.append((m - mr[t]) / (m + mr[t] + eps))
    return out


def characteristic_profile(delta):
    """CP_t = Delta_t / sqrt(sum_t Delta_t^2)   (Eq. 2); all zeros if every Delta is 0."""
    s = 0.0
    for d in delta:
        s = s + d * d
    if s == 0.0:
        return [0.0] * len(delta)
    n = math.sqrt(s)
    return [d / n for d in delta]


def aplus_estimate(raw26, num_wedges, r):
    """Algorithm 5's rescaling: open motifs by |wedges|/(2r), closed by |wedges|/(3r)."""
    opened = set(patterns.open_ids())
    out = []
    for t in range(26):
        w = 2.0 if (t + 1) in opened else 3.0
        out.append((float(int(raw26[t])) * float(num_wedges)) / (w * float(r)))
    return out


def aplus_estimate3(raw431, num_wedges, r):
    """The same rescaling for 3h-motifs: w follows the parent h-motif."""
    opened = set(patterns.open_ids())
    parent = patterns.id3_to_id26()
    out = []
    for t in range(431):
        w = 2.0 if int(parent[t + 1]) in opened else 3.0
        out.append((float(int(raw431[t])) * float(num_wedges)) / (w * float(r)))
    return out


def mochy_a_estimate(raw, num_edges, s):
    """Algorithm 4's rescaling: every count by |E| / (3 s)."""
    return [(float(int(x)) * float(num_edges)) / (3.0 * float(s)) for x in raw]
