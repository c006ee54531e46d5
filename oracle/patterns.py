"""Overlap patterns of hyperedge triples and their ids (oracle side).

Test infrastructure: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may use this package.

Definitions followed (section 2.2 "Hypergraph Motifs"):

* three hyperedges e_i, e_j, e_k split their union into seven regions, in the
  paper's order R1 = e_i - e_j - e_k, R2 = e_j - e_k - e_i, R3 = e_k - e_i - e_j,
  R4 = e_i & e_j - e_k, R5 = e_j & e_k - e_i, R6 = e_k & e_i - e_j,
  R7 = e_i & e_j & e_k;
* an h-motif is the emptiness vector of the seven regions up to relabelling
  the three hyperedges; a pattern is kept only if it can come from three
  *distinct* hyperedges that are *connected* (one of them meets the other
  two).  26 survive;
* a 3h-motif (section 5.1) replaces emptiness by a ternary state of each
  region's cardinality c: 0 if c = 0, 1 if 0 < c <= theta, 2 if c > theta.
  431 survive;
* the k-hyperedge generalisation (appendix "Extensions beyond Three
  Hyperedges", table of the number of h-motifs) uses the 2^k - 1 Venn
  regions of k sets; it is enumerated here for k = 2, 3, 4 to pin the
  counting machinery against the table.

Numbering.  The paper's figure that fixes ids 1..26 is not available, only
facts stated in the text: ids 17-22 are the open motifs, id 16 has all seven
regions non-empty, 17 and 18 are a hyperedge holding two disjoint
hyperedges, 3h-motifs 1-6 subdivide h-motif 1 (one singled-out region plus
two symmetric ones).  The rule used here satisfies all of them:

* canonical form of a pattern = lexicographically smallest (R1, ..., R7)
  tuple over the six relabellings;
* h-motif groups: closed with R7 non-empty -> ids 1..16, open -> 17..22,
  closed with R7 empty -> 23..26; inside a group, order by (number of
  non-empty regions, canonical tuple);
* 3h-motifs ordered by (parent h-motif id, canonical ternary tuple).

Any correspondence with the paper's figure beyond those facts is parity
unpinned.
"""
from __future__ import annotations

import itertools
from functools import lru_cache

import numpy as np

# Region r (0-based, R1..R7) as the set of hyperedges (0=i, 1=j, 2=k) whose
# intersection, minus the others, it is.
REGIONS3 = (frozenset({0}), frozenset({1}), frozenset({2}),
            frozenset({0, 1}), frozenset({1, 2}), frozenset({0, 2}),
            frozenset({0, 1, 2}))
PERMS3 = tuple(itertools.permutations(range(3)))


def relabel(pattern, perm):
    """Pattern of the triple (e_perm[0], e_perm[1], e_perm[2])."""
    out = []
    for s in REGIONS3:
        image = frozenset(perm[x] for x in s)
        out.append(pattern[REGIONS3.index(image)])
    return tuple(out)


def canonical(pattern):
    return min(relabel(tuple(pattern), p) for p in PERMS3)


def adjacent(pattern, x, y):
    return any(pattern[r] > 0 for r, s in enumerate(REGIONS3) if x in s and y in s)


def is_connected(pattern):
    """Some hyperedge of the three meets the other two (section 2.1)."""
    for x in range(3):
        y, z = [w for w in range(3) if w != x]
        if adjacent(pattern, x, y) and adjacent(pattern, x, z):
            return True
    return False


def is_distinct(pattern):
    """No two of the three hyperedges can be forced equal by the pattern."""
    for x, y in ((0, 1), (1, 2), (0, 2)):
        differ = any(pattern[r] > 0 for r, s in enumerate(REGIONS3) if (x in s) != (y in s))
        if not differ:
            return False
    return True


def is_valid(pattern):
    return is_connected(pattern) and is_distinct(pattern)


def is_open(pattern):
    """Open: two of the three hyperedges are disjoint."""
    return not all(adjacent(pattern, x, y) for x, y in ((0, 1), (1, 2), (0, 2)))


def binary_of(pattern):
    return tuple(1 if s > 0 else 0 for s in pattern)


@lru_cache(maxsize=None)
def hmotif_table():
    """List of canonical binary patterns; index 0 is h-motif 1."""
    canon = sorted({canonical(p) for p in itertools.product((0, 1), repeat=7) if is_valid(p)})

    def group(p):
        if not is_open(p):
            return 0 if p[6] else 2
        return 1

    return tuple(sorted(canon, key=lambda p: (group(p), sum(p), p)))


@lru_cache(maxsize=None)
def tmotif_table():
    """List of (canonical ternary pattern, parent h-motif id); index 0 is 3h-motif 1."""
    hid = {p: i + 1 for i, p in enumerate(hmotif_table())}
    canon = {canonical(p) for p in itertools.product((0, 1, 2), repeat=7) if is_valid(binary_of(p))}
    rows = [(hid[canonical(binary_of(p))], p) for p in canon]
    rows.sort()
    return tuple((p, parent) for parent, p in rows)


def code3(pattern):
    """Base-3 integer of a ternary tuple, R1 most significant (lexicographic order)."""
    c = 0
    for s in pattern:
        c = 3 * c + s
    return c


@lru_cache(maxsize=None)
def canonical_code_to_id3():
    """int32[2187]: 3h id (1..431) of every *canonical* ternary code, else 0."""
    table = np.zeros(3 ** 7, dtype=np.int32)
    for idx, (p, _parent) in enumerate(tmotif_table()):
        table[code3(p)] = idx + 1
    return table


@lru_cache(maxsize=None)
def id3_to_id26():
    """int32[432]: parent h-motif id of each 3h-motif id (entry 0 unused)."""
    out = np.zeros(432, dtype=np.int32)
    for idx, (_p, parent) in enumerate(tmotif_table()):
        out[idx + 1] = parent
    return out


def open_ids():
    return [i + 1 for i, p in enumerate(hmotif_table()) if is_open(p)]


def classify_counts(card, theta=1):
    """(h id, 3h id) of a triple from its seven region cardinalities, or None."""
    trit = tuple(0 if c == 0 else (1 if c <= theta else 2) for c in card)
    if not is_valid(binary_of(trit)):
        return None
    cp = canonical(trit)
    i3 = int(canonical_code_to_id3()[code3(cp)])
    return int(id3_to_id26()[i3]), i3


# ---------------------------------------------------------------------------
# General k (k = 2, 3, 4): the pattern census of the table of the number of
# h-motifs with k hyperedges, by vectorised enumeration.

def _regions(k):
    return [frozenset(x for x in range(k) if (m >> x) & 1) for m in range(1, 1 << k)]


def pattern_census(k, states=2):
    """Counts after each filter of the table: raw, orbits, connected, distinct.

    With ``states`` > 2 every region takes one of ``states`` cardinality
    classes; connectivity and distinctness depend only on emptiness.
    """
    regs = _regions(k)
    nreg = len(regs)
    index = {s: r for r, s in enumerate(regs)}
    n = states ** nreg
    codes = np.arange(n, dtype=np.int64)
    digits = np.stack([(codes // states ** (nreg - 1 - r)) % states for r in range(nreg)], axis=1)
    best = None
    for perm in itertools.permutations(range(k)):
        src = [index[frozenset(perm[x] for x in s)] for s in regs]
        relab = digits[:, src]
        val = np.zeros(n, dtype=np.int64)
        for r in range(nreg):
            val = val * states + relab[:, r]
        best = val if best is None else np.minimum(best, val)
    reps = np.nonzero(best == codes)[0]  # lexicographically smallest of its orbit
    nonempty = digits[reps] > 0
    # adjacency of hyperedges x, y: a non-empty region containing both
    adj = np.zeros((reps.size, k, k), dtype=bool)
    for r, s in enumerate(regs):
        for x in s:
            for y in s:
                if x != y:
                    adj[:, x, y] |= nonempty[:, r]
    # connectivity of the k hyperedges by repeated relaxation
    reach = np.zeros((reps.size, k), dtype=bool)
    reach[:, 0] = True
    for _ in range(k):
        reach = reach | np.any(adj & reach[:, :, None], axis=1)
    connected = reach.all(axis=1)
    distinct = np.ones(reps.size, dtype=bool)
    for x in range(k):
        for y in range(x + 1, k):
            differ = np.zeros(reps.size, dtype=bool)
            for r, s in enumerate(regs):
                if (x in s) != (y in s):
                    differ |= nonempty[:, r]
            distinct &= differ
    return {
        "raw": int(n),
        "orbits": int(reps.size),
        "connected": int(connected.sum()),
        "valid": int((connected & distinct).sum()),
    }


def kh_motif_closed_form(k):
    """Number of kh-motifs (appendix on the number of kh-motifs)."""
    return k * (k - 1) * (k ** 5 + k ** 4 + 4 * k ** 3 + k ** 2 - 4 * k + 2) // 6
