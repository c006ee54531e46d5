"""Pins of the oracle's pattern tables against facts the paper states."""
import itertools

import numpy as np
import pytest

from conftest import golden
from oracle import native, patterns as P


@pytest.mark.parametrize("row", golden("hmotif_census.txt"))
def test_census_matches_paper_table(row):
    k, raw, orbits, conn, valid = map(int, row)
    got = P.pattern_census(k)
    assert (got["raw"], got["orbits"], got["connected"], got["valid"]) == (raw, orbits, conn, valid)


@pytest.mark.parametrize("row", golden("khmotif_counts.txt"))
def test_kh_motif_closed_form(row):
    k, n = map(int, row)
    assert P.kh_motif_closed_form(k) == n


@pytest.mark.parametrize("states,expected", [(2, 26), (3, 431), (4, 3076)])
def test_state_census_equals_kh_count(states, expected):
    # k-state refinements of three-hyperedge patterns (section 5.1)
    assert P.pattern_census(3, states)["valid"] == expected


def test_tables_sizes():
    assert len(P.hmotif_table()) == 26
    assert len(P.tmotif_table()) == 431


def test_open_closed_layout():
    # h-motifs 17-22 are open, the others closed (figure caption, section 2.2)
    t = P.hmotif_table()
    assert [i + 1 for i, p in enumerate(t) if P.is_open(p)] == list(range(17, 23))
    # 16 has all seven regions non-empty (section 6.2 discussion of h-motif 16)
    assert t[15] == (1,) * 7


def test_17_18_are_hyperedge_with_two_disjoint_subsets():
    # one hyperedge containing two disjoint hyperedges (section 6.2)
    for p in P.hmotif_table()[16:18]:
        found = False
        for perm in P.PERMS3:
            q = P.relabel(p, perm)
            # e_i, e_j inside e_k, e_i and e_j disjoint: R1=R2=R4=R7=0
            if q[0] == q[1] == q[3] == q[6] == 0:
                found = True
        assert found


def test_duplicate_only_patterns():
    # four connected patterns need identical hyperedges (figure of patterns
    # that cannot be obtained from distinct hyperedges)
    dup = sorted({P.canonical(p) for p in itertools.product((0, 1), repeat=7)
                  if P.is_connected(p) and not P.is_distinct(p)})
    regions = [{f"R{r + 1}" for r in range(7) if p[r]} for p in dup]
    assert len(dup) == 4
    assert sorted(map(sorted, regions)) == sorted(map(sorted, [{"R7"}, {"R6", "R7"}, {"R3", "R7"},
                                                               {"R3", "R4", "R7"}]))


def _automorphisms(p):
    return [perm for perm in P.PERMS3 if P.relabel(p, perm) == p]


def test_3h_children_by_burnside():
    # Children of an h-motif under the ternary refinement counted by Burnside's
    # lemma over the pattern's automorphism group: each non-empty region takes
    # one of 2 non-zero states; a group element fixes a refinement iff it is
    # constant on the element's cycles of non-empty regions.
    counts = {}
    for _p, parent in P.tmotif_table():
        counts[parent] = counts.get(parent, 0) + 1
    for hid, p in enumerate(P.hmotif_table(), start=1):
        aut = _automorphisms(p)
        total = 0
        for perm in aut:
            image = [P.REGIONS3.index(frozenset(perm[x] for x in s)) for s in P.REGIONS3]
            seen, cycles = set(), 0
            for r in range(7):
                if p[r] and r not in seen:
                    cycles += 1
                    q = r
                    while q not in seen:
                        seen.add(q)
                        q = image[q]
            total += 2 ** cycles
        assert total % len(aut) == 0
        assert counts[hid] == total // len(aut), hid


def test_h1_splits_into_six():
    # 3h-motifs 1-6 are the six subdivisions of h-motif 1 (section 5.1)
    t3 = P.tmotif_table()
    assert [parent for _p, parent in t3[:6]] == [1] * 6
    assert t3[6][1] != 1
    h1 = P.hmotif_table()[0]
    # one region singled out, two symmetric ones
    aut = _automorphisms(h1)
    assert len(aut) == 2


def test_native_classifier_agrees_with_python_on_every_ternary_pattern():
    # Feeding cardinalities equal to the states (theta=1) must give the same id
    # from the C++ canonicaliser as from the Python one.
    for trit in itertools.product((0, 1, 2), repeat=7):
        py = P.classify_counts(trit)
        c = native.classify(list(trit))
        assert c == (0 if py is None else py[1]), trit


def test_classifier_relabel_invariant():
    rng = np.random.default_rng(5)
    for _ in range(300):
        card = rng.integers(0, 4, size=7).tolist()
        base = native.classify(card)
        for perm in P.PERMS3:
            assert native.classify(list(P.relabel(card, perm))) == base


def test_theta_buckets():
    # 0 -> empty, 1..theta -> state 1, > theta -> state 2
    base = [0, 0, 0, 0, 3, 3, 3]
    for theta in (1, 2, 3):
        a = native.classify([0, 0, 0, 0, theta, theta, theta], theta)
        b = native.classify([0, 0, 0, 0, theta + 1, theta + 1, theta + 1], theta)
        assert a != b and a and b
    assert native.classify(base, 3) == native.classify([0, 0, 0, 0, 1, 1, 1], 1)
