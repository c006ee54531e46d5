"""Pins of the oracle's MoCHy-A (Algorithm 4): hyperedge sampling."""
import numpy as np

from oracle import cp, native
from workloads import from_edge_lists, make_config, powerlaw_hypergraph


def test_every_hyperedge_once_counts_each_instance_three_times():
    # each connected triple holds three hyperedges, so sampling every
    # hyperedge once counts it exactly three times
    for h in (make_config("tiny"), powerlaw_hypergraph(80, 300, 1, 7, 2.5, 1.0, seed=4)):
        raw26, raw431, inv, E = native.mochy_a_raw(h, indices=np.arange(h.num_edges), nthreads=4)
        assert inv == 0 and E == h.num_edges
        b26, b431, _ = native.bruteforce(h, nthreads=4)
        assert (raw26 == 3 * b26).all() and (raw431 == 3 * b431).all()


def test_single_samples_are_the_instances_of_that_hyperedge():
    h = from_edge_lists([[0, 1], [1, 2], [2, 3], [0, 4], [1, 3]], 5)
    b26, _, _ = native.bruteforce(h, nthreads=1)
    per = [native.mochy_a_raw(h, indices=[i], nthreads=1)[0] for i in range(h.num_edges)]
    assert (sum(per) == 3 * b26).all()
    # hyperedge 4 = {1, 3} meets 0, 1, 2: every connected triple through it
    import itertools
    mine = 0
    for a, b in itertools.combinations([x for x in range(5) if x != 4], 2):
        card = native.region_cards(h, 4, a, b)
        ij, jk, ki = card[3] + card[6] > 0, card[4] + card[6] > 0, card[5] + card[6] > 0
        mine += (ij and ki) or (ij and jk) or (jk and ki)
    assert per[4].sum() == mine


def test_estimates_are_unbiased():
    # the mean over seeds of |E|/(3s) * raw approaches the exact counts
    h = make_config("tiny")
    m26, _, _ = native.mochy_e(h, nthreads=4)
    s, R = 40, 60
    est = np.zeros(26)
    for seed in range(R):
        raw26, _, _, E = native.mochy_a_raw(h, s=s, seed=seed, nthreads=4)
        est += np.array(cp.mochy_a_estimate(raw26, E, s))
    est /= R
    big = m26 > 0.01 * m26.sum()
    rel = np.abs(est[big] - m26[big]) / m26[big]
    assert rel.max() < 0.15, rel


def test_hyperedge_profiles_sum_to_three_times_the_counts():
    # every instance is in the profile of each of its three hyperedges
    for h in (make_config("tiny"), powerlaw_hypergraph(60, 250, 1, 6, 2.5, 1.2, seed=8)):
        hp26, hp431, inv = native.hyperedge_profiles(h, nthreads=4)
        assert (inv == 0).all() and hp26.shape == (h.num_edges, 26)
        b26, b431, _ = native.bruteforce(h, nthreads=4)
        assert (hp26.sum(axis=0) == 3 * b26).all() and (hp431.sum(axis=0) == 3 * b431).all()


def test_hyperedge_profile_by_hand():
    # e0={0,1} e1={1,2} e2={2,3}: the path e0-e1-e2 is the only connected
    # triple (an open motif: e1 holds e0 ∩ e1 and e1 ∩ e2, disjoint)
    h = from_edge_lists([[0, 1], [1, 2], [2, 3]], 4)
    hp26, _, _ = native.hyperedge_profiles(h, nthreads=1)
    assert (hp26.sum(axis=1) == 1).all()
    t = int(np.argmax(hp26[0]))
    assert (hp26[:, t] == 1).all() and t + 1 in range(17, 23)
    b26, _, _ = native.bruteforce(h, nthreads=1)
    assert b26[t] == 1
