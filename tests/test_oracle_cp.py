"""Pins of the oracle's significance (Eq. 1), CP (Eq. 2) and A+ rescaling."""
import math

import numpy as np

from oracle import cp, patterns as P


def test_hand_example():
    M = [3, 0, 5, 2] + [0] * 22
    rand = [[1, 0, 5, 0] + [0] * 22, [1, 2, 5, 0] + [0] * 22]
    d = cp.significance(M, rand, eps=1.0)
    # (3-1)/(3+1+1), (0-1)/(0+1+1), 0, (2-0)/(2+0+1)
    assert d[:4] == [2 / 5, -1 / 2, 0.0, 2 / 3]
    assert all(x == 0.0 for x in d[4:])
    c = cp.characteristic_profile(d)
    n = math.sqrt((2 / 5) ** 2 + (1 / 2) ** 2 + (2 / 3) ** 2)
    assert abs(c[0] - 0.4 / n) < 1e-15 and abs(c[1] + 0.5 / n) < 1e-15


def test_unit_norm_and_bounds():
    rng = np.random.default_rng(0)
    for _ in range(50):
        M = rng.integers(0, 10 ** 12, size=26).tolist()
        rand = [rng.integers(0, 10 ** 12, size=26).tolist() for _ in range(5)]
        c = cp.characteristic_profile(cp.significance(M, rand))
        assert abs(math.fsum(x * x for x in c) - 1.0) < 1e-14
        assert all(-1.0 <= x <= 1.0 for x in c)


def test_sign_and_epsilon():
    d = cp.significance([10, 0, 7], [[4, 0, 7]])
    assert d[0] > 0 and d[1] == 0.0 and d[2] == 0.0
    # eps keeps Delta defined when both counts are zero, and shrinks small counts
    assert cp.significance([1], [[0]], eps=1.0) == [0.5]
    assert cp.significance([1], [[0]], eps=0.0) == [1.0]


def test_degenerate_profile_is_zero():
    assert cp.characteristic_profile([0.0] * 26) == [0.0] * 26


def test_rescale_uses_open_closed_weights():
    raw = [6] * 26
    est = cp.aplus_estimate(raw, num_wedges=100, r=10)
    for t in range(1, 27):
        w = 2.0 if 17 <= t <= 22 else 3.0
        assert est[t - 1] == 6 * 100 / (w * 10)
    raw3 = [6] * 431
    est3 = cp.aplus_estimate3(raw3, 100, 10)
    parent = P.id3_to_id26()
    for t in range(431):
        w = 2.0 if 17 <= parent[t + 1] <= 22 else 3.0
        assert est3[t] == 6 * 100 / (w * 10)
