"""Pins of the oracle's hardware-aware ring (the future work of Sec. VI):
PE m of filter f is in group (f M + m) mod G; the ring visits the groups in a
random order and the members of each group in a random order."""
import itertools

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O


def _group(f, M, G, m):
    return (f * M + m) % G


@pytest.mark.parametrize("M,G,f", [(2, 8, 0), (5, 8, 1), (8, 8, 0), (64, 8, 3), (100, 7, 2),
                                   (257, 16, 1), (30, 30, 0), (1000, 3, 4)])
def test_single_cycle_and_group_crossings(M, G, f):
    for k in (1, 2, 99):
        pi, pred, succ = O.ring_groups(11, f, k, M, G)
        assert sorted(pi.tolist()) == list(range(M))
        # one cycle through all PEs
        m, seen = 0, set()
        for _ in range(M):
            seen.add(m)
            m = int(pred[m])
        assert m == 0 and len(seen) == M
        assert all(succ[pred[i]] == i for i in range(M))
        # each group's PEs are consecutive along the ring; only the edges
        # between groups cross
        groups = [_group(f, M, G, int(x)) for x in pi]
        nonempty = len(set(groups))
        runs = 1 + sum(groups[t] != groups[t - 1] for t in range(1, M))
        assert runs == nonempty
        cross = sum(_group(f, M, G, i) != _group(f, M, G, int(pred[i])) for i in range(M))
        assert cross == (nonempty if nonempty > 1 else 0)


def test_one_group_is_the_plain_ring():
    for M in (1, 2, 9, 64):
        for G in (0, 1):
            a = O.ring_groups(5, 2, 7, M, G)
            b = O.ring(5, 2, 7, M)
            for x, y in zip(a, b):
                assert np.array_equal(x, y)


def test_uniform_over_group_orders_and_member_orders():
    """M = 6, G = 2: 2 group orders x 3! x 3! member orders = 72 equally
    likely ring orders (chi-square over 14400 iterations)."""
    M, G, n = 6, 2, 14400
    counts = {}
    for k in range(1, n + 1):
        pi, _, _ = O.ring_groups(3, 0, k, M, G)
        key = tuple(pi.tolist())
        counts[key] = counts.get(key, 0) + 1
    assert len(counts) == 72
    obs = np.array(list(counts.values()))
    assert stats.chisquare(obs).pvalue > 1e-3
