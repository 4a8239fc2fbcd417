"""Pins for the oracle's IBS distance and complete-linkage clustering
(section "Identity-by-state matrices, complete linkage clustering", under
the readings stated in oracle.c):

- the distance equals 1 - (IBS2 + IBS1/2) / N computed in exact rationals
  and rounded once; it is 0 on the diagonal and +inf without markers;
- a hand-worked 4-sample merge sequence, and one made only of ties (the
  tie rule alone decides it);
- scipy.cluster.hierarchy.linkage(method="complete") on tie-free random
  distances: the same heights and the same partition after every merge;
- invariants: heights never decrease; every height is the largest distance
  between the two merged clusters' members.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy.cluster.hierarchy import linkage
from scipy.spatial.distance import squareform

import oracle
import synth


def test_ibs_distance_exact():
    n, V = 40, 300
    codes = oracle.unpack(synth.hwe(n, V, (0.05, 0.5), 0.05, seed=3), n, V)
    i0, i1, i2, nm = oracle.ibs_matrix(codes, full=True)
    d = oracle.ibs_distance(i0, i1, nm)
    for i in range(0, n, 7):
        for j in range(n):
            s = Fraction(int(i2[i, j]) * 2 + int(i1[i, j]), 2 * int(nm[i, j]))
            assert d[i, j] == float(1 - s)
    assert np.all(np.diag(d) == 0.0)
    z = np.zeros(4, dtype=np.uint32)
    assert np.all(np.isinf(oracle.ibs_distance(z, z, z)))


def test_cluster_hand_worked():
    d = np.array([[0, 1, 4, 5], [1, 0, 3, 6], [4, 3, 0, 2], [5, 6, 2, 0]], float)
    m = oracle.cluster_complete(d)
    assert m.tolist() == [(0, 1, 1.0), (2, 3, 2.0), (0, 2, 6.0)]


def test_cluster_ties_follow_the_index_rule():
    d = np.ones((4, 4)) - np.eye(4)
    m = oracle.cluster_complete(d)
    assert m.tolist() == [(0, 1, 1.0), (0, 2, 1.0), (0, 3, 1.0)]


def _partitions_from_merges(m, n):
    rep = {i: {i} for i in range(n)}
    out = []
    for a, b, _ in m:
        rep[a] = rep[a] | rep.pop(b)
        out.append(frozenset(frozenset(s) for s in rep.values()))
    return out


def _partitions_from_scipy(Z, n):
    members = {i: {i} for i in range(n)}
    out = []
    for t, (x, y, _, _) in enumerate(Z):
        members[n + t] = members.pop(int(x)) | members.pop(int(y))
        out.append(frozenset(frozenset(s) for s in members.values()))
    return out


@pytest.mark.parametrize("n,seed", [(5, 1), (30, 2), (120, 3)])
def test_cluster_matches_scipy_complete_linkage(n, seed):
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 3))
    d = np.sqrt(((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1))
    m = oracle.cluster_complete(d)
    Z = linkage(squareform(d, checks=False), method="complete")
    assert np.allclose(m["height"], Z[:, 2], rtol=0, atol=1e-15)
    assert _partitions_from_merges(m, n) == _partitions_from_scipy(Z, n)


def test_cluster_invariants_on_ibs_distances():
    n, V = 60, 2000
    codes = oracle.unpack(synth.mosaic(n, V, 6, 0.01, 0.001, 0.0, 0.02, seed=4), n, V)
    i0, i1, _, nm = oracle.ibs_matrix(codes, full=True)
    d = oracle.ibs_distance(i0, i1, nm)
    m = oracle.cluster_complete(d)
    assert np.all(np.diff(m["height"]) >= 0)
    members = {i: [i] for i in range(n)}
    for a, b, h in m:
        assert a < b
        assert h == max(d[x, y] for x in members[a] for y in members[b])
        members[a] += members.pop(b)
