"""GPU parity for the IBS distance (bit for bit: the same correctly rounded
quotient of integers) and complete-linkage clustering (the merge sequence
bit for bit: every decision compares maxima of those doubles), including
tie-heavy inputs, samples without markers (+inf distances) and the full
1,000-sample workload; the 10,000-sample workload is checked for a valid,
monotone hierarchy whose first merge is the global closest pair."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

pg = pytest.importorskip("paper_1410_4803_amd")


def _ibs(bed, n):
    c = pg.Cohort.from_numpy(bed, n)
    return pg.ibs_matrix(c, layout="full")


def _cluster(counts, m):
    out = pg.ibs_cluster(*counts)
    torch.cuda.synchronize()
    return pg.merges_to_numpy(out, m)


def test_distance_bit_exact():
    n, V = 150, 900
    bed = synth.hwe(n, V, (0.05, 0.5), 0.03, seed=51)
    counts = _ibs(bed, n)
    d = pg.ibs_distance(counts[0], counts[1], counts[3])
    ref = oracle.ibs_distance(*(t.cpu().numpy().view(np.uint32) for t in (counts[0], counts[1],
                                                                          counts[3])))
    assert np.array_equal(d.cpu().numpy(), ref)


@pytest.mark.parametrize("m,V", [(1, 50), (2, 50), (3, 80), (17, 300), (64, 500), (65, 500),
                                 (300, 2000)])
def test_cluster_parity(m, V):
    bed = synth.mosaic(m, V, 5, 0.02, 0.001, 0.0, 0.02, seed=m + V)
    codes = oracle.unpack(bed, m, V)
    i0, i1, _, nm = oracle.ibs_matrix(codes, full=True)
    ref = oracle.cluster_complete(oracle.ibs_distance(i0, i1, nm))
    got = _cluster(_ibs(bed, m), m)
    assert len(got) == m - 1
    assert np.array_equal(got["a"], ref["a"]) and np.array_equal(got["b"], ref["b"])
    assert np.array_equal(got["height"], ref["height"])


def test_cluster_ties_and_empty_samples():
    """Duplicated samples (distance 0 ties), few markers (coarse distances),
    and two samples without any call (+inf to everyone)."""
    n0, V = 40, 12
    codes = oracle.unpack(synth.hwe(n0, V, (0.2, 0.5), 0.0, seed=52), n0, V)
    codes = np.concatenate([codes, codes[:, :15], codes[:, 5:10]], axis=1)
    codes[:, 3] = 1
    codes[:, 44] = 1
    m = codes.shape[1]
    bed = np.zeros((V, (m + 3) // 4), dtype=np.uint8)
    for k in range(m):
        bed[:, k // 4] |= codes[:, k].astype(np.uint8) << (2 * (k % 4))
    i0, i1, _, nm = oracle.ibs_matrix(codes, full=True)
    ref = oracle.cluster_complete(oracle.ibs_distance(i0, i1, nm))
    assert np.isinf(ref["height"][-1])
    got = _cluster(_ibs(bed, m), m)
    assert np.array_equal(got["a"], ref["a"]) and np.array_equal(got["b"], ref["b"])
    assert np.array_equal(got["height"], ref["height"])


def test_cluster_per_merge_launches_ties_and_empty_samples():
    """From 3,200 samples each merge runs as three launches over the chip:
    3,300 samples over 60 markers (coarse distances, many ties), 300
    duplicated samples (distance-0 ties) and two samples without any call
    (+inf to everyone); the merge sequence equals the oracle's."""
    n0, V = 3000, 60
    codes = oracle.unpack(synth.hwe(n0, V, (0.2, 0.5), 0.0, seed=57), n0, V)
    codes = np.concatenate([codes, codes[:, :300]], axis=1)
    codes[:, 17] = 1
    codes[:, 2999] = 1
    m = codes.shape[1]
    bed = np.zeros((V, (m + 3) // 4), dtype=np.uint8)
    for k in range(m):
        bed[:, k // 4] |= codes[:, k].astype(np.uint8) << (2 * (k % 4))
    i0, i1, _, nm = oracle.ibs_matrix(codes, full=True)
    ref = oracle.cluster_complete(oracle.ibs_distance(i0, i1, nm))
    assert np.isinf(ref["height"][-1]) and (ref["height"] == 0).sum() >= 299
    got = _cluster(_ibs(bed, m), m)
    assert np.array_equal(got["a"], ref["a"]) and np.array_equal(got["b"], ref["b"])
    assert np.array_equal(got["height"], ref["height"])


def test_cluster_full_size_small_workload():
    """Complete linkage of the 1,000-sample relationship-matrix panel (the
    paper's clustering timings use the same two panel sizes)."""
    w = synth.grm_small()
    n, V = w["n"], w["V"]
    codes = oracle.unpack(w["bed"], n, V)
    i0, i1, _, nm = oracle.ibs_matrix(codes, full=True)
    ref = oracle.cluster_complete(oracle.ibs_distance(i0, i1, nm))
    got = _cluster(_ibs(w["bed"], n), n)
    assert np.array_equal(got["a"], ref["a"]) and np.array_equal(got["b"], ref["b"])
    assert np.array_equal(got["height"], ref["height"])


def test_cluster_full_size_large_workload_hierarchy():
    w = synth.grm_large()
    n = w["n"]
    counts = _ibs(w["bed"], n)
    got = _cluster(counts, n)
    d = pg.ibs_distance(counts[0], counts[1], counts[3])
    d.fill_diagonal_(float("inf"))
    flat = int(torch.argmin(d).item())          # first minimal entry in row-major order
    i, j = divmod(flat, n)
    assert (got["a"][0], got["b"][0]) == (min(i, j), max(i, j))
    assert got["height"][0] == d[i, j].item()
    assert np.all(np.diff(got["height"]) >= 0)
    alive = np.ones(n, dtype=bool)
    for a, b in zip(got["a"], got["b"]):
        assert a < b and alive[a] and alive[b]
        alive[b] = False
    assert alive.sum() == 1 and alive[0]


def test_cluster_full_size_large_workload_exact():
    """Complete linkage of the 10,000-sample panel, merge for merge (pair and
    height, ties included) against the oracle's sequence stored by
    tests/golden/make_fullsize.py (oracle IBS counts -> oracle distance ->
    oracle clustering on the same seeded panel, whose hash the file
    records)."""
    import os
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import make_fullsize
    sha, ref = make_fullsize.load_cluster()
    w = synth.grm_large()
    n = w["n"]
    assert make_fullsize.bed_sha256(w["bed"]) == sha, "stored merges were computed from another panel"
    assert len(ref) == n - 1
    got = _cluster(_ibs(w["bed"], n), n)
    assert np.array_equal(got["a"], ref["a"]) and np.array_equal(got["b"], ref["b"])
    assert np.array_equal(got["height"], ref["height"])
