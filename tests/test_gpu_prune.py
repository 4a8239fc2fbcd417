"""GPU parity for greedy LD pruning: the keep flags equal the oracle's
bit for bit (both sides decide r^2 > t on the same double and compare minor
allele frequencies exactly), on both pair-kernel paths, across tile edges,
ragged ranges, sample lists, missing masks, dense offending sets (several
LDS slices per pass), large windows (several passes per window) and more
variants than the kernel's ring of keep bits holds."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

pg = pytest.importorskip("paper_1410_4803_amd")

PATHS = ["mfma", "popc", "sparse", 2 | (1 << 8)]   # the last: the int8 matrix-core tile


def _gpu(bed, n, W, S, t, mask=None, **kw):
    c = pg.Cohort.from_numpy(bed, n, mask)
    keep, n_kept = pg.ld_prune(c, W, S, t, **kw)
    torch.cuda.synchronize()
    k = keep.cpu().numpy()
    assert int(n_kept.item()) == int(k.sum())
    return k


def _check(bed, n, V, W, S, t, path, mask=None):
    codes = oracle.unpack(bed, n, V, mask)
    ref = oracle.ld_prune(codes, W, S, t)
    got = _gpu(bed, n, W, S, t, mask, path=path)
    bad = np.nonzero(got != ref)[0]
    assert bad.size == 0, f"{bad.size} flags differ, first at {bad[:8]}"
    return ref


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("n,V,W,S,t", [
    (1, 5, 2, 1, -1.0), (17, 65, 3, 1, 0.1), (63, 130, 50, 5, 0.5), (129, 1000, 50, 5, 0.5),
    (300, 2000, 200, 20, 0.3), (100, 500, 40, 40, 0.2), (50, 30, 100, 10, 0.1),
    (64, 64, 64, 64, 0.05), (200, 777, 65, 1, 0.4)])
def test_prune_parity(n, V, W, S, t, path):
    bed = synth.mosaic(n, V, 6, 0.02, 0.001, 0.0, 0.02, seed=n + V + W + S, garbage_pad=True)
    ref = _check(bed, n, V, W, S, t, path)
    if t >= 0.1 and V >= 100:
        assert 0 < ref.sum() < V          # something dropped, something kept


@pytest.mark.parametrize("path", PATHS)
def test_prune_dense_offending_pairs(path):
    """Threshold below 0: every defined pair offends, so one pass stages far
    more pairs than one LDS slice holds."""
    n, V = 80, 3000
    bed = synth.hwe(n, V, (0.05, 0.5), 0.01, seed=21)
    ref = _check(bed, n, V, 100, 50, -1.0, path)
    assert ref.sum() < V // 10


@pytest.mark.parametrize("path", PATHS)
def test_prune_large_window(path):
    """A window wider than one pass of (window, row) cells."""
    n, V = 64, 12000
    bed = synth.mosaic(n, V, 4, 0.002, 0.001, 0.0, 0.01, seed=22)
    _check(bed, n, V, 5000, 1000, 0.6, path)


def test_prune_ring_wraps():
    """More variants than the ring of keep bits (2^18) in the greedy kernel."""
    n, V = 16, 300000
    bed = synth.mosaic(n, V, 3, 0.05, 0.001, 0.0, 0.0, seed=23)
    ref = _check(bed, n, V, 20, 7, 0.5, "mfma")
    assert 0 < ref.sum() < V


@pytest.mark.parametrize("path", ["mfma", "sparse"])
def test_prune_step_one(path):
    """Step 1: the most (window, row) cells a window allows, all counted
    grid-wide in the workspace the step-free size query reserves."""
    n, V = 64, 3000
    bed = synth.mosaic(n, V, 4, 0.01, 0.001, 0.0, 0.01, seed=31)
    ref = _check(bed, n, V, 100, 1, 0.4, path)
    assert 0 < ref.sum() < V


def test_prune_cells_beyond_the_count_scratch():
    """More than 2^26 (window, row) cells: the greedy pass counts its cells
    in its own block instead."""
    n, V = 16, 300000
    assert (V - 300 + 1) * 300 > 1 << 26
    bed = synth.mosaic(n, V, 3, 0.05, 0.001, 0.0, 0.0, seed=32)
    ref = _check(bed, n, V, 300, 1, 0.5, "mfma")
    assert 0 < ref.sum() < V


def test_prune_no_threshold_crossing():
    n, V = 100, 400
    bed = synth.mosaic(n, V, 3, 0.01, 0.001, 0.0, 0.0, seed=24)
    assert _gpu(bed, n, 30, 3, 1.0).all()
    assert _gpu(bed, n, 30, 3, float("inf")).all()


@pytest.mark.parametrize("path", PATHS)
def test_prune_mask_selection_range(path):
    n, V = 400, 2500
    bed = synth.mosaic(n, V, 8, 0.01, 0.001, 0.0, 0.01, seed=25, garbage_pad=True)
    mask = synth.missing_mask(n, V, 0.03, seed=26)
    rng = np.random.default_rng(2)
    idx = rng.integers(0, n, 257).astype(np.int32)
    vb, ve = 131, 2411
    codes = oracle.select(oracle.unpack(bed, n, V, mask), idx, vb, ve)
    ref = oracle.ld_prune(codes, 70, 7, 0.5)
    got = _gpu(bed, n, 70, 7, 0.5, mask, sample_idx=torch.from_numpy(idx).cuda(),
               v_range=(vb, ve), path=path)
    assert np.array_equal(got, ref)
    assert 0 < ref.sum() < ve - vb


def test_prune_special_variants_and_repeat():
    """Duplicates and allele flips (r^2 = 1), an all-missing and a
    monomorphic variant (r^2 undefined: never compared); two calls give
    identical flags."""
    n, V = 150, 90
    codes = oracle.unpack(synth.mosaic(n, V, 5, 0.05, 0.001, 0.0, 0.02, seed=27), n, V)
    codes[11] = codes[10]
    codes[12] = np.where(codes[10] == 0, 3, np.where(codes[10] == 3, 0, codes[10]))
    codes[30] = 1
    codes[31] = 3
    bed = np.zeros((V, (n + 3) // 4), dtype=np.uint8)
    for k in range(n):
        bed[:, k // 4] |= codes[:, k].astype(np.uint8) << (2 * (k % 4))
    ref = oracle.ld_prune(codes, 15, 4, 0.3)
    assert ref[11] == 0 and ref[12] == 0 and ref[30] == 1 and ref[31] == 1
    for path in PATHS:
        a = _gpu(bed, n, 15, 4, 0.3, path=path)
        b = _gpu(bed, n, 15, 4, 0.3, path=path)
        assert np.array_equal(a, ref) and np.array_equal(b, ref)


def test_prune_full_size_small_workload():
    """The whole 1,000 x 100,000 --indep-pairwise 50 5 0.5 workload the
    benchmark times, flag for flag."""
    wp = synth.prune_small()
    codes = oracle.unpack(wp["bed"], wp["n"], wp["V"])
    ref = oracle.ld_prune(codes, wp["window"], wp["step"], wp["r2_max"])
    for path in ("mfma", "sparse"):
        got = _gpu(wp["bed"], wp["n"], wp["window"], wp["step"], wp["r2_max"], path=path)
        assert np.array_equal(got, ref), path


def _golden():
    import os
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import make_fullsize
    return make_fullsize


def test_prune_full_size_large_workload():
    """The whole 10,000 x 88,025 --indep-pairwise 700 70 0.7 workload the
    benchmark times, flag for flag against the oracle's flags stored by
    tests/golden/make_fullsize.py (computed from the same seeded panel,
    whose hash the file records), on every pair-kernel path."""
    gold = _golden()
    sha, ref = gold.load_prune()
    wp = synth.prune_large()
    assert gold.bed_sha256(wp["bed"]) == sha, "stored flags were computed from another panel"
    assert len(ref) == wp["V"]
    for path in PATHS:
        got = _gpu(wp["bed"], wp["n"], wp["window"], wp["step"], wp["r2_max"], path=path)
        assert np.array_equal(got, ref), path
