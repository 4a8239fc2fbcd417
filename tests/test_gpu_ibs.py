"""GPU parity for the IBS matrix: every count bit-exact against the oracle.

Small shapes are compared element by element (both paths, both layouts, with
missing masks, sample lists, variant ranges, ragged tails).  The 10,000 x
100,000 workload runs in the configuration the benchmark times and is checked
on sampled pairs the oracle computes one by one, plus whole-matrix properties.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

pg = pytest.importorskip("paper_1410_4803_amd")

PATHS = ["popc", "mfma", "fp4", "fp4rep", "w8", "w8nh"]
# path codes: "fp4" / "fp4rep" are matrix-core variants 3 and 4 (fp4 operands,
# from the 2-bit and from the replicated layout); "w8" / "w8nh" are variants
# 5 and 6 (eight waves of 64x32, with and without scheduling hints)
CODES = {"popc": 1, "mfma": 2, "fp4": 2 | (3 << 8), "fp4rep": 2 | (4 << 8), "w8": 2 | (5 << 8),
         "w8nh": 2 | (6 << 8)}


def _cohort(bed, n, mask=None):
    return pg.Cohort.from_numpy(bed, n, mask)


def _check_full(got, ref):
    for name, g, r in zip(("ibs0", "ibs1", "ibs2", "n"), got, ref):
        g = g.cpu().numpy().view(np.uint32)
        assert g.shape == r.shape
        bad = np.argwhere(g != r)
        assert bad.size == 0, f"{name}: {len(bad)} mismatches, first {bad[:3].tolist()}"


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("n,V", [(1, 1), (2, 1), (3, 17), (5, 31), (63, 33), (64, 256),
                                 (65, 257), (127, 100), (128, 1000), (129, 4097), (300, 515)])
def test_ibs_shapes_full_and_tri(path, n, V):
    bed = synth.hwe(n, V, (0.05, 0.5), 0.05, seed=n * 1000 + V, garbage_pad=True)
    codes = oracle.unpack(bed, n, V)
    ref_full = oracle.ibs_matrix(codes, full=True)
    ref_tri = oracle.ibs_matrix(codes, full=False)
    c = _cohort(bed, n)
    _check_full(pg.ibs_matrix(c, layout="full", path=CODES[path]), ref_full)
    got = pg.ibs_matrix(c, layout="tri", path=CODES[path])
    _check_full(got, ref_tri)


@pytest.mark.parametrize("path", PATHS)
def test_ibs_mask_selection_range(path):
    n, V = 211, 3001
    bed = synth.mosaic(n, V, miss=0.02, seed=77, garbage_pad=True)
    mask = synth.missing_mask(n, V, 0.03, seed=78)
    rng = np.random.default_rng(5)
    idx = rng.integers(0, n, 150).astype(np.int32)
    idx[10] = idx[20]                                        # duplicates allowed
    vb, ve = 123, 2890
    codes = oracle.select(oracle.unpack(bed, n, V, mask), idx, vb, ve)
    ref = oracle.ibs_matrix(codes, full=True)
    c = _cohort(bed, n, mask)
    got = pg.ibs_matrix(c, sample_idx=torch.from_numpy(idx).cuda(), v_range=(vb, ve),
                        layout="full", path=CODES[path])
    _check_full(got, ref)
    ref_t = oracle.ibs_matrix(codes, full=False)
    got_t = pg.ibs_matrix(c, sample_idx=torch.from_numpy(idx).cuda(), v_range=(vb, ve),
                          layout="tri", path=CODES[path])
    _check_full(got_t, ref_t)


@pytest.mark.parametrize("path", PATHS)
def test_ibs_degenerate(path):
    n, V = 70, 200
    bed = synth.hwe(n, V, seed=4)
    codes = oracle.unpack(bed, n, V)
    codes[:, 3] = 1                          # all-missing sample
    codes[:, 9] = 3                          # monomorphic sample
    codes[17, :] = 1                         # all-missing variant
    # repack by hand: variant-major, 4 calls per byte
    packed = np.zeros((V, (n + 3) // 4), dtype=np.uint8)
    for k in range(n):
        packed[:, k // 4] |= (codes[:, k].astype(np.uint8) << (2 * (k % 4)))
    ref = oracle.ibs_matrix(codes, full=True)
    _check_full(pg.ibs_matrix(_cohort(packed, n), layout="full", path=CODES[path]), ref)
    # a sample list with an out-of-range entry reads as all missing
    idx = np.array([0, 5, n + 7, 2], dtype=np.int32)
    got = pg.ibs_matrix(_cohort(packed, n), sample_idx=torch.from_numpy(idx).cuda(), path=CODES[path])
    assert (got[3].cpu().numpy()[2] == 0).all() and (got[3].cpu().numpy()[:, 2] == 0).all()


def test_ibs_paths_agree_and_deterministic():
    w = synth.ibs_small()
    c = _cohort(w["bed"], w["n"])
    a = pg.ibs_matrix(c, layout="tri", path="popc")
    b = pg.ibs_matrix(c, layout="tri", path="mfma")
    b2 = pg.ibs_matrix(c, layout="tri", path="mfma")
    f4 = pg.ibs_matrix(c, layout="tri", path=CODES["fp4"])
    f4r = pg.ibs_matrix(c, layout="tri", path=CODES["fp4rep"])
    for x, y, z, u, r in zip(a, b, b2, f4, f4r):
        assert torch.equal(x, y) and torch.equal(y, z) and torch.equal(z, u) and torch.equal(u, r)


@pytest.mark.parametrize("path", PATHS)
def test_ibs_small_workload_exact(path):
    """500 samples x 5,000 variants, HWE, 1% missing: all 124,750 pairs."""
    w = synth.ibs_small()
    codes = oracle.unpack(w["bed"], w["n"], w["V"])
    ref = oracle.ibs_matrix(codes, full=False)
    got = pg.ibs_matrix(_cohort(w["bed"], w["n"]), layout="tri", path=CODES[path])
    assert got[0].numel() == 124750
    _check_full(got, ref)


@pytest.fixture(scope="module")
def large():
    w = synth.ibs_large()
    c = _cohort(w["bed"], w["n"])
    return w, c


def test_ibs_large_default_matches_variant_one(large):
    """At 10,000 x 100,000 the whole matrix of the default matrix-core kernel
    equals that of variant 1 (the same tile body without scheduling hints),
    every entry, not just the sampled pairs below."""
    w, c = large
    a = pg.ibs_matrix(c, layout="full", path=CODES["mfma"])
    b = pg.ibs_matrix(c, layout="full", path=CODES["mfma"] | (1 << 8))
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.mark.parametrize("path", PATHS)
def test_ibs_large_workload_sampled(large, path):
    """10,000 x 100,000 mosaic, full matrix, in the benchmark's launch
    configuration; 3,000 sampled pairs (plus diagonal entries and the tile
    corners) against the oracle, and whole-matrix properties."""
    w, c = large
    n, V = w["n"], w["V"]
    out = pg.ibs_matrix(c, layout="full", path=CODES[path])
    torch.cuda.synchronize()
    rng = np.random.default_rng(99)
    pi = rng.integers(0, n, 3000)
    pj = rng.integers(0, n, 3000)
    edges = np.array([0, 1, 63, 64, 127, 128, 129, 9983, 9984, 9998, 9999])
    pi = np.concatenate([pi, edges, np.repeat(edges, len(edges))])
    pj = np.concatenate([pj, edges, np.tile(edges, len(edges))])
    codes_sm = oracle.unpack(w["bed"], n, V, sample_major=True)
    ref = oracle.ibs_pairs(codes_sm, pi, pj)
    ti = torch.from_numpy(pi).cuda()
    tj = torch.from_numpy(pj).cuda()
    got = np.stack([o[ti, tj].cpu().numpy().view(np.uint32) for o in out], 1)
    assert np.array_equal(got, ref)
    i0, i1, i2, nm = out
    assert torch.equal(i0 + i1 + i2, nm)
    for o in out:
        assert torch.equal(o, o.T)
    assert (torch.diagonal(i0) == 0).all() and (torch.diagonal(i1) == 0).all()
    nonmiss = (codes_sm != 1).sum(1)
    assert np.array_equal(torch.diagonal(nm).cpu().numpy(), nonmiss)
    assert np.array_equal(torch.diagonal(i2).cpu().numpy(), nonmiss)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("n,extra", [(97, 0), (97, 5), (160, 3), (1000, 0)])
def test_ibs_mask_and_row_stride(path, n, extra):
    """Missing mask with all samples (the transposing layout path), rows
    padded to a stride larger than ceil(n/4) with garbage bytes."""
    V = 777
    bed = synth.hwe(n, V, (0.05, 0.5), 0.02, seed=n + extra, garbage_pad=True)
    mask = synth.missing_mask(n, V, 0.04, seed=n + 1)
    if extra:
        junk = np.random.default_rng(n).integers(0, 256, (V, extra), dtype=np.uint8)
        bed = np.concatenate([bed, junk], axis=1)
    codes = oracle.unpack(bed, n, V, mask)
    ref = oracle.ibs_matrix(codes, full=True)
    got = pg.ibs_matrix(_cohort(bed, n, mask), layout="full", path=CODES[path])
    _check_full(got, ref)
    for variant in (1, 2):
        if path == "mfma":
            got = pg.ibs_matrix(_cohort(bed, n, mask), layout="full", path=2 | (variant << 8))
            _check_full(got, ref)


def _offset_cohort(bed, n, mask, shift):
    """A cohort whose .bed buffer starts `shift` bytes past an allocation's
    start (so its rows need not start on a dword boundary)."""
    flat = np.concatenate([np.full(shift, 0xA5, np.uint8), bed.ravel()])
    t = torch.from_numpy(flat).cuda()[shift:]
    m = None if mask is None else torch.from_numpy(np.ascontiguousarray(mask).view(np.int64)).cuda()
    return pg.Cohort(t, n, bed.shape[0], bed.shape[1], m)


@pytest.mark.parametrize("path", ["popc", "mfma", "fp4rep"])
@pytest.mark.parametrize("n,V,vb,ve,shift,masked", [
    (97, 300, 7, 251, 1, True),      # 25-byte rows, the range starts inside a dword
    (1000, 200, 3, 200, 2, True),    # 250-byte rows, the range ends at the buffer's end
    (160, 90, 0, 90, 0, False),      # 40-byte rows, dword-aligned
    (160, 90, 5, 61, 3, False),      # the same rows off a dword boundary
    (5, 4, 2, 3, 3, True),           # one 2-byte row: too small for dword reads
    (2, 9, 0, 9, 1, False),          # nine 1-byte rows
])
def test_ibs_variant_range_without_sample_list(path, n, V, vb, ve, shift, masked):
    """Variant ranges over all samples: the whole-row reader's edge cases."""
    bed = synth.hwe(n, V, (0.05, 0.5), 0.02, seed=n + V + vb)
    mask = synth.missing_mask(n, V, 0.04, seed=n + 3) if masked else None
    codes = oracle.select(oracle.unpack(bed, n, V, mask), None, vb, ve)
    c = _offset_cohort(bed, n, mask, shift)
    for layout in ("full", "tri"):
        ref = oracle.ibs_matrix(codes, full=layout == "full")
        got = pg.ibs_matrix(c, v_range=(vb, ve), layout=layout, path=CODES[path])
        _check_full(got, ref)


def test_ibs_medium_cohort_k_split():
    """1,800 samples (120 tiles of 128): the default matrix-core kernel splits
    each tile's 32 chunks of 256 variants into two ranges; every pair against
    the oracle."""
    n, V = 1800, 8000
    bed = synth.hwe(n, V, (0.05, 0.5), 0.02, seed=1800)
    codes = oracle.unpack(bed, n, V)
    ref = oracle.ibs_matrix(codes, full=False)
    got = pg.ibs_matrix(_cohort(bed, n), layout="tri", path=CODES["mfma"])
    _check_full(got, ref)
