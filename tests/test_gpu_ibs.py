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

PATHS = ["popc", "mfma", "fp4", "fp4rep", "w8", "w8nh", "pipe", "fp4pipe", "r1"]
# path codes: "fp4" / "fp4rep" are matrix-core variants 3 and 4 (fp4 operands,
# from the 2-bit and from the replicated layout); "w8" / "w8nh" are variants
# 5 and 6 (eight waves of 64x32, with and without scheduling hints); "pipe" is
# variant 7 (int8, the chunk boundaries pipelined), "fp4pipe" variant 8 (the
# same with fp4 operands: the default kernel, "mfma"), "r1" variant 9 (int8,
# unpipelined)
CODES = {"popc": 1, "mfma": 2, "fp4": 2 | (3 << 8), "fp4rep": 2 | (4 << 8), "w8": 2 | (5 << 8),
         "w8nh": 2 | (6 << 8), "pipe": 2 | (7 << 8),
         "fp4pipe": 2 | (8 << 8), "r1": 2 | (9 << 8)}


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
    """The 10,000 x 100,000 workload in the benchmark's launch configuration
    (full layout, default matrix-core kernel), computed once."""
    w = synth.ibs_large()
    c = _cohort(w["bed"], w["n"])
    ref = pg.ibs_matrix(c, layout="full", path=CODES["mfma"])
    torch.cuda.synchronize()
    return w, c, ref


def test_ibs_large_rows_vs_oracle(large):
    """32 whole rows of the 10,000 x 100,000 matrix (320,000 pairs, the tile
    edges among them) against the oracle, every count, plus whole-matrix
    properties of the default kernel's output."""
    w, c, out = large
    n, V = w["n"], w["V"]
    rng = np.random.default_rng(2024)
    edges = np.array([0, 1, 63, 64, 127, 128, 4999, 9871, 9983, 9984, 9998, 9999])
    others = rng.choice(np.setdiff1d(np.arange(n), edges), 20, replace=False)
    rows = np.sort(np.concatenate([edges, others]))
    assert len(rows) == 32
    codes_sm = oracle.unpack(w["bed"], n, V, sample_major=True)
    pi = np.repeat(rows, n)
    pj = np.tile(np.arange(n), len(rows))
    ref = oracle.ibs_pairs(codes_sm, pi, pj).reshape(len(rows), n, 4)
    tr = torch.from_numpy(rows).cuda()
    for k, o in enumerate(out):
        got = o[tr].cpu().numpy().view(np.uint32)
        bad = np.argwhere(got != ref[:, :, k])
        assert bad.size == 0, f"count {k}: {len(bad)} mismatches, first {bad[:3].tolist()}"
    i0, i1, i2, nm = out
    assert torch.equal(i0 + i1 + i2, nm)
    for o in out:
        assert torch.equal(o, o.T)
    assert (torch.diagonal(i0) == 0).all() and (torch.diagonal(i1) == 0).all()


@pytest.mark.parametrize("path", PATHS + ["mfma_v1"])
def test_ibs_large_paths_equal_whole_matrix(large, path):
    """Every other path and kernel variant gives the default kernel's whole
    10,000 x 10,000 output, all four counts, entry for entry (the default is
    pinned to the oracle by the rows above); 300 random pairs of each path
    also go to the oracle directly."""
    w, c, ref = large
    code = CODES["mfma"] | (1 << 8) if path == "mfma_v1" else CODES[path]
    out = pg.ibs_matrix(c, layout="full", path=code)
    torch.cuda.synchronize()
    for k, (x, y) in enumerate(zip(out, ref)):
        assert torch.equal(x, y), f"{path}: count {k} differs from the default kernel"
    n, V = w["n"], w["V"]
    rng = np.random.default_rng(sum(map(ord, path)))
    pi, pj = rng.integers(0, n, 300), rng.integers(0, n, 300)
    codes_sm = oracle.unpack(w["bed"], n, V, sample_major=True)
    r = oracle.ibs_pairs(codes_sm, pi, pj)
    ti, tj = torch.from_numpy(pi).cuda(), torch.from_numpy(pj).cuda()
    got = np.stack([o[ti, tj].cpu().numpy().view(np.uint32) for o in out], 1)
    assert np.array_equal(got, r)


def test_ibs_large_triangle_equals_full(large):
    """The packed upper-triangle layout at 10,000 x 100,000 holds exactly the
    full layout's strict upper triangle."""
    w, c, ref = large
    n = w["n"]
    tri = pg.ibs_matrix(c, layout="tri", path=CODES["mfma"])
    iu = torch.triu_indices(n, n, 1, device="cuda")
    for k, (t, f) in enumerate(zip(tri, ref)):
        assert torch.equal(t, f[iu[0], iu[1]]), f"count {k}"
