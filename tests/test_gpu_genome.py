"""GPU parity for the IBS similarity and the IBD report (--distance ibs,
--Z-genome), bit for bit against the oracle: both evaluate the same IEEE
double operations in the same order (per-marker terms, their sums in marker
order, the per-pair moment estimates), so every output double, and every NaN
position, must agree.  Covers both output layouts, sample lists, variant
ranges, missing-call masks, the undefined cases (no calls in common, no
informative marker), a small pedigree whose duplicate pair is exactly
Z2 = 1, and the 10,000 x 100,000 IBS workload on sampled rows."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

pg = pytest.importorskip("paper_1410_4803_amd")


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _same(got, ref):
    """Bit-for-bit equality of float64 arrays, NaN positions included."""
    g = np.ascontiguousarray(got, dtype=np.float64).view(np.uint64)
    r = np.ascontiguousarray(ref, dtype=np.float64).view(np.uint64)
    gn, rn = np.isnan(got), np.isnan(ref)
    assert np.array_equal(gn, rn), f"NaN positions differ: {np.argwhere(gn != rn)[:3].tolist()}"
    bad = np.argwhere((g != r) & ~gn)
    assert bad.size == 0, (f"{len(bad)} mismatches, first at {bad[:3].tolist()}: "
                           f"{got.reshape(-1)[bad[0][0]] if got.ndim == 1 else got[tuple(bad[0])]} "
                           f"vs {ref.reshape(-1)[bad[0][0]] if ref.ndim == 1 else ref[tuple(bad[0])]}")


def _bed_from_codes(codes_vm):
    V, m = codes_vm.shape
    bed = np.zeros((V, (m + 3) // 4), dtype=np.uint8)
    for k in range(m):
        bed[:, k // 4] |= codes_vm[:, k].astype(np.uint8) << (2 * (k % 4))
    return bed


def _gpu_genome(c, layout, sample_idx=None, v_range=None):
    sidx = None if sample_idx is None else torch.as_tensor(sample_idx, dtype=torch.int32).cuda()
    counts = pg.ibs_matrix(c, sample_idx=sidx, v_range=v_range, layout=layout)
    z = pg.ibs_genome(c, counts[0], counts[1], counts[3], sample_idx=sidx, v_range=v_range)
    torch.cuda.synchronize()
    return counts, [t.cpu().numpy() for t in z]


def _check(codes_sel, counts, z, layout):
    i0, i1, _, nm = oracle.ibs_matrix(codes_sel, full=(layout == "full"))
    for got, ref in zip((counts[0], counts[1], counts[3]), (i0, i1, nm)):
        assert np.array_equal(_u32(got).reshape(ref.shape), ref)
    ref = oracle.genome(codes_sel, i0, i1, nm)
    for g, r in zip(z, ref):
        _same(g.reshape(r.shape), r)


@pytest.mark.parametrize("layout", ["full", "tri"])
def test_similarity_bit_exact(layout):
    n, V = 130, 700
    bed = synth.hwe(n, V, (0.05, 0.5), 0.03, seed=61)
    codes = oracle.unpack(bed, n, V)
    codes[:, 7] = 1                                  # a sample without calls: N = 0 -> NaN
    c = pg.Cohort.from_numpy(_bed_from_codes(codes), n)
    counts = pg.ibs_matrix(c, layout=layout)
    s = pg.ibs_similarity(counts[1], counts[2], counts[3])
    ref = oracle.ibs_similarity(_u32(counts[1]), _u32(counts[2]), _u32(counts[3]))
    _same(s.cpu().numpy(), ref)
    assert np.isnan(s.cpu().numpy()).any()


@pytest.mark.parametrize("m,V,kind,layout", [
    (2, 10, "hwe", "full"), (3, 50, "hwe", "tri"), (17, 300, "mosaic", "full"),
    (64, 1000, "hwe", "tri"), (65, 1001, "mosaic", "full"), (300, 2000, "mosaic", "tri"),
    (129, 4099, "hwe", "full")])
def test_genome_parity(m, V, kind, layout):
    if kind == "hwe":
        bed = synth.hwe(m, V, (0.01, 0.5), 0.02, seed=m * 7 + V)
    else:
        bed = synth.mosaic(m, V, 6, 0.02, 0.001, 0.0, 0.02, seed=m * 7 + V)
    c = pg.Cohort.from_numpy(bed, m)
    counts, z = _gpu_genome(c, layout)
    _check(oracle.unpack(bed, m, V), counts, z, layout)


def test_genome_selection_and_range():
    """A shuffled sample list with a repeated sample (a duplicate pair: Z2 = 1)
    over a variant range that starts and ends inside 16-sample words."""
    n, V = 211, 3000
    bed = synth.mosaic(n, V, 8, 0.02, 0.001, 0.0, 0.03, seed=62)
    rng = np.random.default_rng(62)
    idx = rng.choice(n, 90, replace=False)
    idx = np.concatenate([idx, idx[:1]]).astype(np.int32)
    vr = (37, 2911)
    c = pg.Cohort.from_numpy(bed, n)
    for layout in ("full", "tri"):
        counts, z = _gpu_genome(c, layout, idx, vr)
        sel = oracle.select(oracle.unpack(bed, n, V), idx, *vr)
        _check(sel, counts, z, layout)
    full = _gpu_genome(c, "full", idx, vr)[1]
    assert full[2][0, 90] == 1.0 and full[3][0, 90] == 1.0


def test_genome_missing_mask():
    n, V = 150, 1500
    bed = synth.hwe(n, V, (0.05, 0.5), 0.0, seed=63)
    mask = synth.missing_mask(n, V, 0.05, seed=63)
    c = pg.Cohort.from_numpy(bed, n, mask)
    counts, z = _gpu_genome(c, "tri")
    _check(oracle.unpack(bed, n, V, mask), counts, z, "tri")


def test_genome_pedigree_duplicate_is_exact():
    """Founders, two children, an unrelated sample and a duplicate of the
    first founder, inside 120 unrelated samples."""
    V = 6000
    rng = np.random.default_rng(64)
    p = rng.uniform(0.05, 0.5, V)
    hap = lambda: (rng.random(V) < p).astype(np.int8)          # noqa: E731
    f0, f1, u = (hap(), hap()), (hap(), hap()), (hap(), hap())
    kids = []
    for _ in range(2):
        a, b = rng.integers(0, 2, V).astype(bool), rng.integers(0, 2, V).astype(bool)
        kids.append((np.where(a, f0[0], f0[1]), np.where(b, f1[0], f1[1])))
    ped = [f0, f1, kids[0], kids[1], u, f0] + [(hap(), hap()) for _ in range(120)]
    dos = np.stack([h[0] + h[1] for h in ped], 1)
    codes = np.choose(dos, [0, 2, 3]).astype(np.int8)
    m = codes.shape[1]
    c = pg.Cohort.from_numpy(_bed_from_codes(codes), m)
    counts, z = _gpu_genome(c, "full")
    _check(codes, counts, z, "full")
    assert (z[0][0, 5], z[1][0, 5], z[2][0, 5], z[3][0, 5]) == (0.0, 0.0, 1.0, 1.0)
    assert z[1][0, 2] > 0.8 and z[3][2, 3] > 0.3


def test_genome_undefined_cases():
    # only one call per marker: no marker has four observed alleles -> all NaN
    m, V = 6, 40
    codes = np.full((V, m), 1, dtype=np.int8)
    codes[np.arange(V), np.arange(V) % m] = 3
    c = pg.Cohort.from_numpy(_bed_from_codes(codes), m)
    counts, z = _gpu_genome(c, "full")
    _check(codes, counts, z, "full")
    assert all(np.isnan(a).all() for a in z)
    # exactly two calls on one marker (n = 4 counts), others with one call
    codes[0, :] = 1
    codes[0, 0], codes[0, 1] = 0, 3
    codes[5, 2] = 2
    c = pg.Cohort.from_numpy(_bed_from_codes(codes), m)
    counts, z = _gpu_genome(c, "full")
    _check(codes, counts, z, "full")
    # one sample, triangle layout: nothing to write, the call still succeeds
    c1 = pg.Cohort.from_numpy(synth.hwe(1, 30, seed=65), 1)
    counts, z = _gpu_genome(c1, "tri")
    assert all(a.size == 0 for a in z)


def test_genome_full_size_large_workload():
    """The 10,000 x 100,000 IBS workload (full layout): the report over all
    10,000 samples, checked on 16 sampled rows (160,000 pairs, tile edges
    among them) against the oracle's report for the oracle's counts of the
    same pairs; the per-marker averages come from all 10,000 samples on both
    sides."""
    w = synth.ibs_large()
    n, V = w["n"], w["V"]
    c = pg.Cohort.from_numpy(w["bed"], n)
    counts = pg.ibs_matrix(c, layout="full")
    z = pg.ibs_genome(c, counts[0], counts[1], counts[3])
    torch.cuda.synchronize()
    del counts
    rng = np.random.default_rng(66)
    edges = np.array([0, 63, 64, 5000, 9983, 9984, 9999])
    rows = np.sort(np.concatenate([edges, rng.choice(np.setdiff1d(np.arange(n), edges), 9,
                                                     replace=False)]))
    codes_sm = oracle.unpack(w["bed"], n, V, sample_major=True)
    pi, pj = np.repeat(rows, n), np.tile(np.arange(n), len(rows))
    cnt = oracle.ibs_pairs(codes_sm, pi, pj)
    del codes_sm
    ref = oracle.genome(oracle.unpack(w["bed"], n, V), cnt[:, 0], cnt[:, 1], cnt[:, 3])
    tr = torch.from_numpy(rows).cuda()
    for g, r in zip(z, ref):
        _same(g[tr].cpu().numpy().reshape(-1), r)
    Z0, Z1, Z2, PI = z
    assert torch.allclose(Z0 + Z1 + Z2, torch.ones_like(Z0), atol=1e-12, equal_nan=True)
    assert bool(torch.isnan(torch.diagonal(Z0)).logical_not().all())
    assert bool((torch.diagonal(Z2) == 1.0).all())
