"""Pins for the CPU oracle: each check reaches the expected value by a route
that does not reuse the oracle's code or formulation.

- hand-worked fixtures (tests/golden/*.txt);
- the paper's literal per-marker IBS rule on the raw 2-bit codes (section
  "Bitwise parallelism": equal calls -> IBS2, both bits differ -> IBS0, else
  IBS1), brute force on tiny inputs -- the oracle instead uses allele dosage;
- products of indicator matrices (numpy int64 matmul) for the IBS matrix;
- numpy.corrcoef for r^2, and the paper's 2-bit dot-product identity (section
  "Bit population count") as an independent route to sum x*y;
- invariants and special cases (symmetry, diagonal, inclusion-exclusion,
  identical / allele-flipped samples, duplicated / negated variants).
"""
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _unpack_numpy(bed, n, V, mask=None):
    """Independent .bed decode via numpy.unpackbits (little bit order)."""
    bits = np.unpackbits(bed[:V], axis=1, bitorder="little").astype(np.int8)
    codes = bits[:, 0:2 * n:2] + 2 * bits[:, 1:2 * n:2]
    if mask is not None:
        mbits = np.unpackbits(mask.view(np.uint8), axis=1, bitorder="little")[:, :n]
        codes = np.where(mbits == 1, 1, codes)
    return codes.astype(np.int8)


def _literal_ibs(ci, cj):
    """The paper's per-marker rule on raw 2-bit codes (no dosage)."""
    ibs0 = ibs1 = ibs2 = 0
    for a, b in zip(ci, cj):
        if a == 1 or b == 1:        # either call missing (.bed code 01): skip
            continue
        if a == b:
            ibs2 += 1
        elif (a ^ b) == 3:          # both bits differ
            ibs0 += 1
        else:
            ibs1 += 1
    return ibs0, ibs1, ibs2, ibs0 + ibs1 + ibs2


# --- generators -------------------------------------------------------------

def test_prng_published_vectors():
    lib = synth._load()
    # SplitMix64 from state 0; xoshiro256** from state {1,2,3,4}
    assert lib.synth_splitmix64_first(0) == 0xE220A8397B1DCDAF
    assert lib.synth_xoshiro_first(1, 2, 3, 4) == 11520


def test_hwe_generator_statistics():
    n, V = 4000, 200
    bed = synth.hwe(n, V, (0.3, 0.3), 0.0, seed=7)
    c = _unpack_numpy(bed, n, V)
    q = 0.3
    freq = [(c == k).mean() for k in (0, 1, 2, 3)]
    assert abs(freq[0] - q * q) < 0.005
    assert freq[1] == 0.0
    assert abs(freq[2] - 2 * q * (1 - q)) < 0.006
    assert abs(freq[3] - (1 - q) ** 2) < 0.006
    bed = synth.hwe(n, V, (0.05, 0.5), 0.02, seed=8)
    assert abs((_unpack_numpy(bed, n, V) == 1).mean() - 0.02) < 0.002


def test_mosaic_generator_maf_and_decay():
    n, V = 600, 3000
    bed = synth.mosaic(n, V, switch=0.01, miss=0.0, seed=9)
    c = _unpack_numpy(bed, n, V).astype(np.float64)
    dos = np.where(c == 0, 0, np.where(c == 2, 1, 2))
    f = dos.mean(axis=1) / 2
    assert (np.minimum(f, 1 - f) >= 0.01 - 1e-12).all()
    # r^2 decays with distance
    def mean_r2(d):
        x, y = dos[:-d], dos[d:]
        xc = x - x.mean(1, keepdims=True)
        yc = y - y.mean(1, keepdims=True)
        r = (xc * yc).sum(1) / np.sqrt((xc ** 2).sum(1) * (yc ** 2).sum(1))
        return np.nanmean(r ** 2)
    assert mean_r2(1) > mean_r2(20) > mean_r2(400)


def test_determinism_and_padding():
    a = synth.hwe(13, 50, seed=3, garbage_pad=True)
    b = synth.hwe(13, 50, seed=3, garbage_pad=True)
    assert np.array_equal(a, b)
    assert (a[:, -1] >> 2).any()          # padding bits carry garbage
    assert np.array_equal(_unpack_numpy(a, 13, 50), _unpack_numpy(synth.hwe(13, 50, seed=3), 13, 50))


# --- unpack -----------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 3, 4, 5, 63, 64, 65, 130])
def test_unpack_matches_unpackbits(n):
    V = 37
    bed = synth.hwe(n, V, seed=n, garbage_pad=True)
    mask = synth.missing_mask(n, V, 0.1, seed=n + 1)
    ref = _unpack_numpy(bed, n, V, mask)
    assert np.array_equal(oracle.unpack(bed, n, V, mask), ref)
    assert np.array_equal(oracle.unpack(bed, n, V, mask, sample_major=True), ref.T)


# --- IBS --------------------------------------------------------------------

def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_ibs_golden_hand_worked():
    rows = _read_golden("ibs_tiny.txt")
    n = int([r for r in rows if r[0] == "n"][0][1])
    V = int([r for r in rows if r[0] == "V"][0][1])
    data = [r for r in rows if r[0] == "row"]
    bed = np.array([[int(r[4], 16)] for r in data], dtype=np.uint8)
    codes = oracle.unpack(bed, n, V)
    assert codes.tolist() == [[int(x) for x in r[1:4]] for r in data]
    i0, i1, i2, nm = oracle.ibs_matrix(codes, full=True)
    for r in (r for r in rows if r[0] == "pair"):
        i, j, e0, e1, e2, en = map(int, r[1:])
        assert (i0[i, j], i1[i, j], i2[i, j], nm[i, j]) == (e0, e1, e2, en), (i, j)
        assert (i0[j, i], i1[j, i], i2[j, i], nm[j, i]) == (e0, e1, e2, en)


def test_ibs_all_code_pairs():
    """V = 1, every ordered pair of the four codes, against the literal rule."""
    codes = np.array([[0, 1, 2, 3]], dtype=np.int8)
    i0, i1, i2, nm = oracle.ibs_matrix(codes, full=True)
    for a in range(4):
        for b in range(4):
            assert (i0[a, b], i1[a, b], i2[a, b], nm[a, b]) == _literal_ibs([a], [b])


@settings(max_examples=60, deadline=None)
@given(n=st.integers(1, 9), V=st.integers(1, 70), seed=st.integers(0, 2 ** 31),
       masked=st.booleans())
def test_ibs_brute_force_tiny(n, V, seed, masked):
    bed = synth.hwe(n, V, (0.0, 0.5), 0.15, seed=seed, garbage_pad=True)
    mask = synth.missing_mask(n, V, 0.1, seed + 1) if masked else None
    codes = oracle.unpack(bed, n, V, mask)
    assert np.array_equal(codes, _unpack_numpy(bed, n, V, mask))
    full = oracle.ibs_matrix(codes, full=True)
    tri = oracle.ibs_matrix(codes, full=False)
    t = 0
    for i in range(n):
        for j in range(n):
            exp = _literal_ibs(codes[:, i], codes[:, j])
            assert tuple(int(f[i, j]) for f in full) == exp
            if i < j:
                assert i * n - i * (i + 1) // 2 + (j - i - 1) == t
                assert tuple(int(f[t]) for f in tri) == exp
                t += 1


def _indicator_ibs(codes):
    """IBS via int64 matrix products of per-genotype indicator matrices."""
    a1 = (codes == 0).astype(np.int64)
    ht = (codes == 2).astype(np.int64)
    a2 = (codes == 3).astype(np.int64)
    m = (codes != 1).astype(np.int64)
    ibs0 = a1.T @ a2 + a2.T @ a1
    ibs1 = (a1 + a2).T @ ht + ht.T @ (a1 + a2)
    ibs2 = a1.T @ a1 + ht.T @ ht + a2.T @ a2
    return ibs0, ibs1, ibs2, m.T @ m


def test_ibs_matches_indicator_products_small_workload():
    w = synth.ibs_small()
    codes = oracle.unpack(w["bed"], w["n"], w["V"])
    sub = codes[:, :160]
    got = oracle.ibs_matrix(sub, full=True)
    ref = _indicator_ibs(sub)
    for g, r in zip(got, ref):
        assert np.array_equal(g.astype(np.int64), r)
    # the tri layout of the whole 500 x 5000 workload agrees with the products
    tri = oracle.ibs_matrix(codes, full=False)
    ref = _indicator_ibs(codes)
    iu = np.triu_indices(w["n"], 1)
    for g, r in zip(tri, ref):
        assert np.array_equal(g.astype(np.int64), r[iu])


def test_ibs_invariants():
    n, V = 40, 900
    bed = synth.mosaic(n, V, miss=0.05, seed=11)
    codes = oracle.unpack(bed, n, V)
    # append an identical copy of sample 0 and an allele-flipped copy of sample 1
    flip = codes[:, 1].copy()
    flip = np.where(flip == 0, 3, np.where(flip == 3, 0, flip))
    codes = np.concatenate([codes, codes[:, :1], flip[:, None]], axis=1)
    n2 = n + 2
    i0, i1, i2, nm = [x.astype(np.int64) for x in oracle.ibs_matrix(codes, full=True)]
    assert np.array_equal(i0 + i1 + i2, nm)
    for x in (i0, i1, i2, nm):
        assert np.array_equal(x, x.T)
    miss = (codes == 1).astype(np.int64)
    nonmiss = V - miss.sum(0)
    assert np.array_equal(np.diag(i2), nonmiss) and np.array_equal(np.diag(nm), nonmiss)
    assert not np.diag(i0).any() and not np.diag(i1).any()
    both_missing = miss.T @ miss
    m_i = miss.sum(0)
    assert np.array_equal(nm, V - m_i[:, None] - m_i[None, :] + both_missing)
    # identical copy: IBS2 = N, nothing else
    assert i2[0, n] == nm[0, n] and i0[0, n] == 0 and i1[0, n] == 0
    # allele-flipped copy: homozygotes become IBS0, heterozygotes stay IBS2
    c1 = codes[:, 1]
    assert i0[1, n + 1] == np.isin(c1, (0, 3)).sum()
    assert i2[1, n + 1] == (c1 == 2).sum()
    assert i1[1, n + 1] == 0
    # pair lists agree with the matrix
    pi = np.array([0, 3, n + 1, 7]); pj = np.array([5, 3, 1, n2 - 1])
    got = oracle.ibs_pairs(np.ascontiguousarray(codes.T), pi, pj)
    for k in range(len(pi)):
        assert tuple(got[k]) == (i0[pi[k], pj[k]], i1[pi[k], pj[k]], i2[pi[k], pj[k]], nm[pi[k], pj[k]])


# --- LD ---------------------------------------------------------------------

def test_ld_golden_hand_worked():
    rows = _read_golden("ld_tiny.txt")
    n = int([r for r in rows if r[0] == "n"][0][1])
    V = int([r for r in rows if r[0] == "V"][0][1])
    bed = np.array([[int(x, 16) for x in r[1:]] for r in rows if r[0] == "bed"], dtype=np.uint8)
    exp = [int(x) for x in [r for r in rows if r[0] == "sums"][0][1:]]
    num = int([r for r in rows if r[0] == "r2_num"][0][1])
    den = int([r for r in rows if r[0] == "r2_den"][0][1])
    codes = oracle.unpack(bed, n, V)
    sums, r2 = oracle.ld_pairs(codes, [0], [1])
    assert sums[0].tolist() == exp
    assert abs(r2[0] - num / den) < 1e-15


def _xvals(c):
    return np.where(c == 0, -1, np.where(c == 2, 0, 1)).astype(np.int64)


def _pack_lanes(vals):
    """Encode per-sample values into the paper's 2-bit lanes for the dot
    product: 00 hom minor (x=-1), 01 het or missing (0), 10 hom major (+1)."""
    word = 0
    for k, v in enumerate(vals):
        word |= {-1: 0, 0: 1, 1: 2}[int(v)] << (2 * k)
    return word


def _dot_by_popcount2(xs, ys):
    """sum_S x*y by the 2-bit identity of section "Bit population count":
    Gz = (Gx | Gy) & 0101..; result = |S| - popcount2(((Gx ^ Gy) & (1010.. - Gz)) | Gz)."""
    S = len(xs)
    gx, gy = _pack_lanes(xs), _pack_lanes(ys)
    lo = int("01" * S, 2)
    hi = int("10" * S, 2)
    gz = (gx | gy) & lo
    t = ((gx ^ gy) & (hi - gz)) | gz
    pc2 = sum((t >> (2 * k)) & 3 for k in range(S))
    return S - pc2


def test_dot_product_identity_exhaustive_lanes():
    vals = [-1, 0, 1]
    for a in vals:
        for b in vals:
            assert _dot_by_popcount2([a], [b]) == a * b
    rng = np.random.default_rng(5)
    for _ in range(50):
        xs = rng.integers(-1, 2, 31)
        ys = rng.integers(-1, 2, 31)
        assert _dot_by_popcount2(xs, ys) == int((xs * ys).sum())


@settings(max_examples=60, deadline=None)
@given(n=st.integers(2, 40), seed=st.integers(0, 2 ** 31))
def test_ld_pairs_vs_corrcoef_and_popcount2(n, seed):
    V = 6
    bed = synth.hwe(n, V, (0.1, 0.5), 0.1, seed=seed, garbage_pad=True)
    codes = oracle.unpack(bed, n, V)
    pa, pb = np.triu_indices(V, 1)
    sums, r2 = oracle.ld_pairs(codes, pa, pb)
    for k, (a, b) in enumerate(zip(pa, pb)):
        keep = (codes[a] != 1) & (codes[b] != 1)
        x, y = _xvals(codes[a][keep]), _xvals(codes[b][keep])
        assert sums[k].tolist() == [int(keep.sum()), int(x.sum()), int(y.sum()),
                                    int(np.count_nonzero(x)), int(np.count_nonzero(y)),
                                    _dot_by_popcount2(x, y) if len(x) else 0]
        # missing calls are x = 0 in the paper's full-S dot product
        xa = np.where(codes[a] == 1, 0, _xvals(codes[a]))
        yb = np.where(codes[b] == 1, 0, _xvals(codes[b]))
        assert sums[k][5] == int((xa * yb).sum())
        if len(x) < 2 or x.std() == 0 or y.std() == 0:
            assert np.isnan(r2[k])
        else:
            assert abs(r2[k] - np.corrcoef(x, y)[0, 1] ** 2) < 1e-12
            assert -1e-15 <= r2[k] <= 1 + 1e-15


def test_ld_special_cases():
    n, V = 300, 50
    bed = synth.mosaic(n, V, switch=0.02, miss=0.03, seed=21)
    codes = oracle.unpack(bed, n, V)
    flip = np.where(codes[3] == 0, 3, np.where(codes[3] == 3, 0, codes[3]))
    mono = np.full(n, 3, dtype=np.int8)
    allmiss = np.full(n, 1, dtype=np.int8)
    codes = np.concatenate([codes, codes[3:4], flip[None], mono[None], allmiss[None]], 0)
    dup, neg, mo, am = V, V + 1, V + 2, V + 3
    sums, r2 = oracle.ld_pairs(codes, [3, 3, 3, 3, 0], [dup, neg, mo, am, 1])
    assert r2[0] == 1.0                       # duplicated variant: exactly 1
    assert sums[0][5] == sums[0][3]           # Sxy = Sxx
    assert abs(r2[1] - 1.0) < 1e-15           # negated variant
    assert sums[1][5] == -sums[1][3]
    assert np.isnan(r2[2]) and np.isnan(r2[3])
    assert sums[3][0] == 0
    s = sums[4]
    assert s[0] * s[3] - s[1] ** 2 >= 0 and s[0] * s[4] - s[2] ** 2 >= 0


def test_ld_window_emission():
    n, V, W = 200, 300, 25
    bed = synth.mosaic(n, V, switch=0.01, miss=0.01, seed=31)
    codes = oracle.unpack(bed, n, V)
    rec = oracle.ld_window(codes, W, 0.2)
    pa, pb = [], []
    for a in range(V):
        for b in range(a + 1, min(a + W, V - 1) + 1):
            pa.append(a); pb.append(b)
    sums, r2 = oracle.ld_pairs(codes, pa, pb)
    keep = r2 >= 0.2
    assert len(rec) == keep.sum() > 0
    assert np.array_equal(rec["a"], np.array(pa)[keep]) and np.array_equal(rec["b"], np.array(pb)[keep])
    got = np.stack([rec[f] for f in ("n", "sx", "sy", "sxx", "syy", "sxy")], 1)
    assert np.array_equal(got, sums[keep])
    assert np.array_equal(rec["r2"], r2[keep])
    # (a, b) order, and truncation keeps the first `capacity` records
    keys = rec["a"].astype(np.int64) * V + rec["b"]
    assert (np.diff(keys) > 0).all()
    part = oracle.ld_window(codes, W, 0.2, capacity=10)
    assert np.array_equal(part, rec[:10])
    # a row sub-range gives the matching slice
    sub = oracle.ld_window(codes, W, 0.2, a_begin=100, a_end=180)
    sel = (rec["a"] >= 100) & (rec["a"] < 180)
    assert np.array_equal(sub, rec[sel])
