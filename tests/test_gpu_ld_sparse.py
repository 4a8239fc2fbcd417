"""GPU parity of the LD missing-call correction path (PG_PATH_SPARSE).

Its diagnostic variant writes the correction kernel's own record of every pair
of every tile it takes, so the six sums are compared with the oracle pair by
pair (exactly) and r^2 within 1e-12; the emitting variants are compared with
the oracle like the other LD paths, and byte for byte with the dense path."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

pg = pytest.importorskip("paper_1410_4803_amd")

from ldcheck import compare_records as _compare

SPARSE, FORCE, DIAG = 3, 3 | (1 << 8), 3 | (2 << 8)
FIELDS = ("n", "sx", "sy", "sxx", "syy", "sxy")


def _cap(m):
    """List slot length: ceil(m / 16) rounded up to a multiple of 8, in [64, 65528]."""
    c = (m + 15) // 16
    c = (c + 7) // 8 * 8
    return min(max(64, c), 65528)


def _pack(codes):
    V, n = codes.shape
    packed = np.zeros((V, (n + 3) // 4), dtype=np.uint8)
    for k in range(n):
        packed[:, k // 4] |= codes[:, k].astype(np.uint8) << (2 * (k % 4))
    return packed


def _r2(s):
    """r^2 from exact sums as the library defines it (products, one division)."""
    n, sx, sy, sxx, syy, sxy = (s[:, i] for i in range(6))
    cov, vx, vy = n * sxy - sx * sy, n * sxx - sx * sx, n * syy - sy * sy
    with np.errstate(divide="ignore", invalid="ignore"):
        r2 = (cov.astype(np.float64) * cov) / (vx.astype(np.float64) * vy.astype(np.float64))
    r2 = np.minimum(r2, 1.0)
    r2[(n == 0) | (vx == 0) | (vy == 0)] = np.nan
    return r2


def _diag(c, W, nv, sample_idx=None, v_range=None):
    slots = nv * W
    out = torch.full((slots, 64), 0xFF, dtype=torch.uint8, device="cuda")
    out, n_out = pg.ld_window(c, W, 0.0, capacity=slots, path=DIAG,
                              out=out, sample_idx=sample_idx, v_range=v_range)
    assert int(n_out.item()) == slots
    return pg.records_to_numpy(out, slots)


def _check_diag(rec, codes, W, v0=0):
    """codes: the selected (V, m) codes; rec: diagnostic slots.  Every pair in
    a tile whose two 64-variant groups have at most cap missing calls per
    variant must be written and exact; every other slot untouched."""
    V, m = codes.shape
    cap = _cap(m)
    miss = (codes == 1).sum(axis=1)
    groups = -(-V // 64)
    gmax = np.array([miss[64 * g:64 * g + 64].max() for g in range(groups)])
    a = np.repeat(np.arange(V), W)
    d = np.tile(np.arange(W), V)
    b = a + d + 1
    inside = b < V
    taken = inside & (gmax[a // 64] <= cap) & (gmax[np.minimum(b, V - 1) // 64] <= cap)
    written = rec["a"] != -1
    assert np.array_equal(written, taken), (np.nonzero(written != taken)[0][:5])
    pa, pb = a[taken], b[taken]
    got = rec[taken]
    assert np.array_equal(got["a"], pa + v0) and np.array_equal(got["b"], pb + v0)
    sums, _ = oracle.ld_pairs(codes, pa, pb)
    for i, f in enumerate(FIELDS):
        assert np.array_equal(got[f], sums[:, i]), f
    ref = _r2(sums)
    assert np.array_equal(np.isnan(got["r2"]), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.max(np.abs(got["r2"][ok] - ref[ok]), initial=0.0) <= 1e-12
    return int(taken.sum())


@pytest.mark.parametrize("n,V,W,miss", [(1, 5, 3, 0.05), (2, 40, 7, 0.05), (17, 65, 64, 0.05),
                                        (63, 130, 65, 0.0), (64, 300, 1, 0.05),
                                        (129, 257, 100, 0.02), (300, 700, 257, 0.01),
                                        (1000, 400, 1000, 0.05)])
def test_sparse_diag_all_pairs(n, V, W, miss):
    bed = synth.mosaic(n, V, switch=0.02, miss=miss, seed=n + V + W, garbage_pad=True)
    codes = oracle.unpack(bed, n, V)
    rec = _diag(pg.Cohort.from_numpy(bed, n), W, V)
    assert _check_diag(rec, codes, W) > 0


def test_sparse_diag_counter_flush():
    """More than 248 missing calls per variant: the byte counters are flushed
    into the per-pair cells more than once."""
    n, V, W = 8192, 200, 64
    bed = synth.mosaic(n, V, switch=0.02, miss=0.04, seed=77)
    codes = oracle.unpack(bed, n, V)
    miss = (codes == 1).sum(axis=1)
    assert miss.max() > 248 and miss.max() <= _cap(n)
    rec = _diag(pg.Cohort.from_numpy(bed, n), W, V)
    assert _check_diag(rec, codes, W) == sum(min(W, V - 1 - a) for a in range(V))


def test_sparse_diag_long_lists():
    """Lists of mixed length in one tile: 20 variants with 300 missing calls
    each (byte-counter flushes), one whose 200 missing calls are consecutive
    samples (adjacent rows of the strip), one missing only the first and last
    sample, and light variants."""
    n, V, W = 8192, 200, 150
    codes = oracle.unpack(synth.mosaic(n, V, switch=0.02, miss=0.002, seed=71), n, V).copy()
    rng = np.random.default_rng(72)
    for v in list(range(0, 10)) + list(range(64, 74)):
        codes[v, rng.choice(n, 300, replace=False)] = 1
    codes[130, 4000:4200] = 1
    codes[131, [0, n - 1]] = 1
    rec = _diag(pg.Cohort.from_numpy(_pack(codes), n), W, V)
    assert _check_diag(rec, codes, W) == sum(min(W, V - 1 - a) for a in range(V))


def test_sparse_diag_many_samples():
    """66,000 selected samples: strip offsets past 2^20 bytes, list slots of
    4,128 entries; the sums stay exact."""
    n, V, W = 66000, 100, 40
    bed = synth.mosaic(n, V, switch=0.02, miss=0.002, seed=73)
    codes = oracle.unpack(bed, n, V)
    rec = _diag(pg.Cohort.from_numpy(bed, n), W, V)
    assert _check_diag(rec, codes, W) == sum(min(W, V - 1 - a) for a in range(V))


def test_sparse_diag_list_slot_boundary():
    """A variant with exactly cap missing calls keeps its tiles on the path;
    one with cap + 1 sends every tile of its group to the dense kernel."""
    n, V, W = 1000, 256, 100
    cap = _cap(n)
    codes = oracle.unpack(synth.mosaic(n, V, switch=0.02, miss=0.0, seed=5), n, V).copy()
    rng = np.random.default_rng(6)
    codes[10, rng.choice(n, cap, replace=False)] = 1
    codes[150, rng.choice(n, cap + 1, replace=False)] = 1
    codes[200, :] = 1
    codes[201, :] = 3
    rec = _diag(pg.Cohort.from_numpy(_pack(codes), n), W, V)
    written = _check_diag(rec, codes, W)
    assert 0 < written < sum(min(W, V - 1 - a) for a in range(V))
    # the emitting path is exact on every tile, taken or not
    c = pg.Cohort.from_numpy(_pack(codes), n)
    ref = oracle.ld_window(codes, W, -np.inf)
    got = pg.ld_records(c, W, -np.inf, path=FORCE)
    assert len(got) == len(ref)
    _compare(got, ref, -np.inf)


def test_sparse_diag_mask_selection_range():
    n, V, W = 400, 1000, 150
    bed = synth.mosaic(n, V, switch=0.01, miss=0.01, seed=8, garbage_pad=True)
    mask = synth.missing_mask(n, V, 0.03, seed=9)
    rng = np.random.default_rng(1)
    idx = rng.integers(0, n, 333).astype(np.int32)
    vb, ve = 77, 911
    codes = oracle.select(oracle.unpack(bed, n, V, mask), idx, vb, ve)
    c = pg.Cohort.from_numpy(bed, n, mask)
    rec = _diag(c, W, ve - vb, sample_idx=torch.from_numpy(idx).cuda(), v_range=(vb, ve),
                )
    assert _check_diag(rec, codes, W, v0=vb) > 0


@pytest.mark.parametrize("path", [SPARSE, FORCE])
def test_sparse_mixed_tiles_emission(path):
    """Variants 600-700 miss 40% of their calls, so their tiles exceed the
    budget (and the list slots); the dense kernel takes those, the correction
    kernel the rest, and the records equal the oracle's and the dense path's."""
    n, V, W = 500, 1500, 300
    codes = oracle.unpack(synth.mosaic(n, V, switch=0.005, miss=0.01, seed=31), n, V).copy()
    rng = np.random.default_rng(32)
    heavy = rng.random((101, n)) < 0.4
    codes[600:701][heavy] = 1
    c = pg.Cohort.from_numpy(_pack(codes), n)
    for r2_min in (-np.inf, 0.2):
        ref = oracle.ld_window(codes, W, r2_min)
        got = pg.ld_records(c, W, r2_min, path=path)
        assert _compare(got, ref, r2_min) > 0
        assert got.tobytes() == pg.ld_records(c, W, r2_min, path="mfma").tobytes()


def test_sparse_no_missing_calls():
    """Without missing calls every tile takes the path and the corrections
    are empty: only the Gram and the totals remain."""
    n, V, W = 777, 2000, 500
    bed = synth.mosaic(n, V, switch=0.005, miss=0.0, seed=41)
    codes = oracle.unpack(bed, n, V)
    c = pg.Cohort.from_numpy(bed, n)
    ref = oracle.ld_window(codes, W, 0.3)
    got = pg.ld_records(c, W, 0.3, path=SPARSE)
    assert _compare(got, ref, 0.3) > 0
    rec = _diag(c, 64, V)
    assert _check_diag(rec, codes, 64) == sum(min(64, V - 1 - a) for a in range(V))


@pytest.mark.parametrize("miss", [0.0, 0.003, 0.01])
def test_auto_gate_follows_missing_rate(miss):
    """PG_PATH_AUTO from 5,000 samples and windows of 500 is the correction
    path behind a sampled missing-call gate: without missing calls the path
    runs, at 1% the gate leaves every tile to the dense kernel, and in
    between the tiles decide; the records equal the dense path's in every
    case."""
    n, V, W = 5000, 3000, 500
    bed = synth.mosaic(n, V, switch=0.005, miss=miss, seed=81)
    c = pg.Cohort.from_numpy(bed, n)
    assert pg.api.resolve_path("ld", n, V, W, "auto") == SPARSE | (8 << 8)
    for r2_min in (0.2, -np.inf):
        got = pg.ld_records(c, W, r2_min, path="auto")
        ref = pg.ld_records(c, W, r2_min, path="mfma")
        assert len(got) > 0 and got.tobytes() == ref.tobytes()
