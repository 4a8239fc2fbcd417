"""Pins for the oracle's LD pruning (section "Linkage disequilibrium-based
variant pruning", under the reading stated in oracle.c) and for the r^2 value
its decisions use.  Every expected value comes from a route that shares no
code with the oracle:

- r^2 in exact rational arithmetic (fractions.Fraction) from the paper's
  mean-based expression, rounded once to double;
- a brute-force restatement of the greedy rule in pure Python with exact
  rationals, written as "repeatedly find the first offending pair in the
  window and drop one side" rather than the oracle's single pass;
- closed forms: duplicate runs keep their first member; a threshold of 1
  drops nothing; with a negative threshold and non-overlapping windows the
  survivor of each window is its first variant of highest minor allele
  frequency; pairs that never share a window are never compared.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

XV = {0: -1, 2: 0, 3: 1}


def _exact_r2(ca, cb):
    """Mean-based r^2 over S_xy as an exact rational (None if undefined)."""
    xs = [(XV[a], XV[b]) for a, b in zip(ca, cb) if a != 1 and b != 1]
    n = len(xs)
    if n == 0:
        return None
    mx = Fraction(sum(x for x, _ in xs), n)
    my = Fraction(sum(y for _, y in xs), n)
    vx = Fraction(sum(x * x for x, _ in xs), n) - mx * mx
    vy = Fraction(sum(y * y for _, y in xs), n) - my * my
    if vx == 0 or vy == 0:
        return None
    cov = Fraction(sum(x * y for x, y in xs), n) - mx * my
    return cov * cov / (vx * vy)


def _sums(ca, cb):
    xs = [(XV[a], XV[b]) for a, b in zip(ca, cb) if a != 1 and b != 1]
    return np.array([len(xs), sum(x for x, _ in xs), sum(y for _, y in xs),
                     sum(x * x for x, _ in xs), sum(y * y for _, y in xs),
                     sum(x * y for x, y in xs)], dtype=np.int64)


def _exact_maf(c):
    calls = [v for v in c if v != 1]
    if not calls:
        return Fraction(0)
    a2 = sum({0: 0, 2: 1, 3: 2}[v] for v in calls)
    return Fraction(min(a2, 2 * len(calls) - a2), 2 * len(calls))


def _brute_prune(codes, W, S, t):
    V = codes.shape[0]
    tq = Fraction(t)
    maf = [_exact_maf(codes[v]) for v in range(V)]
    r2 = {}

    def offending(a, b):
        if (a, b) not in r2:
            r2[(a, b)] = _exact_r2(codes[a], codes[b])
        return r2[(a, b)] is not None and r2[(a, b)] > tq

    keep = [True] * V
    start = 0
    while True:
        end = min(start + W, V)
        while True:
            hit = next(((a, b) for a in range(start, end) for b in range(a + 1, end)
                        if keep[a] and keep[b] and offending(a, b)), None)
            if hit is None:
                break
            a, b = hit
            keep[a if maf[a] < maf[b] else b] = False
        if end == V:
            break
        start += S
    return np.array(keep, dtype=np.uint8)


def _pack(codes):
    V, n = codes.shape
    bed = np.zeros((V, (n + 3) // 4), dtype=np.uint8)
    for k in range(n):
        bed[:, k // 4] |= codes[:, k].astype(np.uint8) << (2 * (k % 4))
    return bed


# --- the decision value ----------------------------------------------------------

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_r2_counts_is_the_correctly_rounded_exact_ratio(seed):
    n, V = 120, 40
    codes = oracle.unpack(synth.mosaic(n, V, 6, 0.05, 0.001, 0.0, 0.05, seed=seed), n, V)
    checked = 0
    for a in range(V):
        for b in range(a + 1, min(a + 8, V)):
            exact = _exact_r2(codes[a], codes[b])
            got = oracle.r2_counts(_sums(codes[a], codes[b]))
            if exact is None:
                assert np.isnan(got)
                continue
            # n^4 < 2^53: the integer products are exact and one division rounds
            assert got == float(exact)
            assert abs(got - oracle.r2_from_sums(_sums(codes[a], codes[b]))) <= 1e-12
            checked += 1
    assert checked > 50


def test_r2_counts_undefined_cases():
    assert np.isnan(oracle.r2_counts(np.zeros(6, dtype=np.int64)))
    assert np.isnan(oracle.r2_counts(np.array([5, 5, 1, 5, 3, 1])))   # x constant
    assert oracle.r2_counts(np.array([4, 0, 0, 4, 4, 4])) == 1.0          # y = x


# --- the greedy pass -------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(8))
def test_prune_matches_restart_formulation(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(8, 40))
    V = int(rng.integers(2, 45))
    W = int(rng.integers(2, 12))
    S = int(rng.integers(1, W + 1))
    t = float(rng.choice([0.1, 0.3, 0.6]))
    codes = oracle.unpack(synth.mosaic(n, V, 4, 0.05, 0.001, 0.0, 0.05, seed=100 + seed), n, V)
    assert np.array_equal(oracle.ld_prune(codes, W, S, t), _brute_prune(codes, W, S, t))


def test_prune_duplicate_runs_keep_their_first_member():
    n, base_v = 400, 60
    base = oracle.unpack(synth.hwe(n, base_v, (0.2, 0.5), 0.0, seed=5), n, base_v)
    rng = np.random.default_rng(9)
    rows, expect = [], []
    for v in range(base_v):
        k = int(rng.integers(1, 5))
        flip = np.where(base[v] == 0, 3, np.where(base[v] == 3, 0, base[v]))
        for j in range(k):
            rows.append(flip if (j % 2 and rng.random() < 0.5) else base[v])
            expect.append(1 if j == 0 else 0)
    codes = np.array(rows, dtype=np.int8)
    keep = oracle.ld_prune(codes, 10, 3, 0.95)
    assert np.array_equal(keep, np.array(expect, dtype=np.uint8))


def test_prune_threshold_one_drops_nothing():
    n, V = 100, 300
    codes = oracle.unpack(synth.mosaic(n, V, 3, 0.01, 0.001, 0.0, 0.0, seed=4), n, V)
    codes[5] = codes[4]
    assert oracle.ld_prune(codes, 20, 5, 1.0).all()


def test_prune_negative_threshold_tournament():
    """Every defined pair offends; with step == window each window keeps
    exactly its first variant of highest minor allele frequency."""
    n, V, W = 300, 97, 10
    codes = oracle.unpack(synth.hwe(n, V, (0.05, 0.5), 0.0, seed=6), n, V)
    maf = [_exact_maf(codes[v]) for v in range(V)]
    assert all(m > 0 for m in maf)
    expect = np.zeros(V, dtype=np.uint8)
    for s in range(0, V, W):
        block = range(s, min(s + W, V))
        best = max(maf[v] for v in block)
        expect[next(v for v in block if maf[v] == best)] = 1
    assert np.array_equal(oracle.ld_prune(codes, W, W, -1.0), expect)


def test_prune_pairs_outside_every_window_are_not_compared():
    """window 4, step 2: windows [0,4), [2,6), [4,8).  Variants 1 and 4 are
    3 apart but never share a window; 2 and 5 share [2,6)."""
    n, V = 400, 8
    codes = oracle.unpack(synth.hwe(n, V, (0.3, 0.5), 0.0, seed=7), n, V)
    codes[4] = codes[1]
    codes[5] = codes[2]
    keep = oracle.ld_prune(codes, 4, 2, 0.9)
    assert keep[1] == 1 and keep[4] == 1
    assert keep[2] == 1 and keep[5] == 0
    assert keep.sum() == V - 1


def test_prune_drops_the_lower_maf_side():
    n = 400
    base = oracle.unpack(synth.hwe(n, 1, (0.3, 0.3), 0.0, seed=8), n, 1)[0]
    hi = base.copy()
    # A1 is the minor allele here (frequency 0.3): turning a few heterozygous
    # calls homozygous A1 raises the minor allele frequency and keeps the two
    # variants strongly correlated
    idx = np.nonzero(base == 2)[0][:6]
    hi[idx] = 0
    assert _exact_maf(hi) > _exact_maf(base)
    r2 = _exact_r2(base, hi)
    assert r2 > Fraction(0.8)
    for first, second, dropped in ((base, hi, 0), (hi, base, 1)):
        codes = np.array([first, second], dtype=np.int8)
        keep = oracle.ld_prune(codes, 2, 1, 0.8)
        assert keep[dropped] == 0 and keep[1 - dropped] == 1


def test_prune_packed_roundtrip_matches_codes():
    """The oracle prunes unpacked codes; packing and unpacking them again
    changes nothing (guards the fixtures the GPU tests build)."""
    n, V = 37, 50
    codes = oracle.unpack(synth.mosaic(n, V, 4, 0.05, 0.001, 0.0, 0.05, seed=11), n, V)
    again = oracle.unpack(_pack(codes), n, V)
    assert np.array_equal(oracle.ld_prune(codes, 7, 3, 0.3), oracle.ld_prune(again, 7, 3, 0.3))
