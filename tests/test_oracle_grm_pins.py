"""Pins for the oracle's relationship matrix (section "Partial sum lookup",
under the reading stated in oracle.c).  The oracle sums per-marker increment
tables pair by pair; the pins reach the values by other routes:

- a hand-worked fixture with a missing call and an undefined marker
  (tests/golden/grm_tiny.txt);
- numpy: standardize every call, (x - 2p) / sqrt(2p(1-p)), zero for
  missing calls and left-out markers, then one matrix product for the
  numerators and one for the denominators;
- invariants: with no missing call every numerator row sums to zero;
  re-coding a marker with its alleles swapped changes nothing; a duplicated
  sample has the same row as the original.
"""
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    rows = []
    with open(os.path.join(GOLDEN, "grm_tiny.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_grm_golden_hand_worked():
    rows = _golden()
    n = int([r for r in rows if r[0] == "n"][0][1])
    V = int([r for r in rows if r[0] == "V"][0][1])
    bed = np.array([[int(r[1], 16)] for r in rows if r[0] == "bed"], dtype=np.uint8)
    codes = oracle.unpack(bed, n, V)
    A, N, _ = oracle.grm(codes, full=True)
    for r in (r for r in rows if r[0] == "pair"):
        i, j, num, den, cnt = map(int, r[1:])
        for a, b in ((i, j), (j, i)):
            assert abs(A[a, b] - num / den) < 1e-15, (a, b)
            assert N[a, b] == cnt


def _numpy_grm(codes_vm):
    dos = np.select([codes_vm == 0, codes_vm == 2, codes_vm == 3], [0.0, 1.0, 2.0], 0.0)
    m = codes_vm != 1
    calls = m.sum(1)
    a2 = (dos * m).sum(1)
    used = (calls > 0) & (a2 > 0) & (a2 < 2 * calls)
    p = np.where(used, a2 / np.maximum(2 * calls, 1), 0.5)
    z = np.where(m & used[:, None], (dos - 2 * p[:, None]) / np.sqrt(2 * p * (1 - p))[:, None], 0.0)
    mu = (m & used[:, None]).astype(np.float64)
    num = z.T @ z
    den = mu.T @ mu
    with np.errstate(invalid="ignore", divide="ignore"):
        return num / den, den


@pytest.mark.parametrize("n,V,miss,seed", [(40, 500, 0.02, 1), (97, 1300, 0.05, 2),
                                           (13, 60, 0.3, 3)])
def test_grm_matches_standardized_matrix_product(n, V, miss, seed):
    codes = oracle.unpack(synth.hwe(n, V, (0.01, 0.5), miss, seed=seed), n, V)
    codes[5] = 3                                    # monomorphic: left out
    A, N, S = oracle.grm(codes, full=True)
    A2, N2 = _numpy_grm(codes)
    assert np.array_equal(N, N2.astype(np.uint32))
    ok = N > 0
    assert np.all(np.isnan(A[~ok]))
    assert np.all(np.abs(A[ok] - A2[ok]) <= 1e-12 * (1 + S[ok] / N[ok]))


def test_grm_rows_sum_to_zero_without_missing_calls():
    n, V = 60, 800
    codes = oracle.unpack(synth.hwe(n, V, (0.05, 0.5), 0.0, seed=4), n, V)
    A, N, S = oracle.grm(codes, full=True)
    num = A * N
    assert np.all(np.abs(num.sum(1)) <= 1e-9 * S.sum(1))


def test_grm_allele_swap_and_duplicate_sample():
    n, V = 50, 400
    codes = oracle.unpack(synth.mosaic(n, V, 6, 0.02, 0.001, 0.0, 0.03, seed=5), n, V)
    A, N, S = oracle.grm(codes, full=True)
    flipped = codes.copy()
    rows = np.arange(0, V, 3)
    sub = flipped[rows]
    flipped[rows] = np.where(sub == 0, 3, np.where(sub == 3, 0, sub))
    Af, Nf, _ = oracle.grm(flipped, full=True)
    assert np.array_equal(N, Nf)
    assert np.all(np.abs(A - Af) <= 1e-12 * (1 + S / np.maximum(N, 1)))
    dup = np.concatenate([codes, codes[:, 7:8]], axis=1)
    Ad, Nd, _ = oracle.grm(dup, full=True)
    assert np.array_equal(Ad[:n, n], Ad[:n, 7]) and np.array_equal(Nd[:n, n], Nd[:n, 7])
    assert Ad[n, n] == Ad[7, 7]


def test_grm_triangle_layout_matches_full():
    n, V = 31, 200
    codes = oracle.unpack(synth.hwe(n, V, (0.05, 0.5), 0.02, seed=6), n, V)
    A, N, _ = oracle.grm(codes, full=True)
    At, Nt, _ = oracle.grm(codes, full=False)
    iu = np.triu_indices(n, 1)
    assert np.array_equal(At, A[iu]) and np.array_equal(Nt, N[iu])


def test_grm_pair_list_matches_matrix():
    n, V = 23, 150
    codes = oracle.unpack(synth.hwe(n, V, (0.05, 0.5), 0.05, seed=7), n, V)
    A, N, S = oracle.grm(codes, full=True)
    rng = np.random.default_rng(3)
    pi, pj = rng.integers(0, n, 40), rng.integers(0, n, 40)
    Ap, Np, Sp = oracle.grm_pairs(np.ascontiguousarray(codes.T), pi, pj)
    assert np.array_equal(Ap, A[pi, pj]) and np.array_equal(Np, N[pi, pj])
    assert np.array_equal(Sp, S[pi, pj])
