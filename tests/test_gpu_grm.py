"""GPU parity for the relationship matrix: N bit-exact; A within the
rounding bound of double-precision dot products,
    |A_gpu - A_oracle| <= ((2V + 32) * 2^-53 * S + 4 * 2^-53 * |A| * N) / N,
with S the sum of |increments| of the pair (the oracle reports it) -- both
sides sum V rounded double terms in different orders, and each term carries
a few roundings (sqrt, divisions, products).  NaN exactly where N = 0."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

pg = pytest.importorskip("paper_1410_4803_amd")

U = 2.0 ** -53


def _bound(V, S, A, N):
    return ((2 * V + 32) * U * S + 4 * U * np.abs(np.nan_to_num(A)) * N) / np.maximum(N, 1)


def _compare(A, N, Ar, Nr, Sr, V):
    assert np.array_equal(N.astype(np.uint32), Nr)
    nan = Nr == 0
    assert np.all(np.isnan(A[nan])) and np.all(np.isnan(Ar[nan]))
    ok = ~nan
    err = np.abs(A[ok] - Ar[ok])
    bound = _bound(V, Sr[ok], Ar[ok], Nr[ok])
    assert np.all(err <= bound), f"max err {err.max()} vs bound {bound[np.argmax(err - bound)]}"


def _gpu(bed, n, layout, mask=None, **kw):
    c = pg.Cohort.from_numpy(bed, n, mask)
    A, N = pg.grm_matrix(c, layout=layout, **kw)
    torch.cuda.synchronize()
    return A.cpu().numpy(), N.cpu().numpy().view(np.uint32)


# kernel variants: 1 = four waves of 64x64, 2 = eight waves of 32x64 (the
# default), 3 = sixteen waves of 32x32
VARIANTS = {"w4": 2 | (1 << 8), "w8": 2 | (2 << 8), "w16": 2 | (3 << 8)}


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("layout", ["full", "tri"])
@pytest.mark.parametrize("n,V", [(1, 10), (2, 17), (5, 100), (127, 300), (128, 1000),
                                 (129, 1025), (300, 2000), (513, 700)])
def test_grm_parity(n, V, layout, variant):
    bed = synth.hwe(n, V, (0.01, 0.5), 0.02, seed=n * 7 + V, garbage_pad=True)
    codes = oracle.unpack(bed, n, V)
    Ar, Nr, Sr = oracle.grm(codes, full=layout == "full")
    if n < 2 and layout == "tri":
        return
    A, N = _gpu(bed, n, layout, path=VARIANTS[variant])
    _compare(A.reshape(Ar.shape), N.reshape(Nr.shape), Ar, Nr, Sr, V)


def test_grm_undefined_markers_and_empty_sample():
    """Monomorphic and all-missing markers are left out; a sample with no
    call has N = 0 and NaN in its whole row."""
    n, V = 70, 400
    codes = oracle.unpack(synth.mosaic(n, V, 6, 0.02, 0.001, 0.0, 0.03, seed=31), n, V)
    codes[3] = 0
    codes[4] = 3
    codes[5] = 1
    codes[:, 9] = 1
    bed = np.zeros((V, (n + 3) // 4), dtype=np.uint8)
    for k in range(n):
        bed[:, k // 4] |= codes[:, k].astype(np.uint8) << (2 * (k % 4))
    Ar, Nr, Sr = oracle.grm(codes, full=True)
    assert np.all(Nr[9] == 0)
    A, N = _gpu(bed, n, "full")
    _compare(A, N, Ar, Nr, Sr, V)


def test_grm_mask_selection_range():
    n, V = 300, 3000
    bed = synth.mosaic(n, V, 8, 0.01, 0.001, 0.0, 0.01, seed=32, garbage_pad=True)
    mask = synth.missing_mask(n, V, 0.04, seed=33)
    rng = np.random.default_rng(4)
    idx = rng.integers(0, n, 211).astype(np.int32)     # duplicates allowed
    vb, ve = 17, 2950
    codes = oracle.select(oracle.unpack(bed, n, V, mask), idx, vb, ve)
    Ar, Nr, Sr = oracle.grm(codes, full=True)
    A, N = _gpu(bed, n, "full", mask, sample_idx=torch.from_numpy(idx).cuda(), v_range=(vb, ve))
    _compare(A, N, Ar, Nr, Sr, ve - vb)


@pytest.mark.parametrize("variant", list(VARIANTS))
def test_grm_full_size_sampled(variant):
    """The 10,000 x 71,307 workload the benchmark times: sampled pairs,
    the diagonal and the first row against the oracle, and symmetry."""
    w = synth.grm_large()
    n, V = w["n"], w["V"]
    codes_sm = np.ascontiguousarray(oracle.unpack(w["bed"], n, V).T)
    A, N = _gpu(w["bed"], n, "full", path=VARIANTS[variant])
    assert np.array_equal(A, A.T, equal_nan=True) and np.array_equal(N, N.T)
    rng = np.random.default_rng(5)
    pi = np.concatenate([rng.integers(0, n, 3000), np.arange(n), np.zeros(n, dtype=np.int64)])
    pj = np.concatenate([rng.integers(0, n, 3000), np.arange(n), np.arange(n)])
    Ar, Nr, Sr = oracle.grm_pairs(codes_sm, pi, pj)
    _compare(A[pi, pj], N[pi, pj], Ar, Nr, Sr, V)


def test_grm_medium_cohort_k_split():
    """2,000 samples (136 tiles of 128, more than half a round of the CUs):
    the default kernel splits each tile's variants into three ranges."""
    n, V = 2000, 4096
    bed = synth.hwe(n, V, (0.01, 0.5), 0.02, seed=2024)
    codes = oracle.unpack(bed, n, V)
    Ar, Nr, Sr = oracle.grm(codes, full=False)
    A, N = _gpu(bed, n, "tri")
    _compare(A.reshape(Ar.shape), N.reshape(Nr.shape), Ar, Nr, Sr, V)
