"""Pins of the oracle's IBS similarity and IBD report (--distance ibs,
--Z-genome; section "Identity-by-state matrices, complete linkage
clustering" and the IBD report timed in Table 2), from outside its own
formulas:
- every expected-IBS term equals an exact count of ordered allele draws
  without replacement, enumerated by brute force over labelled alleles;
- the terms tend to the Hardy-Weinberg closed forms as the pool grows;
- on simulated pedigrees the estimates recover the relationship: duplicates
  (Z2 = 1 exactly), parent-offspring (Z1 near 1), full siblings (Z near
  1/4, 1/2, 1/4) and unrelated samples (Z0 near 1);
- the similarity is the correctly rounded rational and complements the
  distance."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle


def _draws(x, y, k):
    """Ordered draws of k alleles without replacement from x labelled A2
    alleles and y labelled A1 alleles, as tuples of allele types."""
    pool = [1] * x + [0] * y
    return [tuple(pool[i] for i in perm) for perm in itertools.permutations(range(x + y), k)]


def _ibs(g1, g2):
    """Shared alleles IBS between two unordered genotypes (allele pairs)."""
    d1, d2 = sum(g1), sum(g2)
    return 2 - abs(d1 - d2)


def _exact_terms(x, y):
    four = _draws(x, y, 4)
    c = [0, 0, 0]
    for d in four:
        c[_ibs(d[:2], d[2:])] += 1
    three = _draws(x, y, 3)
    c1 = [0, 0, 0]
    for s, a, b in three:
        c1[_ibs((s, a), (s, b))] += 1
    n4, n3 = len(four), len(three)
    return [Fraction(c[0], n4), Fraction(c[1], n4), Fraction(c[2], n4),
            Fraction(c1[1], n3), Fraction(c1[2], n3)], c1[0]


@pytest.mark.parametrize("x,y", [(x, n - x) for n in range(4, 9) for x in range(0, n + 1)])
def test_terms_equal_enumerated_draws(x, y):
    exact, ibs0_given_ibd1 = _exact_terms(x, y)
    assert ibs0_given_ibd1 == 0                    # sharing one allele IBD excludes IBS0
    got = oracle.genome_terms(x, y)
    for g, e in zip(got, exact):
        assert abs(g - float(e)) <= 4e-16 * max(1.0, float(e)), (x, y, got, exact)


@pytest.mark.parametrize("x,y", [(3, 9), (17, 4), (250, 750), (12345, 98765)])
def test_terms_are_distributions(x, y):
    t = oracle.genome_terms(x, y)
    assert abs(t[0] + t[1] + t[2] - 1.0) <= 1e-15
    assert abs(t[3] + t[4] - 1.0) <= 1e-15
    assert (t >= 0).all()


@pytest.mark.parametrize("p", [0.05, 0.2, 0.5])
def test_terms_tend_to_hardy_weinberg(p):
    n = 2_000_000
    x = int(round(p * n))
    q = 1.0 - p
    t = oracle.genome_terms(x, n - x)
    hwe = [2 * p * p * q * q, 4 * p ** 3 * q + 4 * p * q ** 3, p ** 4 + q ** 4 + 4 * p * p * q * q,
           2 * p * q, 1 - 2 * p * q]
    assert np.allclose(t, hwe, atol=2e-6)


def _pedigree(V, seed):
    """Haplotype pairs (allele 1 = A2) of: founders f0, f1 (parents), their
    two children c0, c1, an unrelated u, and a duplicate of f0."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.05, 0.5, V)
    founders = [(rng.random(V) < p).astype(np.int8) for _ in range(6)]
    f0 = (founders[0], founders[1])
    f1 = (founders[2], founders[3])
    u = (founders[4], founders[5])

    def child():
        pick0 = rng.integers(0, 2, V).astype(bool)
        pick1 = rng.integers(0, 2, V).astype(bool)
        return (np.where(pick0, f0[0], f0[1]), np.where(pick1, f1[0], f1[1]))

    c0, c1 = child(), child()
    samples = [f0, f1, c0, c1, u, f0]
    code = {0: 0, 1: 2, 2: 3}                      # A2 dosage -> .bed code
    dos = np.stack([h[0] + h[1] for h in samples], 1)     # (V, samples)
    return np.vectorize(code.get)(dos).astype(np.int8)


def test_estimates_recover_relationships():
    """A population of 200 unrelated samples (for the allele frequencies) plus
    a small pedigree; the estimates of the pedigree pairs."""
    V = 20000
    rng = np.random.default_rng(5)
    p = rng.uniform(0.05, 0.5, V)
    pop = (rng.random((V, 200)) < p[:, None]).astype(np.int8) + \
          (rng.random((V, 200)) < p[:, None]).astype(np.int8)
    pop = np.vectorize({0: 0, 1: 2, 2: 3}.get)(pop).astype(np.int8)
    ped = _pedigree(V, 6)
    codes = np.ascontiguousarray(np.concatenate([ped, pop], 1))
    i0, i1, i2, nm = oracle.ibs_matrix(codes, full=True)
    z0, z1, z2, pi = oracle.genome(codes, i0, i1, nm)
    # duplicate of f0: exactly Z2 = 1
    assert (z0[0, 5], z1[0, 5], z2[0, 5], pi[0, 5]) == (0.0, 0.0, 1.0, 1.0)
    for a, b in ((0, 2), (0, 3), (1, 2), (1, 3)):           # parent-offspring
        assert z1[a, b] > 0.9 and z0[a, b] < 0.05 and abs(pi[a, b] - 0.5) < 0.05, (a, b)
    assert abs(z0[2, 3] - 0.25) < 0.05 and abs(z1[2, 3] - 0.5) < 0.08 \
        and abs(z2[2, 3] - 0.25) < 0.05 and abs(pi[2, 3] - 0.5) < 0.05   # full siblings
    for a, b in ((0, 1), (0, 4), (2, 4), (10, 11), (50, 60)):         # unrelated
        assert z0[a, b] > 0.9 and pi[a, b] < 0.05, (a, b)
    assert np.allclose(z0 + z1 + z2, 1.0, atol=1e-12)
    assert (z1 >= 0).all() and (z0 <= 1).all()


def test_undefined_cases_are_nan():
    codes = np.array([[0, 3, 2], [1, 1, 1]], dtype=np.int8)   # second marker all missing
    i0, i1, i2, nm = oracle.ibs_matrix(codes, full=True)
    z = oracle.genome(codes, i0, i1, nm)
    assert all(np.isnan(a[0, 0]) == (nm[0, 0] == 0) for a in z)
    codes = np.full((3, 4), 1, dtype=np.int8)                 # no informative marker at all
    i0, i1, i2, nm = oracle.ibs_matrix(codes, full=True)
    assert all(np.isnan(a).all() for a in oracle.genome(codes, i0, i1, nm))


def test_similarity_is_the_rounded_rational():
    rng = np.random.default_rng(9)
    nm = rng.integers(0, 100000, 500).astype(np.uint32)
    i1 = (rng.random(500) * nm).astype(np.uint32)
    i2 = (rng.random(500) * (nm - i1)).astype(np.uint32)
    i0 = nm - i1 - i2
    s = oracle.ibs_similarity(i1, i2, nm)
    d = oracle.ibs_distance(i0, i1, nm)
    for k in range(500):
        if nm[k] == 0:
            assert np.isnan(s[k]) and np.isinf(d[k])
            continue
        assert s[k] == float(Fraction(2 * int(i2[k]) + int(i1[k]), 2 * int(nm[k])))
        assert abs(s[k] + d[k] - 1.0) <= 2.3e-16


def test_means_within_rounding_bound_of_exact_mean():
    """The five means over 2,500 markers (two full runs of 1,024 and a ragged
    third): within the rounding bound of the exact rational mean of the same
    per-marker terms (each term pinned above), and K equals the markers with
    at least 4 observed alleles, counted directly.  Includes markers with no
    call, one call and two calls."""
    rng = np.random.default_rng(21)
    V, n = 2500, 40
    codes = rng.choice(np.array([0, 1, 2, 3], dtype=np.int8), size=(V, n),
                       p=[0.3, 0.05, 0.4, 0.25])
    codes[7] = 1
    codes[1500] = 1
    codes[1500, 3] = 2
    codes[2100] = 1
    codes[2100, [0, 9]] = 3
    E, K = oracle.genome_means(codes)
    called = (codes != 1).sum(axis=1)
    use = 2 * called >= 4
    assert K == int(use.sum()) and K == V - 2 and not use[7] and not use[1500] and use[2100]
    exact = [Fraction(0)] * 5
    for v in np.nonzero(use)[0]:
        a2 = int(np.where(codes[v] == 3, 2, np.where(codes[v] == 2, 1, 0)).sum())
        t = oracle.genome_terms(a2, 2 * int(called[v]) - a2)
        exact = [e + Fraction(float(x)) for e, x in zip(exact, t)]
    for q in range(5):
        mean = exact[q] / K
        bound = Fraction(V + 2, 2 ** 53) * mean
        assert abs(Fraction(float(E[q])) - mean) <= bound, q
