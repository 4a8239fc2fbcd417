"""CPU oracle (test infrastructure only).

The plain definitions of the IBS and LD statistics of Chang et al. 2015
(arXiv 1410.4803), section "Bitwise parallelism" (the per-marker IBS loop)
and section "Bit population count" (r between two markers with missing
data), the greedy LD pruning of section "Linkage disequilibrium-based
variant pruning" and the genomic relationship matrix of section "Partial sum
lookup", and the IBS distance with complete-linkage clustering of section
"Identity-by-state matrices, complete linkage clustering" (under the readings
stated in ``oracle.c``), written in ``oracle.c``.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the GPU library
(``paper_1410_4803_amd``) and imports nothing from it.

Every function here is pinned by tests that do not re-use it: brute force of
the paper's literal bit rule on tiny inputs, invariants, numpy matrix products
of indicator matrices and ``numpy.corrcoef`` (``tests/test_oracle_pins.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

LD_RECORD = np.dtype([("a", "<i4"), ("b", "<i4"), ("n", "<i8"), ("sx", "<i8"), ("sy", "<i8"),
                      ("sxx", "<i8"), ("syy", "<i8"), ("sxy", "<i8"), ("r2", "<f8")])
assert LD_RECORD.itemsize == 64


def build(force: bool = True) -> str:
    """Compile liboracle.so: plain C, -O2, OpenMP, strict IEEE double (no
    fast-math, no contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off",
             os.path.join(_HERE, "oracle.c"), "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        i64, i32, dbl, p = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        lib.oracle_unpack.argtypes = [p, i64, i64, i64, p, i32, p]
        lib.oracle_unpack.restype = None
        lib.oracle_ibs_pairs.argtypes = [p, i64, i64, p, p, i64, p]
        lib.oracle_ibs_pairs.restype = None
        lib.oracle_ibs_matrix.argtypes = [p, i64, i64, i32, p, p, p, p]
        lib.oracle_ibs_matrix.restype = None
        lib.oracle_r2.argtypes = [p]
        lib.oracle_r2.restype = dbl
        lib.oracle_ld_pairs.argtypes = [p, i64, i64, p, p, i64, p, p]
        lib.oracle_ld_pairs.restype = None
        lib.oracle_ld_window.argtypes = [p, i64, i64, i64, i64, i64, dbl, p, i64]
        lib.oracle_ld_window.restype = i64
        lib.oracle_r2_counts.argtypes = [p]
        lib.oracle_r2_counts.restype = dbl
        lib.oracle_ld_prune.argtypes = [p, i64, i64, i64, i64, dbl, p]
        lib.oracle_ld_prune.restype = i64
        lib.oracle_grm.argtypes = [p, i64, i64, i32, p, p, p]
        lib.oracle_grm.restype = None
        lib.oracle_grm_pairs.argtypes = [p, i64, i64, p, p, i64, p, p, p]
        lib.oracle_grm_pairs.restype = None
        lib.oracle_ibs_distance.argtypes = [p, p, p, i64, p]
        lib.oracle_ibs_distance.restype = None
        lib.oracle_ibs_similarity.argtypes = [p, p, p, i64, p]
        lib.oracle_ibs_similarity.restype = None
        lib.oracle_genome_terms.argtypes = [i64, i64, p]
        lib.oracle_genome_terms.restype = None
        lib.oracle_genome.argtypes = [p, i64, i64, p, p, p, i64, p, p, p, p]
        lib.oracle_genome.restype = None
        lib.oracle_genome_means.argtypes = [p, i64, i64, p, p]
        lib.oracle_genome_means.restype = None
        lib.oracle_cluster_complete.argtypes = [p, i64, p]
        lib.oracle_cluster_complete.restype = i32
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = i32
        _lib = lib
    return _lib


def threads() -> int:
    return int(_load().oracle_threads())


def _c(a: np.ndarray, dtype) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


def unpack(bed: np.ndarray, n: int, V: int, missing_mask: np.ndarray | None = None,
           sample_major: bool = False) -> np.ndarray:
    """int8 codes: (n, V) if sample_major else (V, n)."""
    bed = _c(bed, np.uint8)
    if bed.ndim != 2 or bed.shape[0] < V or bed.shape[1] < (n + 3) // 4:
        raise ValueError("bed must be (>=V, >=ceil(n/4)) uint8")
    out = np.empty((n, V) if sample_major else (V, n), dtype=np.int8)
    mp = None
    if missing_mask is not None:
        missing_mask = _c(missing_mask, np.uint64)
        if missing_mask.shape != (V, (n + 63) // 64):
            raise ValueError("missing_mask must be (V, ceil(n/64)) uint64")
        mp = missing_mask.ctypes.data
    _load().oracle_unpack(bed.ctypes.data, n, V, bed.shape[1], mp, int(sample_major),
                          out.ctypes.data)
    return out


def select(codes_vm: np.ndarray, sample_idx=None, v_begin: int = 0, v_end: int | None = None):
    """Restrict variant-major codes to a sample list (in the given order,
    duplicates allowed) and a variant range [v_begin, v_end)."""
    c = codes_vm[v_begin:v_end]
    if sample_idx is not None:
        c = c[:, np.asarray(sample_idx, dtype=np.int64)]
    return np.ascontiguousarray(c)


def ibs_matrix(codes_vm: np.ndarray, full: bool = True):
    """(IBS0, IBS1, IBS2, N) as uint32 arrays: (n, n) if full else the packed
    strict upper triangle of length n(n-1)/2."""
    V, n = codes_vm.shape
    sm = np.ascontiguousarray(codes_vm.T)
    size = n * n if full else n * (n - 1) // 2
    outs = [np.zeros(size, dtype=np.uint32) for _ in range(4)]
    _load().oracle_ibs_matrix(sm.ctypes.data, n, V, int(full), *[o.ctypes.data for o in outs])
    if full:
        outs = [o.reshape(n, n) for o in outs]
    return tuple(outs)


def ibs_pairs(codes_sm: np.ndarray, pi, pj) -> np.ndarray:
    """(npairs, 4) uint32: IBS0, IBS1, IBS2, N for each pair; codes_sm is (n, V)."""
    n, V = codes_sm.shape
    codes_sm = _c(codes_sm, np.int8)
    pi = _c(pi, np.int64)
    pj = _c(pj, np.int64)
    out = np.zeros((len(pi), 4), dtype=np.uint32)
    _load().oracle_ibs_pairs(codes_sm.ctypes.data, n, V, pi.ctypes.data, pj.ctypes.data,
                             len(pi), out.ctypes.data)
    return out


def ld_pairs(codes_vm: np.ndarray, pa, pb):
    """(sums (npairs, 6) int64 [n, Sx, Sy, Sxx, Syy, Sxy], r2 (npairs,) float64)."""
    V, n = codes_vm.shape
    codes_vm = _c(codes_vm, np.int8)
    pa = _c(pa, np.int64)
    pb = _c(pb, np.int64)
    sums = np.zeros((len(pa), 6), dtype=np.int64)
    r2 = np.zeros(len(pa), dtype=np.float64)
    _load().oracle_ld_pairs(codes_vm.ctypes.data, n, V, pa.ctypes.data, pb.ctypes.data,
                            len(pa), sums.ctypes.data, r2.ctypes.data)
    return sums, r2


def r2_from_sums(s) -> float:
    s = _c(s, np.int64)
    return float(_load().oracle_r2(s.ctypes.data))


def ld_window(codes_vm: np.ndarray, window: int, r2_min: float, a_begin: int = 0,
              a_end: int | None = None, capacity: int | None = None) -> np.ndarray:
    """Kept LD records in (a, b) order, as a structured array of LD_RECORD."""
    V, n = codes_vm.shape
    codes_vm = _c(codes_vm, np.int8)
    a_end = V if a_end is None else a_end
    lib = _load()
    if capacity is None:
        total = lib.oracle_ld_window(codes_vm.ctypes.data, n, V, a_begin, a_end, window,
                                     float(r2_min), None, 0)
        capacity = total
    out = np.zeros(max(capacity, 1), dtype=LD_RECORD)
    total = lib.oracle_ld_window(codes_vm.ctypes.data, n, V, a_begin, a_end, window,
                                 float(r2_min), out.ctypes.data, capacity)
    if total < 0:
        raise MemoryError("oracle_ld_window")
    return out[:min(total, capacity)]


def r2_counts(s) -> float:
    """r^2 as the pruning decision takes it: exact integer cov, vx, vy, then
    (cov*cov)/(vx*vy) in IEEE double, clamped to 1 (NaN when undefined)."""
    s = _c(s, np.int64)
    return float(_load().oracle_r2_counts(s.ctypes.data))


def ld_prune(codes_vm: np.ndarray, window: int, step: int, r2_max: float) -> np.ndarray:
    """Greedy --indep-pairwise pruning; uint8 keep flag per variant."""
    V, n = codes_vm.shape
    codes_vm = _c(codes_vm, np.int8)
    keep = np.zeros(V, dtype=np.uint8)
    kept = _load().oracle_ld_prune(codes_vm.ctypes.data, n, V, int(window), int(step),
                                   float(r2_max), keep.ctypes.data)
    if kept < 0:
        raise MemoryError("oracle_ld_prune")
    return keep


def grm(codes_vm: np.ndarray, full: bool = True):
    """(A float64, N uint32, abs_sum float64): the relationship matrix from
    per-marker increment tables; (n, n) if full else the packed strict upper
    triangle."""
    V, n = codes_vm.shape
    sm = np.ascontiguousarray(codes_vm.T)
    size = n * n if full else n * (n - 1) // 2
    A = np.zeros(size, dtype=np.float64)
    N = np.zeros(size, dtype=np.uint32)
    S = np.zeros(size, dtype=np.float64)
    _load().oracle_grm(sm.ctypes.data, n, V, int(full), A.ctypes.data, N.ctypes.data,
                       S.ctypes.data)
    if full:
        A, N, S = A.reshape(n, n), N.reshape(n, n), S.reshape(n, n)
    return A, N, S


def grm_pairs(codes_sm: np.ndarray, pi, pj):
    """(A, N, abs_sum) of the relationship matrix for listed sample pairs;
    codes_sm is (n, V) sample-major."""
    n, V = codes_sm.shape
    codes_sm = _c(codes_sm, np.int8)
    pi = _c(pi, np.int64)
    pj = _c(pj, np.int64)
    A = np.zeros(len(pi), dtype=np.float64)
    N = np.zeros(len(pi), dtype=np.uint32)
    S = np.zeros(len(pi), dtype=np.float64)
    _load().oracle_grm_pairs(codes_sm.ctypes.data, n, V, pi.ctypes.data, pj.ctypes.data, len(pi),
                             A.ctypes.data, N.ctypes.data, S.ctypes.data)
    return A, N, S


MERGE = np.dtype([("a", "<i4"), ("b", "<i4"), ("height", "<f8")])
assert MERGE.itemsize == 16


def ibs_distance(ibs0, ibs1, nonmiss) -> np.ndarray:
    """(2*IBS0 + IBS1) / (2*N) elementwise (+inf where N = 0), same shape."""
    i0, i1, nm = (_c(x, np.uint32) for x in (ibs0, ibs1, nonmiss))
    out = np.zeros(i0.shape, dtype=np.float64)
    _load().oracle_ibs_distance(i0.ctypes.data, i1.ctypes.data, nm.ctypes.data, i0.size,
                                out.ctypes.data)
    return out


def ibs_similarity(ibs1, ibs2, nonmiss) -> np.ndarray:
    """(2*IBS2 + IBS1) / (2*N) elementwise (NaN where N = 0), same shape."""
    i1, i2, nm = (_c(x, np.uint32) for x in (ibs1, ibs2, nonmiss))
    out = np.zeros(i1.shape, dtype=np.float64)
    _load().oracle_ibs_similarity(i1.ctypes.data, i2.ctypes.data, nm.ctypes.data, i1.size,
                                  out.ctypes.data)
    return out


def genome_terms(x: int, y: int) -> np.ndarray:
    """The five expected-IBS-given-IBD terms of one marker with x A2 and y A1
    alleles observed: P(IBS0|IBD0), P(IBS1|IBD0), P(IBS2|IBD0), P(IBS1|IBD1),
    P(IBS2|IBD1)."""
    t = np.zeros(5, dtype=np.float64)
    _load().oracle_genome_terms(int(x), int(y), t.ctypes.data)
    return t


def genome_means(codes_vm: np.ndarray):
    """((E00, E10, E20, E11, E21), K): the means of the five terms over the
    markers of codes_vm with at least 4 observed alleles, and their count."""
    V, n = codes_vm.shape
    codes_vm = _c(codes_vm, np.int8)
    e = np.zeros(5, dtype=np.float64)
    k = np.zeros(1, dtype=np.int64)
    _load().oracle_genome_means(codes_vm.ctypes.data, n, V, e.ctypes.data, k.ctypes.data)
    return e, int(k[0])


def genome(codes_vm: np.ndarray, ibs0, ibs1, nonmiss):
    """(Z0, Z1, Z2, PI_HAT) float64 arrays shaped like the counts: the IBD
    report for IBS counts computed over the samples and variants of
    codes_vm."""
    V, n = codes_vm.shape
    codes_vm = _c(codes_vm, np.int8)
    i0, i1, nm = (_c(x, np.uint32) for x in (ibs0, ibs1, nonmiss))
    outs = [np.zeros(i0.shape, dtype=np.float64) for _ in range(4)]
    _load().oracle_genome(codes_vm.ctypes.data, n, V, i0.ctypes.data, i1.ctypes.data,
                          nm.ctypes.data, i0.size, *[o.ctypes.data for o in outs])
    return tuple(outs)


def cluster_complete(dist: np.ndarray) -> np.ndarray:
    """Complete-linkage merge sequence (m-1 MERGE records) of an m x m
    distance matrix; ties by the smallest (a, b)."""
    d = _c(dist, np.float64)
    m = d.shape[0]
    out = np.zeros(max(m - 1, 1), dtype=MERGE)
    if _load().oracle_cluster_complete(d.ctypes.data, m, out.ctypes.data) != 0:
        raise MemoryError("oracle_cluster_complete")
    return out[:m - 1]
