"""Seeded synthetic genotype panels in PLINK 1 binary (.bed) layout.

Shared by the tests, the benchmark and the oracle's checks; holds none of the
pairwise statistics.  The C generator (``synth.c``) is built with gcc into
``libsynth.so`` next to this file.

Code table (one 2-bit code per call, low bits first, four calls per byte,
variant-major rows, no file header): 0 homozygous A1, 1 missing,
2 heterozygous, 3 homozygous A2.

The workloads below stand in for the paper's datasets (HAPGEN2 /
simuRare / 1000 Genomes panels, which are not available): they take the
shapes and the value distributions the workloads are specified with.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile libsynth.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
             os.path.join(_HERE, "synth.c"), "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        i64, u64, dbl, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int
        ptr = ctypes.c_void_p
        lib.synth_hwe.argtypes = [i64, i64, dbl, dbl, dbl, u64, i32, ptr]
        lib.synth_hwe.restype = i32
        lib.synth_mosaic.argtypes = [i64, i64, i32, dbl, dbl, dbl, dbl, u64, i32, ptr]
        lib.synth_mosaic.restype = i64
        lib.synth_missing_mask.argtypes = [i64, i64, dbl, u64, ptr]
        lib.synth_missing_mask.restype = i32
        lib.synth_splitmix64_first.argtypes = [u64]
        lib.synth_splitmix64_first.restype = u64
        lib.synth_xoshiro_first.argtypes = [u64, u64, u64, u64]
        lib.synth_xoshiro_first.restype = u64
        _lib = lib
    return _lib


def bytes_per_variant(n: int) -> int:
    return (n + 3) // 4


def hwe(n: int, V: int, q=(0.05, 0.5), miss: float = 0.01, seed: int = 1000,
        garbage_pad: bool = False) -> np.ndarray:
    """Hardy-Weinberg panel; returns a (V, ceil(n/4)) uint8 array."""
    out = np.empty((V, bytes_per_variant(n)), dtype=np.uint8)
    rc = _load().synth_hwe(n, V, float(q[0]), float(q[1]), float(miss), seed,
                           int(garbage_pad), out.ctypes.data)
    if rc != 0:
        raise ValueError("synth_hwe: bad arguments")
    return out


def mosaic(n: int, V: int, founders: int = 20, switch: float = 0.01, mu: float = 0.001,
           maf_min: float = 0.01, miss: float = 0.02, seed: int = 1001,
           garbage_pad: bool = False) -> np.ndarray:
    """Founder-mosaic panel; returns a (V, ceil(n/4)) uint8 array."""
    out = np.empty((V, bytes_per_variant(n)), dtype=np.uint8)
    rc = _load().synth_mosaic(n, V, founders, float(switch), float(mu), float(maf_min),
                              float(miss), seed, int(garbage_pad), out.ctypes.data)
    if rc < 0:
        raise ValueError("synth_mosaic: bad arguments")
    return out


def missing_mask(n: int, V: int, rate: float, seed: int) -> np.ndarray:
    """(V, ceil(n/64)) uint64 mask, bit set = call missing."""
    out = np.empty((V, (n + 63) // 64), dtype=np.uint64)
    if _load().synth_missing_mask(n, V, float(rate), seed, out.ctypes.data) != 0:
        raise ValueError("synth_missing_mask: bad arguments")
    return out


# --- workloads ---------------------------------------------------------------

def ibs_small(seed: int = 1000) -> dict:
    """IBS matrix, 500 samples x 5,000 variants, HWE, MAF~U[0.05,0.5], 1% missing.
    Output: the 124,750 strict-upper-triangle pair counts."""
    n, V = 500, 5000
    return dict(name="ibs_500x5000_hwe", n=n, V=V, layout="tri",
                bed=hwe(n, V, (0.05, 0.5), 0.01, seed))


def ibs_large(seed: int = 1001) -> dict:
    """IBS matrix, 10,000 samples x 100,000 variants, founder mosaic (20
    founders, switch 0.01, mutation 0.001, MAF>=0.01), 2% missing.  Output:
    full 10k x 10k matrices."""
    n, V = 10000, 100000
    return dict(name="ibs_10000x100000_mosaic", n=n, V=V, layout="full",
                bed=mosaic(n, V, 20, 0.01, 0.001, 0.01, 0.02, seed))


def ld_large(seed: int = 1002) -> dict:
    """LD windows, 5,000 samples x 500,000 variants, founder mosaic (switch
    0.005), 1% missing; window 1,000 variants, emit r^2 >= 0.2."""
    n, V = 5000, 500000
    return dict(name="ld_5000x500000_mosaic_w1000", n=n, V=V, window=1000, r2_min=0.2,
                bed=mosaic(n, V, 20, 0.005, 0.001, 0.01, 0.01, seed))


def ld_large_nomiss(seed: int = 1002) -> dict:
    """The LD window workload without missing calls (same generator and
    seed, missing rate 0): the case where only sum x_a x_b varies per pair."""
    n, V = 5000, 500000
    return dict(name="ld_5000x500000_mosaic_w1000_nomiss", n=n, V=V, window=1000, r2_min=0.2,
                bed=mosaic(n, V, 20, 0.005, 0.001, 0.01, 0.0, seed))


def prune_small(seed: int = 1005) -> dict:
    """LD pruning, 1,000 samples x 100,000 variants, founder mosaic (10
    founders, switch 0.01, mutation 0.001, MAF>=0.01), no missing calls;
    --indep-pairwise 50 5 0.5.  The founder count is chosen so that about
    three quarters of the variants survive, as in the paper's pruned
    1,000-sample panel."""
    n, V = 1000, 100000
    return dict(name="prune_1000x100000_mosaic_50_5_0.5", n=n, V=V, window=50, step=5,
                r2_max=0.5, bed=mosaic(n, V, 10, 0.01, 0.001, 0.01, 0.0, seed))


def prune_large(seed: int = 1006) -> dict:
    """LD pruning, 10,000 samples x 88,025 variants, founder mosaic (8
    founders, switch 0.01, mutation 0.001, MAF>=0.01), no missing calls;
    --indep-pairwise 700 70 0.7.  About four fifths of the variants survive,
    as in the paper's pruned 10,000-sample panel."""
    n, V = 10000, 88025
    return dict(name="prune_10000x88025_mosaic_700_70_0.7", n=n, V=V, window=700, step=70,
                r2_max=0.7, bed=mosaic(n, V, 8, 0.01, 0.001, 0.01, 0.0, seed))


def grm_small(seed: int = 1007) -> dict:
    """Relationship matrix, 1,000 samples x 76,124 variants (the size of the
    paper's pruned 1,000-sample panel), founder mosaic (10 founders, switch
    0.01), 1% missing; full matrix."""
    n, V = 1000, 76124
    return dict(name="grm_1000x76124_mosaic", n=n, V=V, layout="full",
                bed=mosaic(n, V, 10, 0.01, 0.001, 0.01, 0.01, seed))


def grm_large(seed: int = 1008) -> dict:
    """Relationship matrix, 10,000 samples x 71,307 variants (the size of
    the paper's pruned 10,000-sample panel), founder mosaic (8 founders,
    switch 0.01), 1% missing; full matrix."""
    n, V = 10000, 71307
    return dict(name="grm_10000x71307_mosaic", n=n, V=V, layout="full",
                bed=mosaic(n, V, 8, 0.01, 0.001, 0.01, 0.01, seed))


def batch_problems(seed: int = 1003, count: int = 64, make_bed: bool = True) -> list:
    """Batched workload: `count` cohorts, samples log-uniform in [200, 20000],
    variants log-uniform in [2000, 50000], HWE MAF~U[0.01,0.5], 1% missing;
    even index IBS (upper triangle), odd index LD window 500, r^2 >= 0.2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    probs = []
    for p in range(count):
        n = int(round(math.exp(rng.uniform(math.log(200), math.log(20000)))))
        V = int(round(math.exp(rng.uniform(math.log(2000), math.log(50000)))))
        kind = "ibs" if p % 2 == 0 else "ld"
        d = dict(kind=kind, n=n, V=V, seed=seed * 1000 + p)
        if kind == "ld":
            d.update(window=500, r2_min=0.2)
        else:
            d.update(layout="tri")
        if make_bed:
            d["bed"] = hwe(n, V, (0.01, 0.5), 0.01, d["seed"])
        probs.append(d)
    return probs


def serve_cohorts(seed: int = 1004, count: int = 8) -> list:
    """Serving workload cohorts: samples log-uniform in [1k, 50k], variants
    log-uniform in [10k, 200k] (PCG64 `seed`), HWE MAF~U[0.01,0.5], 1%
    missing.  Returns dicts with n, V and the .bed seed; call hwe() (or
    serve_cohort_bed) for the payload."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(count):
        n = int(round(math.exp(rng.uniform(math.log(1000), math.log(50000)))))
        V = int(round(math.exp(rng.uniform(math.log(10000), math.log(200000)))))
        out.append(dict(n=n, V=V, seed=2000 + k))
    return out


def serve_cohort_bed(d: dict) -> np.ndarray:
    return hwe(d["n"], d["V"], (0.01, 0.5), 0.01, d["seed"])
