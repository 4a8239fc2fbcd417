"""Writes the stored oracle results of the two full-size workloads whose
oracle runs take CPU-minutes, so the GPU tests can compare against them:

  prune_10000x88025_700_70_0.7.txt
      keep flags of --indep-pairwise 700 70 0.7 on the 10,000-sample x
      88,025-variant pruning panel (section "Linkage disequilibrium-based
      variant pruning", Table 4), from oracle.ld_prune;
  cluster_10000x71307.txt.gz
      the complete-linkage merge sequence of the 10,000-sample x
      71,307-variant panel (section "Identity-by-state matrices, complete
      linkage clustering", Table 2): oracle IBS counts -> oracle.ibs_distance
      -> oracle.cluster_complete.

Only the oracle computes anything here; the inputs come from the seeded
generators in synth/.  Each file records the SHA-256 of the .bed payload it
was computed from, and the tests refuse a file whose payload hash differs.

    python tests/golden/make_fullsize.py [prune] [cluster]
"""
from __future__ import annotations

import gzip
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

PRUNE_FILE = os.path.join(HERE, "prune_10000x88025_700_70_0.7.txt")
CLUSTER_FILE = os.path.join(HERE, "cluster_10000x71307.txt.gz")


def bed_sha256(bed: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(bed).tobytes()).hexdigest()


def make_prune() -> None:
    w = synth.prune_large()
    codes = oracle.unpack(w["bed"], w["n"], w["V"])
    t = time.time()
    keep = oracle.ld_prune(codes, w["window"], w["step"], w["r2_max"])
    dt = time.time() - t
    bits = np.packbits(keep.astype(np.uint8), bitorder="little")
    hexs = bits.tobytes().hex()
    with open(PRUNE_FILE, "w") as f:
        f.write(f"# {w['name']}: keep flags from oracle.ld_prune "
                f"(window {w['window']}, step {w['step']}, r2 > {w['r2_max']} drops)\n")
        f.write("# section 'Linkage disequilibrium-based variant pruning', Table 4 workload shape\n")
        f.write(f"# bed_sha256 {bed_sha256(w['bed'])}\n")
        f.write(f"# variants {w['V']} kept {int(keep.sum())}\n")
        f.write(f"# oracle time {dt:.1f} s on {oracle.threads()} threads\n")
        f.write("# flags: bit v%8 of byte v/8 (little bit order), hex, 64 bytes a line\n")
        for k in range(0, len(hexs), 128):
            f.write(hexs[k:k + 128] + "\n")
    print(f"prune: kept {int(keep.sum())} of {w['V']} in {dt:.1f} s", flush=True)


def load_prune():
    """(bed_sha256, keep uint8 array) from the stored file."""
    sha, lines, V = None, [], None
    with open(PRUNE_FILE) as f:
        for line in f:
            if line.startswith("# bed_sha256"):
                sha = line.split()[2]
            elif line.startswith("# variants"):
                V = int(line.split()[2])
            elif not line.startswith("#"):
                lines.append(line.strip())
    bits = np.frombuffer(bytes.fromhex("".join(lines)), dtype=np.uint8)
    return sha, np.unpackbits(bits, bitorder="little")[:V]


def make_cluster() -> None:
    w = synth.grm_large()
    n, V = w["n"], w["V"]
    codes = oracle.unpack(w["bed"], n, V)
    t = time.time()
    i0, i1, _, nm = oracle.ibs_matrix(codes, full=False)
    t_ibs = time.time() - t
    del codes
    d_tri = oracle.ibs_distance(i0, i1, nm)
    del i0, i1, nm
    dist = np.zeros((n, n), dtype=np.float64)
    iu = np.triu_indices(n, 1)
    dist[iu] = d_tri
    dist.T[iu] = d_tri
    del d_tri, iu
    t = time.time()
    merges = oracle.cluster_complete(dist)
    t_cl = time.time() - t
    with gzip.open(CLUSTER_FILE, "wt") as f:
        f.write(f"# {w['name']}: complete-linkage merges from oracle.cluster_complete on "
                f"oracle.ibs_distance of the oracle IBS counts\n")
        f.write("# section 'Identity-by-state matrices, complete linkage clustering', Table 2\n")
        f.write(f"# bed_sha256 {bed_sha256(w['bed'])}\n")
        f.write(f"# oracle time: IBS {t_ibs:.0f} s on {oracle.threads()} threads, "
                f"clustering {t_cl:.0f} s on 1\n")
        f.write("# a b height (float.hex)\n")
        for r in merges:
            f.write(f"{int(r['a'])} {int(r['b'])} {float(r['height']).hex()}\n")
    print(f"cluster: {len(merges)} merges, IBS {t_ibs:.0f} s, clustering {t_cl:.0f} s",
          flush=True)


def load_cluster():
    """(bed_sha256, MERGE-like structured array) from the stored file."""
    sha, rows = None, []
    with gzip.open(CLUSTER_FILE, "rt") as f:
        for line in f:
            if line.startswith("# bed_sha256"):
                sha = line.split()[2]
            elif not line.startswith("#"):
                a, b, h = line.split()
                rows.append((int(a), int(b), float.fromhex(h)))
    out = np.zeros(len(rows), dtype=oracle.MERGE)
    for k, (a, b, h) in enumerate(rows):
        out[k] = (a, b, h)
    return sha, out


if __name__ == "__main__":
    what = sys.argv[1:] or ["prune", "cluster"]
    if "prune" in what:
        make_prune()
    if "cluster" in what:
        make_cluster()
