"""Autotuner: picks the kernel path (popcount or matrix core) and kernel
variant per problem shape by timing the candidates on the GPU.

Decisions are cached by shape bucket -- (kind, ceil(log2 m), ceil(log2 V),
ceil(log2 window)) -- in a JSON file, so one measurement serves every
problem of a similar shape.  Without a measurement the rule of thumb below
applies.  Timing uses HIP events on the launch stream around the whole
library call (layout + pair kernel + LD finish).
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import _native as N
from . import api

IBS_CANDIDATES = {"mfma": N.PG_PATH_MFMA, "mfma_int8": N.PG_PATH_MFMA | (7 << 8),
                  "mfma_fp4": N.PG_PATH_MFMA | (3 << 8), "mfma_fp4rep": N.PG_PATH_MFMA | (4 << 8),
                  "mfma_w8": N.PG_PATH_MFMA | (5 << 8), "popc": N.PG_PATH_POPC}
# a batch hosts the pipelined fp4 and int8 matrix-core tiles and the popcount
# tile, so the tile and the path are chosen per problem there
IBS_BATCH_CANDIDATES = {"mfma": N.PG_PATH_MFMA, "mfma_int8": N.PG_PATH_MFMA | (7 << 8),
                        "popc": N.PG_PATH_POPC}
# batches run the fp4 and int8 matrix-core and the popcount LD tiles;
# one-problem calls (the serving loop) also have the missing-call correction
# path
LD_BATCH_CANDIDATES = {"mfma": N.PG_PATH_MFMA, "mfma_int8": N.PG_PATH_MFMA | (1 << 8),
                       "popc": N.PG_PATH_POPC}
LD_CANDIDATES = {"mfma": N.PG_PATH_MFMA, "mfma_int8": N.PG_PATH_MFMA | (1 << 8),
                 "popc": N.PG_PATH_POPC, "sparse": N.PG_PATH_SPARSE}


def _bucket(x: int) -> int:
    return int(math.ceil(math.log2(max(int(x), 1))))


def shape_key(kind: str, m: int, nv: int, window: int | None = None) -> str:
    k = f"{kind}:{_bucket(m)}:{_bucket(nv)}"
    if kind == "ld":
        k += f":{_bucket(window)}"
    return k


def rule_of_thumb(kind: str, m: int, nv: int, window: int | None = None) -> int:
    """Default without a measurement: what the library's PG_PATH_AUTO resolves
    to for the shape (pg_resolve_path): the matrix-core path, except LD
    windows of 500 and up over 5,000 samples and up, where it is the
    correction path behind its sampled missing-call gate."""
    return api.resolve_path(kind, m, nv, window or 0, "auto")


class Tuner:
    def __init__(self, cache_path: str | None = None):
        self.cache_path = cache_path
        self.cache: dict[str, dict] = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    def save(self) -> None:
        if self.cache_path:
            tmp = self.cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)
            os.replace(tmp, self.cache_path)

    def choose(self, kind: str, m: int, nv: int, window: int | None = None) -> int:
        rec = self.cache.get(shape_key(kind, m, nv, window))
        if rec:
            return int(rec["path"])
        return rule_of_thumb(kind, m, nv, window)

    @staticmethod
    def _time(fn, reps: int) -> float:
        fn()                                   # warm-up
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            best = min(best, a.elapsed_time(b))
        return best

    def tune(self, kind: str, cohort: api.Cohort, *, sample_idx=None, v_range=None,
             layout: str = "tri", window: int | None = None, r2_min: float = 0.2,
             reps: int = 2, force: bool = False, for_batch: bool = False) -> int:
        """Measures every candidate on this problem (outputs discarded) unless
        its shape bucket is already decided; returns the chosen path code."""
        m = sample_idx.numel() if sample_idx is not None else cohort.n_samples
        nv = (v_range[1] - v_range[0]) if v_range else cohort.n_variants
        key = shape_key(kind, m, nv, window) + (":batch" if for_batch else "")
        if not force and key in self.cache:
            return int(self.cache[key]["path"])
        times = {}
        if kind == "ibs":
            out = tuple(torch.empty(api.ibs_output_size(m, layout), dtype=torch.int32,
                                    device=cohort.bed.device) for _ in range(4))
            cands = IBS_BATCH_CANDIDATES if for_batch else IBS_CANDIDATES
            for name, code in cands.items():
                ws = torch.empty(max(api.ibs_workspace_bytes(cohort, sample_idx.numel()
                                                             if sample_idx is not None else 0,
                                                             v_range, code), 1),
                                 dtype=torch.uint8, device=cohort.bed.device)
                times[name] = self._time(lambda: api.ibs_matrix(
                    cohort, sample_idx=sample_idx, v_range=v_range, layout=layout, path=code,
                    out=out, workspace=ws), reps)
                del ws
        else:
            cap = max(1024, 4 * nv)
            o = torch.empty((cap, 64), dtype=torch.uint8, device=cohort.bed.device)
            n_out = torch.empty(1, dtype=torch.int64, device=cohort.bed.device)
            cands = LD_BATCH_CANDIDATES if for_batch else LD_CANDIDATES
            for name, code in cands.items():
                times[name] = self._time(lambda: api.ld_window(
                    cohort, window, r2_min, capacity=cap, sample_idx=sample_idx, v_range=v_range,
                    path=code, out=o, n_out=n_out), reps)
        best = min(times, key=times.get)
        self.cache[key] = {"path": cands[best], "choice": best,
                           "ms": {k: round(v, 4) for k, v in times.items()}}
        return cands[best]
