"""Batched execution over the pg_batch_* C ABI.

    probs = [IbsProblem(cohort_a, layout="tri"), LdProblem(cohort_b, window=500, r2_min=0.2)]
    b = Batch(probs)          # plan, workspace, tile table upload; outputs allocated
    b.capture()               # one HIP graph: layouts, persistent kernels, LD finish
    b.replay()                # asynchronous on the current stream
    b.results()               # per problem: IBS tensors or LD records (synchronises)

Every problem's outputs equal a separate pg_ibs_matrix / pg_ld_window call
with the same path; the library runs all tiles of all problems in one
persistent kernel per kind of tile body (IBS, LD matrix-core, LD popcount).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _native as N
from .api import Cohort, _ptr, _require_cuda, _stream_handle, ibs_output_size, records_to_numpy


@dataclass
class IbsProblem:
    cohort: Cohort
    sample_idx: torch.Tensor | None = None
    v_range: tuple | None = None
    layout: str = "tri"
    path: int | str = "auto"
    out: tuple | None = None          # four int32 tensors (int16 with counts "u16"); allocated if None
    counts: str = "u32"               # "u16": 16-bit counts (fewer than 65,536 variants)


@dataclass
class LdProblem:
    cohort: Cohort
    window: int
    r2_min: float
    capacity: int = 0                 # 0 -> 4 * selected variants
    sample_idx: torch.Tensor | None = None
    v_range: tuple | None = None
    path: int | str = "auto"
    out: torch.Tensor | None = None   # capacity x 64 uint8
    n_out: torch.Tensor | None = None  # int64[1]


def _path_code(path) -> int:
    return N.PATHS[path] if isinstance(path, str) else int(path)


def _selection(c: Cohort, sample_idx, v_range):
    if sample_idx is not None:
        _require_cuda(sample_idx, "sample_idx", torch.int32)
        n_sel, m = sample_idx.numel(), sample_idx.numel()
    else:
        n_sel, m = 0, c.n_samples
    vb, ve = (0, 0) if v_range is None else (int(v_range[0]), int(v_range[1]))
    nv = (ve - vb) if (vb, ve) != (0, 0) else c.n_variants
    return n_sel, m, vb, ve, nv


class Batch:
    def __init__(self, problems: list, device=None):
        if not problems:
            raise ValueError("empty batch")
        self.lib = N.load()
        self.problems = problems
        self.device = device or problems[0].cohort.bed.device
        arr = (N.Problem * len(problems))()
        self._keep = []
        for k, p in enumerate(problems):
            q = arr[k]
            n_sel, m, vb, ve, nv = _selection(p.cohort, p.sample_idx, p.v_range)
            q.g = p.cohort.struct()
            q.path = _path_code(p.path)
            q.sample_idx = _ptr(p.sample_idx)
            q.n_sel, q.v_begin, q.v_end = n_sel, vb, ve
            if isinstance(p, IbsProblem):
                q.kind = N.PG_KIND_IBS
                size = ibs_output_size(m, p.layout)
                dtype = torch.int16 if p.counts == "u16" else torch.int32
                if p.out is None:
                    shape = (m, m) if p.layout == "full" else (size,)
                    p.out = tuple(torch.empty(shape, dtype=dtype, device=self.device)
                                  for _ in range(4))
                for k, t in enumerate(p.out):
                    _require_cuda(t, f"out[{k}]", dtype)
                    if t.numel() < size:
                        raise ValueError("output tensor too small")
                q.out_layout = N.LAYOUTS[p.layout] | (N.PG_COUNTS_U16 if p.counts == "u16" else 0)
                q.ibs0, q.ibs1, q.ibs2, q.nonmiss = [_ptr(t) for t in p.out]
            else:
                q.kind = N.PG_KIND_LD
                if not p.capacity:
                    p.capacity = max(1024, 4 * nv)
                if p.out is None:
                    p.out = torch.empty((p.capacity, 64), dtype=torch.uint8, device=self.device)
                if p.n_out is None:
                    p.n_out = torch.empty(1, dtype=torch.int64, device=self.device)
                q.window, q.r2_min = int(p.window), float(p.r2_min)
                q.out, q.capacity, q.n_out = _ptr(p.out), int(p.capacity), _ptr(p.n_out)
        self._arr = arr
        plan = ctypes.c_void_p()
        N.check(self.lib.pg_batch_plan(arr, len(problems), ctypes.byref(plan)), "pg_batch_plan")
        self.plan = plan
        nbytes = ctypes.c_size_t()
        N.check(self.lib.pg_batch_workspace_bytes(plan, ctypes.byref(nbytes)),
                "pg_batch_workspace_bytes")
        self.workspace = torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device=self.device)
        N.check(self.lib.pg_batch_upload(plan, _ptr(self.workspace), self.workspace.numel(),
                                         _stream_handle(None)), "pg_batch_upload")
        self.graph = None
        self._graph_stream = None

    @property
    def tiles(self) -> tuple[int, int]:
        t, g = ctypes.c_int64(), ctypes.c_int()
        N.check(self.lib.pg_batch_tiles(self.plan, ctypes.byref(t), ctypes.byref(g)),
                "pg_batch_tiles")
        return t.value, g.value

    def launch(self, stream=None) -> None:
        N.check(self.lib.pg_batch_launch(self.plan, _ptr(self.workspace), self.workspace.numel(),
                                         _stream_handle(stream)), "pg_batch_launch")

    def capture(self) -> None:
        """Captures the whole batch into a HIP graph on a private stream."""
        if self.graph is not None:
            return
        self._graph_stream = torch.cuda.Stream(device=self.device)
        torch.cuda.synchronize(self.device)
        exe = ctypes.c_void_p()
        N.check(self.lib.pg_batch_capture(self.plan, _ptr(self.workspace), self.workspace.numel(),
                                          _stream_handle(self._graph_stream), ctypes.byref(exe)),
                "pg_batch_capture")
        self.graph = exe

    def replay(self, stream=None) -> None:
        if self.graph is None:
            raise RuntimeError("capture() first")
        N.check(self.lib.pg_graph_launch(self.graph, _stream_handle(stream)), "pg_graph_launch")

    def results(self) -> list:
        torch.cuda.synchronize(self.device)
        res = []
        for p in self.problems:
            if isinstance(p, IbsProblem):
                res.append(p.out)
            else:
                total = int(p.n_out.item())
                res.append(records_to_numpy(p.out, min(total, p.capacity)))
        return res

    def close(self) -> None:
        if getattr(self, "graph", None) is not None:
            self.lib.pg_graph_destroy(self.graph)
            self.graph = None
        if getattr(self, "plan", None):
            self.lib.pg_plan_free(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
