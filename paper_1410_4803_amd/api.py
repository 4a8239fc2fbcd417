"""Python API over libpg.so: device buffers and streams come from PyTorch,
every computation runs in the library's HIP kernels.

    cohort = Cohort.from_numpy(bed, n_samples)          # resident in HBM
    ibs0, ibs1, ibs2, n = ibs_matrix(cohort, layout="full")
    recs = ld_records(cohort, window=1000, r2_min=0.2)  # numpy LD_PAIR array
    keep, n_kept = ld_prune(cohort, window=50, step=5, r2_threshold=0.5)
    A, N = grm_matrix(cohort, layout="full")            # relationship matrix
    merges = ibs_cluster(*ibs_matrix(cohort, layout="full"))   # complete linkage
"""
from __future__ import annotations

import contextlib
import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _native as N


def _require_cuda(t: torch.Tensor, name: str, dtype) -> None:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


def _on(stream):
    """Context in which buffers for a call on `stream` are allocated: the
    caching allocator then ties them to that stream, so a workspace freed
    when the call returns is not handed to other streams' work while the
    library's kernels may still use it."""
    return torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()


@dataclass
class Cohort:
    """A .bed genotype matrix resident in device memory.

    bed: CUDA uint8 tensor holding n_variants rows of bytes_per_variant bytes
    (variant-major PLINK 1 binary payload, no header).  missing_mask: optional
    CUDA int64/uint64 tensor of n_variants x ceil(n_samples/64) words, bit set =
    call missing."""
    bed: torch.Tensor
    n_samples: int
    n_variants: int
    bytes_per_variant: int = 0
    missing_mask: torch.Tensor | None = None

    def __post_init__(self):
        _require_cuda(self.bed, "bed", torch.uint8)
        bpv = self.bytes_per_variant or (self.n_samples + 3) // 4
        if self.bed.numel() < self.n_variants * bpv:
            raise ValueError("bed holds fewer than n_variants * bytes_per_variant bytes")
        if self.missing_mask is not None:
            if self.missing_mask.dtype not in (torch.int64, torch.uint64):
                raise TypeError("missing_mask must be a 64-bit integer tensor")
            if not self.missing_mask.is_cuda or not self.missing_mask.is_contiguous():
                raise ValueError("missing_mask must be a contiguous CUDA tensor")
            if self.missing_mask.numel() < self.n_variants * ((self.n_samples + 63) // 64):
                raise ValueError("missing_mask is too small")

    @classmethod
    def from_numpy(cls, bed: np.ndarray, n_samples: int, missing_mask: np.ndarray | None = None,
                   device="cuda") -> "Cohort":
        bed = np.ascontiguousarray(bed, dtype=np.uint8)
        t = torch.from_numpy(bed).to(device)
        m = None
        if missing_mask is not None:
            m = torch.from_numpy(np.ascontiguousarray(missing_mask).view(np.int64)).to(device)
        return cls(t, n_samples, bed.shape[0], bed.shape[1] if bed.ndim == 2 else 0, m)

    def struct(self) -> N.Genotypes:
        return N.Genotypes(self.bed.data_ptr(), self.n_samples, self.n_variants,
                           self.bytes_per_variant, _ptr(self.missing_mask))

    @property
    def nbytes(self) -> int:
        n = self.bed.numel()
        if self.missing_mask is not None:
            n += self.missing_mask.numel() * 8
        return n


def _sel(cohort: Cohort, sample_idx, v_range):
    if sample_idx is not None:
        _require_cuda(sample_idx, "sample_idx", torch.int32)
        n_sel = sample_idx.numel()
    else:
        n_sel = 0
    vb, ve = (0, 0) if v_range is None else (int(v_range[0]), int(v_range[1]))
    return n_sel, vb, ve


def _path(path) -> int:
    return N.PATHS[path] if isinstance(path, str) else int(path)


def ibs_workspace_bytes(cohort: Cohort, n_sel: int = 0, v_range=None, path="auto") -> int:
    vb, ve = (0, 0) if v_range is None else v_range
    out = ctypes.c_size_t(0)
    g = cohort.struct()
    N.check(N.load().pg_ibs_workspace_bytes(ctypes.byref(g), n_sel, vb, ve, _path(path),
                                            ctypes.byref(out)), "pg_ibs_workspace_bytes")
    return out.value


def ibs_output_size(m: int, layout: str) -> int:
    return m * m if layout == "full" else m * (m - 1) // 2


def ibs_matrix(cohort: Cohort, *, sample_idx: torch.Tensor | None = None, v_range=None,
               layout: str = "full", path="auto", out=None, workspace: torch.Tensor | None = None,
               stream=None, counts: str = "u32"):
    """IBS0, IBS1, IBS2, N as four CUDA tensors: (m, m) for layout "full",
    m(m-1)/2 packed upper triangle for "tri".  counts "u32": int32 tensors
    holding uint32 counts (all < 2^31); "u16": int16 tensors holding uint16
    counts (PG_COUNTS_U16; fewer than 65,536 selected variants), half the
    bytes.  Asynchronous on `stream` (default: the current stream)."""
    lib = N.load()
    if counts not in ("u32", "u16"):
        raise ValueError("counts must be 'u32' or 'u16'")
    dtype = torch.int16 if counts == "u16" else torch.int32
    n_sel, vb, ve = _sel(cohort, sample_idx, v_range)
    m = n_sel or cohort.n_samples
    size = ibs_output_size(m, layout)
    with _on(stream):
        if out is None:
            shape = (m, m) if layout == "full" else (size,)
            out = tuple(torch.empty(shape, dtype=dtype, device=cohort.bed.device)
                        for _ in range(4))
        else:
            for k, t in enumerate(out):
                _require_cuda(t, f"out[{k}]", dtype)
                if t.numel() < size:
                    raise ValueError("output tensor too small")
        need = ibs_workspace_bytes(cohort, n_sel, (vb, ve), path)
        if workspace is None:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=cohort.bed.device)
    g = cohort.struct()
    lay = N.LAYOUTS[layout] | (N.PG_COUNTS_U16 if counts == "u16" else 0)
    st = lib.pg_ibs_matrix(ctypes.byref(g), _ptr(sample_idx), n_sel, vb, ve, lay,
                           _path(path), *[_ptr(t) for t in out], _ptr(workspace),
                           workspace.numel(), _stream_handle(stream))
    N.check(st, "pg_ibs_matrix")
    return out


def resolve_path(kind: str, m: int, nv: int, window: int = 0, path="auto") -> int:
    """The path | variant << 8 code a call of `kind` ("ibs" or "ld") runs for
    m samples, nv variants and window (pg_resolve_path)."""
    out = ctypes.c_int(0)
    N.check(N.load().pg_resolve_path(N.PG_KIND_IBS if kind == "ibs" else N.PG_KIND_LD, int(m),
                                     int(nv), int(window), _path(path), ctypes.byref(out)),
            "pg_resolve_path")
    return out.value


def noalloc_scratch_bytes() -> int:
    """Size of the static scratch array pg_ibs_matrix_noalloc works in."""
    out = ctypes.c_size_t(0)
    N.check(N.load().pg_noalloc_scratch_bytes(ctypes.byref(out)), "pg_noalloc_scratch_bytes")
    return out.value


def ibs_matrix_noalloc(cohort: Cohort, out, *, sample_idx: torch.Tensor | None = None,
                       v_range=None, layout: str = "full", path="auto", stream=None,
                       counts: str = "u32"):
    """pg_ibs_matrix_noalloc: the IBS matrix into the caller's four tensors
    `out` (int32, or int16 with counts "u16"), with the library's static
    scratch array as workspace (no allocation anywhere in the call).  Calls
    that overlap on one GPU race."""
    lib = N.load()
    if counts not in ("u32", "u16"):
        raise ValueError("counts must be 'u32' or 'u16'")
    n_sel, vb, ve = _sel(cohort, sample_idx, v_range)
    m = n_sel or cohort.n_samples
    size = ibs_output_size(m, layout)
    for k, t in enumerate(out):
        _require_cuda(t, f"out[{k}]", torch.int16 if counts == "u16" else torch.int32)
        if t.numel() < size:
            raise ValueError("output tensor too small")
    g = cohort.struct()
    lay = N.LAYOUTS[layout] | (N.PG_COUNTS_U16 if counts == "u16" else 0)
    st = lib.pg_ibs_matrix_noalloc(ctypes.byref(g), _ptr(sample_idx), n_sel, vb, ve, lay,
                                   _path(path), *[_ptr(t) for t in out],
                                   _stream_handle(stream))
    N.check(st, "pg_ibs_matrix_noalloc")
    return out


def ld_workspace_bytes(cohort: Cohort, window: int, n_sel: int = 0, v_range=None,
                       path="auto") -> int:
    vb, ve = (0, 0) if v_range is None else v_range
    out = ctypes.c_size_t(0)
    g = cohort.struct()
    N.check(N.load().pg_ld_workspace_bytes(ctypes.byref(g), n_sel, vb, ve, window, _path(path),
                                           ctypes.byref(out)), "pg_ld_workspace_bytes")
    return out.value


def ld_window(cohort: Cohort, window: int, r2_min: float, *, capacity: int,
              sample_idx: torch.Tensor | None = None, v_range=None, path="auto", out=None,
              n_out=None, workspace: torch.Tensor | None = None, stream=None):
    """Asynchronous LD window call.  Returns (out, n_out): out is a CUDA
    uint8 tensor of capacity x 64 bytes (pg_ld_pair records in (a, b) order),
    n_out a CUDA int64 tensor holding the total number of emitted pairs."""
    lib = N.load()
    n_sel, vb, ve = _sel(cohort, sample_idx, v_range)
    dev = cohort.bed.device
    with _on(stream):
        if out is None:
            out = torch.empty((max(capacity, 1), 64), dtype=torch.uint8, device=dev)
        if n_out is None:
            n_out = torch.empty(1, dtype=torch.int64, device=dev)
        need = ld_workspace_bytes(cohort, window, n_sel, (vb, ve), path)
        if workspace is None:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    g = cohort.struct()
    st = lib.pg_ld_window(ctypes.byref(g), _ptr(sample_idx), n_sel, vb, ve, int(window),
                          float(r2_min), _ptr(out), int(capacity), _ptr(n_out), _path(path),
                          _ptr(workspace), workspace.numel(), _stream_handle(stream))
    N.check(st, "pg_ld_window")
    return out, n_out


def records_to_numpy(out: torch.Tensor, count: int) -> np.ndarray:
    """First `count` records of an LD output buffer as a numpy LD_PAIR array."""
    raw = out[:count].contiguous().cpu().numpy()
    return raw.reshape(-1).view(N.LD_PAIR)[:count].copy()


def ld_records(cohort: Cohort, window: int, r2_min: float, *, capacity: int | None = None,
               **kw) -> np.ndarray:
    """Synchronous LD window: all emitted pairs as a numpy LD_PAIR array.
    Re-issues the call once with a larger buffer if the first one overflows."""
    if capacity is None:
        capacity = max(1024, 4 * cohort.n_variants)
    out, n_out = ld_window(cohort, window, r2_min, capacity=capacity, **kw)
    total = int(n_out.item())
    if total > capacity:
        out, n_out = ld_window(cohort, window, r2_min, capacity=total, **kw)
        total = int(n_out.item())
    return records_to_numpy(out, total)


def prune_workspace_bytes(cohort: Cohort, window: int, n_sel: int = 0, v_range=None,
                          path="auto") -> int:
    vb, ve = (0, 0) if v_range is None else v_range
    out = ctypes.c_size_t(0)
    g = cohort.struct()
    N.check(N.load().pg_prune_workspace_bytes(ctypes.byref(g), n_sel, vb, ve, int(window),
                                              _path(path), ctypes.byref(out)),
            "pg_prune_workspace_bytes")
    return out.value


def ld_prune(cohort: Cohort, window: int, step: int, r2_threshold: float, *,
             sample_idx: torch.Tensor | None = None, v_range=None, path="auto", keep=None,
             n_kept=None, workspace: torch.Tensor | None = None, stream=None):
    """Asynchronous greedy LD pruning (--indep-pairwise window step threshold).
    Returns (keep, n_kept): keep is a CUDA uint8 tensor with one flag per
    selected variant (1 = kept), n_kept a CUDA int64 tensor."""
    lib = N.load()
    n_sel, vb, ve = _sel(cohort, sample_idx, v_range)
    dev = cohort.bed.device
    nv = (ve - vb) if (vb, ve) != (0, 0) else cohort.n_variants
    with _on(stream):
        if keep is None:
            keep = torch.empty(nv, dtype=torch.uint8, device=dev)
        if n_kept is None:
            n_kept = torch.empty(1, dtype=torch.int64, device=dev)
        need = prune_workspace_bytes(cohort, window, n_sel, (vb, ve), path)
        if workspace is None:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    g = cohort.struct()
    st = lib.pg_ld_prune(ctypes.byref(g), _ptr(sample_idx), n_sel, vb, ve, int(window), int(step),
                         float(r2_threshold), _ptr(keep), _ptr(n_kept), _path(path),
                         _ptr(workspace), workspace.numel(), _stream_handle(stream))
    N.check(st, "pg_ld_prune")
    return keep, n_kept


def grm_workspace_bytes(cohort: Cohort, n_sel: int = 0, v_range=None) -> int:
    vb, ve = (0, 0) if v_range is None else v_range
    out = ctypes.c_size_t(0)
    g = cohort.struct()
    N.check(N.load().pg_grm_workspace_bytes(ctypes.byref(g), n_sel, vb, ve, ctypes.byref(out)),
            "pg_grm_workspace_bytes")
    return out.value


def grm_matrix(cohort: Cohort, *, sample_idx: torch.Tensor | None = None, v_range=None,
               layout: str = "full", path="auto", out=None,
               workspace: torch.Tensor | None = None, stream=None):
    """Asynchronous relationship matrix.  Returns (A, N): A float64 and N
    int32 (holding uint32 counts) CUDA tensors, (m, m) for the full layout or
    the packed strict upper triangle."""
    lib = N.load()
    n_sel, vb, ve = _sel(cohort, sample_idx, v_range)
    m = n_sel if sample_idx is not None else cohort.n_samples
    dev = cohort.bed.device
    if out is None:
        shape = (m, m) if layout == "full" else (ibs_output_size(m, layout),)
        with _on(stream):
            out = (torch.empty(shape, dtype=torch.float64, device=dev),
                   torch.empty(shape, dtype=torch.int32, device=dev))
    A, Nn = out
    size = ibs_output_size(m, layout)
    _require_cuda(A, "A", torch.float64)
    _require_cuda(Nn, "N", torch.int32)
    if A.numel() < size or Nn.numel() < size:
        raise ValueError(f"outputs need {size} entries")
    need = grm_workspace_bytes(cohort, n_sel, (vb, ve))
    if workspace is None:
        with _on(stream):
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    g = cohort.struct()
    st = lib.pg_grm_matrix(ctypes.byref(g), _ptr(sample_idx), n_sel, vb, ve, N.LAYOUTS[layout],
                           _path(path), _ptr(A), _ptr(Nn), _ptr(workspace), workspace.numel(),
                           _stream_handle(stream))
    N.check(st, "pg_grm_matrix")
    return A, Nn


def ibs_distance(ibs0: torch.Tensor, ibs1: torch.Tensor, nonmiss: torch.Tensor, *, out=None,
                 stream=None) -> torch.Tensor:
    """(2*IBS0 + IBS1) / (2*N) elementwise (+inf where N = 0), float64, the
    shape of the inputs (any pg_ibs_matrix layout)."""
    for t, name in ((ibs0, "ibs0"), (ibs1, "ibs1"), (nonmiss, "nonmiss")):
        _require_cuda(t, name, torch.int32)
    if out is None:
        with _on(stream):
            out = torch.empty(ibs0.shape, dtype=torch.float64, device=ibs0.device)
    _require_cuda(out, "out", torch.float64)
    if not (ibs0.numel() == ibs1.numel() == nonmiss.numel() == out.numel()):
        raise ValueError("inputs and output must have the same number of entries")
    N.check(N.load().pg_ibs_distance(_ptr(ibs0), _ptr(ibs1), _ptr(nonmiss), ibs0.numel(),
                                     _ptr(out), _stream_handle(stream)), "pg_ibs_distance")
    return out


def ibs_similarity(ibs1: torch.Tensor, ibs2: torch.Tensor, nonmiss: torch.Tensor, *,
                   out=None, stream=None) -> torch.Tensor:
    """(2*IBS2 + IBS1) / (2*N) elementwise (NaN where N = 0), float64, the
    shape of the inputs (any pg_ibs_matrix layout)."""
    for t, name in ((ibs1, "ibs1"), (ibs2, "ibs2"), (nonmiss, "nonmiss")):
        _require_cuda(t, name, torch.int32)
    if out is None:
        with _on(stream):
            out = torch.empty(ibs1.shape, dtype=torch.float64, device=ibs1.device)
    _require_cuda(out, "out", torch.float64)
    if not (ibs1.numel() == ibs2.numel() == nonmiss.numel() == out.numel()):
        raise ValueError("inputs and output must have the same number of entries")
    N.check(N.load().pg_ibs_similarity(_ptr(ibs1), _ptr(ibs2), _ptr(nonmiss), ibs1.numel(),
                                       _ptr(out), _stream_handle(stream)), "pg_ibs_similarity")
    return out


def genome_workspace_bytes(cohort: Cohort, n_sel: int = 0, v_range=None) -> int:
    vb, ve = (0, 0) if v_range is None else v_range
    out = ctypes.c_size_t(0)
    g = cohort.struct()
    N.check(N.load().pg_genome_workspace_bytes(ctypes.byref(g), n_sel, vb, ve,
                                               ctypes.byref(out)), "pg_genome_workspace_bytes")
    return out.value


def ibs_genome(cohort: Cohort, ibs0: torch.Tensor, ibs1: torch.Tensor, nonmiss: torch.Tensor,
               *, sample_idx: torch.Tensor | None = None, v_range=None, out=None,
               workspace: torch.Tensor | None = None, stream=None):
    """IBD report (Z0, Z1, Z2, PI_HAT) by the method of moments from the IBS
    counts of the same selection (pass the sample_idx and v_range the counts
    were computed with).  Returns four float64 CUDA tensors shaped like ibs0
    (any pg_ibs_matrix layout)."""
    lib = N.load()
    for t, name in ((ibs0, "ibs0"), (ibs1, "ibs1"), (nonmiss, "nonmiss")):
        _require_cuda(t, name, torch.int32)
    if not (ibs0.numel() == ibs1.numel() == nonmiss.numel()):
        raise ValueError("inputs must have the same number of entries")
    n_sel, vb, ve = _sel(cohort, sample_idx, v_range)
    dev = cohort.bed.device
    with _on(stream):
        if out is None:
            out = tuple(torch.empty(ibs0.shape, dtype=torch.float64, device=dev)
                        for _ in range(4))
        if workspace is None:
            workspace = torch.empty(max(genome_workspace_bytes(cohort, n_sel, (vb, ve)), 1),
                                    dtype=torch.uint8, device=dev)
    for t in out:
        _require_cuda(t, "out", torch.float64)
        if t.numel() != ibs0.numel():
            raise ValueError("outputs must have as many entries as the inputs")
    g = cohort.struct()
    N.check(lib.pg_ibs_genome(ctypes.byref(g), _ptr(sample_idx), n_sel, vb, ve, _ptr(ibs0),
                              _ptr(ibs1), _ptr(nonmiss), ibs0.numel(), *(_ptr(t) for t in out),
                              _ptr(workspace), workspace.numel(), _stream_handle(stream)),
            "pg_ibs_genome")
    return out


def cluster_workspace_bytes(m: int) -> int:
    out = ctypes.c_size_t(0)
    N.check(N.load().pg_cluster_workspace_bytes(int(m), ctypes.byref(out)),
            "pg_cluster_workspace_bytes")
    return out.value


def ibs_cluster(ibs0: torch.Tensor, ibs1: torch.Tensor, ibs2: torch.Tensor | None = None,
                nonmiss: torch.Tensor | None = None, *, out=None,
                workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Complete-linkage clustering on the IBS distance of a full (m, m)
    pg_ibs_matrix result (pass its four tensors as returned; ibs2 is not
    needed).  Returns a CUDA uint8 tensor of (m - 1) x 16 bytes: pg_merge
    records in merge order (see merges_to_numpy)."""
    if nonmiss is None:
        raise TypeError("pass the four pg_ibs_matrix outputs (ibs0, ibs1, ibs2, nonmiss)")
    m = ibs0.shape[0]
    if ibs0.dim() != 2 or ibs0.shape != (m, m):
        raise ValueError("clustering needs the full (m, m) layout")
    for t, name in ((ibs0, "ibs0"), (ibs1, "ibs1"), (nonmiss, "nonmiss")):
        _require_cuda(t, name, torch.int32)
    dev = ibs0.device
    with _on(stream):
        if out is None:
            out = torch.empty((max(m - 1, 1), 16), dtype=torch.uint8, device=dev)
        if workspace is None:
            workspace = torch.empty(cluster_workspace_bytes(m), dtype=torch.uint8, device=dev)
    N.check(N.load().pg_ibs_cluster(_ptr(ibs0), _ptr(ibs1), _ptr(nonmiss), m, _ptr(out),
                                    _ptr(workspace), workspace.numel(), _stream_handle(stream)),
            "pg_ibs_cluster")
    return out


def merges_to_numpy(out: torch.Tensor, m: int) -> np.ndarray:
    """The m - 1 merge records of an ibs_cluster output as a numpy MERGE array."""
    raw = out[:max(m - 1, 0)].contiguous().cpu().numpy()
    return raw.reshape(-1).view(N.MERGE)[:max(m - 1, 0)].copy()


def peak_rates(workspace_bytes: int = 2 << 30) -> dict:
    """Measured int8 / fp64 matrix-core, popcount and HBM-copy throughput of
    the current device (pg_peak_rates)."""
    ws = torch.empty(workspace_bytes, dtype=torch.uint8, device="cuda")
    out = (ctypes.c_double * 4)()
    N.check(N.load().pg_peak_rates(_ptr(ws), ws.numel(), out), "pg_peak_rates")
    del ws
    return {"int8_mfma_tops": out[0], "fp64_mfma_tflops": out[1], "valu_bcnt_tops": out[2],
            "hbm_copy_gbs": out[3]}
