"""Serving: IBS-matrix and LD-window queries over cohorts resident in HBM.

Continuous batching over stream slots: each admitted request runs on its own
slot (a HIP stream with its own pinned result buffers), so requests that
arrive while others are on the GPU start as soon as a slot and enough device
memory are free, and their kernels overlap on the device.  Admission is by
memory footprint (outputs + workspace + sample list) against a budget, in
arrival order; a request larger than the whole budget is rejected.  Latency
is arrival -> result in host memory; device time is measured with events on
the slot's stream.

The arithmetic is the library's (pg_ibs_matrix / pg_ld_window); the server
only schedules.  A request's result does not depend on what else runs.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import _native as N
from .api import Cohort, ibs_matrix, ibs_output_size, ibs_workspace_bytes, ld_window, \
    ld_workspace_bytes


@dataclass
class Request:
    rid: int
    kind: str                       # "ibs" or "ld"
    cohort: int
    sample_idx: np.ndarray          # int32 sample indices into the cohort
    v_range: tuple                  # [begin, end) variants
    window: int = 500
    r2_min: float = 0.2
    layout: str = "tri"
    arrival: float = 0.0            # seconds after the run starts
    # set by the server
    admitted: float | None = None
    done: float | None = None
    device_ms: float | None = None
    footprint: int = 0
    result: object = None
    error: str | None = None
    ld_capacity: int = 0            # 0: default; set to the needed size after an overflow


class GpuBackend:
    """Runs requests through the library on per-slot streams."""

    def __init__(self, cohorts: list[Cohort], n_slots: int, device=None, tuner=None,
                 keep_results: bool | str = True, ld_capacity: int = 1 << 18,
                 ibs_counts: str = "auto"):
        """keep_results: True keeps each result (numpy arrays) on its
        request, False keeps nothing, "digest" keeps a 128-bit hash of the
        result's bytes (for comparing many large results).  ibs_counts:
        "auto" returns IBS counts as uint16 when the request's variant range
        is shorter than 65,536 (half the device memory and the copy to the
        host), else uint32; "u32" always uint32."""
        if ibs_counts not in ("auto", "u32"):
            raise ValueError("ibs_counts must be 'auto' or 'u32'")
        self.ibs_counts = ibs_counts
        self.cohorts = cohorts
        self.device = device or cohorts[0].bed.device
        self.tuner = tuner
        self.keep = keep_results
        self.ld_capacity = ld_capacity
        self.slots = []
        for _ in range(n_slots):
            self.slots.append({
                "stream": torch.cuda.Stream(device=self.device),
                "host": None,               # pinned result buffer, grown on demand
                "idx": torch.empty(1 << 18, dtype=torch.int32, pin_memory=True),
            })

    # -- sizing ---------------------------------------------------------------
    def _path(self, req: Request) -> int:
        m = len(req.sample_idx)
        nv = req.v_range[1] - req.v_range[0]
        if self.tuner is None:
            return N.PG_PATH_AUTO
        return self.tuner.choose(req.kind, m, nv, req.window if req.kind == "ld" else None)

    def _counts(self, req: Request) -> str:
        """Width of an IBS request's counts: "u16" or "u32"."""
        short = req.v_range[1] - req.v_range[0] < 65536
        return "u16" if self.ibs_counts == "auto" and short else "u32"

    def footprint(self, req: Request) -> int:
        c = self.cohorts[req.cohort]
        m = len(req.sample_idx)
        path = self._path(req)
        if req.kind == "ibs":
            ws = ibs_workspace_bytes(c, m, req.v_range, path)
            width = 2 if self._counts(req) == "u16" else 4
            return ws + 4 * width * ibs_output_size(m, req.layout) + 4 * m
        ws = ld_workspace_bytes(c, req.window, m, req.v_range, path)
        return ws + 64 * self._ld_cap(req) + 8 + 4 * m

    def _ld_cap(self, req: Request) -> int:
        if req.ld_capacity:
            return req.ld_capacity
        return max(1024, min(self.ld_capacity, 4 * (req.v_range[1] - req.v_range[0])))

    def _host_buf(self, slot, nbytes: int) -> torch.Tensor:
        h = slot["host"]
        if h is None or h.numel() < nbytes:
            slot["host"] = torch.empty(max(nbytes, 1 << 20), dtype=torch.uint8, pin_memory=True)
        return slot["host"]

    # -- execution ------------------------------------------------------------
    def start(self, req: Request, slot_id: int):
        slot = self.slots[slot_id]
        st = slot["stream"]
        c = self.cohorts[req.cohort]
        m = len(req.sample_idx)
        path = self._path(req)
        with torch.cuda.stream(st):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            if m > slot["idx"].numel():
                slot["idx"] = torch.empty(m, dtype=torch.int32, pin_memory=True)
            hidx = slot["idx"][:m]
            hidx.numpy()[:] = req.sample_idx
            idx = hidx.to(self.device, non_blocking=True)
            e0.record(st)
            if req.kind == "ibs":
                size = ibs_output_size(m, req.layout)
                counts = self._counts(req)
                dtype, width = (torch.int16, 2) if counts == "u16" else (torch.int32, 4)
                out = tuple(torch.empty(size, dtype=dtype, device=self.device)
                            for _ in range(4))
                ibs_matrix(c, sample_idx=idx, v_range=req.v_range, layout=req.layout, path=path,
                           out=out, stream=st, counts=counts)
                e1.record(st)
                host = self._host_buf(slot, 4 * width * size)
                views = [host[k * width * size:(k + 1) * width * size].view(dtype)
                         for k in range(4)]
                for v, o in zip(views, out):
                    v.copy_(o, non_blocking=True)
                keep = (out, idx)
                h = {"kind": "ibs", "views": views, "keep": keep,
                     "np": np.uint16 if counts == "u16" else np.uint32}
            else:
                cap = self._ld_cap(req)
                out, n_out = ld_window(c, req.window, req.r2_min, capacity=cap, sample_idx=idx,
                                       v_range=req.v_range, path=path, stream=st)
                e1.record(st)
                host = self._host_buf(slot, 64 * cap + 64)
                hv_n = host[:8].view(torch.int64)
                hv_out = host[64:64 + 64 * cap]
                hv_n.copy_(n_out, non_blocking=True)
                hv_out.copy_(out.view(-1)[:64 * cap], non_blocking=True)
                h = {"kind": "ld", "n": hv_n, "out": hv_out, "cap": cap, "keep": (out, n_out, idx)}
            done = torch.cuda.Event()
            done.record(st)
        h.update(event=done, e0=e0, e1=e1)
        return h

    def poll(self, h) -> bool:
        return h["event"].query()

    def finish(self, req: Request, h):
        """Moves the result into host memory (numpy).  Returns False when an
        LD query overflowed its buffer: req.ld_capacity is then set to the
        needed size and the server re-issues the request."""
        req.device_ms = h["e0"].elapsed_time(h["e1"])
        res = None
        if h["kind"] == "ibs":
            if self.keep == "digest":
                res = _digest(v.numpy() for v in h["views"])
            elif self.keep:
                res = tuple(v.numpy().view(h["np"]).copy() for v in h["views"])
        else:
            total = int(h["n"].item())
            if total > h["cap"]:
                req.ld_capacity = total
                return False
            if self.keep == "digest":
                res = _digest([h["out"][:64 * total].numpy()])
            elif self.keep:
                raw = h["out"][:64 * total].numpy().copy()
                res = raw.view(N.LD_PAIR)
        req.result = res
        return True


def _digest(arrays) -> str:
    """128-bit hash of the concatenated bytes of numpy arrays."""
    try:
        import xxhash
        h = xxhash.xxh3_128()
    except ImportError:                       # pragma: no cover
        import hashlib
        h = hashlib.blake2b(digest_size=16)
    for a in arrays:
        h.update(np.ascontiguousarray(a).reshape(-1).view(np.uint8))
    return h.hexdigest()


class Server:
    def __init__(self, backend, n_slots: int, memory_budget: int):
        self.backend = backend
        self.n_slots = n_slots
        self.budget = memory_budget
        self.used = 0
        self.queue: collections.deque[Request] = collections.deque()
        self.running: dict[int, tuple] = {}    # slot -> (req, handle)
        self.finished: list[Request] = []
        self.rejected: list[Request] = []
        self.t0 = time.perf_counter()
        self.peak_used = 0
        self.max_running = 0
        self.memory_holds = 0               # admissions deferred for memory
        self._held: Request | None = None

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request) -> None:
        req.footprint = self.backend.footprint(req)
        if req.footprint > self.budget:
            req.error = "footprint exceeds the memory budget"
            req.done = self.now()
            self.rejected.append(req)
            return
        self.queue.append(req)

    def _admit(self) -> None:
        free = [s for s in range(self.n_slots) if s not in self.running]
        while self.queue and free:
            req = self.queue[0]
            if self.used + req.footprint > self.budget:
                if self._held is not req:            # count each deferred request once
                    self.memory_holds += 1
                    self._held = req
                break                                # wait for memory (arrival order)
            self.queue.popleft()
            slot = free.pop(0)
            req.admitted = self.now()
            try:
                h = self.backend.start(req, slot)
            except Exception as e:                   # a failed request does not stop the server
                req.error = f"{type(e).__name__}: {e}"
                req.done = self.now()
                self.rejected.append(req)
                free.insert(0, slot)
                continue
            self.used += req.footprint
            self.peak_used = max(self.peak_used, self.used)
            self.running[slot] = (req, h)
        self.max_running = max(self.max_running, len(self.running))

    def step(self) -> None:
        for slot in list(self.running):
            req, h = self.running[slot]
            if not self.backend.poll(h):
                continue
            del self.running[slot]
            self.used -= req.footprint
            try:
                ok = self.backend.finish(req, h)
            except Exception as e:
                req.error = f"{type(e).__name__}: {e}"
                req.done = self.now()
                self.rejected.append(req)
                continue
            if not ok:                                # re-issue with a larger buffer, at the front
                req.footprint = self.backend.footprint(req)
                if req.footprint > self.budget:       # the larger buffer can never fit
                    req.error = "footprint after LD overflow exceeds the memory budget"
                    req.done = self.now()
                    self.rejected.append(req)
                    continue
                self.queue.appendleft(req)
                continue
            req.done = self.now()
            self.finished.append(req)
        self._admit()

    def idle(self) -> bool:
        return not self.queue and not self.running

    def run(self, requests: list[Request], poll_s: float = 0.0002) -> dict:
        """Replays the arrival schedule in real time until every request is
        done; returns latency and throughput statistics."""
        pending = sorted(requests, key=lambda r: r.arrival)
        self.t0 = time.perf_counter()
        k = 0
        while k < len(pending) or not self.idle():
            now = self.now()
            while k < len(pending) and pending[k].arrival <= now:
                self.submit(pending[k])
                k += 1
            self.step()
            if k < len(pending) and self.idle():
                time.sleep(max(0.0, min(pending[k].arrival - self.now(), 0.01)))
            elif poll_s:
                time.sleep(poll_s)
        return self.stats()

    def stats(self) -> dict:
        lat = np.array([r.done - r.arrival for r in self.finished])
        dev = np.array([r.device_ms for r in self.finished if r.device_ms is not None])
        wait = np.array([r.admitted - r.arrival for r in self.finished])
        span = max((r.done for r in self.finished), default=0.0) - \
            min((r.arrival for r in self.finished), default=0.0)
        out = {"completed": len(self.finished), "rejected": len(self.rejected),
               "throughput_rps": round(len(self.finished) / span, 2) if span > 0 else 0.0,
               "max_concurrent": self.max_running, "peak_device_bytes": self.peak_used,
               "memory_holds": self.memory_holds}
        if len(lat):
            out.update(p50_ms=round(float(np.percentile(lat, 50)) * 1e3, 3),
                       p99_ms=round(float(np.percentile(lat, 99)) * 1e3, 3),
                       mean_ms=round(float(lat.mean()) * 1e3, 3),
                       queue_wait_p99_ms=round(float(np.percentile(wait, 99)) * 1e3, 3))
        if len(dev):
            out.update(device_p50_ms=round(float(np.percentile(dev, 50)), 3),
                       device_p99_ms=round(float(np.percentile(dev, 99)), 3))
        return out


def poisson_requests(cohort_shapes: list[tuple[int, int]], rate: float, seconds: float,
                     seed: int, p_ibs: float = 0.7, window: int = 500, r2_min: float = 0.2,
                     max_samples: int = 5000, range_len=(1000, 20000)) -> list[Request]:
    """The serving workload: Poisson arrivals; each request picks a cohort
    uniformly, IBS with probability p_ibs else LD; a sample subset of size
    U{100..min(max_samples, n)} without replacement; a variant range of length
    U{range_len} (capped at V) at a uniform start."""
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs, t, rid = [], 0.0, 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > seconds:
            break
        ci = int(rng.integers(0, len(cohort_shapes)))
        n, V = cohort_shapes[ci]
        s = int(rng.integers(100, min(max_samples, n) + 1))
        idx = np.sort(rng.choice(n, size=s, replace=False)).astype(np.int32)
        L = int(rng.integers(range_len[0], min(range_len[1], V) + 1))
        b = int(rng.integers(0, V - L + 1))
        kind = "ibs" if rng.random() < p_ibs else "ld"
        reqs.append(Request(rid, kind, ci, idx, (b, b + L), window, r2_min, "tri", t))
        rid += 1
    return reqs
