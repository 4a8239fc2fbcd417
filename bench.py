"""Benchmark: genotype-pair comparisons per second on one MI355X.

Default workload: the 10,000-sample x 100,000-variant identity-by-state
matrix (founder-mosaic genotypes, 2% missing, full 10k x 10k output), one
pg_ibs_matrix call per step (operand layout + pair kernel), inputs resident in
HBM.  Prints ONE JSON line.

    python bench.py [--steps K] [--warmup W] [--path auto|mfma|popc]
                    [--no-cpu] [--quick] [--copy-calibration]

Extras in the same line: the LD window workload (5,000 x 500,000, window
1,000, r^2 >= 0.2), the 500 x 5,000 matrix latency, and the other IBS path at
the default workload.  `roofline` comes from per-launch HIP-event timings of
the pair kernel recorded by the library on the launch stream
(pg_profile_events); `cpu_baseline` times the CPU oracle on a bounded sample
of the same workload on this host's cores.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_INT8_TOPS = 5000.0        # MI355X dense int8 MFMA, 5.0 POP/s
PEAK_FP4_TFLOPS = 10100.0      # MI355X dense fp4 MFMA, 10.1 PFLOP/s
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12   # 32-bit integer VALU lane-ops/s, 39.3 T
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6         # MI355X dense fp64 MFMA
# algorithmic work per unique genotype-pair comparison (one pair, one variant)
IBS_MFMA_OPS = 4 * 2          # four contractions: 4 multiply-adds = 8 ops (int8 or fp4)
IBS_FP4_VARIANTS = (0, 8)      # the default kernel: pipelined, fp4 operands
IBS_POPC_OPS = 8 / 32         # per 32-variant word: AND, 2 XOR, 2 bitop3, 3 popcount-adds
LD_MFMA_OPS = 6 * 2           # six int8 contractions
LD_POPC_OPS = 16 / 32         # 16 VALU ops per 32-sample word
LD_INT8 = 2 | (1 << 8)         # the LD matrix-core path's int8 tile (variant 1)
LD_SPARSE_ALL = 3 | (1 << 8)   # the correction path on every tile (variant 1)
LD_PATH_NAMES = {LD_INT8: "mfma_int8", LD_SPARSE_ALL: "sparse_all_tiles"}
IBS_FP4_KERNELS = "k_ibs_head<true>+k_ibs_tail<true>+k_ibs_tail_reduce"
IBS_INT8_KERNELS = "k_ibs_head<false>+k_ibs_tail<false>+k_ibs_tail_reduce"


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class HipEvents:
    """hipEvent_t handles through the HIP runtime (libpg links it)."""

    def __init__(self):
        self.rt = ctypes.CDLL("libamdhip64.so")
        self.rt.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.rt.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                                ctypes.c_void_p]
        self.rt.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def create(self, n: int):
        evs = []
        for _ in range(n):
            e = ctypes.c_void_p()
            if self.rt.hipEventCreate(ctypes.byref(e)) != 0:
                raise RuntimeError("hipEventCreate failed")
            evs.append(e.value)
        return evs

    def ms(self, a, b) -> float:
        out = ctypes.c_float()
        if self.rt.hipEventElapsedTime(ctypes.byref(out), ctypes.c_void_p(a), ctypes.c_void_p(b)) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(out.value)

    def destroy(self, evs):
        for e in evs:
            self.rt.hipEventDestroy(ctypes.c_void_p(e))


def set_stage_events(lib, evs):
    if evs is None:
        lib.pg_profile_events(None, 0)
    else:
        arr = (ctypes.c_void_p * len(evs))(*evs)
        if lib.pg_profile_events(arr, len(evs)) != 0:
            raise RuntimeError("pg_profile_events failed")


def timed_steps(torch, lib, hip, call, steps, warmup, n_events):
    """Runs warmup + timed steps of `call`; returns (ms_per_step, per-stage
    per-launch durations in ms)."""
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    evs = [hip.create(n_events) for _ in range(steps)] if n_events else []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        if n_events:
            set_stage_events(lib, evs[k])
        call()
    set_stage_events(lib, None)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = [[hip.ms(e[s], e[s + 1]) for e in evs] for s in range(max(n_events - 1, 0))]
    for e in evs:
        hip.destroy(e)
    return (t1 - t0) * 1e3 / steps, stages


def mean(xs):
    return sum(xs) / len(xs)


def traffic_from_profile(kernel: str):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(kernel)
    if not rec:
        return None
    h = hashlib.sha256()
    for src in rec.get("sources", []):
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if rec.get("source_sha256") != h.hexdigest():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_ibs(bed, n, V, budget_s: float):
    """Times the CPU oracle on the first s samples (all variants, strict upper
    triangle), s chosen for about `budget_s` seconds of host work."""
    import numpy as np
    import oracle
    codes = oracle.unpack(bed, n, V)          # variant-major int8 (V, n)

    def run(s):
        sub = np.ascontiguousarray(codes[:, :s])
        t = time.perf_counter()
        oracle.ibs_matrix(sub, full=False)
        return time.perf_counter() - t

    s0 = 160
    t0 = run(s0)
    rate = s0 * (s0 - 1) / 2 * V / max(t0, 1e-6)
    s = int(math.sqrt(2 * budget_s * rate / V))
    s = max(s0, min(s, n))
    t = run(s)
    comps = s * (s - 1) / 2 * V
    return {"value": round(comps / t / 1e9, 3), "unit": "G/s", "cores": oracle.threads(),
            "kind": "oracle", "cpu": cpu_model(),
            "sample": f"first {s} samples x all {V} variants of the workload, strict upper "
                      f"triangle ({comps:.3e} comparisons, {t:.1f} s)"}


def bench_prune(torch, lib, hip, pg, wp, dev, steps):
    """Greedy LD pruning (--indep-pairwise window step r2): whole-call time
    and its stages; comparisons = in-window variant pairs x samples of the
    pair kernel (largest distance window - 1)."""
    n, V, W, S, t = wp["n"], wp["V"], wp["window"], wp["step"], wp["r2_max"]
    c = pg.Cohort.from_numpy(wp["bed"], n, device=dev)
    keep = torch.empty(V, dtype=torch.uint8, device=dev)
    n_kept = torch.empty(1, dtype=torch.int64, device=dev)
    ws = torch.empty(pg.prune_workspace_bytes(c, W, path="mfma"), dtype=torch.uint8, device=dev)
    ms, st = timed_steps(torch, lib, hip, lambda: pg.ld_prune(
        c, W, S, t, path="mfma", keep=keep, n_kept=n_kept, workspace=ws), steps, 2, 5)
    pairs = sum(min(W - 1, V - 1 - a) for a in range(V))
    comps = pairs * n
    band_ms = mean(st[1])
    ach = comps * LD_MFMA_OPS / (band_ms * 1e-3) / 1e12   # pipelined fp4 band kernel
    kept = int(n_kept.item())
    assert kept == int(keep.sum().item())
    # the missing-call correction path on the same call (these panels have no
    # missing calls); identical flags
    ref_keep = keep.clone()
    ws_s = torch.empty(pg.prune_workspace_bytes(c, W, path="sparse"), dtype=torch.uint8,
                       device=dev)
    ms_s, st_s = timed_steps(torch, lib, hip, lambda: pg.ld_prune(
        c, W, S, t, path="sparse", keep=keep, n_kept=n_kept, workspace=ws_s), steps, 2, 5)
    assert torch.equal(keep, ref_keep)
    del ws_s
    sparse = {"ms_per_call": round(ms_s, 3),
              "stages_ms": {"layout": round(mean(st_s[0]), 3),
                            "band_kernel": round(mean(st_s[1]), 3),
                            "allele_counts": round(mean(st_s[2]), 3),
                            "greedy": round(mean(st_s[3]), 3)}}
    return {"workload": wp["name"], "path": "mfma", "ms_per_call": round(ms, 3), "sparse": sparse,
            "value": round(comps / (ms * 1e-3) / 1e9, 1), "unit": "G/s",
            "kept": kept, "variants": V,
            "stages_ms": {"layout": round(mean(st[0]), 3), "band_kernel": round(band_ms, 3),
                          "allele_counts": round(mean(st[2]), 3),
                          "greedy": round(mean(st[3]), 3)},
            "roofline": {"bound": "mfma", "kernel": "k_ld_mfma<fp4>", "unit": "TFLOP/s",
                         "dtype": "fp4", "achieved": round(ach, 2), "peak": PEAK_FP4_TFLOPS,
                         "frac": round(ach / PEAK_FP4_TFLOPS, 4)}}


def bench_grm(torch, lib, hip, pg, wg, dev, steps, path="auto"):
    """Relationship matrix (full layout): whole-call time and its stages.
    Algorithmic work: one fp64 multiply-add per (unique pair incl. the
    diagonal) x variant, i.e. 2 * m(m+1)/2 * V flops."""
    n, V = wg["n"], wg["V"]
    c = pg.Cohort.from_numpy(wg["bed"], n, device=dev)
    A = torch.empty((n, n), dtype=torch.float64, device=dev)
    Nn = torch.empty((n, n), dtype=torch.int32, device=dev)
    ws = torch.empty(pg.grm_workspace_bytes(c), dtype=torch.uint8, device=dev)
    ms, st = timed_steps(torch, lib, hip, lambda: pg.grm_matrix(
        c, layout="full", path=path, out=(A, Nn), workspace=ws), steps, 2, 3)
    flops = 2.0 * n * (n + 1) / 2 * V
    pair_ms = mean(st[1])
    ach = flops / (pair_ms * 1e-3) / 1e12
    torch.cuda.synchronize()
    assert torch.equal(Nn, Nn.T)
    return {"workload": wg["name"], "ms_per_call": round(ms, 3),
            "value": round(n * (n - 1) / 2 * V / (ms * 1e-3) / 1e9, 1), "unit": "G/s",
            "stages_ms": {"layout_and_tables": round(mean(st[0]), 3),
                          "pair_kernel": round(pair_ms, 3)},
            "roofline": {"bound": "mfma", "kernel": "k_grm_mfma", "unit": "TFLOP/s",
                         "achieved": round(ach, 2), "peak": PEAK_FP64_TFLOPS,
                         "frac": round(ach / PEAK_FP64_TFLOPS, 4)}}


def bench_cluster(torch, lib, hip, pg, wc, dev, steps):
    """IBS matrix (full) then complete-linkage clustering of all samples; the
    clustering call is timed on its own (its input is the IBS result)."""
    n = wc["n"]
    c = pg.Cohort.from_numpy(wc["bed"], n, device=dev)
    counts = pg.ibs_matrix(c, layout="full")
    out = torch.empty((n - 1, 16), dtype=torch.uint8, device=dev)
    ws = torch.empty(pg.cluster_workspace_bytes(n), dtype=torch.uint8, device=dev)
    ms, st = timed_steps(torch, lib, hip, lambda: pg.ibs_cluster(*counts, out=out, workspace=ws),
                         steps, 1, 3)
    merges = pg.merges_to_numpy(out, n)
    assert (merges["a"] < merges["b"]).all()
    return {"workload": wc["name"], "samples": n, "ms_per_call": round(ms, 3),
            "unit": "ms", "merges_per_s": round((n - 1) / (ms * 1e-3), 1),
            "stages_ms": {"distances_and_neighbours": round(mean(st[0]), 3),
                          "merge_loop": round(mean(st[1]), 3)}}


def bench_genome(torch, lib, hip, pg, cohort, counts, dev, steps):
    """IBS similarity and the IBD report over the default workload's full
    10,000 x 10,000 counts.  The report's per-pair kernel is bound by HBM:
    per entry it reads three uint32 counts and writes four doubles (44 B);
    the similarity reads three counts and writes one double (20 B)."""
    i0, i1, i2, nm = counts
    n = i0.shape[0]
    z = tuple(torch.empty((n, n), dtype=torch.float64, device=dev) for _ in range(4))
    ws = torch.empty(pg.genome_workspace_bytes(cohort), dtype=torch.uint8, device=dev)
    ms, st = timed_steps(torch, lib, hip, lambda: pg.ibs_genome(
        cohort, i0, i1, nm, out=z, workspace=ws), steps, 2, 3)
    pairs_ms = mean(st[1])
    gbs = 44.0 * n * n / (pairs_ms * 1e-3) / 1e9
    sim = z[0]
    ms_s, _ = timed_steps(torch, lib, hip, lambda: pg.ibs_similarity(i1, i2, nm, out=sim),
                          steps, 2, 0)
    gbs_s = 20.0 * n * n / (ms_s * 1e-3) / 1e9
    torch.cuda.synchronize()
    assert bool((torch.diagonal(z[2]) == 1.0).all())
    return {"samples": n, "ms_per_call": round(ms, 3), "unit": "ms",
            "stages_ms": {"layout_terms_and_averages": round(mean(st[0]), 3),
                          "pair_estimates": round(pairs_ms, 3)},
            "roofline": {"bound": "hbm", "kernel": "k_genome_pairs", "unit": "GB/s",
                         "bytes_per_entry": 44, "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                         "frac": round(gbs / PEAK_HBM_GBS, 4)},
            "similarity": {"ms_per_call": round(ms_s, 3), "bytes_per_entry": 20,
                           "achieved_gbs": round(gbs_s, 1),
                           "frac": round(gbs_s / PEAK_HBM_GBS, 4)}}


def cpu_baseline_cluster(wc):
    """The oracle's O(m^3) complete linkage on the same distances."""
    import oracle
    codes = oracle.unpack(wc["bed"], wc["n"], wc["V"])
    i0, i1, _, nm = oracle.ibs_matrix(codes, full=True)
    d = oracle.ibs_distance(i0, i1, nm)
    t0 = time.perf_counter()
    oracle.cluster_complete(d)
    dt = time.perf_counter() - t0
    return {"value": round(dt * 1e3, 1), "unit": "ms", "cores": 1, "kind": "oracle", "cpu": cpu_model(),
            "sample": "clustering of the whole workload (distances given)"}


def cpu_baseline_prune(wp):
    """The oracle's pruning on the whole workload (OpenMP r^2 table, then its
    sequential greedy pass)."""
    import oracle
    codes = oracle.unpack(wp["bed"], wp["n"], wp["V"])
    t0 = time.perf_counter()
    keep = oracle.ld_prune(codes, wp["window"], wp["step"], wp["r2_max"])
    dt = time.perf_counter() - t0
    return {"value": round(dt * 1e3, 1), "unit": "ms", "cores": oracle.threads(), "cpu": cpu_model(),
            "kind": "oracle", "sample": "whole workload", "kept": int(keep.sum())}


def bench_batch(torch, lib, hip, pg, synth, dev, steps):
    """64 uneven problems: the autotuner picks each problem's path; then the
    one-call-per-problem loop and the captured persistent batch are timed on
    the same problems and outputs."""
    log("batched workload: generating 64 problems")
    specs = synth.batch_problems()
    tuner = pg.Tuner()
    probs, comps, calls = [], 0.0, []
    t_tune = time.perf_counter()
    for d in specs:
        c = pg.Cohort.from_numpy(d["bed"], d["n"], device=dev)
        d.pop("bed")
        n, V = d["n"], d["V"]
        if d["kind"] == "ibs":
            path = tuner.tune("ibs", c, layout="tri", reps=3, for_batch=True)
            p = pg.IbsProblem(c, layout="tri", path=path)
            comps += n * (n - 1) / 2 * V
        else:
            W = d["window"]
            path = tuner.tune("ld", c, window=W, r2_min=d["r2_min"], reps=3, for_batch=True)
            cap = max(1 << 16, 64 * V)
            p = pg.LdProblem(c, window=W, r2_min=d["r2_min"], capacity=cap, path=path)
            comps += sum(min(W, V - 1 - a) for a in range(V)) * n
        probs.append(p)
    t_tune = time.perf_counter() - t_tune
    b = pg.Batch(probs)        # allocates every problem's outputs
    tiles, grid = b.tiles
    # one call per problem, same paths, outputs of their own, workspaces
    # allocated up front
    loop_out = []
    for p in probs:
        if isinstance(p, pg.IbsProblem):
            ws = torch.empty(max(pg.ibs_workspace_bytes(p.cohort, path=p.path), 1),
                             dtype=torch.uint8, device=dev)
            o = tuple(torch.empty_like(t) for t in p.out)
            calls.append(lambda p=p, ws=ws, o=o: pg.ibs_matrix(p.cohort, layout="tri",
                                                               path=p.path, out=o, workspace=ws))
        else:
            ws = torch.empty(max(pg.ld_workspace_bytes(p.cohort, p.window, path=p.path), 1),
                             dtype=torch.uint8, device=dev)
            o = (torch.empty_like(p.out), torch.empty_like(p.n_out))
            calls.append(lambda p=p, ws=ws, o=o: pg.ld_window(
                p.cohort, p.window, p.r2_min, capacity=p.capacity, path=p.path, out=o[0],
                n_out=o[1], workspace=ws))
        loop_out.append(o)

    def loop():
        for f in calls:
            f()

    ms_loop, _ = timed_steps(torch, lib, hip, loop, steps, 2, 0)
    b.capture()
    ms_graph, _ = timed_steps(torch, lib, hip, b.replay, steps, 2, 0)
    ms_direct, st_d = timed_steps(torch, lib, hip, b.launch, steps, 2, 3)
    torch.cuda.synchronize()
    # every output of the batch equals its one-call-per-problem counterpart
    for k, (p, o) in enumerate(zip(probs, loop_out)):
        if isinstance(p, pg.IbsProblem):
            assert all(torch.equal(x, y) for x, y in zip(p.out, o)), f"IBS problem {k}"
        else:
            total = int(o[1].item())
            assert int(p.n_out.item()) == total, f"LD problem {k}: emitted count"
            kept = min(total, p.capacity)
            assert torch.equal(p.out[:kept], o[0][:kept]), f"LD problem {k}: records"
    del loop_out, calls
    choice = {}
    for p in probs:
        k = ("ibs_" if isinstance(p, pg.IbsProblem) else "ld_") + \
            {1: "popc", 2: "mfma"}[int(p.path) & 0xFF]
        choice[k] = choice.get(k, 0) + 1
    b.close()
    return {"workload": "batch_64_hwe", "problems": len(probs), "comparisons": comps,
            "tiles": tiles, "persistent_grid": grid, "path_choices": choice,
            "tune_s": round(t_tune, 2),
            "graph": {"value": round(comps / (ms_graph * 1e-3) / 1e9, 1), "unit": "G/s",
                      "ms_per_step": round(ms_graph, 3)},
            "direct_launch": {"ms_per_step": round(ms_direct, 3),
                              "ibs_branch_ms": round(mean(st_d[0]), 3),
                              "both_branches_ms": round(mean(st_d[0]) + mean(st_d[1]), 3)},
            "one_call_per_problem": {"value": round(comps / (ms_loop * 1e-3) / 1e9, 1),
                                     "unit": "G/s", "ms_per_step": round(ms_loop, 3)},
            "speedup_vs_loop": round(ms_loop / ms_graph, 3)}


def bench_serve(torch, pg, synth, dev, seconds, serial_seconds, rates, rate_seconds):
    """8 resident cohorts (samples log-uniform in [1k, 50k], variants in
    [10k, 200k], HWE, MAF~U[0.01,0.5], 1% missing); Poisson 200 requests/s,
    70% IBS matrices (strict upper triangle) / 30% LD windows (500, r^2 >=
    0.2); subsets of 100-5,000 samples, ranges of 1k-20k variants.  The
    8-slot server and one request at a time run the same arrivals for the
    same time; then both at higher arrival rates (`rates`, `rate_seconds`
    each), and the server once more at the highest rate under a 384 MiB
    memory budget, where admission has to hold requests back."""
    import numpy as np
    from paper_1410_4803_amd.serve import GpuBackend, Server, poisson_requests
    specs = synth.serve_cohorts()
    shapes = [(d["n"], d["V"]) for d in specs]
    log(f"serving: generating 8 cohorts {shapes}")
    cohorts = [pg.Cohort.from_numpy(synth.serve_cohort_bed(d), d["n"], device=dev)
               for d in specs]
    resident = sum(c.nbytes for c in cohorts)
    budget = 64 << 30

    def work(r):
        m, L = len(r.sample_idx), r.v_range[1] - r.v_range[0]
        if r.kind == "ibs":
            return m * (m - 1) / 2 * L
        return sum(min(r.window, L - 1 - a) for a in range(L)) * m

    def run(slots, rate, secs, mem=budget):
        reqs = poisson_requests(shapes, rate=rate, seconds=secs, seed=1005)
        srv = Server(GpuBackend(cohorts, slots, keep_results=False), slots, mem)
        st = srv.run(reqs)
        done = srv.finished
        span = max(r.done for r in done) - min(r.arrival for r in done)
        st["value"] = round(sum(work(r) for r in done) / span / 1e9, 1)
        st["unit"] = "G/s"
        st["offered_rps"] = rate
        st["requests"] = len(reqs)
        st["queue_wait_p50_ms"] = round(float(np.percentile(
            [r.admitted - r.arrival for r in done], 50)) * 1e3, 3)
        return st

    # warm-up: a handful of requests (kernels, allocator pools, pinned buffers)
    warm = poisson_requests(shapes, rate=200.0, seconds=0.1, seed=99)
    Server(GpuBackend(cohorts, 8, keep_results=False), 8, budget).run(warm)
    log(f"serving {seconds} s of 200 requests/s with 8 slots")
    st = run(8, 200.0, seconds)
    log(f"serving {serial_seconds} s of 200 requests/s one at a time")
    sst = run(1, 200.0, serial_seconds)
    sweep = []
    for rate in rates:
        log(f"serving {rate_seconds} s of {rate} requests/s: 8 slots, then one at a time")
        sweep.append({"offered_rps": rate, "server_8_slots": run(8, rate, rate_seconds),
                      "serial_one_at_a_time": run(1, rate, rate_seconds)})
    tight = None
    if rates:
        log(f"serving {rate_seconds} s of {max(rates)} requests/s with a 384 MiB budget")
        tight = run(8, max(rates), rate_seconds, mem=384 << 20)
        tight["memory_budget"] = 384 << 20
    return {"workload": "serve_8_cohorts_poisson200", "cohorts": shapes,
            "resident_bytes": resident, "memory_budget": budget, "seconds": seconds,
            "requests": st["requests"], "server_8_slots": st,
            "serial_one_at_a_time": dict(sst, seconds=serial_seconds),
            "rate_sweep": sweep, "rate_sweep_seconds": rate_seconds,
            "budget_bound_run": tight}


def sweep(torch, lib, hip, pg, synth, dev, which: str, reps: int) -> None:
    """Path crossover: whole-call time of every kernel path per shape, one
    JSON line per shape (then a summary line with the fastest path per
    shape).  IBS: HWE panels (MAF~U[0.05,0.5], 1% missing), strict upper
    triangle, m in 64..10,000 samples x V in {5,000, 20,000, 100,000}.  LD:
    HWE panels of 20,000 variants, m in 500..20,000 samples x window in {50,
    500, 1,000} x missing rate in {0, 0.5%, 1%}, r^2 >= 0.2."""
    best = {}
    if which in ("ibs", "all"):
        for V in (5000, 20000, 100000):
            for m in (64, 128, 256, 512, 1024, 2048, 4096, 10000):
                bed = synth.hwe(m, V, (0.05, 0.5), 0.01, seed=7000 + m + V)
                c = pg.Cohort.from_numpy(bed, m, device=dev)
                size = m * (m - 1) // 2
                out = tuple(torch.empty(max(size, 1), dtype=torch.int32, device=dev)
                            for _ in range(4))
                rec = {"sweep": "ibs", "m": m, "V": V, "ms": {}}
                for path in ("mfma", "popc"):
                    ws = torch.empty(max(pg.ibs_workspace_bytes(c, path=path), 1),
                                     dtype=torch.uint8, device=dev)
                    ms, st = timed_steps(torch, lib, hip, lambda: pg.ibs_matrix(
                        c, layout="tri", path=path, out=out, workspace=ws), reps, 2, 3)
                    rec["ms"][path] = round(min(ms, 1e9), 4)
                    rec.setdefault("pair_kernel_ms", {})[path] = round(mean(st[1]), 4)
                    del ws
                rec["auto"] = {1: "popc", 2: "mfma"}[pg.api.resolve_path("ibs", m, V) & 0xFF]
                rec["fastest"] = min(rec["ms"], key=rec["ms"].get)
                best[f"ibs:{m}x{V}"] = rec["fastest"]
                print(json.dumps(rec), flush=True)
                del c, out
                torch.cuda.empty_cache()
    if which in ("ld", "all"):
        V = 20000
        cap = 1 << 22
        ol = torch.empty((cap, 64), dtype=torch.uint8, device=dev)
        nl = torch.empty(1, dtype=torch.int64, device=dev)
        for miss in (0.0, 0.005, 0.01):
            for m in (500, 1000, 2000, 5000, 10000, 20000):
                bed = synth.hwe(m, V, (0.05, 0.5), miss, seed=8000 + m + int(miss * 1e4))
                c = pg.Cohort.from_numpy(bed, m, device=dev)
                for W in (50, 500, 1000):
                    rec = {"sweep": "ld", "m": m, "V": V, "window": W, "miss": miss, "ms": {}}
                    for path in ("mfma", "sparse", "popc"):
                        ws = torch.empty(pg.ld_workspace_bytes(c, W, path=path),
                                         dtype=torch.uint8, device=dev)
                        ms, st = timed_steps(torch, lib, hip, lambda: pg.ld_window(
                            c, W, 0.2, capacity=cap, out=ol, n_out=nl, workspace=ws,
                            path=path), reps, 2, 5)
                        rec["ms"][path] = round(ms, 4)
                        rec.setdefault("band_kernel_ms", {})[path] = round(mean(st[1]), 4)
                        del ws
                    rec["auto"] = {1: "popc", 2: "mfma", 3: "sparse"}[
                        pg.api.resolve_path("ld", m, V, W) & 0xFF]
                    rec["fastest"] = min(rec["ms"], key=rec["ms"].get)
                    best[f"ld:{m}:{W}:{miss}"] = rec["fastest"]
                    print(json.dumps(rec), flush=True)
                del c
                torch.cuda.empty_cache()
    print(json.dumps({"sweep": "summary", "fastest": best}), flush=True)




def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--path", default="mfma", choices=["auto", "mfma", "popc"])
    ap.add_argument("--variant", type=int, default=0, help="kernel variant of the path (tuning)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--quick", action="store_true", help="default workload only, no extras")
    ap.add_argument("--extras", default="all",
                    help="comma list of extras: other,int8,small,ld,prune,grm,cluster,genome,peaks,batch,"
                         "serve "
                         "(or all / none)")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serial-seconds", type=float, default=60.0)
    ap.add_argument("--serve-rates", default="400,800,1600",
                    help="arrival rates (requests/s) of the serving sweep")
    ap.add_argument("--serve-rate-seconds", type=float, default=6.0)
    ap.add_argument("--grm-path", type=int, default=0,
                    help="path code of the relationship-matrix calls (0 = library default)")
    ap.add_argument("--sweep", choices=["ibs", "ld", "all"], default=None,
                    help="print the path crossover sweep (JSON lines) instead of the benchmark")
    ap.add_argument("--sweep-reps", type=int, default=3)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_1410_4803_amd as pg
    from paper_1410_4803_amd import _native as N

    torch.cuda.set_device(0)
    lib = N.load()
    hip = HipEvents()
    dev = torch.device("cuda:0")
    if args.sweep:
        sweep(torch, lib, hip, pg, synth, dev, args.sweep, args.sweep_reps)
        return

    # ---- default workload: IBS 10,000 x 100,000, full matrix ----
    log("generating the 10000 x 100000 mosaic panel")
    w = synth.ibs_large()
    n, V = w["n"], w["V"]
    cohort = pg.Cohort.from_numpy(w["bed"], n, device=dev)
    comps = n * (n - 1) / 2 * V

    def ibs_runner(path, variant=0):
        out = tuple(torch.empty((n, n), dtype=torch.int32, device=dev) for _ in range(4))
        code = pg.PATHS[path] | (variant << 8)
        ws = torch.empty(pg.ibs_workspace_bytes(cohort, path=code), dtype=torch.uint8, device=dev)
        return lambda: pg.ibs_matrix(cohort, layout="full", path=code, out=out, workspace=ws), out

    path = "mfma" if args.path == "auto" else args.path
    call, out = ibs_runner(path, args.variant)
    log(f"timing {args.steps} steps ({args.warmup} warmup), path {path}")
    ms, stages = timed_steps(torch, lib, hip, call, args.steps, args.warmup, 3)
    layout_ms, pair_ms = mean(stages[0]), mean(stages[1])
    fp4 = path == "mfma" and args.variant in IBS_FP4_VARIANTS
    if fp4:
        # the pair stage: whole tiles, the last round's tiles in K ranges, and
        # the reduce of those ranges (one launch each)
        ops = comps * IBS_MFMA_OPS
        roof = {"bound": "mfma", "achieved": ops / (pair_ms * 1e-3) / 1e12,
                "peak": PEAK_FP4_TFLOPS, "unit": "TFLOP/s", "kernel": IBS_FP4_KERNELS}
    elif path == "mfma":
        ops = comps * IBS_MFMA_OPS
        roof = {"bound": "mfma", "achieved": ops / (pair_ms * 1e-3) / 1e12, "peak": PEAK_INT8_TOPS,
                "unit": "TOP/s", "kernel": "k_ibs_mfma"}
    else:
        ops = comps * IBS_POPC_OPS
        roof = {"bound": "alu", "achieved": ops / (pair_ms * 1e-3) / 1e12, "peak": PEAK_VALU_TOPS,
                "unit": "TOP/s", "kernel": "k_ibs_popc"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = traffic_from_profile(roof["kernel"])
    roof["achieved"] = round(roof["achieved"], 2)
    roof["frac"] = round(roof["frac"], 4)
    roof["launch_ms"] = round(pair_ms, 4)

    result = {
        "metric": "genotype-pair comparisons/sec (G/s)",
        "value": round(comps / (ms * 1e-3) / 1e9, 1),
        "unit": "G/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp4" if fp4 else "int8" if path == "mfma" else "u32",
        "data": "synthetic",
        "config": {"workload": w["name"], "n_samples": n, "n_variants": V, "layout": "full",
                   "path": path, "variant": args.variant, "comparisons_per_step": comps},
        "roofline": roof,
        "stages_ms": {"layout": round(layout_ms, 4), "pair_kernel": round(pair_ms, 4)},
    }
    # sanity: the timed output is the IBS matrix (symmetric, sums agree)
    torch.cuda.synchronize()
    i0, i1, i2, nm = out
    assert torch.equal(i0 + i1 + i2, nm) and torch.equal(nm, nm.T)
    del i0, i1, i2, nm, call

    extras = {}
    want = set()
    if not args.quick:
        everything = {"other", "int8", "small", "ld", "prune", "grm", "cluster", "genome", "peaks",
                      "batch", "serve"}
        want = everything if args.extras == "all" else \
            set(x for x in args.extras.split(",") if x and x != "none")
    if "genome" in want:
        log("timing the IBD report and the similarity on the full counts")
        extras["genome_" + w["name"]] = bench_genome(torch, lib, hip, pg, cohort, out, dev,
                                                     max(3, args.steps // 2))
    del out
    torch.cuda.empty_cache()
    if "other" in want:
        other = "popc" if path == "mfma" else "mfma"
        call2, out2 = ibs_runner(other)
        log(f"timing the {other} path")
        ms2, st2 = timed_steps(torch, lib, hip, call2, max(3, args.steps // 2), 1, 3)
        pk2 = mean(st2[1])
        rec2 = {"value": round(comps / (ms2 * 1e-3) / 1e9, 1), "unit": "G/s",
                "ms_per_step": round(ms2, 3), "pair_kernel_ms": round(pk2, 3)}
        if other == "popc":
            ach2 = comps * IBS_POPC_OPS / (pk2 * 1e-3) / 1e12
            rec2["roofline"] = {"bound": "alu", "kernel": "k_ibs_popc", "unit": "TOP/s",
                                "ops_per_32_comparisons": 8, "achieved": round(ach2, 2),
                                "peak": round(PEAK_VALU_TOPS, 2),
                                "frac": round(ach2 / PEAK_VALU_TOPS, 4)}
        extras[f"ibs_large_{other}"] = rec2
        del call2, out2
        torch.cuda.empty_cache()

    if "int8" in want and path == "mfma":
        # the same tile schedule with int8 operands, against the int8 peak
        call3, out3 = ibs_runner("mfma", 7)
        log("timing the int8 matrix-core kernel (variant 7)")
        ms3, st3 = timed_steps(torch, lib, hip, call3, max(3, args.steps // 2), 1, 3)
        pk3 = mean(st3[1])
        ach3 = comps * IBS_MFMA_OPS / (pk3 * 1e-3) / 1e12
        extras["ibs_large_int8"] = {
            "value": round(comps / (ms3 * 1e-3) / 1e9, 1), "unit": "G/s", "variant": 7,
            "ms_per_step": round(ms3, 3), "pair_kernel_ms": round(pk3, 3),
            "roofline": {"bound": "mfma", "kernel": IBS_INT8_KERNELS, "unit": "TOP/s",
                         "achieved": round(ach3, 2), "peak": PEAK_INT8_TOPS,
                         "frac": round(ach3 / PEAK_INT8_TOPS, 4)}}
        del call3, out3
        torch.cuda.empty_cache()

    if "small" in want:
        # IBS 500 x 5,000 (strict upper triangle): latency-bound
        ws_ = synth.ibs_small()
        c1 = pg.Cohort.from_numpy(ws_["bed"], ws_["n"], device=dev)
        comps1 = ws_["n"] * (ws_["n"] - 1) / 2 * ws_["V"]
        for p1 in ("mfma", "popc"):
            o1 = tuple(torch.empty(124750, dtype=torch.int32, device=dev) for _ in range(4))
            wk1 = torch.empty(pg.ibs_workspace_bytes(c1, path=p1), dtype=torch.uint8, device=dev)
            ms1, st1 = timed_steps(torch, lib, hip, lambda: pg.ibs_matrix(
                c1, layout="tri", path=p1, out=o1, workspace=wk1), 20, 5, 3)
            extras[f"ibs_small_{p1}"] = {"value": round(comps1 / (ms1 * 1e-3) / 1e9, 1),
                                         "unit": "G/s", "us_per_call": round(ms1 * 1e3, 1),
                                         "pair_kernel_us": round(mean(st1[1]) * 1e3, 1)}

    if "ld" in want:
        # LD 5,000 x 500,000, window 1,000, r^2 >= 0.2 (1% missing calls), and the
        # same panel without missing calls, where the correction path pays
        cap = 4_000_000
        ol = torch.empty((cap, 64), dtype=torch.uint8, device=dev)
        nl = torch.empty(1, dtype=torch.int64, device=dev)
        for wl, key, lpaths in ((synth.ld_large(), "ld_large",
                                 ("mfma", "auto", "sparse", LD_SPARSE_ALL, "popc", LD_INT8)),
                                (synth.ld_large_nomiss(), "ld_large_nomiss",
                                 ("mfma", "auto", "sparse"))):
            log(f"timing LD windows on {wl['name']}")
            cl = pg.Cohort.from_numpy(wl["bed"], wl["n"], device=dev)
            W = wl["window"]
            Vl = wl["V"]
            pairs = sum(min(W, Vl - 1 - a) for a in range(Vl))
            compsl = pairs * wl["n"]
            for lpath in lpaths:
                wkl = torch.empty(pg.ld_workspace_bytes(cl, W, path=lpath), dtype=torch.uint8,
                                  device=dev)
                msl, stl = timed_steps(torch, lib, hip, lambda: pg.ld_window(
                    cl, W, wl["r2_min"], capacity=cap, out=ol, n_out=nl, workspace=wkl,
                    path=lpath), args.steps if lpath != "popc" else 3,
                    2 if lpath != "popc" else 1, 5)
                band_ms = mean(stl[1])
                rec = {"workload": wl["name"], "path": lpath,
                       "value": round(compsl / (msl * 1e-3) / 1e9, 1), "unit": "G/s",
                       "ms_per_step": round(msl, 3), "pairs": pairs, "emitted": int(nl.item()),
                       "stages_ms": {"layout": round(mean(stl[0]), 3),
                                     "band_kernel": round(band_ms, 3),
                                     "scan": round(mean(stl[2]), 3),
                                     "emit": round(mean(stl[3]), 3)}}
                if lpath == "mfma":
                    ach = compsl * LD_MFMA_OPS / (band_ms * 1e-3) / 1e12
                    rec["roofline"] = {"bound": "mfma", "kernel": "k_ld_mfma<fp4>",
                                       "unit": "TFLOP/s", "dtype": "fp4",
                                       "achieved": round(ach, 2), "peak": PEAK_FP4_TFLOPS,
                                       "frac": round(ach / PEAK_FP4_TFLOPS, 4),
                                       "traffic": traffic_from_profile("k_ld_mfma<fp4>")
                                       if key == "ld_large" else None}
                elif lpath == LD_INT8:
                    ach = compsl * LD_MFMA_OPS / (band_ms * 1e-3) / 1e12
                    rec["roofline"] = {"bound": "mfma", "kernel": "k_ld_mfma<int8>",
                                       "unit": "TOP/s", "dtype": "int8",
                                       "achieved": round(ach, 2), "peak": PEAK_INT8_TOPS,
                                       "frac": round(ach / PEAK_INT8_TOPS, 4)}
                elif lpath == "popc":
                    ach = compsl * LD_POPC_OPS / (band_ms * 1e-3) / 1e12
                    rec["roofline"] = {"bound": "alu", "kernel": "k_ld_popc", "unit": "TOP/s",
                                       "achieved": round(ach, 2), "peak": round(PEAK_VALU_TOPS, 2),
                                       "frac": round(ach / PEAK_VALU_TOPS, 4),
                                       "traffic": traffic_from_profile("k_ld_popc")}
                else:
                    rec["vs_mfma"] = round(extras[f"{key}_mfma"]["ms_per_step"] / msl, 3)
                    if lpath == LD_SPARSE_ALL:
                        rec["traffic_bytes_per_launch"] = traffic_from_profile("k_ld_sparse")
                rec["path"] = lpath if isinstance(lpath, str) else LD_PATH_NAMES[lpath]
                extras[f"{key}_{rec['path']}"] = rec
                del wkl
            del cl
        del ol

    prune_runs = []
    if "prune" in want:
        for wp in (synth.prune_small(), synth.prune_large()):
            log(f"timing LD pruning on {wp['name']}")
            extras[wp["name"]] = bench_prune(torch, lib, hip, pg, wp, dev, args.steps)
            prune_runs.append(wp)
        torch.cuda.empty_cache()

    if "grm" in want:
        for wg in (synth.grm_small(), synth.grm_large()):
            log(f"timing the relationship matrix on {wg['name']}")
            extras[wg["name"]] = bench_grm(torch, lib, hip, pg, wg, dev, max(3, args.steps // 2),
                                           args.grm_path)
            torch.cuda.empty_cache()

    cluster_runs = []
    if "cluster" in want:
        for wc in (synth.grm_small(), synth.grm_large()):
            log(f"timing complete-linkage clustering on {wc['name']}")
            key = "cluster_" + wc["name"].split("_")[1]
            extras[key] = bench_cluster(torch, lib, hip, pg, wc, dev, 3)
            cluster_runs.append((key, wc))
            torch.cuda.empty_cache()

    if "peaks" in want:
        log("measuring unit throughputs (peak probes)")
        pk = pg.peak_rates()
        pk = {k: round(v, 1) for k, v in pk.items()}
        pk["published"] = {"int8_mfma_tops": PEAK_INT8_TOPS, "fp64_mfma_tflops": PEAK_FP64_TFLOPS,
                           "valu_bcnt_tops": round(PEAK_VALU_TOPS, 1), "hbm_copy_gbs": PEAK_HBM_GBS}
        pk["ibs_int8_kernel_frac_of_measured_int8"] = round(
            extras["ibs_large_int8"]["roofline"]["achieved"] / pk["int8_mfma_tops"], 4) \
            if "ibs_large_int8" in extras else None
        extras["peaks"] = pk

    if "batch" in want:
        extras["batch"] = bench_batch(torch, lib, hip, pg, synth, dev, args.steps)
        torch.cuda.empty_cache()
    if "serve" in want and args.serve_seconds > 0:
        rates = [float(x) for x in args.serve_rates.split(",") if x]
        extras["serve"] = bench_serve(torch, pg, synth, dev, args.serve_seconds,
                                      args.serial_seconds, rates, args.serve_rate_seconds)
        torch.cuda.empty_cache()

    if args.copy_calibration:
        # an elementwise kernel that reads exactly 1 GiB and writes 1 GiB, for the
        # HBM byte counters (a plain tensor copy may go to the DMA engines,
        # which the kernel counters do not see)
        src = torch.zeros(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    if extras:
        result["extras"] = extras
    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample")
        result["cpu_baseline"] = cpu_baseline_ibs(w["bed"], n, V, args.cpu_budget)
        for key, wc in cluster_runs:
            if wc["n"] <= 2000:
                log(f"timing the CPU oracle's clustering on {wc['name']}")
                extras[key]["cpu_baseline"] = cpu_baseline_cluster(wc)
        for wp in prune_runs:
            if wp["n"] * wp["V"] * wp["window"] <= 1e10:     # whole problem in ~a second
                log(f"timing the CPU oracle on {wp['name']}")
                extras[wp["name"]]["cpu_baseline"] = cpu_baseline_prune(wp)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
