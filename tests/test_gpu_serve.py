"""GPU serving: requests run concurrently on stream slots (the mix) give
byte-identical results to the same requests run one at a time (alone), and
sampled responses match the oracle."""
import numpy as np
import pytest

import oracle
import synth
from ldcheck import compare_records

pytestmark = pytest.mark.gpu

pg = pytest.importorskip("paper_1410_4803_amd")
from paper_1410_4803_amd.serve import GpuBackend, Request, Server, poisson_requests  # noqa: E402


@pytest.fixture(scope="module")
def cohorts():
    shapes = [(2000, 12000), (1200, 30000), (3000, 15000)]
    beds = [synth.hwe(n, V, (0.01, 0.5), 0.01, seed=500 + k) for k, (n, V) in enumerate(shapes)]
    return shapes, beds, [pg.Cohort.from_numpy(b, n) for b, (n, V) in zip(beds, shapes)]


def _copy(r):
    return Request(r.rid, r.kind, r.cohort, r.sample_idx, r.v_range, r.window, r.r2_min,
                   r.layout, r.arrival)


def _same(a, b):
    if isinstance(a, tuple):
        return all(np.array_equal(x, y) for x, y in zip(a, b))
    return a.tobytes() == b.tobytes()


def test_mix_equals_alone_and_oracle(cohorts):
    shapes, beds, cs = cohorts
    reqs = poisson_requests(shapes, rate=2000, seconds=0.03, seed=7, max_samples=600,
                            range_len=(1000, 5000), window=200, r2_min=0.05)
    assert len(reqs) >= 20
    mix = Server(GpuBackend(cs, n_slots=6), n_slots=6, memory_budget=8 << 30)
    stats = mix.run([_copy(r) for r in reqs])
    assert stats["completed"] == len(reqs) and stats["max_concurrent"] > 1
    alone = {}
    for r in reqs:
        srv = Server(GpuBackend(cs, n_slots=1), n_slots=1, memory_budget=8 << 30)
        srv.run([_copy(r)])
        alone[r.rid] = srv.finished[0].result
    for r in mix.finished:
        assert _same(r.result, alone[r.rid]), f"request {r.rid} differs in the mix"
    # oracle on one IBS and one LD response
    by_kind = {}
    for r in mix.finished:
        by_kind.setdefault(r.kind, r)
    r = by_kind["ibs"]
    n, V = shapes[r.cohort]
    codes = oracle.select(oracle.unpack(beds[r.cohort], n, V), r.sample_idx, *r.v_range)
    for g, e in zip(r.result, oracle.ibs_matrix(codes, full=False)):
        assert np.array_equal(g, e)
    r = by_kind["ld"]
    n, V = shapes[r.cohort]
    codes = oracle.select(oracle.unpack(beds[r.cohort], n, V), r.sample_idx, *r.v_range)
    ref = oracle.ld_window(codes, r.window, r.r2_min)
    ref["a"] += r.v_range[0]
    ref["b"] += r.v_range[0]
    compare_records(r.result, ref, r.r2_min)


def test_overflowing_ld_request_is_reissued(cohorts):
    shapes, beds, cs = cohorts
    idx = np.arange(0, 300, dtype=np.int32)
    r = Request(0, "ld", 1, idx, (100, 2100), window=300, r2_min=-np.inf)
    srv = Server(GpuBackend(cs, n_slots=2, ld_capacity=1024), n_slots=2, memory_budget=8 << 30)
    srv.run([r])
    got = srv.finished[0]
    assert got.ld_capacity > 1024 and len(got.result) == got.ld_capacity
    ref = pg.ld_records(cs[1], 300, -np.inf, sample_idx=pg.api.torch.from_numpy(idx).cuda(),
                        v_range=(100, 2100))
    assert got.result.tobytes() == ref.tobytes()


def test_serving_workload_cohorts():
    """The serving workload's eight resident cohorts (up to 12,312 samples
    and 180,243 variants) and the first second of its 200 requests/s Poisson
    arrivals: every response of the 8-slot mix equals the same request run
    alone (a one-slot server, nothing else on the GPU), compared by a 128-bit
    hash of the result bytes; the smallest IBS and LD responses are checked
    whole against the oracle, and the IBS response with the most samples on
    sampled pairs."""
    specs = synth.serve_cohorts()
    shapes = [(d["n"], d["V"]) for d in specs]
    beds = [synth.serve_cohort_bed(d) for d in specs]
    cs = [pg.Cohort.from_numpy(b, n) for b, (n, V) in zip(beds, shapes)]
    reqs = poisson_requests(shapes, rate=200.0, seconds=1.0, seed=1005)
    assert len(reqs) >= 150
    budget = 64 << 30
    mix = Server(GpuBackend(cs, 8, keep_results="digest"), 8, budget)
    st = mix.run([_copy(r) for r in reqs])
    assert st["completed"] == len(reqs) and st["rejected"] == 0
    alone_reqs = [_copy(r) for r in reqs]
    for r in alone_reqs:
        r.arrival = 0.0
    alone = Server(GpuBackend(cs, 1, keep_results="digest"), 1, budget)
    alone.run(alone_reqs)
    assert alone.max_running == 1
    dig = {r.rid: r.result for r in alone.finished}
    assert len(dig) == len(reqs)
    for r in mix.finished:
        assert r.result == dig[r.rid], f"request {r.rid} ({r.kind}) differs in the mix"

    def work(r):
        return len(r.sample_idx) ** 2 * (r.v_range[1] - r.v_range[0])

    ibs = [r for r in reqs if r.kind == "ibs"]
    ld = [r for r in reqs if r.kind == "ld"]
    picks = [min(ibs, key=work), min(ld, key=work), max(ibs, key=lambda r: len(r.sample_idx))]
    keep = Server(GpuBackend(cs, 1, keep_results=True), 1, budget)
    keep.run([_copy(r) for r in picks])
    by_rid = {r.rid: r for r in keep.finished}
    from paper_1410_4803_amd.serve import _digest
    for k, p in enumerate(picks):
        r = by_rid[p.rid]
        n, V = shapes[r.cohort]
        raw = r.result
        assert _digest(raw if isinstance(raw, tuple) else [raw]) == dig[r.rid]
        codes = oracle.select(oracle.unpack(beds[r.cohort], n, V), r.sample_idx, *r.v_range)
        if r.kind == "ld":
            ref = oracle.ld_window(codes, r.window, r.r2_min)
            ref["a"] += r.v_range[0]
            ref["b"] += r.v_range[0]
            compare_records(r.result, ref, r.r2_min)
        elif k == 0:
            for g, e in zip(r.result, oracle.ibs_matrix(codes, full=False)):
                assert np.array_equal(g, e)
        else:
            m = len(r.sample_idx)
            rng = np.random.default_rng(8)
            pi = rng.integers(0, m - 1, 4000)
            pj = pi + 1 + (rng.integers(0, 1 << 30, 4000) % (m - 1 - pi))
            ref = oracle.ibs_pairs(np.ascontiguousarray(codes.T), pi, pj)
            t = pi * m - pi * (pi + 1) // 2 + (pj - pi - 1)
            got = np.stack([x[t] for x in r.result], 1)
            assert np.array_equal(got, ref)
