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
