"""GPU: a batch of uneven problems in one persistent launch (direct and
captured in a HIP graph, replayed several times with other GPU work in
between) gives byte-identical outputs to one call per problem, and both
match the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from ldcheck import compare_records

pytestmark = pytest.mark.gpu

pg = pytest.importorskip("paper_1410_4803_amd")


def _problems(seed=0):
    rng = np.random.default_rng(seed)
    specs = []
    shapes = [(130, 900), (257, 1500), (64, 4000), (500, 700), (90, 333), (1, 50), (700, 2100)]
    for k, (n, V) in enumerate(shapes):
        bed = synth.hwe(n, V, (0.01, 0.5), 0.01, seed=seed * 100 + k, garbage_pad=True)
        mask = synth.missing_mask(n, V, 0.02, seed=k) if k % 3 == 0 else None
        specs.append((n, V, bed, mask))
    c = [pg.Cohort.from_numpy(b, n, m) for (n, V, b, m) in specs]
    idx = torch.from_numpy(rng.integers(0, 500, 211).astype(np.int32)).cuda()
    probs = [
        pg.IbsProblem(c[0], layout="tri", path="mfma"),
        pg.LdProblem(c[1], window=100, r2_min=0.05, capacity=200000, path="mfma"),
        pg.IbsProblem(c[2], layout="full", path="popc"),
        pg.LdProblem(c[3], window=64, r2_min=-np.inf, capacity=60000, path="popc"),
        pg.IbsProblem(c[3], sample_idx=idx, v_range=(50, 650), layout="full", path="mfma"),
        pg.IbsProblem(c[4], layout="tri", path=2 | (1 << 8)),
        pg.IbsProblem(c[5], layout="tri", path="popc"),
        pg.LdProblem(c[6], window=300, r2_min=0.02, capacity=200000, sample_idx=idx,
                     v_range=(10, 2000),
                     path="mfma"),
        pg.IbsProblem(c[6], layout="tri", path="auto"),
        pg.IbsProblem(c[2], layout="full", path=2 | (4 << 8)),
        pg.IbsProblem(c[0], sample_idx=idx[:90], layout="tri", path=2 | (3 << 8)),
        # the int8 tiles the batch hosts beside the fp4 ones
        pg.IbsProblem(c[6], layout="full", path=2 | (7 << 8)),
        pg.LdProblem(c[3], window=200, r2_min=0.0, capacity=200000, path=2 | (1 << 8)),
    ]
    return specs, probs, idx


def _single(p):
    if isinstance(p, pg.IbsProblem):
        return pg.ibs_matrix(p.cohort, sample_idx=p.sample_idx, v_range=p.v_range,
                             layout=p.layout, path=p.path)
    return pg.ld_records(p.cohort, p.window, p.r2_min, sample_idx=p.sample_idx,
                         v_range=p.v_range, path=p.path)


def _same(a, b):
    if isinstance(a, tuple):
        return all(torch.equal(x, y) for x, y in zip(a, b))
    return a.tobytes() == b.tobytes()


def test_batch_equals_single_calls_and_oracle():
    specs, probs, idx = _problems()
    singles = [_single(p) for p in probs]
    b = pg.Batch(probs)
    tiles, grid = b.tiles
    assert tiles > 0 and grid > 0
    b.launch()
    got = b.results()
    for k, (g, s) in enumerate(zip(got, singles)):
        assert _same(g, s), f"problem {k} differs from its single call"
    # oracle for two of them
    n, V, bed, mask = specs[0]
    ref = oracle.ibs_matrix(oracle.unpack(bed, n, V, mask), full=False)
    for g, r in zip(got[0], ref):
        assert np.array_equal(g.cpu().numpy().view(np.uint32), r)
    n, V, bed, mask = specs[6]
    codes = oracle.select(oracle.unpack(bed, n, V, mask), idx.cpu().numpy(), 10, 2000)
    refl = oracle.ld_window(codes, 300, 0.02)
    refl["a"] += 10
    refl["b"] += 10
    assert compare_records(got[7], refl, 0.02) > 40000
    b.close()


def test_batch_capacity_protocol():
    """An LD problem whose emitted pairs exceed its capacity: n_out holds the
    total, the buffer holds the first `capacity` pairs in (a, b) order."""
    n, V = 300, 800
    c = pg.Cohort.from_numpy(synth.mosaic(n, V, switch=0.01, miss=0.01, seed=4), n)
    full = pg.ld_records(c, 50, -np.inf)
    b = pg.Batch([pg.LdProblem(c, window=50, r2_min=-np.inf, capacity=100),
                  pg.IbsProblem(c, layout="tri")])
    b.launch()
    got = b.results()[0]
    assert int(b.problems[0].n_out.item()) == len(full)
    assert got.tobytes() == full[:100].tobytes()
    b.close()


def test_batch_graph_replays():
    specs, probs, idx = _problems(seed=1)
    singles = [_single(p) for p in probs]
    b = pg.Batch(probs)
    b.capture()
    for rep in range(3):
        # scribble over the outputs, replay, and check every replay
        for p in probs:
            if isinstance(p, pg.IbsProblem):
                for t in p.out:
                    t.fill_(-7)
            else:
                p.out.zero_()
                p.n_out.fill_(-1)
        junk = torch.randn(512, 512, device="cuda") @ torch.randn(512, 512, device="cuda")
        torch.cuda.synchronize()
        b.replay()
        got = b.results()
        for k, (g, s) in enumerate(zip(got, singles)):
            assert _same(g, s), f"replay {rep}: problem {k} differs"
        del junk
    b.close()


def test_batch_generated_workload_subset():
    """A slice of the batched workload generator (HWE, log-uniform shapes),
    shrunk so the single calls stay quick; the tuner picks paths."""
    probs_spec = synth.batch_problems(count=8, make_bed=False)
    tuner = pg.Tuner()
    probs = []
    for d in probs_spec:
        n, V = min(d["n"], 1500), min(d["V"], 6000)
        bed = synth.hwe(n, V, (0.01, 0.5), 0.01, seed=d["seed"])
        c = pg.Cohort.from_numpy(bed, n)
        if d["kind"] == "ibs":
            path = tuner.tune("ibs", c, layout="tri", reps=1, for_batch=True)
            probs.append(pg.IbsProblem(c, layout="tri", path=path))
        else:
            path = tuner.tune("ld", c, window=d["window"], r2_min=d["r2_min"], reps=1,
                              for_batch=True)
            probs.append(pg.LdProblem(c, window=d["window"], r2_min=d["r2_min"], path=path))
    singles = [_single(p) for p in probs]
    b = pg.Batch(probs)
    b.capture()
    b.replay()
    got = b.results()
    for k, (g, s) in enumerate(zip(got, singles)):
        assert _same(g, s), f"problem {k}"
    b.close()


def _tri_row_pairs(m, rows):
    """Packed upper-triangle indices and (i, j) pairs of whole rows: every
    pair of each listed sample with every other sample."""
    idx, pi, pj = [], [], []
    for i in rows:
        j = np.delete(np.arange(m), i)
        a, b = np.minimum(i, j), np.maximum(i, j)
        idx.append(a * m - a * (a + 1) // 2 + (b - a - 1))
        pi.append(a)
        pj.append(b)
    return np.concatenate(idx), np.concatenate(pi), np.concatenate(pj)


def test_batch_full_workload():
    """The whole 64-problem batched workload (samples log-uniform in [200,
    20,000], variants in [2,000, 50,000], HWE, 1% missing; even problems IBS
    triangles, odd problems LD windows of 500 at r^2 >= 0.2) as the
    benchmark runs it: tuner-chosen paths, captured in one HIP graph and
    replayed twice.  Every problem's outputs, in buffers of their own, equal
    a separate call per problem byte for byte (IBS: all four counts; LD: the
    total and the record list), and whole rows of the three largest IBS
    problems and row ranges of the three largest LD problems match the
    oracle."""
    specs = synth.batch_problems()
    assert len(specs) == 64
    tuner = pg.Tuner()
    probs = []
    for d in specs:
        c = pg.Cohort.from_numpy(d["bed"], d["n"])
        if d["kind"] == "ibs":
            path = tuner.tune("ibs", c, layout="tri", reps=1, for_batch=True)
            probs.append(pg.IbsProblem(c, layout="tri", path=path))
        else:
            path = tuner.tune("ld", c, window=d["window"], r2_min=d["r2_min"], reps=1,
                              for_batch=True)
            probs.append(pg.LdProblem(c, window=d["window"], r2_min=d["r2_min"],
                                      capacity=max(1 << 16, 64 * d["V"]), path=path))
    b = pg.Batch(probs)
    b.capture()
    b.replay()
    b.replay()
    got = b.results()
    for k, p in enumerate(probs):
        s = _single(p)
        if isinstance(p, pg.IbsProblem):
            for x, y in zip(got[k], s):
                assert torch.equal(x, y), f"problem {k} (IBS {specs[k]['n']} x {specs[k]['V']})"
        else:
            assert int(p.n_out.item()) == len(s), f"problem {k}: emitted count"
            assert got[k].tobytes() == s.tobytes(), f"problem {k} (LD)"
        del s
    ibs_k = sorted((k for k in range(64) if specs[k]["kind"] == "ibs"),
                   key=lambda k: specs[k]["n"] ** 2 * specs[k]["V"])[-3:]
    for k in ibs_k:
        d = specs[k]
        m, V = d["n"], d["V"]
        rows = np.array([0, 1, m // 2, m - 2, m - 1])
        tidx, pi, pj = _tri_row_pairs(m, rows)
        ref = oracle.ibs_pairs(oracle.unpack(d["bed"], m, V, sample_major=True), pi, pj)
        t = torch.from_numpy(tidx).cuda()
        g = np.stack([o[t].cpu().numpy().view(np.uint32) for o in got[k]], 1)
        assert np.array_equal(g, ref), f"problem {k}: rows differ from the oracle"
    ld_k = sorted((k for k in range(64) if specs[k]["kind"] == "ld"),
                  key=lambda k: specs[k]["n"] * specs[k]["V"])[-3:]
    for k in ld_k:
        d = specs[k]
        codes = oracle.unpack(d["bed"], d["n"], d["V"])
        for a0 in (0, d["V"] // 2, d["V"] - 60):
            ref = oracle.ld_window(codes, d["window"], d["r2_min"], a_begin=a0, a_end=a0 + 60)
            sel = got[k][(got[k]["a"] >= a0) & (got[k]["a"] < a0 + 60)]
            compare_records(sel, ref, d["r2_min"])
    b.close()


def test_batch_auto_ld_is_the_matrix_core_path():
    """A shape where one-problem calls resolve AUTO to the gated correction
    path: in a batch AUTO is the matrix-core path, with the same records."""
    n, V = 5000, 1200
    c = pg.Cohort.from_numpy(synth.mosaic(n, V, switch=0.01, miss=0.0, seed=61), n)
    b = pg.Batch([pg.LdProblem(c, window=500, r2_min=0.1, capacity=400000, path="auto")])
    b.launch()
    got = b.results()[0]
    assert got.tobytes() == pg.ld_records(c, 500, 0.1, path="mfma").tobytes()
    assert got.tobytes() == pg.ld_records(c, 500, 0.1, path="auto").tobytes()
    b.close()
