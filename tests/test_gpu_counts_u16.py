"""GPU: 16-bit counts (PG_COUNTS_U16).  Every path and kernel variant of the
IBS matrix, in both layouts, gives the same counts with the flag as without
it; so do a batch problem and the allocation-free call.  Shapes cover a
ragged last tile, odd row lengths (rows whose 16-bit entries are not 8-byte
aligned take the scalar stores), the K-split small-cohort launch, the
tail-split launch, and a range of exactly 65,535 variants whose diagonal
reaches the largest 16-bit count.  One shape is also checked against the
oracle directly."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

pg = pytest.importorskip("paper_1410_4803_amd")

MFMA, POPC = 2, 1


def _wide(t16):
    return t16.to(torch.int32) & 0xFFFF


def _same(a16, b32, what):
    for k, (x, y) in enumerate(zip(a16, b32)):
        assert x.dtype == torch.int16 and y.dtype == torch.int32
        assert torch.equal(_wide(x), y), f"{what}: count {k} differs with 16-bit counts"


def _cohort(n, V, seed, mask=True):
    bed = synth.hwe(n, V, (0.01, 0.5), 0.02, seed=seed, garbage_pad=True)
    mm = synth.missing_mask(n, V, 0.01, seed=seed + 1) if mask else None
    return bed, mm, pg.Cohort.from_numpy(bed, n, mm)


@pytest.mark.parametrize("path", ["auto", POPC] + [MFMA | (v << 8) for v in range(1, 10)])
@pytest.mark.parametrize("layout", ["full", "tri"])
def test_u16_equals_u32_every_variant(path, layout):
    n, V = 333, 2500
    bed, mm, c = _cohort(n, V, 11)
    vr = (7, 2491)
    a = pg.ibs_matrix(c, v_range=vr, layout=layout, path=path, counts="u16")
    b = pg.ibs_matrix(c, v_range=vr, layout=layout, path=path)
    torch.cuda.synchronize()
    _same(a, b, f"path {path}, {layout}")


@pytest.mark.parametrize("n,m,V,layout", [
    (600, 500, 5000, "tri"),      # small cohort: K split over several ranges, then a reduce
    (700, 257, 9000, "full"),     # K split, a ragged last tile and odd rows
    (4100, 4001, 6000, "full"),   # tail split: whole-tile head, K-range tail, reduce
    (5200, 4900, 5000, "tri"),
])
def test_u16_split_launches(n, m, V, layout):
    bed, mm, c = _cohort(n, V, n + m)
    rng = np.random.default_rng(m)
    idx = torch.from_numpy(rng.choice(n, m, replace=False).astype(np.int32)).cuda()
    a = pg.ibs_matrix(c, sample_idx=idx, layout=layout, counts="u16")
    b = pg.ibs_matrix(c, sample_idx=idx, layout=layout)
    torch.cuda.synchronize()
    _same(a, b, f"{m} of {n} samples x {V}")


def test_u16_largest_count_and_oracle():
    """65,535 selected variants, no missing calls: each diagonal entry is
    N = IBS2 = 65,535, the largest 16-bit count; every count equals the
    oracle's."""
    n, V = 150, 66000
    bed = synth.hwe(n, V, (0.01, 0.5), 0.0, seed=5, garbage_pad=True)
    c = pg.Cohort.from_numpy(bed, n, None)
    vr = (300, 300 + 65535)
    got = pg.ibs_matrix(c, v_range=vr, layout="full", counts="u16")
    ref = oracle.ibs_matrix(oracle.select(oracle.unpack(bed, n, V, None), None, *vr), full=True)
    for k, (g, r) in enumerate(zip(got, ref)):
        assert np.array_equal(g.cpu().numpy().view(np.uint16).astype(np.uint32), r.reshape(n, n)), k
    assert int(_wide(got[3]).diagonal().min()) == 65535
    assert int(_wide(got[2]).diagonal().min()) == 65535
    with pytest.raises(RuntimeError):
        pg.ibs_matrix(c, v_range=(300, 300 + 65536), counts="u16")


def test_u16_batch_problem():
    _, _, c0 = _cohort(300, 3000, 21)
    _, _, c1 = _cohort(130, 900, 22, mask=False)
    probs = [pg.IbsProblem(c0, layout="tri", counts="u16"),
             pg.IbsProblem(c1, layout="full", path="popc", counts="u16"),
             pg.IbsProblem(c0, v_range=(11, 2900), layout="full", counts="u16"),
             pg.LdProblem(c1, window=50, r2_min=0.1, capacity=50000)]
    b = pg.Batch(probs)
    b.launch()
    got = b.results()
    torch.cuda.synchronize()
    for k, p in enumerate(probs[:3]):
        ref = pg.ibs_matrix(p.cohort, v_range=p.v_range, layout=p.layout, path=p.path)
        _same(got[k], ref, f"batch problem {k}")


def test_u16_noalloc_two_calls():
    _, _, c = _cohort(900, 4000, 31)
    for m, vr in [(900, (0, 4000)), (401, (33, 3001))]:
        idx = torch.arange(m, dtype=torch.int32, device="cuda") * 2 % 900
        out = tuple(torch.empty((m, m), dtype=torch.int16, device="cuda") for _ in range(4))
        pg.ibs_matrix_noalloc(c, out, sample_idx=idx, v_range=vr, counts="u16")
        ref = pg.ibs_matrix(c, sample_idx=idx, v_range=vr)
        torch.cuda.synchronize()
        _same(out, ref, f"no-alloc, {m} samples")


def test_u16_served_results():
    """The server returns uint16 counts for ranges under 65,536 variants
    ("auto"), equal to the uint32 counts it returns with ibs_counts "u32"."""
    from paper_1410_4803_amd.serve import GpuBackend, Request, Server
    _, _, c = _cohort(800, 70000, 41, mask=False)
    rng = np.random.default_rng(3)
    reqs = []
    for k, vr in enumerate([(0, 5000), (100, 65635), (0, 70000)]):
        idx = np.sort(rng.choice(800, 300 + 50 * k, replace=False)).astype(np.int32)
        reqs.append(Request(k, "ibs", 0, idx, vr, 0, 0.0, "tri", 0.0))
    res = {}
    for mode in ("auto", "u32"):
        srv = Server(GpuBackend([c], 2, ibs_counts=mode), 2, 8 << 30)
        srv.run([Request(r.rid, r.kind, r.cohort, r.sample_idx, r.v_range, r.window, r.r2_min,
                         r.layout, r.arrival) for r in reqs])
        res[mode] = {r.rid: r.result for r in srv.finished}
    for r in reqs:
        a, b = res["auto"][r.rid], res["u32"][r.rid]
        want = np.uint16 if r.v_range[1] - r.v_range[0] < 65536 else np.uint32
        assert all(x.dtype == want for x in a) and all(y.dtype == np.uint32 for y in b)
        assert all(np.array_equal(x, y) for x, y in zip(a, b)), f"request {r.rid}"
