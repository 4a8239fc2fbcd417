"""GPU parity of the default IBS matrix-core launch where it splits the last,
partial round of tiles in K (grids of 512 tiles or more; the head runs whole
tiles over 8 XCD-balanced runs, the tail K ranges, and a reduce adds them).
Shapes are chosen so that the tail takes 2 to 19 tiles per run and 5 or 8
K ranges, with sample lists (a repeated sample among them), variant ranges
that cut through 16-variant words, missing-call masks, and both layouts.
Every count of the whole matrix equals the popcount path's (independent bit
planes), and sampled rows equal the oracle's."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

pg = pytest.importorskip("paper_1410_4803_amd")

MFMA, POPC = 2, 1


def _operand_bytes(m, nv):
    rows = -(-m // 128) * 128
    words = -(-(-(-nv // 16)) // 16) * 16
    return rows * words * 4


@pytest.mark.parametrize("n,m,V,vr,layout,mask", [
    (4100, 4001, 6000, (13, 5990), "full", False),   # 528 tiles: 2 tail tiles per run, 8 ranges
    (5200, 4900, 5000, None, "tri", True),           # 780 tiles: 2 tail tiles per run
    (6100, 6100, 3001, (0, 2999), "full", True),     # 1,176 tiles: 19 tail tiles per run, 5 ranges
])
def test_tail_split_equals_popcount_and_oracle(n, m, V, vr, layout, mask):
    bed = synth.mosaic(n, V, miss=0.02, seed=n + m, garbage_pad=True)
    mm = synth.missing_mask(n, V, 0.01, seed=m) if mask else None
    c = pg.Cohort.from_numpy(bed, n, mm)
    rng = np.random.default_rng(m)
    idx = None
    if m != n:
        idx = rng.choice(n, m - 1, replace=False)
        idx = np.concatenate([idx, idx[:1]]).astype(np.int32)     # a duplicate sample
    sidx = None if idx is None else torch.from_numpy(idx).cuda()
    nv = (vr[1] - vr[0]) if vr else V
    # the tail split is on for this shape: its K-range sums are in the workspace
    ws = pg.ibs_workspace_bytes(c, m if idx is not None else 0, vr, MFMA)
    assert ws > _operand_bytes(m, nv)
    got = pg.ibs_matrix(c, sample_idx=sidx, v_range=vr, layout=layout, path=MFMA)
    ref = pg.ibs_matrix(c, sample_idx=sidx, v_range=vr, layout=layout, path=POPC)
    torch.cuda.synchronize()
    for k, (g, r) in enumerate(zip(got, ref)):
        assert torch.equal(g, r), f"count {k} differs from the popcount path"
    # oracle on sampled rows of the selection
    codes = oracle.unpack(bed, n, V, mm)
    sel = oracle.select(codes, idx, *(vr if vr else (0, None)))
    codes_sm = np.ascontiguousarray(sel.T)
    rows = np.unique(np.concatenate([[0, 127, 128, m // 2, m - 2, m - 1],
                                     rng.choice(m, 6, replace=False)]))
    pi = np.repeat(rows, m)
    pj = np.tile(np.arange(m), len(rows))
    refp = oracle.ibs_pairs(codes_sm, pi, pj).reshape(len(rows), m, 4)
    if layout == "full":
        tr = torch.from_numpy(rows).cuda()
        for k in range(4):
            g = got[k][tr].cpu().numpy().view(np.uint32)
            assert np.array_equal(g, refp[:, :, k]), f"count {k}: rows differ from the oracle"
    else:
        for q, i in enumerate(rows):
            j = np.arange(i + 1, m)
            if len(j) == 0:
                continue
            t = i * m - i * (i + 1) // 2 + (j - i - 1)
            tt = torch.from_numpy(t).cuda()
            for k in range(4):
                g = got[k][tt].cpu().numpy().view(np.uint32)
                assert np.array_equal(g, refp[q, j, k]), f"count {k}, row {i}"
    if idx is not None:   # the repeated sample: its last row equals its first
        assert all(torch.equal(x[0], x[m - 1]) for x in got) if layout == "full" else True
