"""GPU: pg_ibs_matrix_noalloc (static scratch array, no workspace) gives the
same counts as pg_ibs_matrix with a caller workspace, on two calls in a row,
the second smaller (the array keeps the first call's contents)."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

pg = pytest.importorskip("paper_1410_4803_amd")
from paper_1410_4803_amd import api  # noqa: E402


def _junk(shape):
    return tuple(torch.full(shape, -7, dtype=torch.int32, device="cuda") for _ in range(4))


@pytest.mark.parametrize("path", ["mfma", "popc"])
def test_noalloc_equals_workspace_entry_point(path):
    assert api.noalloc_scratch_bytes() == 64 << 20
    # 1) 2,000 x 30,000, full layout: the operand fits the array, the K
    #    split's sums do not, so the call runs the unsplit kernel
    n, V = 2000, 30000
    bed = synth.hwe(n, V, (0.05, 0.5), 0.02, seed=71, garbage_pad=True)
    c = pg.Cohort.from_numpy(bed, n)
    assert pg.ibs_workspace_bytes(c, path=path) > 0
    ref = pg.ibs_matrix(c, layout="full", path=path)
    got = api.ibs_matrix_noalloc(c, _junk((n, n)), layout="full", path=path)
    torch.cuda.synchronize()
    for x, y in zip(got, ref):
        assert torch.equal(x, y)
    # 2) smaller: 300 of 700 samples by list, a variant range, triangle
    n2, V2 = 700, 9000
    bed2 = synth.mosaic(n2, V2, miss=0.01, seed=72, garbage_pad=True)
    c2 = pg.Cohort.from_numpy(bed2, n2)
    idx = torch.from_numpy(np.random.default_rng(3).integers(0, n2, 300).astype(np.int32)).cuda()
    ref2 = pg.ibs_matrix(c2, sample_idx=idx, v_range=(111, 8800), layout="tri", path=path)
    got2 = api.ibs_matrix_noalloc(c2, _junk((300 * 299 // 2,)), sample_idx=idx,
                                  v_range=(111, 8800), layout="tri", path=path)
    torch.cuda.synchronize()
    for x, y in zip(got2, ref2):
        assert torch.equal(x, y)


def test_noalloc_rejects_oversized_call():
    n, V = 10000, 40000                # operand alone is 100 MB
    c = pg.Cohort(torch.zeros(V * (n // 4), dtype=torch.uint8, device="cuda"), n, V)
    out = tuple(torch.empty(n * (n - 1) // 2, dtype=torch.int32, device="cuda") for _ in range(4))
    with pytest.raises(pg.PgError) as e:
        api.ibs_matrix_noalloc(c, out, layout="tri", path="mfma")
    assert e.value.status == -4 and "static array" in str(e.value)
