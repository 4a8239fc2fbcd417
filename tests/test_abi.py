"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments with the documented status codes
before touching the device (no compute calls here)."""
import ctypes
import os
import re

import pytest

from paper_1410_4803_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "pg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pg_\w+)\s*\(", text)))


def test_every_header_symbol_is_exported():
    lib = N.load()
    names = _header_functions()
    assert set(names) == set(N.SYMBOLS)
    for name in names:
        assert hasattr(lib, name), name
    assert lib.pg_version() == 1


def test_status_strings():
    assert N.status_str(0) == "ok"
    assert N.status_str(-2) == "workspace too small"
    assert N.status_str(99) == "unknown status"


def _g(n=100, V=50, bpv=0, bed=0x1000):
    return N.Genotypes(bed, n, V, bpv, None)


def _ibs_ws(g, n_sel=0, vb=0, ve=0, path=0):
    b = ctypes.c_size_t(0)
    rc = N.load().pg_ibs_workspace_bytes(ctypes.byref(g), n_sel, vb, ve, path, ctypes.byref(b))
    return rc, b.value


def _ld_ws(g, W, n_sel=0, vb=0, ve=0, path=0):
    b = ctypes.c_size_t(0)
    rc = N.load().pg_ld_workspace_bytes(ctypes.byref(g), n_sel, vb, ve, W, path, ctypes.byref(b))
    return rc, b.value


def test_workspace_sizes():
    # 10,000 x 100,000: the operand (10,112 rows x 6,256 words), then the tail
    # split's sums: 3,160 tiles in 8 runs of 395, 384 whole tiles each
    # (12 rounds of 32 CUs), 11 tail tiles x 5 K ranges x 196,608 bytes per run
    rc, b = _ibs_ws(_g(10000, 100000), path=N.PG_PATH_MFMA)
    assert rc == 0 and b == 10112 * 6256 * 4 + 8 * 11 * 5 * 192 * 256 * 4
    rc, b = _ibs_ws(_g(10000, 100000), path=N.PG_PATH_MFMA | (2 << 8))   # a whole-tile variant
    assert rc == 0 and b == 10112 * 6256 * 4
    rc, b = _ibs_ws(_g(10000, 100000), path=N.PG_PATH_POPC)
    assert rc == 0 and b == 3 * 10048 * 3136 * 4
    rc, b = _ibs_ws(_g(100, 50), n_sel=7)
    assert rc == 0 and b == 128 * 16 * 4
    # small cohorts: the default matrix-core kernel splits each tile's chunks
    # of 256 variants into ranges (500 x 5,000: 10 tiles, 20 chunks, 10 ranges
    # of 2) whose raw sums (192 x 256 int32 per tile and range) follow the
    # operand, 256-byte aligned
    rc, b = _ibs_ws(_g(500, 5000), path=N.PG_PATH_MFMA)
    assert rc == 0 and b == 512 * 320 * 4 + 10 * 10 * 192 * 256 * 4
    rc, b = _ibs_ws(_g(500, 5000), path=N.PG_PATH_MFMA | (1 << 8))   # variant 1: no split
    assert rc == 0 and b == 512 * 320 * 4
    rc, b = _ld_ws(_g(5000, 500000), 1000, path=N.PG_PATH_MFMA)
    assert rc == 0 and b > 500000 * 320 * 4
    # correction path: + sample-major operand (5120 x 31264 words), lists of
    # 320 entries per variant, 16 bytes of totals per variant
    rc, bs = _ld_ws(_g(5000, 500000), 1000, path=N.PG_PATH_SPARSE)
    assert rc == 0 and bs >= b + 5120 * 31264 * 4 + 500032 * 320 * 4 + 500032 * 16
    assert bs < b + 5120 * 31264 * 4 + 500032 * 320 * 4 + 500032 * 16 + (1 << 20)
    # AUTO at this shape is the correction path behind its sampled gate
    rc, ba = _ld_ws(_g(5000, 500000), 1000)
    assert rc == 0 and ba == bs
    # list slots: max(64, ceil(m/16) rounded up to 8), at most 65528
    for m, cap in [(1, 64), (1000, 64), (1040, 72), (5000, 320), (2000000, 65528)]:
        rc, b0 = _ld_ws(_g(m, 64), 1, path=N.PG_PATH_MFMA)
        rc1, b1 = _ld_ws(_g(m, 64), 1, path=N.PG_PATH_SPARSE)
        t_rows = -(-m // 128) * 128
        assert rc == rc1 == 0
        # operand, lists, totals, then group sums, group maxima and a flag
        # (each carve rounded up to 256 bytes)
        assert b1 - b0 == t_rows * 16 * 4 + 64 * cap * 4 + 64 * 16 + 3 * 256, (m, b1 - b0)


@pytest.mark.parametrize("kw,code", [
    (dict(n=0), N.PG_EINVAL), (dict(V=0), N.PG_EINVAL), (dict(n=1 << 31), N.PG_EINVAL),
    (dict(bpv=3, n=100), N.PG_EINVAL), (dict(bed=0), N.PG_EINVAL)])
def test_bad_matrix(kw, code):
    rc, _ = _ibs_ws(_g(**kw))
    assert rc == code
    assert N.last_error() != ""


def test_bad_selection_and_range():
    g = _g(100, 50)
    assert _ibs_ws(g, vb=10, ve=5)[0] == N.PG_EINVAL
    assert _ibs_ws(g, vb=0, ve=51)[0] == N.PG_EINVAL
    assert _ibs_ws(g, vb=-1, ve=5)[0] == N.PG_EINVAL
    assert _ibs_ws(g, path=7)[0] == N.PG_EINVAL
    assert _ld_ws(g, 0)[0] == N.PG_EINVAL
    assert _ld_ws(g, 10, path=N.PG_PATH_POPC)[0] == 0
    assert _ld_ws(g, 10, path=9)[0] == N.PG_EINVAL
    assert _ld_ws(g, 10, path=1 << 16)[0] == N.PG_EINVAL
    assert _ibs_ws(g, vb=10, ve=20)[0] == 0


def test_calls_reject_before_launch():
    lib = N.load()
    g = _g(100, 50)
    fake = 0x2000
    # short workspace
    rc = lib.pg_ibs_matrix(ctypes.byref(g), None, 0, 0, 0, N.PG_FULL, 0, fake, fake, fake, fake,
                           fake, 16, None)
    assert rc == N.PG_ENOMEM
    # NULL output
    rc = lib.pg_ibs_matrix(ctypes.byref(g), None, 0, 0, 0, N.PG_FULL, 0, None, fake, fake, fake,
                           fake, 1 << 30, None)
    assert rc == N.PG_EINVAL
    # bad layout
    rc = lib.pg_ibs_matrix(ctypes.byref(g), None, 0, 0, 0, 5, 0, fake, fake, fake, fake,
                           fake, 1 << 30, None)
    assert rc == N.PG_EINVAL
    # 16-bit counts: only for ranges under 65,536 variants; unknown flag bits rejected
    for lay, V, vb, ve in [(N.PG_FULL | N.PG_COUNTS_U16, 70000, 0, 0),
                           (N.PG_TRI_UPPER | N.PG_COUNTS_U16, 70000, 1000, 66536),
                           (N.PG_FULL | 0x200, 50, 0, 0), (5 | N.PG_COUNTS_U16, 50, 0, 0)]:
        gv = _g(100, V)
        rc = lib.pg_ibs_matrix(ctypes.byref(gv), None, 0, vb, ve, lay, 0, fake, fake, fake, fake,
                               fake, 1 << 30, None)
        assert rc == N.PG_EINVAL, (lay, V)
        why = "65,536" if V > 65535 else "unknown layout"
        assert why in N.last_error()
        rc = lib.pg_ibs_matrix_noalloc(ctypes.byref(gv), None, 0, vb, ve, lay, 0, fake, fake,
                                       fake, fake, None)
        assert rc == N.PG_EINVAL and why in N.last_error(), (lay, V)
    # one sample, triangle layout: nothing to do, NULL outputs accepted
    g1 = _g(1, 50)
    rc = lib.pg_ibs_matrix(ctypes.byref(g1), None, 0, 0, 0, N.PG_TRI_UPPER, 0, None, None, None,
                           None, None, 0, None)
    assert rc == N.PG_OK
    # LD: NULL n_out, negative capacity, NULL out with capacity
    rc = lib.pg_ld_window(ctypes.byref(g), None, 0, 0, 0, 10, 0.2, fake, 10, None, 0, fake,
                          1 << 30, None)
    assert rc == N.PG_EINVAL
    rc = lib.pg_ld_window(ctypes.byref(g), None, 0, 0, 0, 10, 0.2, fake, -1, fake, 0, fake,
                          1 << 30, None)
    assert rc == N.PG_EINVAL
    rc = lib.pg_ld_window(ctypes.byref(g), None, 0, 0, 0, 10, 0.2, None, 5, fake, 0, fake,
                          1 << 30, None)
    assert rc == N.PG_EINVAL
    rc = lib.pg_ld_window(ctypes.byref(g), None, 0, 0, 0, 10, 0.2, fake, 5, fake, 0, fake,
                          8, None)
    assert rc == N.PG_ENOMEM
    # diagnostic variant of the correction path: one slot per (variant, distance)
    rc = lib.pg_ld_window(ctypes.byref(g), None, 0, 0, 0, 10, 0.2, fake, 5, fake,
                          N.PG_PATH_SPARSE | (2 << 8), fake, 1 << 30, None)
    assert rc == N.PG_EINVAL and "slots" in N.last_error()


def test_batch_plan_validation_names_problem():
    lib = N.load()
    arr = (N.Problem * 3)()
    for k in range(3):
        arr[k].kind = N.PG_KIND_IBS
        arr[k].g = _g(100, 50)
        arr[k].out_layout = N.PG_TRI_UPPER
        arr[k].ibs0 = arr[k].ibs1 = arr[k].ibs2 = arr[k].nonmiss = 0x3000
    arr[2].kind = N.PG_KIND_LD
    arr[2].window = 0                   # invalid window
    arr[2].n_out = 0x4000
    plan = ctypes.c_void_p()
    rc = lib.pg_batch_plan(arr, 3, ctypes.byref(plan))
    assert rc == N.PG_EINVAL and plan.value is None
    assert "problem 2" in N.last_error()
    arr[2].window = 10
    rc = lib.pg_batch_plan(arr, 3, ctypes.byref(plan))
    assert rc == N.PG_OK and plan.value
    nbytes = ctypes.c_size_t()
    assert lib.pg_batch_workspace_bytes(plan, ctypes.byref(nbytes)) == 0 and nbytes.value > 0
    tiles = ctypes.c_int64()
    assert lib.pg_batch_tiles(plan, ctypes.byref(tiles), None) == 0
    # two 128-tile IBS problems (1 tile each) + LD 64-row tiles: 1 row tile x 2 band tiles
    assert tiles.value == 1 + 1 + 2
    # launching with a workspace that was never uploaded is rejected before any launch
    rc = lib.pg_batch_launch(plan, 0x5000, nbytes.value, None)
    assert rc == N.PG_EINVAL
    lib.pg_plan_free(plan)
    assert lib.pg_batch_plan(arr, 0, ctypes.byref(plan)) == N.PG_EINVAL
    arr[2].path = N.PG_PATH_SPARSE      # the correction path is for one-problem calls
    rc = lib.pg_batch_plan(arr, 3, ctypes.byref(plan))
    assert rc == N.PG_EUNSUPPORTED and "problem 2" in N.last_error()
    arr[2].path = 0
    arr[1].g = _g(100, 65536)          # 16-bit counts need fewer than 65,536 variants
    arr[1].out_layout = N.PG_TRI_UPPER | N.PG_COUNTS_U16
    rc = lib.pg_batch_plan(arr, 3, ctypes.byref(plan))
    assert rc == N.PG_EINVAL and "problem 1" in N.last_error()
    arr[1].g = _g(100, 65535)
    rc = lib.pg_batch_plan(arr, 3, ctypes.byref(plan))
    assert rc == N.PG_OK and plan.value
    lib.pg_plan_free(plan)


def _prune_ws(g, W, n_sel=0, vb=0, ve=0, path=0):
    b = ctypes.c_size_t(0)
    rc = N.load().pg_prune_workspace_bytes(ctypes.byref(g), n_sel, vb, ve, W, path,
                                           ctypes.byref(b))
    return rc, b.value


def test_prune_workspace_and_validation():
    lib = N.load()
    g = _g(1000, 100000)
    rc, b = _prune_ws(g, 50)
    _, ld = _ld_ws(g, 49)
    # the LD scratch of the pair kernel (largest distance window - 1), one
    # int2 of allele counts per padded variant, a drop-side bitmap of the
    # pair kernel's bitmap size (2 words per row for window 50), and uint16
    # counts of the (window, row) cells for the smallest step (at most one
    # window per variant: 100,000 x 50 cells), rounded up to passes of 16,384
    cells = -(-100000 * 50 // 16384) * 16384
    assert rc == 0 and b == ld + 100032 * 8 + 100032 * 2 * 4 + cells * 2
    # capped at 2^26 cells
    rc, b2 = _prune_ws(_g(1000, 2000000), 1000)
    _, ld2 = _ld_ws(_g(1000, 2000000), 999)
    assert rc == 0 and b2 == ld2 + 2000000 * 8 + 2000000 * 32 * 4 + (1 << 26) * 2
    assert _prune_ws(g, 1)[0] == N.PG_EINVAL
    assert _prune_ws(g, (1 << 16) + 1)[0] == N.PG_EINVAL
    assert _prune_ws(g, 1 << 16)[0] == 0
    fake = 0x2000

    def call(W=50, S=5, t=0.5, keep=fake, ws=1 << 30, path=0):
        return lib.pg_ld_prune(ctypes.byref(g), None, 0, 0, 0, W, S, t, keep, None, path, fake,
                               ws, None)
    assert call(S=0) == N.PG_EINVAL
    assert call(S=51) == N.PG_EINVAL
    assert call(W=1, S=1) == N.PG_EINVAL
    assert call(t=float("nan")) == N.PG_EINVAL
    assert call(keep=None) == N.PG_EINVAL
    assert call(path=9) == N.PG_EINVAL
    assert call(path=N.PG_PATH_SPARSE | (2 << 8)) == N.PG_EINVAL
    assert call(ws=16) == N.PG_ENOMEM
    assert "workspace" in N.last_error()


def test_grm_workspace_and_validation():
    lib = N.load()
    g = _g(10000, 71307)
    b = ctypes.c_size_t(0)
    assert lib.pg_grm_workspace_bytes(ctypes.byref(g), 0, 0, 0, ctypes.byref(b)) == 0
    wp = -(-(-(-71307 // 16)) // 16) * 16
    # sample-major 2-bit operand, four doubles per padded variant, one mask
    # word per 16 variants (each piece aligned to 256 bytes)
    assert b.value >= 10112 * wp * 4 + wp * 16 * 32 + wp * 4
    fake = 0x2000
    g2 = _g(100, 50)

    def call(layout=N.PG_FULL, A=fake, n=fake, ws=1 << 30, path=0):
        return lib.pg_grm_matrix(ctypes.byref(g2), None, 0, 0, 0, layout, path, A, n, fake, ws,
                                 None)
    assert call(layout=7) == N.PG_EINVAL
    assert call(path=N.PG_PATH_POPC) == N.PG_EINVAL
    assert call(path=1 << 16) == N.PG_EINVAL
    assert call(A=None) == N.PG_EINVAL
    assert call(n=None) == N.PG_EINVAL
    assert call(ws=64) == N.PG_ENOMEM
    g1 = _g(1, 50)
    assert lib.pg_grm_matrix(ctypes.byref(g1), None, 0, 0, 0, N.PG_TRI_UPPER, 0, None, None, None,
                             0, None) == N.PG_OK


def test_distance_and_cluster_validation():
    lib = N.load()
    fake = 0x2000
    assert lib.pg_ibs_distance(fake, fake, fake, -1, fake, None) == N.PG_EINVAL
    assert lib.pg_ibs_distance(None, fake, fake, 10, fake, None) == N.PG_EINVAL
    assert lib.pg_ibs_distance(None, None, None, 0, None, None) == N.PG_OK
    b = ctypes.c_size_t(0)
    assert lib.pg_cluster_workspace_bytes(0, ctypes.byref(b)) == N.PG_EINVAL
    assert lib.pg_cluster_workspace_bytes(10000, ctypes.byref(b)) == N.PG_OK
    assert b.value >= 10000 * 10000 * 8 + 10000 * 12
    assert lib.pg_ibs_cluster(fake, fake, None, 100, fake, fake, 1 << 30, None) == N.PG_EINVAL
    assert lib.pg_ibs_cluster(fake, fake, fake, 100, None, fake, 1 << 30, None) == N.PG_EINVAL
    assert lib.pg_ibs_cluster(fake, fake, fake, 100, fake, fake, 1000, None) == N.PG_ENOMEM


def test_peak_rates_validation():
    lib = N.load()
    out = (ctypes.c_double * 4)()
    assert lib.pg_peak_rates(0x2000, 1 << 30, None) == N.PG_EINVAL
    assert lib.pg_peak_rates(0x2000, 1 << 20, out) == N.PG_ENOMEM
    assert lib.pg_peak_rates(None, 1 << 30, out) == N.PG_ENOMEM


def test_noalloc_rejects_oversized_before_the_device():
    """pg_ibs_matrix_noalloc refuses, on the host and before any HIP call, a
    call whose scratch would exceed the static array; the size query reports
    the array's size."""
    lib = N.load()
    b = ctypes.c_size_t(0)
    assert lib.pg_noalloc_scratch_bytes(ctypes.byref(b)) == 0 and b.value == 64 << 20
    g = _g(10000, 40000)
    fake = ctypes.c_void_p(0x1000)
    rc = lib.pg_ibs_matrix_noalloc(ctypes.byref(g), None, 0, 0, 0, N.PG_TRI_UPPER, N.PG_PATH_MFMA,
                                   fake, fake, fake, fake, None)
    assert rc == N.PG_EUNSUPPORTED
    assert "static array" in N.last_error()
    assert lib.pg_ibs_matrix_noalloc(None, None, 0, 0, 0, 0, 0, fake, fake, fake, fake,
                                     None) == N.PG_EINVAL


@pytest.mark.parametrize("m,nv", [(1, 1), (64, 5000), (500, 5000), (10000, 100000),
                                  (20000, 50000), (3, (1 << 24) + 5)])
def test_resolve_path_ibs(m, nv):
    """PG_PATH_AUTO resolves to the matrix-core path at every measured IBS
    shape, kernel variant 8 (pipelined fp4) below 2^24 variants and variant 7
    (pipelined int8: fp32 sums would no longer be exact) from there; explicit
    paths and variants pass through, undefined variants become the default."""
    lib = N.load()
    out = ctypes.c_int(-1)

    def res(path):
        assert lib.pg_resolve_path(N.PG_KIND_IBS, m, nv, 0, path, ctypes.byref(out)) == 0
        return out.value

    fp4 = nv < (1 << 24)
    default = N.PG_PATH_MFMA | ((8 if fp4 else 7) << 8)
    assert res(N.PG_PATH_AUTO) == default
    assert res(N.PG_PATH_MFMA) == default
    assert res(N.PG_PATH_MFMA | (99 << 8)) == default
    assert res(N.PG_PATH_MFMA | (9 << 8)) == N.PG_PATH_MFMA | (9 << 8)
    assert res(N.PG_PATH_MFMA | (3 << 8)) == N.PG_PATH_MFMA | ((3 if fp4 else 7) << 8)
    assert res(N.PG_PATH_POPC) == N.PG_PATH_POPC


@pytest.mark.parametrize("m,nv,w", [(1, 2, 1), (500, 20000, 50), (5000, 500000, 1000),
                                    (20000, 20000, 1000), (4999, 20000, 1000), (5000, 20000, 499),
                                    (20000, 20000, 50)])
def test_resolve_path_ld(m, nv, w):
    """LD: PG_PATH_AUTO resolves to the matrix-core path (variant 0, the
    pipelined fp4 tile), or from 5,000 samples and windows of 500 to the
    correction path with its sampled gate (variant bit 8); variant 1 is the
    int8 tile; the correction and popcount paths pass through."""
    lib = N.load()
    out = ctypes.c_int(-1)

    def res(path):
        assert lib.pg_resolve_path(N.PG_KIND_LD, m, nv, w, path, ctypes.byref(out)) == 0
        return out.value

    gated = m >= 5000 and w >= 500
    assert res(N.PG_PATH_AUTO) == (N.PG_PATH_SPARSE | (8 << 8) if gated else N.PG_PATH_MFMA)
    assert res(N.PG_PATH_MFMA | (1 << 8)) == N.PG_PATH_MFMA | (1 << 8)
    assert res(N.PG_PATH_SPARSE) == N.PG_PATH_SPARSE
    assert res(N.PG_PATH_POPC) == N.PG_PATH_POPC
    assert lib.pg_resolve_path(7, m, nv, w, 0, ctypes.byref(out)) == N.PG_EINVAL
    assert lib.pg_resolve_path(N.PG_KIND_LD, m, nv, 0, 0, ctypes.byref(out)) == N.PG_EINVAL
