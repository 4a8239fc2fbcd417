"""Comparison of LD records against the oracle, shared by the GPU tests.

Counts must match exactly and r^2 within 1e-12.  The two sides evaluate r^2 by
different double expressions (the oracle through means, the library from the
exact integer sums), so a pair whose r^2 lies within 1e-12 of the threshold
may be emitted by one side only; every other pair must be on both sides."""
import numpy as np

TOL = 1e-12
FIELDS = ("n", "sx", "sy", "sxx", "syy", "sxy")


def compare_records(got, ref, r2_min):
    kg = got["a"].astype(np.int64) * (1 << 32) + got["b"]
    kr = ref["a"].astype(np.int64) * (1 << 32) + ref["b"]
    assert (np.diff(kg) > 0).all(), "GPU records not in (a, b) order"
    common, ig, ir = np.intersect1d(kg, kr, return_indices=True)
    only_g = np.setdiff1d(np.arange(len(kg)), ig)
    only_r = np.setdiff1d(np.arange(len(kr)), ir)
    assert all(abs(got["r2"][k] - r2_min) <= TOL for k in only_g), got[only_g][:5]
    assert all(abs(ref["r2"][k] - r2_min) <= TOL for k in only_r), ref[only_r][:5]
    for f in FIELDS:
        assert np.array_equal(got[f][ig], ref[f][ir]), f
    d = np.abs(got["r2"][ig] - ref["r2"][ir])
    assert np.nanmax(d, initial=0.0) <= TOL
    return len(common)
