"""Acceptance bounds for GPU results against the FP64 oracle.

Relative tolerance 1e-5, measured against the scale the sum itself sets:
for V, |V - V*| <= tol (|V*| + T' A0) and for each gradient component
|g - g*| <= tol (|g*| + T' A_i), where A0 = sum |w K| and A_i = sum |w dK/ds_i|
are the oracle's condition sums and T' = dV/dh is the transform slope. For a
plain bias with positive heights the first bound is plain relative error; the
second is the componentwise bound of a compensated sum, which stays
meaningful where the gradient crosses zero.

When the path computes in FP64 but returns FP32 outputs, the bound is the
output rounding (1e-6 covers 2^-24 relative). FP32 arithmetic also gets an
absolute floor for hill terms below the FP32 normal range (fp32_floor).
"""
import numpy as np

TOL = 1e-5


def fp32_floor(heights):
    """Absolute floor for FP32 arithmetic: each hill term below the smallest
    normal FP32 number (2^-126, times its height) may be flushed to zero."""
    h = np.asarray(heights, dtype=np.float64)
    return float(h.size * (np.abs(h).max() if h.size else 0.0) * 2.0 ** -126)


def check_bound(name, got, want, scale, tol=TOL, floor=0.0):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    scale = np.asarray(scale, dtype=np.float64)
    err = np.abs(got - want)
    lim = tol * (np.abs(want) + scale) + floor
    bad = ~(err <= lim)
    if bad.any():
        i = np.flatnonzero(bad.ravel())[0]
        raise AssertionError(
            f"{name}: {bad.sum()} of {bad.size} outside tolerance; first at flat index {i}: "
            f"got {got.ravel()[i]!r}, want {want.ravel()[i]!r}, err {err.ravel()[i]:.3e}, "
            f"limit {lim.ravel()[i]:.3e}")
    ratio = err / np.where(lim > 0, lim, 1.0)
    return float(ratio.max()) if ratio.size else 0.0


def rel_err(got, want, scale):
    """max |got - want| / (|want| + scale), the quantity the bound limits."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    den = np.abs(want) + np.asarray(scale, dtype=np.float64)
    den = np.where(den > 0, den, 1.0)
    return float(np.max(np.abs(got - want) / den)) if got.size else 0.0
