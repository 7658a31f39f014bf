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


def fp32_kernel_condition(spec, centers, heights, q, snap=None, chunk=512):
    """Extra FP32 error scale of the compact kernel S_a^p (eq. compacthill).

    A term's relative rounding error in FP32 is about its condition number
    times the unit roundoff: with u = |delta|/a, d ln S / d ln u = 2p u^2/(1-u^2)^2,
    which grows without bound near the edge of the support (about 290 at
    p = 20 where S = 1e-20). Returns per query (C0, C) with
    C0 = sum_k |w_k K_k| kappa_k and C_i = sum_k |w_k dK_k/ds_i| kappa_k,
    kappa_k = sum_i 2(p + 2) u_i^2 / (1 - u_i^2)^2 (the +2 covers the
    derivative factor). Gaussian kernels: zeros. `snap(axis, x)` maps
    coordinates to grid nodes in the quantised mode.
    """
    q = np.asarray(q, dtype=np.float64)
    d, nq = q.shape
    C0 = np.zeros(nq)
    C = np.zeros((d, nq))
    if spec.kernel != 1:
        return C0, C
    c = np.asarray(centers, dtype=np.float64)
    w = np.asarray(heights, dtype=np.float64)
    if snap is not None:
        q = np.array([[snap(i, x) for x in q[i]] for i in range(d)])
        c = np.array([[snap(i, x) for x in c[i]] for i in range(d)])
    p = spec.p
    for j0 in range(0, nq, chunk):
        qq = q[:, j0:j0 + chunk]
        val = np.ones((qq.shape[1], c.shape[1]))
        der = [np.ones_like(val) for _ in range(d)]
        kappa = np.zeros_like(val)
        for i in range(d):
            delta = qq[i][:, None] - c[i][None, :]
            if spec.periodic[i]:
                L = spec.hi[i] - spec.lo[i]
                delta = delta - L * np.round(delta / L)
            a = spec.width[i]
            u = np.abs(delta) / a
            inside = u < 1.0
            om = np.where(inside, 1.0 - u * u, 1.0)
            s = np.where(inside, np.exp(p - p / om), 0.0)
            ds = np.where(inside, -2.0 * p * delta / (a * a * om * om) * s, 0.0)
            kappa += np.where(inside, 2.0 * (p + 2) * u * u / (om * om), 0.0)
            val *= s
            for k in range(d):
                der[k] *= ds if k == i else s
        C0[j0:j0 + chunk] = (np.abs(w)[None, :] * val * kappa).sum(axis=1)
        for k in range(d):
            C[k, j0:j0 + chunk] = (np.abs(w)[None, :] * np.abs(der[k]) * kappa).sum(axis=1)
    return C0, C
