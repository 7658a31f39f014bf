"""Acceptance bounds for GPU results against the FP64 oracle.

Relative tolerance 1e-5, measured against the scale the sum itself sets:
for V, |V - V*| <= tol max(|V*|, T' A0) and for each gradient component
|g - g*| <= tol max(|g*|, T' A_i), where A0 = sum |w K| and A_i = sum |w dK/ds_i|
are the oracle's condition sums and T' = dV/dh is the transform slope. For a
plain bias with positive heights A0 = V*, so the first bound is plain relative
error 1e-5 (and for mABP V* >= T' A0, so it is relative error in V); since
T' A_i >= |g*| the second is tol T' A_i, the componentwise bound of a
compensated sum, which stays meaningful where the gradient crosses zero.

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
    lim = tol * np.maximum(np.abs(want), scale) + floor
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
    """max |got - want| / max(|want|, scale), the quantity the bound limits."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    den = np.maximum(np.abs(want), np.asarray(scale, dtype=np.float64))
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


def working_coord_error(spec, fp64):
    """Per-axis model of how the working form of the coordinates moves a
    displacement d_i = q_i - c_i, as (absolute, relative) pairs: the error of
    d_i is absolute + relative (|q_i| + |c_i|).

    FP32 sums: every coordinate is a 32-bit fixed-point word, rounded to half
    a step: a period in 2^32 steps on a periodic axis, the window
    [lo - E, hi + E] (E = max((hi - lo)/2, 16 width)) in 2^31 steps otherwise.
    FP64 sums: a periodic coordinate becomes a fraction of the period, rounded
    to 2^-53 of a turn; a non-periodic one stays as given (no rounding) and
    the subtraction rounds at 2^-53 of the operands.
    """
    out = []
    for i in range(spec.ndim):
        L = spec.hi[i] - spec.lo[i]
        if fp64:
            out.append((2.0 ** -52 * L, 0.0) if spec.periodic[i] else (0.0, 2.0 ** -53))
        elif spec.periodic[i]:
            out.append((L * 2.0 ** -32, 0.0))
        else:
            E = max(0.5 * L, 16.0 * spec.width[i])
            out.append(((L + 2.0 * E) * 2.0 ** -31, 0.0))
    return out


def rounding_error_scales(spec, centers, heights, q, unit, coord_err, snap=None, chunk=256):
    """Absolute error estimates (E0 for h, E_i for dh/ds_i) of a sum whose
    terms are evaluated in a format with unit roundoff `unit`, from the
    conditioning of each term, before the transform:

      * the exponent: a relative error `unit` in the exponent's argument
        changes a term by |argument| * unit; the argument is
        |ln w| + sum_i d_i^2/(2 sigma_i^2) (Gaussian) or
        |ln w| + sum_i p u_i^2/(1 - u_i^2) with u = |d|/a (compact), and
        the compact argument's own sensitivity to u adds 2p u^2/(1-u^2)^2;
      * the coordinates: the working form moves d_i by
        abs_i + rel_i (|q_i| + |c_i|), with (abs_i, rel_i) = coord_err[i]
        (working_coord_error), which changes the value by that times
        |dK/dd_i| and the gradient by that times |d^2K/dd_i^2|.

    Each term's estimate is multiplied by 4 (several roundings per term).
    Returns (E0[nq], E[ndim][nq]).
    """
    q = np.asarray(q, dtype=np.float64)
    d, nq = q.shape
    c = np.asarray(centers, dtype=np.float64).reshape(d, -1)
    w = np.asarray(heights, dtype=np.float64)
    E0 = np.zeros(nq)
    E = np.zeros((d, nq))
    if w.size == 0:
        return E0, E
    if snap is not None:
        q = np.array([[snap(i, x) for x in q[i]] for i in range(d)])
        c = np.array([[snap(i, x) for x in c[i]] for i in range(d)])
    p = spec.p
    lnw = np.abs(np.log(np.where(w > 0, w, 1.0)))[None, :]
    for j0 in range(0, nq, chunk):
        qq = q[:, j0:j0 + chunk]
        m = qq.shape[1]
        val = np.ones((m, c.shape[1]))
        arg = np.tile(lnw, (m, 1))
        dlog = []          # d ln K / d d_i per axis
        d2 = []            # (d^2 K / d d_i^2) / K per axis
        ecoord = []
        for i in range(d):
            delta = qq[i][:, None] - c[i][None, :]
            if spec.periodic[i]:
                L = spec.hi[i] - spec.lo[i]
                delta = delta - L * np.round(delta / L)
            ea, er = coord_err[i]
            ec = ea + er * (np.abs(qq[i])[:, None] + np.abs(c[i])[None, :])
            a = spec.width[i]
            if spec.kernel == 0:
                s = np.exp(-0.5 * (delta / a) ** 2)
                arg = arg + 0.5 * (delta / a) ** 2
                g = -delta / a ** 2
                h2 = (delta ** 2 / a ** 2 - 1.0) / a ** 2
            else:
                u = np.abs(delta) / a
                inside = u < 1.0
                om = np.where(inside, 1.0 - u * u, 1.0)
                s = np.where(inside, np.exp(-p * u * u / om), 0.0)
                arg = arg + np.where(inside, p * u * u / om + 2.0 * p * u * u / (om * om), 0.0)
                g = np.where(inside, -2.0 * p * delta / (a * a * om * om), 0.0)
                h2 = np.where(inside, g * g + np.abs(2.0 * p * (1.0 + 3.0 * u * u) / (a * a * om ** 3)), 0.0)
            val = val * s
            dlog.append(g)
            d2.append(np.abs(h2))
            ecoord.append(ec)
        wk = np.abs(w)[None, :] * val
        rel = unit * arg
        E0[j0:j0 + m] = 4.0 * (wk * (rel + sum(np.abs(dlog[i]) * ecoord[i] for i in range(d)))).sum(axis=1)
        for k in range(d):
            gk = wk * np.abs(dlog[k])
            extra = sum((d2[i] if i == k else np.abs(dlog[i]) * np.abs(dlog[k])) * ecoord[i] for i in range(d))
            E[k, j0:j0 + m] = 4.0 * (gk * rel + wk * extra).sum(axis=1)
    return E0, E
