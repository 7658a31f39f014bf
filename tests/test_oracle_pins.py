"""Pins for the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a value the
paper prints (tests/golden), a closed form, an invariant, a textbook property,
or an independent numerical route (finite differences of the oracle's own
values check its analytic derivatives). A dropped term, a wrong sign, a wrong
index or a transposed operand in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1609_09833_amd import workloads as W
from tests import golden_io

PI = math.pi


def spec1(width=0.35, kernel=W.KERNEL_GAUSS, p=1, periodic=True, lo=-PI, hi=PI, transform=W.TRANSFORM_PLAIN,
          grid_n=0, **kw):
    return W.BiasSpec(ndim=1, periodic=(1 if periodic else 0,), lo=(lo,), hi=(hi,), width=(width,),
                      kernel=kernel, p=p, transform=transform, grid_n=(grid_n,), **kw)


# --------------------------------------------------------------------------
# K1: single Gaussian hill (eq. ghill with alpha = sqrt(2) sigma)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_single_gaussian_value_and_derivative(ndim):
    sig = [0.3, 0.5, 0.2][:ndim]
    c = np.array([0.1, -0.4, 1.0][:ndim])
    w = 0.7
    spec = W.BiasSpec(ndim=ndim, periodic=(1,) * ndim, lo=(-PI,) * ndim, hi=(PI,) * ndim, width=tuple(sig))
    cen = c.reshape(ndim, 1)
    # at the centre: V = w, gradient 0
    h, dh, _, _ = oracle.hill_sum(spec, cen, [w], c.reshape(ndim, 1))
    assert h[0] == pytest.approx(w, rel=1e-15)
    assert np.all(np.abs(dh) < 1e-15)
    for i in range(ndim):
        for sgn in (+1, -1):
            q = c.copy()
            q[i] += sgn * sig[i]
            h, dh, _, _ = oracle.hill_sum(spec, cen, [w], q.reshape(ndim, 1))
            assert h[0] == pytest.approx(w * math.exp(-0.5), rel=1e-14)
            # dV/ds_i at c + sigma e_i is -w e^{-1/2} / sigma
            assert dh[i, 0] == pytest.approx(-sgn * w * math.exp(-0.5) / sig[i], rel=1e-13)
            for j in range(ndim):
                if j != i:
                    assert abs(dh[j, 0]) < 1e-15
    # product over axes: one sigma along every axis gives e^{-ndim/2}
    q = c + np.array(sig)
    h, dh, _, _ = oracle.hill_sum(spec, cen, [w], q.reshape(ndim, 1))
    assert h[0] == pytest.approx(w * math.exp(-0.5 * ndim), rel=1e-14)
    for i in range(ndim):
        assert dh[i, 0] == pytest.approx(-w * math.exp(-0.5 * ndim) / sig[i], rel=1e-13)


# --------------------------------------------------------------------------
# K2: periodic wrap
# --------------------------------------------------------------------------
def test_periodic_wrap_and_symmetry():
    spec = spec1(width=0.35)
    rng = np.random.default_rng(3)
    cen = rng.uniform(-PI, PI, size=(1, 50))
    hts = rng.uniform(0.1, 1.2, size=50)
    q = rng.uniform(-PI, PI, size=(1, 20))
    h0, d0, _, _ = oracle.hill_sum(spec, cen, hts, q)
    for shift in (2 * PI, -2 * PI, 6 * PI):
        h1, d1, _, _ = oracle.hill_sum(spec, cen, hts, q + shift)
        np.testing.assert_allclose(h1, h0, rtol=1e-12)
        np.testing.assert_allclose(d1, d0, rtol=1e-9, atol=1e-12)
    # a hill just above lo and a query just below hi are 2 eps apart
    eps = 1e-3
    h, dh, _, _ = oracle.hill_sum(spec, [[-PI + eps]], [1.0], [[PI - eps]])
    assert h[0] == pytest.approx(math.exp(-(2 * eps) ** 2 / (2 * 0.35 ** 2)), rel=1e-12)
    # the query sits "below" the hill across the boundary: gradient is positive
    assert dh[0, 0] > 0
    # symmetric queries c +- delta: equal values, opposite gradients
    c = 3.0
    for dlt in (0.05, 0.2, 0.9):
        ha, da, _, _ = oracle.hill_sum(spec, [[c]], [1.0], [[c + dlt]])
        hb, db, _, _ = oracle.hill_sum(spec, [[c]], [1.0], [[c - dlt]])
        assert ha[0] == pytest.approx(hb[0], rel=1e-12)
        assert da[0, 0] == pytest.approx(-db[0, 0], rel=1e-10)


def test_wrap_is_minimum_image():
    L = 2 * PI
    for d in np.linspace(-3 * L, 3 * L, 97):
        w = oracle.wrap(d, L)
        assert -L / 2 <= w <= L / 2
        assert abs((d - w) / L - round((d - w) / L)) < 1e-12


# --------------------------------------------------------------------------
# K3: compact kernel S_a^p (eq. compacthill) and the width relations
# --------------------------------------------------------------------------
@pytest.mark.parametrize("p", [1, 2, 5, 20])
def test_compact_kernel_shape(p):
    a = 0.7
    v, d = oracle.kernel_1d(W.KERNEL_COMPACT, a, p, 0.0)
    assert v == pytest.approx(1.0, rel=1e-15)
    assert d == 0.0
    for x in (a, -a, 1.3 * a, -5 * a):
        v, d = oracle.kernel_1d(W.KERNEL_COMPACT, a, p, x)
        assert v == 0.0 and d == 0.0
    # half height at w_a / 2 = a sqrt(ln2 / (p + ln2))
    half = a * math.sqrt(math.log(2) / (p + math.log(2)))
    v, _ = oracle.kernel_1d(W.KERNEL_COMPACT, a, p, half)
    assert v == pytest.approx(0.5, rel=1e-13)
    # symmetric, strictly decreasing on (0, a), derivative -> 0 at the edge
    xs = np.linspace(0, a, 2001)[1:-1]
    vals = np.array([oracle.kernel_1d(W.KERNEL_COMPACT, a, p, x)[0] for x in xs])
    assert np.all(np.diff(vals) <= 0)
    big = vals > 1e-280                    # beyond that the double exponent underflows
    assert np.all(np.diff(vals[big]) < 0)
    for x in xs[::100]:
        assert oracle.kernel_1d(W.KERNEL_COMPACT, a, p, -x)[0] == oracle.kernel_1d(W.KERNEL_COMPACT, a, p, x)[0]
    _, dedge = oracle.kernel_1d(W.KERNEL_COMPACT, a, p, a * (1 - 1e-4))
    assert abs(dedge) < 1e-100


def test_compact_kernel_worked_example_from_paper():
    """a = 18, p = 1: the Gaussian with the same half-height width has alpha = 13.833."""
    g = golden_io.read("showhill.txt")
    a, p, alpha_paper = g["a"], int(g["p"]), g["alpha"]
    # half-height point of the oracle's compact kernel, found by bisection
    lo, hi = 0.0, a
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if oracle.kernel_1d(W.KERNEL_COMPACT, a, p, mid)[0] > 0.5:
            lo = mid
        else:
            hi = mid
    w_a = 2 * lo
    alpha = w_a / (2 * math.sqrt(math.log(2)))
    assert round(alpha, 3) == alpha_paper
    # the oracle's Gaussian with alpha = sqrt(2) sigma is at half height at w_a / 2
    sigma = alpha_paper / math.sqrt(2)
    v, _ = oracle.kernel_1d(W.KERNEL_GAUSS, sigma, 1, w_a / 2)
    assert v == pytest.approx(0.5, abs=5e-5)     # alpha is printed to 5 digits


def test_compact_kernel_support_node_count():
    """With a = 10 grid spacings, a node-aligned hill touches 19 nodes per axis (strict '<')."""
    n = 480
    spec = W.BiasSpec(ndim=1, periodic=(0,), lo=(0.0,), hi=(12.0,), width=(10 * 12.0 / (n - 1),),
                      kernel=W.KERNEL_COMPACT, p=20, grid_n=(n,))
    c = oracle.grid_coord(spec, 0, 240)
    H = oracle.grid_nodes(spec, [[c]], [1.0], np.arange(n))
    assert int(np.count_nonzero(H[:, 0])) == 19


def test_compact_derivative_matches_finite_difference():
    a, p = 0.9, 3
    for x in (-0.8, -0.3, 0.05, 0.4, 0.85):
        _, d = oracle.kernel_1d(W.KERNEL_COMPACT, a, p, x)
        hstep = 1e-6
        fd = (oracle.kernel_1d(W.KERNEL_COMPACT, a, p, x + hstep)[0]
              - oracle.kernel_1d(W.KERNEL_COMPACT, a, p, x - hstep)[0]) / (2 * hstep)
        assert d == pytest.approx(fd, rel=1e-6, abs=1e-12)


# --------------------------------------------------------------------------
# K4: equally spaced hills on the circle (Poisson summation closed form)
# --------------------------------------------------------------------------
def lattice_closed_form(n, sigma, s_minus_s0):
    """sum_k exp(-(s - s0 - k D)^2 / (2 sigma^2)) over all integers k, D = 2 pi / n."""
    D = 2 * PI / n
    tot = 1.0
    for m in range(1, 50):
        tot += 2 * math.exp(-2 * PI ** 2 * m ** 2 * sigma ** 2 / D ** 2) * math.cos(2 * PI * m * s_minus_s0 / D)
    return sigma * math.sqrt(2 * PI) / D * tot


def test_lattice_sum_closed_form_1d():
    spec, hills, q = W.lattice_1d(n_hills=2000, sigma=0.35, n_queries=64)
    h, dh, _, _ = oracle.hill_sum(spec, hills.centers, hills.heights, q)
    expect = 279.25959628100287
    assert lattice_closed_form(2000, 0.35, 0.123) == pytest.approx(expect, rel=1e-15)
    np.testing.assert_allclose(h, expect, rtol=1e-13)
    assert np.abs(dh).max() < 1e-9 * expect
    # a coarse lattice, where the cosine terms matter
    spec, hills, q = W.lattice_1d(n_hills=12, sigma=0.35, n_queries=32)
    h, dh, _, _ = oracle.hill_sum(spec, hills.centers, hills.heights, q)
    s0 = -PI
    ex = np.array([lattice_closed_form(12, 0.35, qq - s0) for qq in q[0]])
    np.testing.assert_allclose(h, ex, rtol=1e-12)


def test_lattice_sum_closed_form_2d_tensor():
    n0, n1 = 40, 30
    sig = (0.35, 0.4)
    g0 = -PI + 2 * PI / n0 * np.arange(n0)
    g1 = -PI + 2 * PI / n1 * np.arange(n1)
    c0, c1 = np.meshgrid(g0, g1, indexing="ij")
    cen = np.vstack([c0.ravel(), c1.ravel()])
    spec = W.BiasSpec(ndim=2, periodic=(1, 1), lo=(-PI, -PI), hi=(PI, PI), width=sig)
    rng = np.random.default_rng(5)
    q = rng.uniform(-PI, PI, size=(2, 16))
    h, dh, _, _ = oracle.hill_sum(spec, cen, np.full(cen.shape[1], 0.5), q)
    ex = np.array([0.5 * lattice_closed_form(n0, sig[0], a + PI) * lattice_closed_form(n1, sig[1], b + PI)
                   for a, b in q.T])
    np.testing.assert_allclose(h, ex, rtol=1e-12)


# --------------------------------------------------------------------------
# K5: co-located hills sum their heights exactly (correctly rounded reference)
# --------------------------------------------------------------------------
def test_colocated_hills_sum_heights():
    n = 50000
    heights = W.decaying_height(np.arange(n))
    spec = W.BiasSpec(ndim=2, periodic=(1, 1), lo=(-PI, -PI), hi=(PI, PI), width=(0.3, 0.3))
    c = np.array([[0.25], [-1.5]])
    cen = np.repeat(c, n, axis=1)
    h, dh, A0, _ = oracle.hill_sum(spec, cen, heights, c)
    exact = math.fsum(heights.tolist())
    assert h[0] == pytest.approx(exact, rel=2e-16)
    # geometric-series closed form of 1.2 exp(-k/20000), k < 50000
    closed = 1.2 * (1 - math.exp(-2.5)) / (1 - math.exp(-1 / 20000))
    assert closed == pytest.approx(22030.510786598672, rel=1e-15)
    assert h[0] == pytest.approx(closed, rel=1e-11)
    assert A0[0] == pytest.approx(h[0], rel=1e-15)
    assert np.all(dh == 0)


# --------------------------------------------------------------------------
# Condition sums A0 = sum |w K| and A_i = sum |w dK/ds_i| (eq. histos taken in
# absolute value): closed forms for hills away from the query, where K < 1,
# and a symmetric pair whose gradients cancel while A_i does not.
# --------------------------------------------------------------------------
def _kernel_closed(kernel, width, p, delta):
    """1-D kernel value and derivative d/ds written out from eq. ghill (sigma
    form) and eq. compacthill, independent of the oracle's kernel routine."""
    if kernel == W.KERNEL_GAUSS:
        v = math.exp(-delta * delta / (2.0 * width * width))
        return v, -delta / (width * width) * v
    u2 = (delta / width) ** 2
    if u2 >= 1.0:
        return 0.0, 0.0
    v = math.exp(p) * math.exp(-p / (1.0 - u2))
    return v, -2.0 * p * delta / (width * width * (1.0 - u2) ** 2) * v


@pytest.mark.parametrize("kernel", [W.KERNEL_GAUSS, W.KERNEL_COMPACT])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_condition_sums_closed_forms(kernel, ndim):
    width = ((0.3, 0.25, 0.4) if kernel == W.KERNEL_GAUSS else (0.9, 0.7, 1.1))[:ndim]
    p = 4
    spec = W.BiasSpec(ndim=ndim, periodic=(1, 0, 1)[:ndim], lo=(-PI, -2.0, -PI)[:ndim], hi=(PI, 3.0, PI)[:ndim],
                      width=width, kernel=kernel, p=p)
    q = np.array([0.2, 0.5, -1.0][:ndim])
    off = np.array([0.21, -0.17, 0.33][:ndim])          # K < 1 on every axis
    w = 0.8
    # one hill off the query: A0 = w K, A_i = |w dK/ds_i|
    cen = (q - off).reshape(ndim, 1)
    h, dh, A0, A = oracle.hill_sum(spec, cen, [w], q.reshape(ndim, 1))
    vals = [_kernel_closed(kernel, width[i], p, off[i]) for i in range(ndim)]
    K = math.prod(v for v, _ in vals)
    assert K < 0.9
    assert h[0] == pytest.approx(w * K, rel=1e-14)
    assert A0[0] == pytest.approx(w * K, rel=1e-14)
    for i in range(ndim):
        g = w * vals[i][1] * math.prod(vals[j][0] for j in range(ndim) if j != i)
        assert dh[i, 0] == pytest.approx(g, rel=1e-13)
        assert A[i, 0] == pytest.approx(abs(g), rel=1e-13)
        assert A[i, 0] != pytest.approx(w * K, rel=1e-3)   # |w dK| differs from |w K| here
    # two hills at q -+ off: the gradients cancel, A_i is twice one hill's
    cen = np.hstack([(q - off).reshape(ndim, 1), (q + off).reshape(ndim, 1)])
    h, dh, A0, A = oracle.hill_sum(spec, cen, [w, w], q.reshape(ndim, 1))
    assert h[0] == pytest.approx(2 * w * K, rel=1e-14)
    assert A0[0] == pytest.approx(2 * w * K, rel=1e-14)
    for i in range(ndim):
        g = w * vals[i][1] * math.prod(vals[j][0] for j in range(ndim) if j != i)
        assert abs(dh[i, 0]) <= 1e-14 * abs(g)
        assert A[i, 0] == pytest.approx(2 * abs(g), rel=1e-13)
    # unequal heights at unequal distances along axis 0: A0 = sum w_k K_k
    d2 = off.copy()
    d2[0] *= 1.7
    cen = np.hstack([(q - off).reshape(ndim, 1), (q + d2).reshape(ndim, 1)])
    h, dh, A0, A = oracle.hill_sum(spec, cen, [w, 0.3], q.reshape(ndim, 1))
    vals2 = [_kernel_closed(kernel, width[i], p, -d2[i]) for i in range(ndim)]
    K2 = math.prod(v for v, _ in vals2)
    assert A0[0] == pytest.approx(w * K + 0.3 * K2, rel=1e-14)
    g1 = w * vals[0][1] * math.prod(vals[j][0] for j in range(1, ndim))
    g2 = 0.3 * vals2[0][1] * math.prod(vals2[j][0] for j in range(1, ndim))
    assert dh[0, 0] == pytest.approx(g1 + g2, rel=1e-12, abs=1e-15)
    assert A[0, 0] == pytest.approx(abs(g1) + abs(g2), rel=1e-13)


# --------------------------------------------------------------------------
# K6: mABP transform (eq. apfm and eq. btraj-grad)
# --------------------------------------------------------------------------
def test_mabp_gradient_is_derivative_of_potential():
    g = golden_io.read("mabp_params.txt")
    kT = 0.0083144626 * g["T"]
    spec = W.BiasSpec(ndim=2, periodic=(1, 1), lo=(-PI, -PI), hi=(PI, PI), width=(0.3, 0.4),
                      transform=W.TRANSFORM_MABP, kT=kT, b=g["b"], c=g["c"])
    rng = np.random.default_rng(11)
    cen = rng.uniform(-PI, PI, size=(2, 300))
    hts = np.ones(300) * 50.0
    q = rng.uniform(-PI, PI, size=(2, 10))
    V, dV, _, _ = oracle.bias_eval(spec, cen, hts, q)
    step = 1e-6
    for i in range(2):
        e = np.zeros((2, 1))
        e[i] = step
        Vp, _, _, _ = oracle.bias_eval(spec, cen, hts, q + e)
        Vm, _, _, _ = oracle.bias_eval(spec, cen, hts, q - e)
        np.testing.assert_allclose(dV[i], (Vp - Vm) / (2 * step), rtol=1e-6, atol=1e-10)
    # the definition written out
    h, dh, _, _ = oracle.hill_sum(spec, cen, hts, q)
    b, c = g["b"], g["c"]
    np.testing.assert_allclose(V, kT * b / (1 - b) * np.log(c * (1 - b) * h + 1), rtol=1e-12)


def test_mabp_limits():
    spec = spec1(width=0.3, transform=W.TRANSFORM_MABP, kT=2.5, b=0.9, c=1e-9)
    # c -> 0: V -> kT b c h (linear in the histogram, metadynamics-like)
    h, _, _, _ = oracle.hill_sum(spec, [[0.0]], [3.0], [[0.1]])
    V, _, _, _ = oracle.bias_eval(spec, [[0.0]], [3.0], [[0.1]])
    assert V[0] / (2.5 * 0.9 * 1e-9 * h[0]) == pytest.approx(1.0, rel=1e-8)
    # h = 0 gives V = 0 and zero gradient
    V, dV, _, _ = oracle.bias_eval(spec, [[0.0]], [0.0], [[0.1]])
    assert V[0] == 0.0 and dV[0, 0] == 0.0


# --------------------------------------------------------------------------
# Derivatives of the direct sum against finite differences (brute force)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kernel,ndim", [(W.KERNEL_GAUSS, 1), (W.KERNEL_GAUSS, 2), (W.KERNEL_GAUSS, 3),
                                         (W.KERNEL_COMPACT, 2), (W.KERNEL_COMPACT, 3)])
def test_direct_sum_gradient_matches_finite_difference(kernel, ndim):
    rng = np.random.default_rng(17 + ndim)
    periodic = (1, 0, 1)[:ndim]
    lo = (-PI, 0.0, -PI)[:ndim]
    hi = (PI, 1.5, PI)[:ndim]
    width = ((0.3, 0.1, 0.35) if kernel == W.KERNEL_GAUSS else (0.9, 0.3, 1.0))[:ndim]
    spec = W.BiasSpec(ndim=ndim, periodic=periodic, lo=lo, hi=hi, width=width, kernel=kernel, p=3)
    n = 200
    cen = np.vstack([rng.uniform(l, h, size=n) for l, h in zip(lo, hi)])
    hts = rng.uniform(0.1, 1.2, size=n)
    q = np.vstack([rng.uniform(l, h, size=8) for l, h in zip(lo, hi)])
    h, dh, _, _ = oracle.hill_sum(spec, cen, hts, q)
    step = 1e-6
    for i in range(ndim):
        e = np.zeros((ndim, 1))
        e[i] = step
        hp, _, _, _ = oracle.hill_sum(spec, cen, hts, q + e)
        hm, _, _, _ = oracle.hill_sum(spec, cen, hts, q - e)
        np.testing.assert_allclose(dh[i], (hp - hm) / (2 * step), rtol=1e-6, atol=1e-8)


# --------------------------------------------------------------------------
# K7: grid node arrays and Hermite interpolation
# --------------------------------------------------------------------------
def test_grid_node_arrays_are_derivatives_of_the_sum():
    """H_m at a node equals the mixed derivative of the direct sum (finite differences)."""
    rng = np.random.default_rng(23)
    spec = W.BiasSpec(ndim=3, periodic=(0, 1, 1), lo=(0.0, -PI, -PI), hi=(1.2, PI, PI),
                      width=(0.1, 0.3, 0.35), grid_n=(7, 9, 8))
    cen = np.vstack([rng.uniform(0, 1.2, 60), rng.uniform(-PI, PI, 60), rng.uniform(-PI, PI, 60)])
    hts = rng.uniform(0.1, 1.2, 60)
    ids = np.array([0, 5, 77, 200, 7 * 9 * 8 - 1])
    H = oracle.grid_nodes(spec, cen, hts, ids)
    step = 1e-4
    for t, nid in enumerate(ids):
        j0, rem = nid % 7, nid // 7
        j1, j2 = rem % 9, rem // 9
        x = np.array([oracle.grid_coord(spec, 0, j0), oracle.grid_coord(spec, 1, j1),
                      oracle.grid_coord(spec, 2, j2)])
        for m in range(8):
            # finite-difference mixed derivative over the axes set in m
            axes = [i for i in range(3) if (m >> i) & 1]
            acc = 0.0
            for signs in np.ndindex(*([2] * len(axes))):
                pt = x.copy()
                sgn = 1.0
                for a, sbit in zip(axes, signs):
                    pt[a] += step if sbit == 0 else -step
                    sgn *= 1.0 if sbit == 0 else -1.0
                hv, _, _, _ = oracle.hill_sum(spec, cen, hts, pt.reshape(3, 1))
                acc += sgn * hv[0]
            fd = acc / (2 * step) ** len(axes)
            scale = np.abs(H[t]).max()
            assert H[t, m] == pytest.approx(fd, rel=1e-5, abs=1e-6 * scale)


def test_hermite_reproduces_tensor_cubics():
    """Tensor-product cubic Hermite interpolation is exact for products of cubics."""
    rng = np.random.default_rng(29)
    for ndim in (1, 2, 3):
        coef = rng.normal(size=(ndim, 4))
        n = (6, 5, 4)[:ndim]
        spec = W.BiasSpec(ndim=ndim, periodic=(0,) * ndim, lo=(-1.0, 0.5, 2.0)[:ndim], hi=(1.0, 2.0, 3.5)[:ndim],
                          width=(1.0,) * ndim, grid_n=n)

        def f1(i, x, der):
            c = coef[i]
            return (c[1] + 2 * c[2] * x + 3 * c[3] * x * x) if der else (c[0] + c[1] * x + c[2] * x * x + c[3] * x ** 3)

        total = int(np.prod(n))
        H = np.zeros((total, 1 << ndim))
        for nid in range(total):
            rem = nid
            xs = []
            for i in range(ndim):
                xs.append(oracle.grid_coord(spec, i, rem % n[i]))
                rem //= n[i]
            for m in range(1 << ndim):
                v = 1.0
                for i in range(ndim):
                    v *= f1(i, xs[i], (m >> i) & 1)
                H[nid, m] = v
        q = np.vstack([rng.uniform(spec.lo[i], spec.hi[i], 50) for i in range(ndim)])
        h, dh, ncl = oracle.grid_eval(spec, H, q)
        assert ncl == 0
        ex = np.ones(50)
        for i in range(ndim):
            ex = ex * f1(i, q[i], False)
        np.testing.assert_allclose(h, ex, rtol=1e-12, atol=1e-12)
        for k in range(ndim):
            exd = np.ones(50)
            for i in range(ndim):
                exd = exd * f1(i, q[i], i == k)
            np.testing.assert_allclose(dh[k], exd, rtol=1e-11, atol=1e-11)


def test_grid_interpolation_at_nodes_and_error_bound():
    """At nodes the interpolant equals the direct sum; between nodes it obeys the
    cubic Hermite bounds (dx^4/384) max|f''''| and (sqrt(3)/216) dx^3 max|f''''|."""
    sigma, w = 0.3, 0.8
    n = 96
    spec = W.BiasSpec(ndim=1, periodic=(1,), lo=(-PI,), hi=(PI,), width=(sigma,), grid_n=(n,))
    cen = [[0.4321]]
    H = oracle.grid_all(spec, cen, [w])
    nodes = np.array([[oracle.grid_coord(spec, 0, j) for j in range(n)]])
    h, dh, _ = oracle.grid_eval(spec, H, nodes)
    hd, dhd, _, _ = oracle.hill_sum(spec, cen, [w], nodes)
    np.testing.assert_allclose(h, hd, rtol=1e-14, atol=1e-15 * w)
    np.testing.assert_allclose(dh, dhd, rtol=1e-12, atol=1e-13 * w / sigma)
    dx = 2 * PI / n
    f4 = 3 * w / sigma ** 4
    q = np.linspace(-PI, PI, 5001)[None, :-1]
    h, dh, _ = oracle.grid_eval(spec, H, q)
    hd, dhd, _, _ = oracle.hill_sum(spec, cen, [w], q)
    assert np.abs(h - hd).max() <= dx ** 4 / 384 * f4
    assert np.abs(dh - dhd).max() <= math.sqrt(3) / 216 * dx ** 3 * f4
    # and the bound is not vacuous: the observed error is within 10x of it
    assert np.abs(h - hd).max() > dx ** 4 / 384 * f4 / 10


def test_grid_clamps_out_of_range_queries():
    spec = W.BiasSpec(ndim=1, periodic=(0,), lo=(0.0,), hi=(1.0,), width=(0.2,), grid_n=(11,))
    H = oracle.grid_all(spec, [[0.5]], [1.0])
    h, dh, ncl = oracle.grid_eval(spec, H, [[-0.5, 0.0, 1.0, 1.7]])
    assert ncl == 2
    assert h[0] == pytest.approx(h[1], rel=1e-15) and h[3] == pytest.approx(h[2], rel=1e-15)


# --------------------------------------------------------------------------
# Collective variables: K9 invariants, K10 RMSD, torsion geometry
# --------------------------------------------------------------------------
def test_torsion_known_geometries():
    def build(theta):
        # b2 along z; atom 1 along +x from atom 2, atom 4 rotated by theta about z
        return np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 1.5],
                         [math.cos(theta), math.sin(theta), 1.5]])
    assert oracle.torsion(build(0.0))[0] == pytest.approx(0.0, abs=1e-15)         # cis
    assert abs(oracle.torsion(build(PI))[0]) == pytest.approx(PI, rel=1e-15)      # trans
    for th in (PI / 2, -PI / 2, 1.0, -2.5):
        phi, _ = oracle.torsion(build(th))
        # IUPAC sign: looking along b2 (2 -> 3), a clockwise turn of the far bond
        # from the near bond is positive. With b2 = +z, rotating atom 4 by +theta
        # counter-clockwise about +z seen from above is clockwise seen along +z.
        assert phi == pytest.approx(th, abs=1e-13)


def test_torsion_gradient_fd_and_invariants():
    rng = np.random.default_rng(31)
    for _ in range(20):
        x4 = rng.normal(size=(4, 3))
        phi, g = oracle.torsion(x4)
        fd = np.zeros((4, 3))
        step = 1e-6
        for a in range(4):
            for c in range(3):
                xp = x4.copy(); xp[a, c] += step
                xm = x4.copy(); xm[a, c] -= step
                dp = oracle.torsion(xp)[0] - oracle.torsion(xm)[0]
                dp = (dp + PI) % (2 * PI) - PI
                fd[a, c] = dp / (2 * step)
        np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-7)
        np.testing.assert_allclose(g.sum(axis=0), 0.0, atol=1e-12)
        torque = np.cross(x4, g).sum(axis=0)
        np.testing.assert_allclose(torque, 0.0, atol=1e-11)


def test_com_distance_gradient_and_invariants():
    rng = np.random.default_rng(37)
    xa, xb = rng.uniform(0, 6, (50, 3)), rng.uniform(0, 6, (200, 3))
    ma, mb = rng.choice(W.ATOM_MASSES, 50), rng.choice(W.ATOM_MASSES, 200)
    d, ga, gb = oracle.com_distance(xa, ma, xb, mb)
    RA = (ma[:, None] * xa).sum(0) / ma.sum()
    RB = (mb[:, None] * xb).sum(0) / mb.sum()
    assert d == pytest.approx(np.linalg.norm(RA - RB), rel=1e-13)
    np.testing.assert_allclose(ga.sum(0) + gb.sum(0), 0.0, atol=1e-14)
    np.testing.assert_allclose(ga.sum(0), (RA - RB) / d, rtol=1e-12)
    step = 1e-6
    for (arr, g, idx) in ((xa, ga, 3), (xb, gb, 17)):
        for c in range(3):
            arr[idx, c] += step
            dp = oracle.com_distance(xa, ma, xb, mb)[0]
            arr[idx, c] -= 2 * step
            dm = oracle.com_distance(xa, ma, xb, mb)[0]
            arr[idx, c] += step
            assert g[idx, c] == pytest.approx((dp - dm) / (2 * step), rel=1e-5, abs=1e-10)
    # translation invariance
    d2, _, _ = oracle.com_distance(xa + 1.7, ma, xb + 1.7, mb)
    assert d2 == pytest.approx(d, rel=1e-12)


def test_rmsd_offset_definition():
    g = golden_io.read("rmsd_offset.txt")
    rng = np.random.default_rng(41)
    x0 = rng.uniform(0, 3, (8, 3))
    r, grad = oracle.rmsd_off(x0, x0)
    assert r == pytest.approx(g["lower_bound"], rel=1e-15)
    assert np.all(grad == 0)
    for dlt in (0.05, 0.3, 1.0):
        r, _ = oracle.rmsd_off(x0 + dlt, x0)
        assert r == pytest.approx(math.sqrt(3 * dlt * dlt + g["offset"]), rel=1e-14)
    x = x0 + rng.normal(scale=0.2, size=x0.shape)
    r, grad = oracle.rmsd_off(x, x0)
    step = 1e-6
    for a in range(8):
        for c in range(3):
            xp = x.copy(); xp[a, c] += step
            xm = x.copy(); xm[a, c] -= step
            fd = (oracle.rmsd_off(xp, x0)[0] - oracle.rmsd_off(xm, x0)[0]) / (2 * step)
            assert grad[a, c] == pytest.approx(fd, rel=1e-6, abs=1e-10)


# --------------------------------------------------------------------------
# K8: bias forces against finite differences of V(s(x))
# --------------------------------------------------------------------------
def _tiny_walkers(kinds):
    wk = W.ligand_pocket_walkers(seed=3, n_walkers=2, atoms_lo=300, atoms_hi=400, ligand=(6, 9), pocket=(10, 14))
    if kinds == "rmsd":
        wk = W.rmsd_walkers(seed=4, n_walkers=2, n_atoms=50, cv_atoms=4)
    for name in ("x", "y", "z", "mass", "ref_x", "ref_y", "ref_z"):
        setattr(wk, name, getattr(wk, name).astype(np.float64))
    return wk


@pytest.mark.parametrize("kinds,transform,use_grid", [("com_tors", W.TRANSFORM_PLAIN, False),
                                                      ("com_tors", W.TRANSFORM_MABP, False),
                                                      ("rmsd", W.TRANSFORM_MABP, False),
                                                      ("com_tors", W.TRANSFORM_PLAIN, True)])
def test_forces_match_finite_differences(kinds, transform, use_grid):
    wk = _tiny_walkers(kinds)
    rng = np.random.default_rng(43)
    if kinds == "rmsd":
        spec = W.BiasSpec(ndim=2, periodic=(0, 0), lo=(0.0, 0.0), hi=(1.5, 1.5), width=(0.1, 0.12),
                          transform=transform, grid_n=(64, 64))
        cen = rng.uniform(0.05, 0.6, size=(2, 300))
    else:
        spec = W.BiasSpec(ndim=2, periodic=(0, 1), lo=(0.0, -PI), hi=(4.0, PI), width=(0.1, 0.3),
                          transform=transform, grid_n=(161, 64))
        cen = np.vstack([rng.uniform(0.0, 3.0, 600), rng.uniform(-PI, PI, 600)])
    spec.kT, spec.b, spec.c = 2.494, 0.9, 0.01
    hts = rng.uniform(0.1, 1.2, cen.shape[1]) * (50 if transform == W.TRANSFORM_MABP else 1)
    H = oracle.grid_all(spec, cen, hts) if use_grid else None
    N = wk.total_atoms
    zeros = np.zeros(N)
    s, V, dV, fx, fy, fz, st = oracle.bias_force(spec, cen, hts, wk, zeros, zeros, zeros, use_grid=use_grid, H=H)
    assert np.all(st == 0)
    touched = np.unique(np.concatenate([wk.atom_base[w] + wk.list_idx[wk.list_off[a, sl, w]:wk.list_off[a, sl, w + 1]]
                                        for w in range(wk.nw) for a in range(wk.ncv) for sl in range(2)]))
    step = 1e-6
    for g in touched[:: max(1, len(touched) // 12)]:
        w = int(np.searchsorted(wk.atom_base, g, side="right") - 1)
        for arr_name, F in (("x", fx), ("y", fy), ("z", fz)):
            arr = getattr(wk, arr_name)
            arr[g] += step
            Vp = oracle.bias_force(spec, cen, hts, wk, zeros, zeros, zeros, use_grid=use_grid, H=H)[1][w]
            arr[g] -= 2 * step
            Vm = oracle.bias_force(spec, cen, hts, wk, zeros, zeros, zeros, use_grid=use_grid, H=H)[1][w]
            arr[g] += step
            fd = -(Vp - Vm) / (2 * step)
            assert F[g] == pytest.approx(fd, rel=2e-5, abs=1e-7 * (1 + abs(dV[:, w]).max()))
    if kinds == "com_tors":
        # COM-distance and torsion forces sum to zero per walker
        for w in range(wk.nw):
            sl = slice(wk.atom_base[w], wk.atom_base[w] + wk.n_atoms[w])
            np.testing.assert_allclose([fx[sl].sum(), fy[sl].sum(), fz[sl].sum()], 0.0,
                                       atol=1e-11 * (1 + np.abs(dV[:, w]).max()))


def test_bias_force_flags_bad_walkers():
    wk = _tiny_walkers("com_tors")
    spec = W.BiasSpec(ndim=2, periodic=(0, 1), lo=(0.0, -PI), hi=(4.0, PI), width=(0.1, 0.3))
    cen, hts = np.array([[0.5], [0.0]]), np.array([1.0])
    N = wk.total_atoms
    z = np.zeros(N)
    # out-of-range index in walker 1's pocket list
    bad = W.Walkers(**{k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in wk.__dict__.items()})
    bad.list_idx[bad.list_off[0, 1, 1]] = bad.n_atoms[1] + 5
    st = oracle.bias_force(spec, cen, hts, bad, z, z, z)[6]
    assert list(st) == [0, oracle.ORC_E_INDEX]
    # non-finite position of a ligand atom in walker 0
    bad = W.Walkers(**{k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in wk.__dict__.items()})
    bad.x[bad.atom_base[0] + bad.list_idx[bad.list_off[0, 0, 0]]] = np.nan
    out = oracle.bias_force(spec, cen, hts, bad, z, z, z)
    assert list(out[6]) == [oracle.ORC_E_NONFINITE, 0]
    assert np.isnan(out[1][0]) and np.isfinite(out[1][1])


# --------------------------------------------------------------------------
# Quantised mode: the CV value is replaced by its nearest grid node before
# the update (text before eq. update); the force is a look-up at that node
# (eq. btraj-grad at xi*). The paper's discretisation: 480 x 480 nodes over
# [0, 12] nm, compact hills with a = 10 node spacings.
# --------------------------------------------------------------------------
PAPER_DX = 12.0 / 479


def paper_grid_spec(**kw):
    base = dict(ndim=2, periodic=(0, 0), lo=(0.0, 0.0), hi=(12.0, 12.0), kernel=W.KERNEL_COMPACT,
                width=(10 * PAPER_DX, 10 * PAPER_DX), p=20, grid_n=(480, 480), quantize=1)
    base.update(kw)
    return W.BiasSpec(**base)


def test_snap_is_the_nearest_node():
    spec = paper_grid_spec()
    rng = np.random.default_rng(31)
    xs = rng.uniform(0.0, 12.0, 2000)
    nodes = np.arange(480) * PAPER_DX
    for x in xs:
        j = oracle.snap_index(spec, 0, x)
        best = np.abs(nodes - x).min()
        assert abs(nodes[j] - x) <= best + 1e-12            # brute force over every node
        assert oracle.snap(spec, 0, x) == pytest.approx(nodes[j], abs=1e-12)
    # outside the range: the edge nodes
    assert oracle.snap_index(spec, 0, -3.0) == 0 and oracle.snap_index(spec, 0, 40.0) == 479
    # exactly halfway goes to the upper node (node spacing 1 makes the midpoint exact)
    half = W.BiasSpec(ndim=1, periodic=(0,), lo=(0.0,), hi=(10.0,), grid_n=(11,), quantize=1)
    assert oracle.snap_index(half, 0, 2.5) == 3 and oracle.snap_index(half, 0, 2.4999999) == 2
    # periodic axis: nearest node under the wrap
    per = W.BiasSpec(ndim=1, periodic=(1,), lo=(-PI,), hi=(PI,), grid_n=(256,), quantize=1)
    d = 2 * PI / 256
    assert oracle.snap_index(per, 0, PI - 0.1 * d) == 0
    assert oracle.snap_index(per, 0, -PI - 0.6 * d) == 255
    assert oracle.snap_index(per, 0, -PI + 3.4 * d) == 3


def test_quantised_look_up_3d():
    """The look-up indexes a 3-D grid with mixed periodicity correctly."""
    spec = W.BiasSpec(ndim=3, periodic=(0, 1, 1), lo=(0.0, -PI, -PI), hi=(1.2, PI, PI), width=(0.25, 0.9, 1.1),
                      kernel=W.KERNEL_COMPACT, p=2, grid_n=(13, 10, 8), quantize=1)
    rng = np.random.default_rng(33)
    cen = np.vstack([rng.uniform(0.1, 1.1, 25), rng.uniform(-PI, PI, (2, 25))])
    w = rng.uniform(0.5, 1.5, 25)
    q = np.vstack([rng.uniform(0.0, 1.2, 200), rng.uniform(-PI, PI, (2, 200))])
    H = oracle.grid_all(spec, cen, w)
    hg, dhg, _ = oracle.grid_eval(spec, H, q)
    hs, dhs, A0, A = oracle.hill_sum(spec, cen, w, q)
    np.testing.assert_allclose(hg, hs, rtol=1e-12, atol=1e-14 * A0.max())
    np.testing.assert_allclose(dhg, dhs, rtol=1e-12, atol=1e-14 * A.max())


def test_quantised_look_up_equals_sum_at_the_node():
    """Grid arrays at xi* equal the direct sum of the node-centred hills at xi*,
    and the sum at a point equals a brute-force sum built from the 1-D kernel."""
    spec = paper_grid_spec(grid_n=(60, 50), width=(10 * 12.0 / 59, 10 * 12.0 / 49), p=4)
    rng = np.random.default_rng(32)
    cen = rng.uniform(3.0, 9.0, (2, 40))
    w = rng.uniform(0.5, 1.5, 40)
    q = rng.uniform(2.0, 10.0, (2, 300))
    H = oracle.grid_all(spec, cen, w)
    hg, dhg, _ = oracle.grid_eval(spec, H, q)
    hs, dhs, A0, A = oracle.hill_sum(spec, cen, w, q)
    np.testing.assert_allclose(hg, hs, rtol=1e-12, atol=1e-14 * A0.max())
    np.testing.assert_allclose(dhg, dhs, rtol=1e-12, atol=1e-14 * A.max())
    dxs = (12.0 / 59, 12.0 / 49)
    node = lambda x, i: np.floor(x / dxs[i] + 0.5) * dxs[i]
    for j in range(0, 300, 37):
        v = 0.0
        for k in range(40):
            f0 = oracle.kernel_1d(spec.kernel, spec.width[0], spec.p, node(q[0, j], 0) - node(cen[0, k], 0))[0]
            f1 = oracle.kernel_1d(spec.kernel, spec.width[1], spec.p, node(q[1, j], 1) - node(cen[1, k], 1))[0]
            v += w[k] * f0 * f1
        assert hs[j] == pytest.approx(v, rel=1e-12, abs=1e-14)


def test_quantised_hill_stencil_is_nbase_squared():
    """A deposit off the nodes is moved to its node, so it touches 19 x 19
    nodes with a = 10 spacings (eq. Cupdate runs only over those)."""
    spec = paper_grid_spec()
    ids = np.arange(480 * 480)
    for c in ([[5.0], [6.0]], [[5.0 + 0.37 * PAPER_DX], [6.0 - 0.21 * PAPER_DX]]):
        H = oracle.grid_nodes(spec, c, [1.0], ids)
        assert int(np.count_nonzero(H[:, 0])) == 19 * 19
        j0, j1 = oracle.snap_index(spec, 0, c[0][0]), oracle.snap_index(spec, 1, c[1][0])
        assert H[j0 + 480 * j1, 0] == 1.0                   # S(0) = 1 at the hill's own node


# --------------------------------------------------------------------------
# Well-tempered heights w0 exp(-V/dT) (WTmetaD's hill-height factor)
# --------------------------------------------------------------------------
def test_wt_height_closed_forms():
    spec = W.BiasSpec(ndim=2, periodic=(1, 1), lo=(-PI, -PI), hi=(PI, PI), width=(0.3, 0.3))
    c = np.array([[0.4], [-1.0]])
    # empty history: the full height
    assert oracle.wt_heights(spec, np.zeros((2, 0)), np.zeros(0), c, 0.7, 2.5)[0] == 0.7
    # one hill of height w at the same point: V = w
    assert oracle.wt_heights(spec, c, [1.3], c, 0.7, 2.5)[0] == pytest.approx(0.7 * math.exp(-1.3 / 2.5), rel=1e-14)
    # one sigma away on one axis: V = w e^(-1/2)
    c1 = np.array([[0.4 + 0.3], [-1.0]])
    assert oracle.wt_heights(spec, c, [1.3], c1, 0.7, 2.5)[0] == pytest.approx(
        0.7 * math.exp(-1.3 * math.exp(-0.5) / 2.5), rel=1e-13)


def test_wt_repeated_deposits_follow_the_log_law():
    """Deposits at one point, one per step: V_{n+1} = V_n + w0 exp(-V_n/dT),
    whose continuous limit is V(n) = dT ln(1 + n w0 / dT); dT -> infinity gives
    plain metadynamics, V = n w0."""
    spec = W.BiasSpec(ndim=1, periodic=(1,), lo=(-PI,), hi=(PI,), width=(0.35,))
    c = np.array([[0.25]])
    for dT, n, rel in ((2.5, 400, 2e-2), (1e12, 50, 1e-9)):
        cen, hts = np.zeros((1, 0)), np.zeros(0)
        for _ in range(n):
            w = oracle.wt_heights(spec, cen, hts, c, 0.05, dT)[0]
            cen, hts = np.hstack([cen, c]), np.append(hts, w)
        V = hts.sum()
        expect = dT * math.log1p(n * 0.05 / dT) if dT < 1e6 else n * 0.05
        assert V == pytest.approx(expect, rel=rel)
