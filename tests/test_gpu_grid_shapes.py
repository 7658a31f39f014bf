"""Grid deposits at edge shapes, against the oracle's grid.

Gaussian 2-D and 3-D grids take the matrix-core deposit (32 x 32 and
16 x 32 node tiles per wave, hills in groups of four, hill sub-ranges split
over waves and reduced in order); these cases put tile edges, ragged groups
and splits where they can go wrong: grids smaller than one tile (down to two nodes per axis) or one node
past a tile, every periodic mask, hill counts that leave a partial group,
splits whose sub-ranges are not multiples of four, and a grid built by many
small deposits (the in-place accumulation path) against one built at once.
"""
import numpy as np
import pytest

import oracle
from paper_1609_09833_amd import workloads as W
from tests.gpu_common import device, to_dev

pytestmark = pytest.mark.gpu
PI = np.pi


def _spec(ndim, periodic, grid_n, kernel=W.KERNEL_GAUSS):
    lo = tuple(-PI if p else -0.5 for p in periodic)
    hi = tuple(PI if p else 1.5 for p in periodic)
    width = tuple(0.4 if p else 0.3 for p in periodic)
    return W.BiasSpec(ndim=ndim, periodic=periodic, lo=lo, hi=hi, width=width, kernel=kernel, p=3,
                      grid_n=grid_n)


def _hills(spec, n, seed):
    rng = np.random.default_rng(seed)
    cen = np.vstack([rng.uniform(spec.lo[i], spec.hi[i], n) for i in range(spec.ndim)])
    return W.Hills(cen, rng.uniform(0.05, 1.3, n))


def _check(spec, H, hills):
    Ho = oracle.grid_all(spec, hills.centers, hills.heights)
    np.testing.assert_allclose(H, Ho, rtol=1e-9, atol=1e-12 * max(np.abs(Ho).max(), 1e-300))


CASES = [
    (2, (1, 1), (2, 3)), (2, (0, 0), (2, 2)), (2, (1, 0), (33, 2)), (2, (0, 1), (31, 65)),
    (2, (1, 1), (64, 32)), (2, (0, 0), (97, 33)),
    (3, (1, 1, 1), (2, 3, 2)), (3, (0, 0, 0), (2, 2, 2)), (3, (1, 0, 1), (33, 17, 3)),
    (3, (0, 1, 0), (32, 16, 2)), (3, (0, 0, 1), (31, 15, 5)), (3, (1, 1, 0), (65, 31, 4)),
]


@pytest.mark.parametrize("ndim,periodic,grid_n", CASES)
@pytest.mark.parametrize("n_hills", [1, 3, 5, 998])
def test_gauss_grid_edges(ndim, periodic, grid_n, n_hills):
    device()
    from paper_1609_09833_amd import abp
    spec = _spec(ndim, periodic, grid_n)
    hills = _hills(spec, n_hills, 7 * n_hills + ndim)
    ctx = abp.Context(spec, capacity=n_hills)
    abp.bias_deposit(ctx, to_dev(hills.centers), to_dev(hills.heights))
    abp.abp_sync(ctx)
    _check(spec, abp.abp_grid_export(ctx), hills)


@pytest.mark.parametrize("ndim,grid_n", [(2, (40, 24)), (3, (20, 12, 6))])
def test_split_ragged_subranges(ndim, grid_n):
    """16,387 hills on a few tiles: the deposit splits them into many
    sub-ranges, most not multiples of four, reduced in order."""
    device()
    from paper_1609_09833_amd import abp
    spec = _spec(ndim, (1,) * ndim, grid_n)
    hills = _hills(spec, 16387, 91 + ndim)
    ctx = abp.Context(spec, capacity=hills.n)
    abp.bias_deposit(ctx, to_dev(hills.centers), to_dev(hills.heights))
    abp.abp_sync(ctx)
    _check(spec, abp.abp_grid_export(ctx), hills)


@pytest.mark.parametrize("ndim,grid_n", [(2, (45, 37)), (3, (19, 17, 3))])
def test_incremental_deposits_match_one_batch(ndim, grid_n):
    """Many small deposits (one, then three, then five hills, ...) accumulate
    in place into the grid; the result matches the oracle for all hills."""
    device()
    from paper_1609_09833_amd import abp
    spec = _spec(ndim, (0,) + (1,) * (ndim - 1), grid_n)
    hills = _hills(spec, 300, 5 + ndim)
    ctx = abp.Context(spec, capacity=hills.n)
    k, step = 0, 1
    while k < hills.n:
        m = min(step, hills.n - k)
        abp.bias_deposit(ctx, to_dev(np.ascontiguousarray(hills.centers[:, k:k + m])),
                         to_dev(np.ascontiguousarray(hills.heights[k:k + m])))
        k += m
        step = step % 7 + 2
    abp.abp_sync(ctx)
    _check(spec, abp.abp_grid_export(ctx), hills)


@pytest.mark.parametrize("ndim,grid_n", [(2, (48, 40)), (3, (20, 18, 6))])
def test_quantised_gauss_grid(ndim, grid_n):
    """Quantised mode with Gaussian hills: centres snap to their nearest node
    at deposit, then take the matrix-core deposit like any Gaussian grid."""
    device()
    from paper_1609_09833_amd import abp
    import dataclasses
    spec = dataclasses.replace(_spec(ndim, (0,) + (1,) * (ndim - 1), grid_n), quantize=1)
    hills = _hills(spec, 777, 13 + ndim)
    ctx = abp.Context(spec, capacity=hills.n)
    abp.bias_deposit(ctx, to_dev(hills.centers), to_dev(hills.heights))
    abp.abp_sync(ctx)
    cen, _ = abp.abp_hills_export(ctx)
    snapped = np.array([[oracle.snap(spec, i, x) for x in hills.centers[i]] for i in range(ndim)])
    assert np.array_equal(cen, snapped)
    _check(spec, abp.abp_grid_export(ctx), hills)


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("kernel", [W.KERNEL_GAUSS, W.KERNEL_COMPACT])
def test_quantised_direct_sum_offset_grid(ndim, kernel):
    """Quantised direct sums on grids whose lower bounds are not 0: queries
    and centres snap to lo + j dx, so a node coordinate off by an ulp would
    show here. FP64 sums agree with the oracle to 1e-12; the grid look-up
    returns the oracle's node values. The periodic axes have an odd number of
    nodes: on an even one a hill exactly half a period from a query has two
    minimum images, and the two sides may pick different ones (the term's
    value agrees, its gradient changes sign)."""
    device()
    from paper_1609_09833_amd import abp
    from tests.tolerance import check_bound
    import dataclasses
    grid_n = (45, 37, 7)[:ndim]
    spec = dataclasses.replace(_spec(ndim, (0,) + (1,) * (ndim - 1), grid_n, kernel=kernel), quantize=1)
    if kernel == W.KERNEL_COMPACT:
        spec = dataclasses.replace(spec, width=tuple(4.5 * w for w in spec.width))
    hills = _hills(spec, 500, 17 + ndim + kernel)
    ctx = abp.Context(spec, capacity=hills.n)
    abp.bias_deposit(ctx, to_dev(hills.centers), to_dev(hills.heights))
    rng = np.random.default_rng(3 + ndim)
    q = np.vstack([rng.uniform(spec.lo[i], spec.hi[i], 700) for i in range(ndim)])
    V, dV = abp.bias_eval(ctx, to_dev(q), prec=abp.ABP_PREC_FP64)
    abp.abp_sync(ctx)
    Vo, dVo, sV, sG = oracle.bias_eval(spec, hills.centers, hills.heights, q)
    check_bound("quantised V", V.cpu().numpy(), Vo, sV, 1e-12)
    check_bound("quantised dV", dV.cpu().numpy(), dVo, sG, 1e-12)
    Vg, dVg = abp.bias_eval(ctx, to_dev(q), mode=abp.ABP_EVAL_GRID)
    abp.abp_sync(ctx)
    H = oracle.grid_all(spec, hills.centers, hills.heights)
    hq, dhq, _ = oracle.grid_eval(spec, H, q)
    Vq, dVq, _ = oracle.transform(spec, hq, dhq)
    check_bound("quantised look-up V", Vg.cpu().numpy(), Vq, sV, 1e-9)
    check_bound("quantised look-up dV", dVg.cpu().numpy(), dVq, sG, 1e-9)


@pytest.mark.parametrize("ndim,grid_n,quantize", [(2, (150, 100), 0), (2, (150, 100), 1), (3, (70, 40, 6), 0)])
def test_compact_deposits_refresh_the_mirror_where_they_land(ndim, grid_n, quantize):
    """Compact hills deposited one at a time (the VALU deposit marks the tiles
    it reaches, and the FP32 mirror is refreshed only there): after every
    deposit, FP32-mode evaluations (which read the mirror) must agree with
    FP64-mode evaluations (which read the node arrays) everywhere, and the
    node arrays with the oracle's grid."""
    import dataclasses
    from paper_1609_09833_amd import abp
    device()
    periodic = (1,) + (0,) * (ndim - 1)
    spec = dataclasses.replace(_spec(ndim, periodic, grid_n, kernel=W.KERNEL_COMPACT), quantize=quantize)
    hills = _hills(spec, 12, 91 + ndim)
    ctx = abp.Context(spec, capacity=hills.n)
    rng = np.random.default_rng(7)
    q = np.vstack([rng.uniform(spec.lo[i], spec.hi[i], 8192) for i in range(ndim)])
    qd = to_dev(q)
    for k in range(hills.n):
        abp.bias_deposit(ctx, to_dev(hills.centers[:, k:k + 1]), to_dev(hills.heights[k:k + 1]))
        V64, dV64 = abp.bias_eval(ctx, qd, mode=abp.ABP_EVAL_GRID, prec=abp.ABP_PREC_FP64)
        V32, dV32 = abp.bias_eval(ctx, qd, mode=abp.ABP_EVAL_GRID, prec=abp.ABP_PREC_FP32_KAHAN)
        abp.abp_sync(ctx)
        V64, dV64, V32, dV32 = (t.cpu().numpy() for t in (V64, dV64, V32, dV32))
        scale = max(np.abs(V64).max(), 1e-30)
        assert np.abs(V32 - V64).max() <= 1e-5 * scale, (k, np.abs(V32 - V64).max(), scale)
        gscale = max(np.abs(dV64).max(), 1e-30)
        assert np.abs(dV32 - dV64).max() <= 1e-4 * gscale, (k, np.abs(dV32 - dV64).max(), gscale)
    _check(spec, abp.abp_grid_export(ctx), hills)


@pytest.mark.parametrize("periodic,grid_n", [((1, 1), (2, 3)), ((0, 0), (2, 2)), ((1, 0), (33, 2)),
                                             ((0, 1), (31, 65)), ((1, 1), (64, 32))])
def test_grid_eval_ragged_batches_and_cell_edges(periodic, grid_n):
    """2-D Hermite evaluation (four lanes fetch one query's cell data and hand
    it over through LDS): batches that end inside a group of four and inside a
    wave, queries on nodes, on the upper end of a non-periodic axis and
    outside it, in both precisions and both query types, against the
    oracle's interpolation; and every query's result the same, bit for bit,
    whichever batch (and lane) it is evaluated in."""
    from paper_1609_09833_amd import abp
    from tests.tolerance import check_bound
    device()
    spec = _spec(2, periodic, grid_n)
    hills = _hills(spec, 40, 17 + grid_n[0])
    ctx = abp.Context(spec, capacity=hills.n)
    abp.bias_deposit(ctx, to_dev(hills.centers), to_dev(hills.heights))
    Ho = oracle.grid_all(spec, hills.centers, hills.heights)
    rng = np.random.default_rng(grid_n[0] * 7 + grid_n[1])
    n = 257
    q = np.vstack([rng.uniform(spec.lo[i] - 0.2, spec.hi[i] + 0.2, n) for i in range(2)])
    dx = [(spec.hi[i] - spec.lo[i]) / (grid_n[i] if periodic[i] else grid_n[i] - 1) for i in range(2)]
    for i in range(2):                   # nodes, and the upper end of the range
        q[i, :16] = spec.lo[i] + dx[i] * rng.integers(0, grid_n[i], 16)
        q[i, 16:20] = spec.hi[i]
    _, _, A0, A = oracle.hill_sum(spec, hills.centers, hills.heights, q)
    gscale = float(np.abs(Ho).max()) * max(1.0, max(dx)) ** 2
    for qdt in (np.float64, np.float32):
        qq = q.astype(qdt)
        hq, dhq, _ = oracle.grid_eval(spec, Ho, qq.astype(np.float64))
        for prec in (abp.ABP_PREC_FP64, abp.ABP_PREC_FP32_KAHAN):
            fp64 = prec == abp.ABP_PREC_FP64
            full = None
            for m in (1, 3, 5, 63, 65, 257):
                V, dV = abp.bias_eval(ctx, to_dev(qq[:, :m]), mode=abp.ABP_EVAL_GRID, prec=prec)
                abp.abp_sync(ctx)
                V, dV = V.cpu().numpy(), dV.cpu().numpy()
                if full is None or m == 257:
                    tol = (1e-9 if qdt == np.float64 else 1e-6) if fp64 else 1e-6
                    floor = (1e-13 if fp64 else 2.0 ** -22) * gscale
                    check_bound(f"grid V n={m}", V, hq[:m], A0[:m], tol, floor)
                    check_bound(f"grid dV n={m}", dV, dhq[:, :m], A[:, :m], 10 * tol,
                                floor * max(1.0, max(1.0 / h for h in dx)))
                if full is None:
                    full = abp.bias_eval(ctx, to_dev(qq), mode=abp.ABP_EVAL_GRID, prec=prec)
                    abp.abp_sync(ctx)
                    full = tuple(t.cpu().numpy() for t in full)
                assert np.array_equal(V, full[0][:m]) and np.array_equal(dV, full[1][:, :m]), (qdt, prec, m)
            # one query alone, from the middle of a group of four
            V1, dV1 = abp.bias_eval(ctx, to_dev(qq[:, 42:43].copy()), mode=abp.ABP_EVAL_GRID, prec=prec)
            abp.abp_sync(ctx)
            assert V1.cpu().numpy()[0] == full[0][42] and np.array_equal(dV1.cpu().numpy()[:, 0], full[1][:, 42])


@pytest.mark.parametrize("ndim,kernel,quantize", [(2, W.KERNEL_COMPACT, 0), (2, W.KERNEL_COMPACT, 1),
                                                  (3, W.KERNEL_COMPACT, 0), (2, W.KERNEL_GAUSS, 0)])
def test_mirror_catches_up_over_several_deposits(ndim, kernel, quantize):
    """The FP32 mirror follows every deposit: after groups of deposits (single
    hills and small batches; compact hills whose refresh rewrites only the
    tiles they reach, and Gaussian hills on the matrix cores, refreshed
    whole) with FP64 evaluations between some of them, FP32 and FP64 grid
    evaluations agree everywhere, and the node arrays match the oracle's
    grid."""
    import dataclasses
    from paper_1609_09833_amd import abp
    device()
    periodic = (1,) + (0,) * (ndim - 1)
    grid_n = (150, 100) if ndim == 2 else (70, 40, 6)
    spec = dataclasses.replace(_spec(ndim, periodic, grid_n, kernel=kernel), quantize=quantize)
    hills = _hills(spec, 30, 131 + ndim + kernel)
    ctx = abp.Context(spec, capacity=hills.n)
    rng = np.random.default_rng(11)
    qd = to_dev(np.vstack([rng.uniform(spec.lo[i], spec.hi[i], 4096) for i in range(ndim)]))
    k = 0
    for group in ((1, 2, 1), (3,), (1, 1, 1, 1), (5, 2), (1,), (4, 3, 4)):
        for m in group:
            abp.bias_deposit(ctx, to_dev(hills.centers[:, k:k + m]), to_dev(hills.heights[k:k + m]))
            k += m
            if m == 2:                   # FP64 evaluations between deposits
                abp.bias_eval(ctx, qd, mode=abp.ABP_EVAL_GRID, prec=abp.ABP_PREC_FP64)
        V64, dV64 = abp.bias_eval(ctx, qd, mode=abp.ABP_EVAL_GRID, prec=abp.ABP_PREC_FP64)
        V32, dV32 = abp.bias_eval(ctx, qd, mode=abp.ABP_EVAL_GRID, prec=abp.ABP_PREC_FP32_KAHAN)
        abp.abp_sync(ctx)
        V64, dV64, V32, dV32 = (t.cpu().numpy() for t in (V64, dV64, V32, dV32))
        scale = max(np.abs(V64).max(), 1e-30)
        assert np.abs(V32 - V64).max() <= 1e-5 * scale, (k, np.abs(V32 - V64).max(), scale)
        gscale = max(np.abs(dV64).max(), 1e-30)
        assert np.abs(dV32 - dV64).max() <= 1e-4 * gscale, (k, np.abs(dV32 - dV64).max(), gscale)
    assert k == hills.n
    _check(spec, abp.abp_grid_export(ctx), hills)
