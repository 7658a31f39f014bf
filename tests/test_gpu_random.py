"""Randomised parity sweep: seeded random bias definitions (dimension,
periodicity, kernel, widths, exponent p, transform, the quantised mode,
heights including zeros), ragged hill and query counts and both I/O dtypes,
every precision mode and the grid form, each against the FP64 oracle."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from paper_1609_09833_amd import workloads as W
from tests.gpu_common import device, to_dev, host
from tests.tolerance import check_bound, fp32_floor, rounding_error_scales, working_coord_error

pytestmark = pytest.mark.gpu
PI = math.pi


def _random_case(seed):
    rng = np.random.default_rng(1000 + seed)
    d = int(rng.integers(1, 4))
    periodic = tuple(int(x) for x in rng.integers(0, 2, d))
    lo, hi, width = [], [], []
    for i in range(d):
        if periodic[i]:
            lo.append(-PI); hi.append(PI)
            width.append(float(rng.uniform(0.15, 0.8)))
        else:
            a = float(rng.uniform(-2.0, 1.0)); L = float(rng.uniform(1.0, 4.0))
            lo.append(a); hi.append(a + L)
            width.append(float(rng.uniform(0.05, 0.3) * L))
    kernel = int(rng.integers(0, 2))
    if kernel == W.KERNEL_COMPACT:
        width = [w * 2.5 for w in width]
    transform = int(rng.integers(0, 2))
    grid_n = tuple(int(rng.integers(24, 72)) if d < 3 else int(rng.integers(10, 20)) for _ in range(d))
    spec = W.BiasSpec(ndim=d, periodic=periodic, lo=tuple(lo), hi=tuple(hi), kernel=kernel, width=tuple(width),
                      p=int(rng.integers(1, 21)), transform=transform, kT=W.KT_300K, b=float(rng.uniform(0.5, 0.95)),
                      c=float(10 ** rng.uniform(-3, -1)), grid_n=grid_n)
    nh = int(rng.choice([0, 1, 7, 63, 64, 65, 500, 1023, 2500]))
    nq = int(rng.choice([1, 31, 256, 257, 1000]))
    cen = np.vstack([rng.uniform(lo[i], hi[i], nh) for i in range(d)]) if nh else np.zeros((d, 0))
    hts = rng.uniform(0.0, 1.2, nh)
    hts[rng.random(nh) < 0.1] = 0.0                     # some zero-height hills
    span = [(hi[i] - lo[i]) * 0.1 for i in range(d)]
    q = np.vstack([rng.uniform(lo[i] - (0 if periodic[i] else span[i]), hi[i] + (0 if periodic[i] else span[i]), nq)
                   for i in range(d)])
    qdt = np.float32 if rng.random() < 0.5 else np.float64
    if rng.random() < 0.3:
        # the quantised mode; periodic axes get an odd node count, so that no
        # pair of nodes is exactly half a period apart (where the minimum
        # image is not unique)
        gn = tuple(n | 1 if periodic[i] else n for i, n in enumerate(grid_n))
        spec = dataclasses.replace(spec, quantize=1, grid_n=gn)
    return spec, W.Hills(cen, hts), q.astype(qdt)


@pytest.mark.parametrize("seed", range(48))
def test_random_spec_parity(seed):
    device()
    from paper_1609_09833_amd import abp
    spec, hills, q = _random_case(seed)
    ctx = abp.Context(spec, capacity=max(hills.n, 1))
    if hills.n:
        abp.bias_deposit(ctx, to_dev(hills.centers), to_dev(hills.heights))
    qd = to_dev(q)
    qq = q.astype(np.float64)
    Vo, dVo, sV, sG = oracle.bias_eval(spec, hills.centers, hills.heights, qq)
    out32 = q.dtype == np.float32
    _, _, slope = oracle.transform(spec, *oracle.hill_sum(spec, hills.centers, hills.heights, qq)[:2])
    for prec in (abp.ABP_PREC_FP32_KAHAN, abp.ABP_PREC_FP64):
        V, dV = abp.bias_eval(ctx, qd, prec=prec)
        abp.abp_sync(ctx)
        fp64 = prec == abp.ABP_PREC_FP64
        tol = (1e-6 if out32 else 1e-12) if fp64 else 1e-5 + (1e-6 if out32 else 0.0)
        # terms below the FP32 range: flushed in FP32 arithmetic or FP32 outputs
        fl = fp32_floor(hills.heights) if hills.n and (out32 or not fp64) else 0.0
        gfl = fl * 1e4 * max(1.0, max(1.0 / w ** 2 for w in spec.width))
        snap = (lambda i, x: oracle.snap(spec, i, x)) if spec.quantize else None
        E0, E = rounding_error_scales(spec, hills.centers, hills.heights, qq, 2.0 ** -53 if fp64 else 2.0 ** -24,
                                      working_coord_error(spec, fp64), snap=snap)
        got_V, got_dV = host(V), host(dV)
        check_bound(f"seed {seed} prec {prec} V", got_V, Vo, sV, tol, fl + slope * E0)
        check_bound(f"seed {seed} prec {prec} dV", got_dV, dVo, sG, tol, gfl + slope[None, :] * E)
    # the grid form against the oracle's grid and interpolation
    H = abp.abp_grid_export(ctx)
    Ho = oracle.grid_all(spec, hills.centers, hills.heights)
    np.testing.assert_allclose(H, Ho, rtol=1e-9, atol=1e-12 * max(np.abs(Ho).max(), 1e-300))
    V, dV = abp.bias_eval(ctx, qd, mode=abp.ABP_EVAL_GRID)
    abp.abp_sync(ctx)
    hq, dhq, _ = oracle.grid_eval(spec, Ho, qq)
    Vg, dVg, _ = oracle.transform(spec, hq, dhq)
    tolg = 1e-6 if out32 else 1e-9
    # a query outside every hill's support can interpolate corner values that
    # cancel: allow rounding at 1e-13 of the grid's largest entry as well
    dx = [(spec.hi[i] - spec.lo[i]) / (spec.grid_n[i] if spec.periodic[i] else spec.grid_n[i] - 1)
          for i in range(spec.ndim)]
    gscale = float(np.abs(Ho).max()) * max(1.0, max(dx)) ** spec.ndim if Ho.size else 0.0
    _, _, gslope = oracle.transform(spec, hq, dhq)
    gfloor = 1e-13 * gscale * gslope
    check_bound(f"seed {seed} grid V", host(V), Vg, sV, tolg, gfloor)
    check_bound(f"seed {seed} grid dV", host(dV), dVg, sG, tolg, gfloor[None, :] * max(1.0, max(1.0 / h for h in dx)))
    # the FP32 mirror of the node arrays: node values rounded to FP32 (2^-24 of the
    # grid's largest entry absorbs corners that cancel; value nodes enter the
    # gradient divided by the node spacing); V at 1e-6, dV at 1e-5
    V, dV = abp.bias_eval(ctx, qd, mode=abp.ABP_EVAL_GRID, prec=abp.ABP_PREC_FP32_KAHAN)
    abp.abp_sync(ctx)
    ffloor = 2.0 ** -22 * gscale * gslope
    check_bound(f"seed {seed} grid V, FP32 nodes", host(V), Vg, sV, 1e-6, ffloor)
    check_bound(f"seed {seed} grid dV, FP32 nodes", host(dV), dVg, sG, 1e-5,
                ffloor[None, :] * max(1.0, max(1.0 / h for h in dx)))
