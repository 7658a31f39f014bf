"""Randomised bias-force sweep against the oracle: 1, 2 and 3 CVs (the
fixed-case tests cover 2), every CV kind in every position (COM distance,
torsion, offset RMSD), walkers of uneven size, COM groups that sometimes
share atoms (the general chain rule), Gaussian and compact hills, plain and
mABP, the fused, split, chained and grid launch shapes, FP32 + Kahan and FP64."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1609_09833_amd import workloads as W
from tests.gpu_common import cv_atom_grad_abs, device, host, to_dev
from tests.tolerance import check_bound, fp32_floor, rounding_error_scales, working_coord_error

pytestmark = pytest.mark.gpu
PI = np.pi
KINDS = (W.CV_COM_DIST, W.CV_TORSION, W.CV_RMSD_OFF)


def _walkers(rng, kinds, nw):
    """nw walkers of U{40..3000} atoms in a 3 nm box; per CV the lists its kind
    needs (COM groups of 1-200 and 1-300 atoms, disjoint or sharing a few;
    4 distinct torsion atoms; 1-100 RMSD atoms with references jittered by
    U[-0.3, 0.3] nm)."""
    n_atoms = rng.integers(40, 3001, nw).astype(np.int32)
    base = np.concatenate([[0], np.cumsum(n_atoms)[:-1]]).astype(np.int64)
    total = int(n_atoms.sum())
    pos = rng.uniform(0.0, 3.0, (3, total)).astype(np.float32)
    mass = W.ATOM_MASSES[rng.integers(0, len(W.ATOM_MASSES), total)].astype(np.float32)
    D = len(kinds)
    lists = [[] for _ in range(2 * D)]
    refs = [[] for _ in range(2 * D)]
    for w in range(nw):
        n = int(n_atoms[w])
        for a, kind in enumerate(kinds):
            perm = rng.permutation(n)
            if kind == W.CV_COM_DIST:
                na = int(rng.integers(1, min(200, n // 3) + 1))
                nb = int(rng.integers(1, min(300, n // 3) + 1))
                A = np.sort(perm[:na])
                share = int(rng.integers(0, min(na, nb, 5) + 1)) if rng.random() < 0.3 else 0
                B = np.sort(np.concatenate([perm[na:na + nb - share], A[:share]]))
                two = (A, B)
            elif kind == W.CV_TORSION:
                two = (perm[:4].copy(), np.zeros(0, np.int64))
            else:
                two = (np.sort(perm[:int(rng.integers(1, min(100, n) + 1))]), np.zeros(0, np.int64))
            for t in range(2):
                lists[2 * a + t].append(two[t].astype(np.int32))
                g = base[w] + two[t]
                r = np.zeros((3, two[t].size))
                if kind == W.CV_RMSD_OFF and t == 0:
                    r = np.vstack([pos[0][g], pos[1][g], pos[2][g]]) + rng.uniform(-0.3, 0.3, (3, two[t].size))
                refs[2 * a + t].append(r)
    off = np.zeros((D, 2, nw + 1), dtype=np.int64)
    idx_chunks, ref_chunks, start = [], [], 0
    for gi in range(2 * D):
        o = W._csr(lists[gi]) + start
        off[gi // 2, gi % 2] = o
        start = int(o[-1])
        idx_chunks.extend(lists[gi])
        ref_chunks.extend(refs[gi])
    idx = np.concatenate(idx_chunks).astype(np.int32)
    ref = np.concatenate(ref_chunks, axis=1).astype(np.float32)
    return W.Walkers(n_atoms=n_atoms, atom_base=base, x=pos[0].copy(), y=pos[1].copy(), z=pos[2].copy(), mass=mass,
                     kinds=np.array(kinds, dtype=np.int32), list_off=off.astype(np.int32), list_idx=idx,
                     ref_x=ref[0].copy(), ref_y=ref[1].copy(), ref_z=ref[2].copy())


def _case(seed):
    rng = np.random.default_rng(5000 + seed)
    D = 1 + seed % 3
    kinds = tuple(int(k) for k in rng.choice(KINDS, D))
    periodic = tuple(1 if k == W.CV_TORSION else 0 for k in kinds)
    lo = tuple(-PI if k == W.CV_TORSION else 0.0 for k in kinds)
    hi = tuple(PI if k == W.CV_TORSION else (3.5 if k == W.CV_COM_DIST else 1.0) for k in kinds)
    width = tuple(float(rng.uniform(0.2, 0.6)) if k == W.CV_TORSION else
                  float(rng.uniform(0.1, 0.3) if k == W.CV_COM_DIST else rng.uniform(0.03, 0.1)) for k in kinds)
    kernel = int(rng.integers(0, 2))
    if kernel == W.KERNEL_COMPACT:
        width = tuple(2.5 * w for w in width)
    grid_n = {1: (300,), 2: (80, 70), 3: (24, 20, 18)}[D]
    spec = W.BiasSpec(ndim=D, periodic=periodic, lo=lo, hi=hi, kernel=kernel, width=width,
                      p=int(rng.integers(1, 9)), transform=int(rng.integers(0, 2)), kT=W.KT_300K, b=0.9, c=0.001,
                      grid_n=grid_n)
    nh = int(rng.choice([0, 1, 37, 500, 2000]))
    cen = np.vstack([rng.uniform(lo[i], hi[i], nh) for i in range(D)]) if nh else np.zeros((D, 0))
    hills = W.Hills(cen, rng.uniform(0.1, 1.2, nh))
    wk = _walkers(rng, kinds, int(rng.integers(1, 40)))
    shape = ("fused", "split", "chain", "grid")[(seed // 3) % 4]
    prec = int(rng.choice([0, 2]))          # ABP_PREC_FP32_KAHAN, ABP_PREC_FP64
    return spec, hills, wk, shape, prec


def _check_forces(wk, dw, ref, scale_cv, gabs, tol):
    """Per-atom bound: tol (|F*| + sum_a scale_a |ds_a/dx|); zero elsewhere."""
    F = np.stack([host(dw.fx), host(dw.fy), host(dw.fz)]).astype(np.float64)
    Fo = np.stack([ref[3], ref[4], ref[5]])
    atoms = np.array(sorted(gabs))
    scale = np.zeros((3, atoms.size))
    for k, j in enumerate(atoms):
        w = int(np.searchsorted(wk.atom_base, j, side="right") - 1)
        for a in range(wk.ncv):
            scale[:, k] += scale_cv[a, w] * gabs[j][a]
    check_bound("forces", F[:, atoms], Fo[:, atoms], scale, tol)
    mask = np.ones(F.shape[1], dtype=bool)
    mask[atoms] = False
    assert np.all(F[:, mask] == 0.0), "forces written outside the CV atoms"


@pytest.mark.parametrize("seed", range(36))
def test_random_bias_force(seed):
    device()
    from paper_1609_09833_amd import abp
    spec, hills, wk, shape, prec = _case(seed)
    ctx = abp.Context(spec, capacity=max(hills.n, 1))
    if hills.n:
        abp.bias_deposit(ctx, to_dev(hills.centers), to_dev(hills.heights))
    if shape != "grid":
        abp.abp_set_force_shape(ctx, shape)
    dw = abp.DeviceWalkers(wk)
    mode = abp.ABP_EVAL_GRID if shape == "grid" else abp.ABP_EVAL_DIRECT
    s, V, dV = abp.bias_force(ctx, dw, mode=mode, prec=prec)
    abp.abp_sync(ctx)
    z = np.zeros(wk.total_atoms)
    H = abp.abp_grid_export(ctx) if shape == "grid" else None
    ref = oracle.bias_force(spec, hills.centers, hills.heights, wk, z, z, z, use_grid=H is not None, H=H)
    assert np.all(ref[6] == 0)
    so = ref[0]
    s = host(s)
    ds = s - so
    for a in range(spec.ndim):
        if spec.periodic[a]:
            ds[a] = (ds[a] + PI) % (2 * PI) - PI
    assert np.abs(ds).max() < 1e-9, f"CVs differ by {np.abs(ds).max():.3e}"
    # bounds as in the parity tests: relative to the condition sums at the oracle's CVs
    _, _, sV, sG = oracle.bias_eval(spec, hills.centers, hills.heights, so)
    if shape == "grid":
        tol, fl, gfl = 1e-9, 0.0, 0.0
        E0, E = np.zeros_like(sV), np.zeros_like(sG)
    else:
        fp64 = prec == abp.ABP_PREC_FP64
        tol = 1e-12 if fp64 else 1e-5
        fl = 0.0 if fp64 else (fp32_floor(hills.heights) if hills.n else 0.0)
        gfl = fl * 1e4 * max(1.0, max(1.0 / w ** 2 for w in spec.width))
        unit = 2.0 ** -53 if fp64 else 2.0 ** -24
        h, dh = oracle.hill_sum(spec, hills.centers, hills.heights, so)[:2]
        slope = oracle.transform(spec, h, dh)[2]
        E0, E = rounding_error_scales(spec, hills.centers, hills.heights, so, unit, working_coord_error(spec, fp64))
        E0, E = slope * E0, slope[None, :] * E
    check_bound("V", host(V), ref[1], sV, tol, fl + E0)
    check_bound("dV/ds", host(dV), ref[2], sG, tol, gfl + E)
    # forces land in the caller's FP32 arrays: at least their output rounding
    ftol = max(tol, 1e-6)
    scale_cv = np.abs(ref[2]) + sG + (gfl + E) / tol
    _check_forces(wk, dw, ref, scale_cv, cv_atom_grad_abs(wk, so), ftol)
