"""GPU tests of the serving loop (abp_server_*): continuous batching of
bias-force requests from many walkers sharing one hill history.

A request carries the positions of a walker's CV atoms for one MD step and
returns the bias force on them (the per-step exchange of the paper's
"Minimization of Interprocess Communications"). Every request is re-evaluated
by the oracle on the host at the history version it saw (the first `version`
hills of the exported history), with the positions that were submitted: s,
V, dV/ds and the force on every CV atom must agree to the same bounds as a
direct bias_force call. Deposits must land in the slots they report, with the
reported CV value as centre and the height law's height, and the grid the
commits built must equal the oracle's grid of the final history.
"""
import threading
import time

import numpy as np
import pytest

from paper_1609_09833_amd import workloads as W
from tests.gpu_common import device, cv_atom_grad_abs
from tests.tolerance import check_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    device()
    from paper_1609_09833_amd import abp as _abp
    return _abp


@pytest.fixture(scope="module")
def drv(lib):
    from paper_1609_09833_amd.examples import serve_driver
    return serve_driver


AMP = 2.0 ** -7          # nm, exact in float32
N_WALKERS = 48
N_HILLS = 5000


def _setup(lib, n_hills=N_HILLS, capacity_extra=4096):
    import torch
    spec, hills = W.ligand_pocket_hills(seed=3, n_hills=n_hills)
    wk = W.ligand_pocket_walkers(seed=5, n_walkers=N_WALKERS)
    ctx = lib.Context(spec, n_hills + capacity_extra)
    lib.bias_deposit(ctx, torch.tensor(hills.centers, dtype=torch.float64, device="cuda"),
                     torch.tensor(hills.heights, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    return spec, hills, wk, ctx


def _register(srv, wk):
    ids, ncv = [], []
    for w in range(wk.nw):
        b, n = int(wk.atom_base[w]), int(wk.n_atoms[w])
        lens, idx, rx, ry, rz = W.walker_lists(wk, w)
        wid, nc = srv.add_walker(wk.mass[b:b + n], lens, idx, rx, ry, rz)
        ids.append(wid)
        ncv.append(nc)
        atoms = srv.walker_atoms(wid)
        assert np.array_equal(atoms, np.unique(idx)) and nc == atoms.size
    assert ids == list(range(wk.nw))
    return np.array(ncv)


def _cv_budget(lib, ncv, fraction):
    return lib.ABP_SERVER_BYTES_PER_ATOM * int(ncv.astype(np.int64).sum() * fraction)


def _oracle_request(spec, centers, heights, wk, w, atoms, xyz, version, H=None):
    """The oracle's bias force for walker w with its CV atoms at xyz ([3][n_cv]),
    over the first `version` hills (or interpolated from their grid H): (s, V,
    dV, forces on the CV atoms [3][n_cv], A0, A, per-atom force scale [3][n_cv])."""
    from oracle import bias_eval, bias_force
    b, n = int(wk.atom_base[w]), int(wk.n_atoms[w])
    x, y, z = (np.asarray(a[b:b + n], dtype=np.float32).copy() for a in (wk.x, wk.y, wk.z))
    k = atoms.size
    x[atoms], y[atoms], z[atoms] = xyz[:k], xyz[k:2 * k], xyz[2 * k:3 * k]
    one = W.single_walker(wk, w, x, y, z)
    zero = np.zeros(n)
    c, h = centers[:, :version], heights[:version]
    s, V, dV, fx, fy, fz, status = bias_force(spec, c, h, one, zero, zero, zero, use_grid=H is not None, H=H)
    assert status[0] == 0
    _, _, sA0, sA = bias_eval(spec, c, h, s)
    F = np.stack([fx[atoms], fy[atoms], fz[atoms]])
    gabs = cv_atom_grad_abs(one, s)
    scale = np.zeros((3, k))
    for j, at in enumerate(atoms):
        g = gabs[int(at)]                                  # [ncv, 3]
        for a in range(wk.ncv):
            scale[:, j] += np.maximum(np.abs(dV[a, 0]), sA[a, 0]) * g[a]
    return s[:, 0], V[0], dV[:, 0], F, sA0[0], sA[:, 0], scale


def _wrap(d):
    return (d + np.pi) % (2 * np.pi) - np.pi


def _check_request(name, spec, centers, heights, wk, srv, r, w, xyz, version, s, V, dV, F, H=None):
    """One served request against the oracle: the direct sum at 1e-5, or (H
    given) the interpolation of the grid of its version at 1e-9 (forces, being
    FP32, at 1e-6)."""
    atoms = srv.walker_atoms(w)
    s_o, V_o, dV_o, F_o, A0, A, fscale = _oracle_request(spec, centers, heights, wk, w, atoms, xyz, version, H)
    ds = s - s_o
    for a in range(spec.ndim):
        if spec.periodic[a]:
            ds[a] = _wrap(ds[a])
    assert np.abs(ds).max() < 1e-12, (name, r, ds)
    tol = 1e-5 if H is None else 1e-9
    rv = check_bound(f"{name} V (request {r})", np.array([V]), np.array([V_o]), np.array([A0]), tol)
    rg = check_bound(f"{name} dV/ds (request {r})", dV, dV_o, A, tol)
    # forces are FP32: at least their output rounding
    rf = check_bound(f"{name} forces (request {r})", F.reshape(3, -1), F_o, fscale, tol=max(tol, 1e-6), floor=0.0)
    return max(rv, rg, rf)


def test_serving_with_deposits_matches_oracle(lib, drv):
    """Batched, evicting, depositing replay through submit/poll: every request's
    s, V, dV/ds and forces against the oracle, deposits in order, and the grid
    built by the commits (on two streams) equal to the oracle's."""
    import oracle
    spec, hills, wk, ctx = _setup(lib)
    srv = lib.Server(ctx, wk.kinds, hbm_budget_bytes=1 << 20, max_batch=16, streams=2, deposit_every=3,
                     height0=1.2, height_decay=20000.0, max_pending=256)
    ncv = _register(srv, wk)
    srv.close()
    # about a third of the walkers' CV atoms fit
    srv = lib.Server(ctx, wk.kinds, hbm_budget_bytes=_cv_budget(lib, ncv, 1 / 3), max_batch=16, streams=2,
                     deposit_every=3, height0=1.2, height_decay=20000.0, max_pending=256)
    _register(srv, wk)
    eng = drv.Engines(srv, wk)
    srv.start()
    # 120 ms of arrivals: walkers go idle between their requests, so they are evicted and admitted again
    t, w, step = W.serving_requests(seed=1, n_walkers=N_WALKERS, rate=5_000.0, n_requests=600)
    print(f"serving replay: {len(t)} requests, {N_WALKERS} walkers", flush=True)
    out = drv.replay(srv, eng, w, step, t, AMP)
    srv.stop()
    st = srv.stats()
    n = len(t)
    assert st["completed"] == n == st["submitted"]
    assert st["evictions"] > 0 and st["admissions"] > N_WALKERS
    assert st["max_batch_seen"] <= 16 and st["batches"] >= n // 16
    assert np.all(np.isfinite(out["t_done"])) and np.all(out["t_done"] >= out["t_submit"])
    tr = srv.trace()
    assert tr.size == st["batches"] and tr["requests"].sum() == n
    assert np.all(tr["t_formed"] <= tr["t_launched"]) and np.all(tr["t_launched"] <= tr["t_done"])
    # deposits: one per request whose step is a positive multiple of 3, slots dense after the seed hills
    dep = out["deposit_slot"]
    want_dep = (step % 3) == 0
    assert np.array_equal(dep >= 0, want_dep)
    slots = np.sort(dep[dep >= 0])
    assert np.array_equal(slots, np.arange(N_HILLS, N_HILLS + slots.size))
    assert ctx.num_hills == N_HILLS + slots.size == N_HILLS + st["deposits"]
    # versions: seed hills at least, never a request's own deposit, non-decreasing per walker
    ver = out["version"]
    assert np.all(ver >= N_HILLS) and np.all(ver <= ctx.num_hills)
    assert np.all(ver[dep >= 0] <= dep[dep >= 0])
    for wi in range(N_WALKERS):
        v = ver[w == wi]
        assert np.all(np.diff(v) >= 0)
    centers, heights = lib.abp_hills_export(ctx)
    assert np.array_equal(centers[:, :N_HILLS], hills.centers)
    for r in np.flatnonzero(dep >= 0):
        k = int(dep[r])
        assert np.array_equal(centers[:, k], out["s"][:, r])
        assert abs(heights[k] - 1.2 * np.exp(-k / 20000.0)) <= 1e-15 * heights[k]
    # every request against the oracle, forces included
    worst = 0.0
    for r in range(n):
        o, k3 = int(out["offset"][r]), 3 * int(eng.n_cv[w[r]])
        worst = max(worst, _check_request("served", spec, centers, heights, wk, srv, r, int(w[r]),
                                          out["positions"][o:o + k3], int(ver[r]), out["s"][:, r], out["V"][r],
                                          out["dVds"][:, r], out["forces"][o:o + k3]))
    print(f"served requests: worst error / bound {worst:.3e}")
    # the grid the serial commits built equals the oracle's grid of the final history
    H = lib.abp_grid_export(ctx)
    Ho = oracle.grid_all(spec, centers, heights)
    np.testing.assert_allclose(H, Ho, rtol=1e-9, atol=1e-12 * np.abs(Ho).max())
    srv.close()
    ctx.close()


def test_serving_grid_with_deposits_matches_oracle(lib, drv):
    """GRID evaluation: batches read one copy of the grid while the commits of
    the requests' deposits go into the other on their own stream; every
    request must equal the oracle's interpolation of the grid of exactly its
    version, the context's grid must hold every hill after stop, and a restart
    must see hills deposited from outside in between."""
    import dataclasses
    import oracle
    import torch
    spec, hills = W.ligand_pocket_hills(seed=3, n_hills=1000)
    spec = dataclasses.replace(spec, grid_n=(64, 64))
    wk = W.ligand_pocket_walkers(seed=5, n_walkers=N_WALKERS)
    ctx = lib.Context(spec, hills.n + 1024)
    lib.bias_deposit(ctx, torch.tensor(hills.centers, device="cuda"), torch.tensor(hills.heights, device="cuda"))
    torch.cuda.synchronize()
    probe = lib.Server(ctx, wk.kinds)
    ncv = _register(probe, wk)
    probe.close()
    srv = lib.Server(ctx, wk.kinds, hbm_budget_bytes=_cv_budget(lib, ncv, 1 / 3), max_batch=48, streams=2,
                     deposit_every=3, height0=1.2, height_decay=20000.0, eval_mode=lib.ABP_EVAL_GRID)
    _register(srv, wk)
    eng = drv.Engines(srv, wk)
    srv.start()
    # bursts: batches both within and above the 16 requests whose fields ride in the kernel arguments
    t, w, step = W.serving_requests(seed=7, n_walkers=N_WALKERS, rate=60_000.0, n_requests=400)
    out = drv.replay(srv, eng, w, step, t, AMP)
    srv.stop()
    st = srv.stats()
    assert st["completed"] == len(t) and st["evictions"] > 0 and st["deposits"] > 0
    tr = srv.trace()
    print(f"batch sizes: max {tr['requests'].max()}, batches above 16: {(tr['requests'] > 16).sum()}")
    dep = out["deposit_slot"]
    assert np.array_equal(dep >= 0, (step % 3) == 0)
    ver = out["version"]
    for wi in range(N_WALKERS):                 # a walker never sees an older grid
        assert np.all(np.diff(ver[w == wi]) >= 0)
    assert np.unique(ver).size >= 2             # the copies took turns
    assert ctx.num_hills == 1000 + st["deposits"]
    centers, heights = lib.abp_hills_export(ctx)
    grids = {}
    worst = 0.0
    for r in range(len(t)):
        v = int(out["version"][r])
        if v not in grids:
            grids[v] = oracle.grid_all(spec, centers[:, :v], heights[:v])
        o, k3 = int(out["offset"][r]), 3 * int(eng.n_cv[w[r]])
        worst = max(worst, _check_request("grid served", spec, centers, heights, wk, srv, r, int(w[r]),
                                          out["positions"][o:o + k3], v, out["s"][:, r], out["V"][r],
                                          out["dVds"][:, r], out["forces"][o:o + k3], H=grids[v]))
    print(f"grid-served requests: {len(grids)} versions, worst error / bound {worst:.3e}")
    H = lib.abp_grid_export(ctx)
    Ho = oracle.grid_all(spec, centers, heights)
    np.testing.assert_allclose(H, Ho, rtol=1e-9, atol=1e-12 * np.abs(Ho).max())
    # hills from outside between two runs: both copies start from them
    rng = np.random.default_rng(17)
    outside = np.stack([rng.uniform(0.2, 1.0, 64), rng.uniform(-np.pi, np.pi, 64)])
    lib.bias_deposit(ctx, torch.tensor(outside, device="cuda"), torch.tensor(np.full(64, 2.0), device="cuda"))
    torch.cuda.synchronize()
    n0 = ctx.num_hills
    srv.start()
    t2, w2, step2 = W.serving_requests(seed=8, n_walkers=N_WALKERS, rate=60_000.0, n_requests=200)
    out2 = drv.replay(srv, eng, w2, step2, t2, AMP)
    srv.stop()
    assert np.all(out2["version"] >= n0)
    centers, heights = lib.abp_hills_export(ctx)
    grids = {}
    for r in range(0, len(t2), 5):
        v = int(out2["version"][r])
        if v not in grids:
            grids[v] = oracle.grid_all(spec, centers[:, :v], heights[:v])
        o, k3 = int(out2["offset"][r]), 3 * int(eng.n_cv[w2[r]])
        _check_request("grid served after restart", spec, centers, heights, wk, srv, r, int(w2[r]),
                       out2["positions"][o:o + k3], v, out2["s"][:, r], out2["V"][r], out2["dVds"][:, r],
                       out2["forces"][o:o + k3], H=grids[v])
    np.testing.assert_allclose(lib.abp_grid_export(ctx), oracle.grid_all(spec, centers, heights), rtol=1e-9,
                               atol=1e-12 * np.abs(Ho).max())
    srv.close()
    ctx.close()


def test_serving_alone_equals_in_the_mix(lib, drv):
    """Without deposits a request's s, V, dV/ds and forces are bitwise the same
    whether it ran alone (one request per launch, one stream) or inside mixed
    batches on three streams, with DIRECT and with GRID evaluation."""
    spec, hills, wk, ctx = _setup(lib)
    t, w, step = W.serving_requests(seed=2, n_walkers=N_WALKERS, rate=100_000.0, n_requests=400)
    res = []
    for mb, ns, mode in ((1, 1, lib.ABP_EVAL_DIRECT), (64, 3, lib.ABP_EVAL_DIRECT), (1, 1, lib.ABP_EVAL_GRID),
                         (64, 3, lib.ABP_EVAL_GRID)):
        srv = lib.Server(ctx, wk.kinds, hbm_budget_bytes=1 << 30, max_batch=mb, streams=ns, deposit_every=0,
                         eval_mode=mode)
        _register(srv, wk)
        eng = drv.Engines(srv, wk)
        srv.start()
        print(f"replay max_batch={mb} streams={ns}", flush=True)
        out = drv.replay(srv, eng, w, step, t, AMP)
        srv.stop()
        out["stats"] = srv.stats()
        res.append(out)
        srv.close()
    for alone, mix in (res[:2], res[2:]):
        assert alone["stats"]["max_batch_seen"] == 1
        assert mix["stats"]["batches"] < alone["stats"]["batches"]
        for k in ("s", "V", "dVds", "forces", "positions"):
            assert np.array_equal(alone[k], mix[k]), k
        assert np.all(np.isfinite(alone["forces"]))
        assert np.all(alone["version"] == N_HILLS) and np.all(mix["version"] == N_HILLS)
        assert np.all(alone["deposit_slot"] == -1)
    assert not np.array_equal(res[0]["V"], res[2]["V"])          # direct sum and grid differ
    ctx.close()


def test_serving_live_submit_and_poll(lib):
    """Engines in host threads submit each step's CV-atom positions as it
    arrives and a poller collects results while others are on the GPU; every
    result, forces included, against the oracle."""
    spec, hills, wk, ctx = _setup(lib)
    srv = lib.Server(ctx, wk.kinds, hbm_budget_bytes=1 << 30, max_batch=8, streams=2, deposit_every=5,
                     height0=1.0, max_pending=64)
    ncv = _register(srv, wk)
    srv.start()
    rng = np.random.default_rng(9)
    n_threads, per_thread = 4, 40
    sent = {}                                      # request id -> (walker, step, xyz, force_out)
    lock = threading.Lock()
    errors = []

    def engine(tid):
        try:
            walkers = list(range(tid, wk.nw, n_threads))
            steps = {wi: 1 for wi in walkers}
            for k in range(per_thread):
                wi = walkers[k % len(walkers)]
                atoms = srv.walker_atoms(wi)
                b = int(wk.atom_base[wi])
                base = np.concatenate([wk.x[b + atoms], wk.y[b + atoms], wk.z[b + atoms]]).astype(np.float32)
                xyz = base + np.float32(AMP) * rng_local[tid].uniform(-1, 1, base.size).astype(np.float32)
                fo = np.full(base.size, np.nan, dtype=np.float32)
                while True:
                    try:
                        rid = srv.submit(wi, steps[wi], xyz, fo)
                        break
                    except lib.AbpError as e:
                        if e.status != lib.ABP_E_BUSY:
                            raise
                        time.sleep(1e-4)
                with lock:
                    sent[rid] = (wi, steps[wi], xyz, fo)
                steps[wi] += 1
                time.sleep(float(rng_local[tid].exponential(2e-4)))
        except Exception as e:                     # surfaced by the main thread
            errors.append(e)

    rng_local = [np.random.default_rng(100 + i) for i in range(n_threads)]
    threads = [threading.Thread(target=engine, args=(i,)) for i in range(n_threads)]
    for th in threads:
        th.start()
    got = []
    total = n_threads * per_thread
    deadline = time.time() + 60
    while len(got) < total and time.time() < deadline and not errors:
        res = srv.poll(256, wait_us=2000)
        got.extend(res.tolist())
    for th in threads:
        th.join()
    assert not errors, errors
    srv.stop()
    got.extend(srv.poll(4096).tolist())
    assert len(got) == total
    names = lib.SERVER_RESULT.names
    centers, heights = lib.abp_hills_export(ctx)
    worst = 0.0
    for row in got:
        r = dict(zip(names, row))
        wi, stp, xyz, fo = sent[r["request"]]
        assert r["walker"] == wi and r["step"] == stp and r["n_cv_atoms"] == ncv[wi]
        assert (r["deposit_slot"] >= 0) == (stp % 5 == 0)
        worst = max(worst, _check_request("live", spec, centers, heights, wk, srv, r["request"], wi, xyz,
                                          int(r["version"]), np.array(r["s"][:2]), r["V"], np.array(r["dVds"][:2]),
                                          fo))
    print(f"live requests: worst error / bound {worst:.3e}")
    srv.close()
    ctx.close()


def test_serving_rejects_bad_input(lib):
    spec, hills, wk, ctx = _setup(lib, n_hills=100, capacity_extra=16)
    with pytest.raises(lib.AbpError):
        lib.Server(ctx, [W.CV_TORSION, W.CV_TORSION])         # torsion on a non-periodic axis
    with pytest.raises(lib.AbpError):
        lib.Server(ctx, wk.kinds, max_batch=0)
    with pytest.raises(lib.AbpError):
        lib.Server(ctx, wk.kinds, max_pending=0)
    import dataclasses
    import torch
    nogrid = lib.Context(dataclasses.replace(spec, grid_n=(0, 0)), 16)
    with pytest.raises(lib.AbpError):
        lib.Server(nogrid, wk.kinds, eval_mode=lib.ABP_EVAL_GRID)   # GRID needs a grid
    nogrid.close()
    small = lib.Server(ctx, wk.kinds, hbm_budget_bytes=lib.ABP_SERVER_BYTES_PER_ATOM * 100)
    b, n = int(wk.atom_base[0]), int(wk.n_atoms[0])
    lens, idx, rx, ry, rz = W.walker_lists(wk, 0)
    with pytest.raises(lib.AbpError) as e:
        small.add_walker(wk.mass[b:b + n], lens, idx)            # more CV atoms than the budget holds
    assert e.value.status == lib.ABP_E_NOMEM
    srv = lib.Server(ctx, wk.kinds, max_pending=2)
    bad = idx.copy()
    bad[0] = n                                                 # out of range
    with pytest.raises(lib.AbpError):
        srv.add_walker(wk.mass[b:b + n], lens, bad)
    with pytest.raises(lib.AbpError):
        srv.start()                                            # no walkers yet
    wid, ncv = srv.add_walker(wk.mass[b:b + n], lens, idx)
    xyz = np.zeros(3 * ncv, dtype=np.float32)
    with pytest.raises(lib.AbpError):
        srv.submit(wid, 1, xyz)                                # not started
    srv.start()
    with pytest.raises(lib.AbpError):
        srv.add_walker(wk.mass[b:b + n], lens, idx)            # registration is closed
    with pytest.raises(lib.AbpError):
        srv.submit(5, 1, xyz)                                  # unknown walker
    nan = xyz.copy()
    nan[3] = np.nan
    with pytest.raises(lib.AbpError) as e:
        srv.submit(wid, 1, nan)
    assert e.value.status == lib.ABP_E_NONFINITE
    base = np.concatenate([wk.x[b + srv.walker_atoms(wid)], wk.y[b + srv.walker_atoms(wid)],
                           wk.z[b + srv.walker_atoms(wid)]]).astype(np.float32)
    srv.submit(wid, 1, base)
    srv.submit(wid, 2, base)
    with pytest.raises(lib.AbpError) as e:
        srv.submit(wid, 3, base)                               # two outstanding until polled
    assert e.value.status == lib.ABP_E_BUSY
    got = []
    while len(got) < 2:
        got.extend(srv.poll(8, wait_us=100000).tolist())
    srv.submit(wid, 3, base)                                   # room again
    srv.stop()
    assert len(srv.poll(8)) == 1
    assert srv.stats()["completed"] == 3
    srv.close()
    small.close()
    ctx.close()


@pytest.mark.parametrize("kinds", [(W.CV_TORSION,), (W.CV_COM_DIST, W.CV_TORSION, W.CV_RMSD_OFF)])
def test_serving_one_and_three_cvs(lib, drv, kinds):
    """The serving loop in 1-D and 3-D CV spaces (walkers of uneven size with
    a torsion; a COM distance, a torsion and an offset RMSD), with evictions
    and deposits: every request, forces included, against the oracle."""
    import torch
    from tests.test_gpu_force_random import _walkers
    rng = np.random.default_rng(77 + len(kinds))
    wk = _walkers(rng, kinds, 20)
    D = len(kinds)
    periodic = tuple(1 if k == W.CV_TORSION else 0 for k in kinds)
    lo = tuple(-np.pi if k == W.CV_TORSION else 0.0 for k in kinds)
    hi = tuple(np.pi if k == W.CV_TORSION else (3.5 if k == W.CV_COM_DIST else 1.0) for k in kinds)
    width = tuple(0.4 if k == W.CV_TORSION else (0.15 if k == W.CV_COM_DIST else 0.05) for k in kinds)
    spec = W.BiasSpec(ndim=D, periodic=periodic, lo=lo, hi=hi, width=width, grid_n=(0, 0, 0))
    nh = 1500
    cen = np.vstack([rng.uniform(lo[i], hi[i], nh) for i in range(D)])
    hts = rng.uniform(0.1, 1.2, nh)
    ctx = lib.Context(spec, nh + 1024)
    lib.bias_deposit(ctx, torch.tensor(cen, device="cuda"), torch.tensor(hts, device="cuda"))
    torch.cuda.synchronize()
    probe = lib.Server(ctx, wk.kinds)
    ncv = _register(probe, wk)
    probe.close()
    srv = lib.Server(ctx, wk.kinds, hbm_budget_bytes=_cv_budget(lib, ncv, 1 / 3), max_batch=8, streams=2,
                     deposit_every=4, height0=1.0, height_decay=10000.0)
    _register(srv, wk)
    from paper_1609_09833_amd.examples import serve_driver
    eng = serve_driver.Engines(srv, wk)
    srv.start()
    t, w, step = W.serving_requests(seed=4, n_walkers=wk.nw, rate=50_000.0, n_requests=240)
    out = serve_driver.replay(srv, eng, w, step, t, AMP)
    srv.stop()
    st = srv.stats()
    assert st["completed"] == len(t) and st["evictions"] > 0
    centers, heights = lib.abp_hills_export(ctx)
    assert np.array_equal(centers[:, :nh], cen)
    for r in range(len(t)):
        o, k3 = int(out["offset"][r]), 3 * int(eng.n_cv[w[r]])
        _check_request(f"{D}-D served", spec, centers, heights, wk, srv, r, int(w[r]), out["positions"][o:o + k3],
                       int(out["version"][r]), out["s"][:, r], out["V"][r], out["dVds"][:, r],
                       out["forces"][o:o + k3])
    srv.close()
    ctx.close()
