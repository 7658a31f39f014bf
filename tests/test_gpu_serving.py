"""GPU tests of the serving loop (abp_server_*): continuous batching of
bias-force requests from many walkers sharing one hill history.

Every request is re-evaluated by the oracle on the host: the walker's
positions at that step are reproduced bit for bit from the synthetic engine's
hash, the hills it saw are the first `version` hills of the exported history,
and s, V and dV/ds must agree to the same bounds as a direct bias_force call.
Deposits must land in the slots they report, with the reported CV value as
center and the height law's height.
"""
import numpy as np
import pytest

from paper_1609_09833_amd import workloads as W
from tests.gpu_common import device
from tests.tolerance import check_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    device()
    from paper_1609_09833_amd import abp as _abp
    return _abp


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
    ids = []
    for w in range(wk.nw):
        b, n = int(wk.atom_base[w]), int(wk.n_atoms[w])
        lens, idx, rx, ry, rz = W.walker_lists(wk, w)
        ids.append(srv.add_walker(wk.x[b:b + n], wk.y[b:b + n], wk.z[b:b + n], wk.mass[b:b + n], lens, idx,
                                  rx, ry, rz))
    assert ids == list(range(wk.nw))


def _oracle_request(spec, centers, heights, wk, w, step, version):
    from oracle import bias_eval, bias_force
    b, n = int(wk.atom_base[w]), int(wk.n_atoms[w])
    lens, idx, _, _, _ = W.walker_lists(wk, w)
    x, y, z = W.engine_positions(wk.x[b:b + n], wk.y[b:b + n], wk.z[b:b + n], w, step, idx, AMP)
    one = W.single_walker(wk, w, x, y, z)
    zero = np.zeros(n)
    c, h = centers[:, :version], heights[:version]
    s, V, dV, _, _, _, status = bias_force(spec, c, h, one, zero, zero, zero)
    assert status[0] == 0
    _, _, sA0, sA = bias_eval(spec, c, h, s)
    return s[:, 0], V[0], dV[:, 0], sA0[0], sA[:, 0]


def _wrap(d):
    return (d + np.pi) % (2 * np.pi) - np.pi


def test_serving_with_deposits_matches_oracle(lib):
    """Batched, evicting, depositing replay: every request checked against the oracle."""
    spec, hills, wk, ctx = _setup(lib)
    # about a third of the walkers fit
    budget = lib.ABP_SERVER_BYTES_PER_ATOM * int(wk.n_atoms.astype(np.int64).sum() // 3)
    srv = lib.Server(ctx, wk.kinds, hbm_budget_bytes=budget, max_batch=16, streams=2, deposit_every=3,
                     height0=1.2, height_decay=20000.0, amplitude=AMP)
    _register(srv, wk)
    # 120 ms of arrivals: walkers go idle between their requests, so they are evicted and
    # admitted again even if the first launches of the process (code loading) stall the loop
    t, w, step = W.serving_requests(seed=1, n_walkers=N_WALKERS, rate=5_000.0, n_requests=600)
    print(f"serving replay: {len(t)} requests, {N_WALKERS} walkers, budget {budget} B", flush=True)
    out = srv.replay(w, step, t)
    st = out["stats"]
    n = len(t)
    assert st["completed"] == n
    assert st["evictions"] > 0 and st["admissions"] > N_WALKERS
    assert st["max_batch_seen"] <= 16 and st["batches"] >= n // 16
    assert np.all(np.isfinite(out["t_done"])) and np.all(out["t_done"] >= t)
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
    # each deposited hill holds the depositing request's CV value and the height law's height
    for r in np.flatnonzero(dep >= 0):
        k = int(dep[r])
        assert np.array_equal(centers[:, k], out["s"][:, r])
        assert abs(heights[k] - 1.2 * np.exp(-k / 20000.0)) <= 1e-15 * heights[k]
    # oracle re-evaluation of every request
    s_g, V_g, dV_g = out["s"], out["V"], out["dVds"]
    s_o = np.zeros_like(s_g); V_o = np.zeros_like(V_g); dV_o = np.zeros_like(dV_g)
    A0 = np.zeros(n); A = np.zeros((wk.ncv, n))
    for r in range(n):
        s_o[:, r], V_o[r], dV_o[:, r], A0[r], A[:, r] = _oracle_request(
            spec, centers, heights, wk, int(w[r]), int(step[r]), int(ver[r]))
    assert np.abs(s_g[0] - s_o[0]).max() < 1e-12
    assert np.abs(_wrap(s_g[1] - s_o[1])).max() < 1e-12
    check_bound("served V", V_g, V_o, A0)
    check_bound("served dVds", dV_g, dV_o, A)
    srv.close()
    ctx.close()


def test_serving_alone_equals_in_the_mix(lib):
    """Without deposits a request's result is bitwise the same whether it ran
    alone (one request per launch, one stream) or inside mixed batches."""
    spec, hills, wk, ctx = _setup(lib)
    t, w, step = W.serving_requests(seed=2, n_walkers=N_WALKERS, rate=100_000.0, n_requests=400)
    res = []
    for mb, ns in ((1, 1), (64, 3)):
        srv = lib.Server(ctx, wk.kinds, hbm_budget_bytes=1 << 30, max_batch=mb, streams=ns, deposit_every=0,
                         amplitude=AMP)
        _register(srv, wk)
        print(f"replay max_batch={mb} streams={ns}", flush=True)
        res.append(srv.replay(w, step, t))
        srv.close()
    alone, mix = res
    assert alone["stats"]["max_batch_seen"] == 1
    assert mix["stats"]["batches"] < alone["stats"]["batches"]
    for k in ("s", "V", "dVds"):
        assert np.array_equal(alone[k], mix[k]), k
    assert np.all(alone["version"] == N_HILLS) and np.all(mix["version"] == N_HILLS)
    assert np.all(alone["deposit_slot"] == -1)
    ctx.close()


def test_serving_rejects_bad_input(lib):
    spec, hills, wk, ctx = _setup(lib, n_hills=100, capacity_extra=16)
    with pytest.raises(lib.AbpError):
        lib.Server(ctx, [W.CV_TORSION, W.CV_TORSION])         # torsion on a non-periodic axis
    with pytest.raises(lib.AbpError):
        lib.Server(ctx, wk.kinds, max_batch=0)
    small = lib.Server(ctx, wk.kinds, hbm_budget_bytes=lib.ABP_SERVER_BYTES_PER_ATOM * 1000)
    b, n = int(wk.atom_base[0]), int(wk.n_atoms[0])
    lens, idx, rx, ry, rz = W.walker_lists(wk, 0)
    with pytest.raises(lib.AbpError) as e:
        small.add_walker(wk.x[b:b + n], wk.y[b:b + n], wk.z[b:b + n], wk.mass[b:b + n], lens, idx)
    assert e.value.status == lib.ABP_E_NOMEM
    srv = lib.Server(ctx, wk.kinds)
    bad = idx.copy()
    bad[0] = n                                                 # out of range
    with pytest.raises(lib.AbpError):
        srv.add_walker(wk.x[b:b + n], wk.y[b:b + n], wk.z[b:b + n], wk.mass[b:b + n], lens, bad)
    wid = srv.add_walker(wk.x[b:b + n], wk.y[b:b + n], wk.z[b:b + n], wk.mass[b:b + n], lens, idx)
    with pytest.raises(lib.AbpError):
        srv.replay([wid, wid], [1, 2], [0.001, 0.0])           # arrivals out of order
    with pytest.raises(lib.AbpError):
        srv.replay([wid, wid], [2, 2], [0.0, 0.0])             # steps must increase
    with pytest.raises(lib.AbpError):
        srv.replay([5], [1], [0.0])                            # unknown walker
    out = srv.replay([wid], [1], [0.0])                        # still usable afterwards
    assert out["stats"]["completed"] == 1
    srv.close()
    small.close()
    ctx.close()


@pytest.mark.parametrize("kinds", [(W.CV_TORSION,), (W.CV_COM_DIST, W.CV_TORSION, W.CV_RMSD_OFF)])
def test_serving_one_and_three_cvs(lib, kinds):
    """The serving loop in 1-D and 3-D CV spaces (walkers of uneven size with
    a torsion; a COM distance, a torsion and an offset RMSD), with evictions
    and deposits: every request against the oracle."""
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
    budget = lib.ABP_SERVER_BYTES_PER_ATOM * int(wk.n_atoms.astype(np.int64).sum() // 3)
    srv = lib.Server(ctx, wk.kinds, hbm_budget_bytes=budget, max_batch=8, streams=2, deposit_every=4,
                     height0=1.0, height_decay=10000.0, amplitude=AMP)
    _register(srv, wk)
    t, w, step = W.serving_requests(seed=4, n_walkers=wk.nw, rate=50_000.0, n_requests=240)
    out = srv.replay(w, step, t)
    assert out["stats"]["completed"] == len(t) and out["stats"]["evictions"] > 0
    centers, heights = lib.abp_hills_export(ctx)
    assert np.array_equal(centers[:, :nh], cen)
    for r in range(len(t)):
        s_o, V_o, dV_o, A0, A = _oracle_request(spec, centers, heights, wk, int(w[r]), int(step[r]),
                                                int(out["version"][r]))
        ds = out["s"][:, r] - s_o
        for a in range(D):
            if periodic[a]:
                ds[a] = _wrap(ds[a])
        assert np.abs(ds).max() < 1e-12, (r, ds)
        check_bound("served V", np.array([out["V"][r]]), np.array([V_o]), np.array([A0]))
        check_bound("served dVds", out["dVds"][:, r], dV_o, A)
    srv.close()
    ctx.close()
