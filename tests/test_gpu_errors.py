"""GPU tests of error handling and degenerate inputs through the C-ABI.

Every condition here is one the host checks or the kernels' own bounds checks
turn into an error (an atom index outside the walker, a list of the wrong
length, a non-finite input, a full history): the kernels skip the affected
walker or hill and set the context's error word, which abp_sync reports. The
other walkers' results must be exactly those of a clean batch.
"""
import numpy as np
import pytest

import oracle
from paper_1609_09833_amd import workloads as W
from tests.gpu_common import device, to_dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    device()
    from paper_1609_09833_amd import abp
    return abp


@pytest.fixture(scope="module")
def small(lib):
    wk = W.ligand_pocket_walkers(seed=61, n_walkers=8, atoms_lo=1000, atoms_hi=2000)
    spec, hills = W.ligand_pocket_hills(seed=62, n_hills=3000)
    return wk, spec, hills


def _ctx(lib, spec, hills, capacity=None):
    import torch
    ctx = lib.Context(spec, capacity or hills.n)
    if hills.n:
        lib.bias_deposit(ctx, torch.tensor(hills.centers, device="cuda"), torch.tensor(hills.heights, device="cuda"))
    return ctx


def _clean_run(lib, ctx, wk):
    dw = lib.DeviceWalkers(wk)
    s, V, dV = lib.bias_force(ctx, dw)
    lib.abp_sync(ctx)
    return host(s), host(V), host(dV), host(dw.fx)


@pytest.mark.parametrize("shape", ["fused", "split", "chain"])
def test_bad_atom_index_isolated(lib, small, shape):
    wk, spec, hills = small
    ctx = _ctx(lib, spec, hills)
    lib.abp_set_force_shape(ctx, shape)
    s0, V0, dV0, fx0 = _clean_run(lib, ctx, wk)
    bad = W.Walkers(**{**wk.__dict__, "list_idx": wk.list_idx.copy()})
    e = int(wk.list_off[1, 0, 3])                      # walker 3's first torsion atom
    bad.list_idx[e] = int(wk.n_atoms[3]) + 5           # outside walker 3
    dw = lib.DeviceWalkers(bad)
    s, V, dV = lib.bias_force(ctx, dw)
    with pytest.raises(lib.AbpError) as err:
        lib.abp_sync(ctx)
    assert err.value.status == lib.ABP_E_INDEX
    s, V, dV, fx = host(s), host(V), host(dV), host(dw.fx)
    good = [w for w in range(wk.nw) if w != 3]
    assert np.array_equal(V[good], V0[good]) and np.array_equal(s[:, good], s0[:, good])
    assert np.array_equal(dV[:, good], dV0[:, good])
    assert np.isnan(V[3]) and np.all(np.isnan(dV[:, 3]))      # unwritten
    b, n = int(wk.atom_base[3]), int(wk.n_atoms[3])
    assert np.all(fx[b:b + n] == 0.0)                          # no force on the bad walker
    assert np.array_equal(np.delete(fx, np.arange(b, b + n)), np.delete(fx0, np.arange(b, b + n)))
    lib.abp_sync(ctx)                                          # the error word was cleared


def test_non_increasing_com_list_and_wrong_torsion_length(lib, small):
    wk, spec, hills = small
    ctx = _ctx(lib, spec, hills)
    dup = W.Walkers(**{**wk.__dict__, "list_idx": wk.list_idx.copy()})
    e = int(wk.list_off[0, 1, 2])                      # walker 2's pocket list
    dup.list_idx[e + 1] = dup.list_idx[e]              # repeated atom: not strictly increasing
    lib.bias_force(ctx, lib.DeviceWalkers(dup))
    with pytest.raises(lib.AbpError) as err:
        lib.abp_sync(ctx)
    assert err.value.status == lib.ABP_E_INDEX
    short = W.Walkers(**{**wk.__dict__, "list_off": wk.list_off.copy()})
    short.list_off[1, 0, 5] += 1                       # torsion lists of walkers 4 and 5: 5 and 3 atoms
    s, V, dV = lib.bias_force(ctx, lib.DeviceWalkers(short))
    with pytest.raises(lib.AbpError) as err:
        lib.abp_sync(ctx)
    assert err.value.status == lib.ABP_E_INVAL
    V = host(V)
    assert np.isnan(V[4]) and np.isnan(V[5]) and np.all(np.isfinite(np.delete(V, [4, 5])))


def test_non_finite_position_and_height(lib, small):
    wk, spec, hills = small
    ctx = _ctx(lib, spec, hills, capacity=hills.n + 4)
    nan = W.Walkers(**{**wk.__dict__, "x": wk.x.copy()})
    atom = int(wk.atom_base[6] + wk.list_idx[int(wk.list_off[0, 0, 6])])
    nan.x[atom] = np.nan
    s, V, dV = lib.bias_force(ctx, lib.DeviceWalkers(nan))
    with pytest.raises(lib.AbpError) as err:
        lib.abp_sync(ctx)
    assert err.value.status == lib.ABP_E_NONFINITE
    assert np.isnan(host(V)[6]) and np.all(np.isfinite(np.delete(host(V), 6)))
    import torch
    lib.bias_deposit(ctx, torch.zeros((2, 2), dtype=torch.float64, device="cuda"),
                     torch.tensor([1.0, float("inf")], dtype=torch.float64, device="cuda"))
    with pytest.raises(lib.AbpError) as err:
        lib.abp_sync(ctx)
    assert err.value.status == lib.ABP_E_NONFINITE
    _, h = lib.abp_hills_export(ctx)
    assert h[-2] == 1.0 and h[-1] == 0.0               # the bad hill is kept with height 0


def test_capacity_and_reservations(lib, small):
    import torch
    wk, spec, hills = small
    ctx = _ctx(lib, spec, W.Hills(hills.centers[:, :10], hills.heights[:10]), capacity=12)
    c = torch.zeros((2, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(lib.AbpError) as err:
        lib.bias_deposit(ctx, c, torch.ones(3, dtype=torch.float64, device="cuda"))
    assert err.value.status == lib.ABP_E_CAPACITY
    assert ctx.num_hills == 10                          # nothing appended
    first = lib.abp_reserve(ctx, 2)
    assert first == 10
    with pytest.raises(lib.AbpError):
        lib.abp_reserve(ctx, 1)                         # full
    with pytest.raises(lib.AbpError):
        lib.bias_deposit(ctx, c[:, :1].contiguous(), torch.ones(1, dtype=torch.float64, device="cuda"))
    lib.abp_commit(ctx, 12)                             # slots never written are zero-height hills
    V, dV = lib.bias_eval(ctx, to_dev(np.array([[0.5], [0.0]])), prec=lib.ABP_PREC_FP64)
    Vo = oracle.bias_eval(spec, hills.centers[:, :10], hills.heights[:10], np.array([[0.5], [0.0]]))[0]
    assert host(V)[0] == pytest.approx(Vo[0], rel=1e-12)
    with pytest.raises(lib.AbpError):
        lib.abp_commit(ctx, 13)


def test_empty_inputs_and_empty_history(lib, small):
    import torch
    wk, spec, hills = small
    ctx = _ctx(lib, spec, W.Hills(np.zeros((2, 0)), np.zeros(0)), capacity=8)
    V, dV = lib.bias_eval(ctx, torch.zeros((2, 0), dtype=torch.float64, device="cuda"))
    assert V.numel() == 0
    dw = lib.DeviceWalkers(wk)
    s, V, dV = lib.bias_force(ctx, dw)                  # no hills: zero bias, zero force
    lib.abp_sync(ctx)
    assert np.all(host(V) == 0.0) and np.all(host(dV) == 0.0)
    assert np.all(host(dw.fx) == 0.0)
    z = np.zeros(wk.total_atoms)
    ref = oracle.bias_force(spec, np.zeros((2, 0)), np.zeros(0), wk, z, z, z)
    assert np.abs(host(s) - ref[0]).max() < 1e-12
    import dataclasses
    nogrid = lib.Context(dataclasses.replace(spec, grid_n=(0, 0)), 4)
    with pytest.raises(lib.AbpError) as err:
        lib.bias_eval(nogrid, torch.zeros((2, 4), dtype=torch.float64, device="cuda"), mode=lib.ABP_EVAL_GRID)
    assert err.value.status == lib.ABP_E_INVAL


@pytest.mark.parametrize("mode,prec", [("direct", 0), ("direct", 1), ("direct", 2), ("grid", 0)])
@pytest.mark.parametrize("q_f64", [False, True])
def test_non_finite_queries_give_nan_rows(lib, small, mode, prec, q_f64):
    """NaN and +-inf query coordinates give NaN outputs for those queries
    only; every other query's result is bitwise that of a clean batch."""
    import torch
    wk, spec, hills = small
    ctx = _ctx(lib, spec, hills)
    rng = np.random.default_rng(8)
    q = np.vstack([rng.uniform(0.0, 1.5, 700), rng.uniform(-np.pi, np.pi, 700)])
    q = q.astype(np.float64 if q_f64 else np.float32)
    bad = q.copy()
    rows = [3, 4, 5, 600, 699]
    bad[0, 3], bad[1, 4], bad[0, 5], bad[1, 600], bad[0, 699] = np.nan, np.inf, -np.inf, np.nan, np.inf
    m = lib.ABP_EVAL_GRID if mode == "grid" else lib.ABP_EVAL_DIRECT
    V0, dV0 = lib.bias_eval(ctx, to_dev(q), mode=m, prec=prec)
    V1, dV1 = lib.bias_eval(ctx, to_dev(bad), mode=m, prec=prec)
    lib.abp_sync(ctx)                                   # not an error
    V0, dV0, V1, dV1 = host(V0), host(dV0), host(V1), host(dV1)
    assert np.all(np.isnan(V1[rows])) and np.all(np.isnan(dV1[:, rows]))
    keep = np.setdiff1d(np.arange(q.shape[1]), rows)
    assert np.array_equal(V1[keep], V0[keep]) and np.array_equal(dV1[:, keep], dV0[:, keep])
    assert np.all(np.isfinite(V1[keep]))
