"""HIP graph capture of the bias path (torch.cuda.graph over the C-ABI calls).

bias_eval and bias_force enqueue kernels only (no allocation once the
context's workspace exists, no memset), so a caller can capture a step in a
graph and replay it. Every replay, with eager work and synchronisations in
between, must reproduce the eager result bitwise.
"""
import numpy as np
import pytest

from paper_1609_09833_amd import workloads as W
from tests.gpu_common import device, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    device()
    from paper_1609_09833_amd import abp
    return abp


@pytest.mark.parametrize("n_hills,shape", [(3000, None), (20000, None), (20000, "chain")])   # fused, split, chained
@pytest.mark.parametrize("mode", ["direct", "grid"])
def test_bias_force_graph_replays(lib, n_hills, shape, mode):
    import torch
    wk = W.ligand_pocket_walkers(seed=71, n_walkers=64, atoms_lo=1000, atoms_hi=3000)
    spec, hills = W.ligand_pocket_hills(seed=72, n_hills=n_hills)
    ctx = lib.Context(spec, hills.n)
    if shape:
        lib.abp_set_force_shape(ctx, shape)      # the chained launch's counters must be back at zero after every replay
    lib.bias_deposit(ctx, torch.tensor(hills.centers, device="cuda"), torch.tensor(hills.heights, device="cuda"))
    dw = lib.DeviceWalkers(wk)
    m = lib.ABP_EVAL_GRID if mode == "grid" else lib.ABP_EVAL_DIRECT
    s = torch.empty((2, wk.nw), dtype=torch.float64, device="cuda")
    V = torch.empty(wk.nw, dtype=torch.float64, device="cuda")
    dV = torch.empty((2, wk.nw), dtype=torch.float64, device="cuda")

    def step():
        for f in (dw.fx, dw.fy, dw.fz):
            f.zero_()
        lib.bias_force(ctx, dw, mode=m, s=s, V=V, dVds=dV)

    step()                                   # eager; allocates the workspace
    torch.cuda.synchronize()
    lib.abp_sync(ctx)
    want = [host(t).copy() for t in (s, V, dV, dw.fx, dw.fy, dw.fz)]
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()                               # warm the side stream (no new allocations)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        step()
    for rep in range(4):
        for t in (s, V, dV, dw.fx):
            t.fill_(float("nan"))            # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [host(t) for t in (s, V, dV, dw.fx, dw.fy, dw.fz)]
        for a, b in zip(got, want):
            assert np.array_equal(a, b), f"replay {rep} differs"
    lib.abp_sync(ctx)


def test_bias_eval_graph_replays(lib):
    import torch
    spec, hills, q = W.torsion_2d(seed=73, n_hills=5000, n_queries=100000)
    ctx = lib.Context(spec, hills.n)
    lib.bias_deposit(ctx, torch.tensor(hills.centers, device="cuda"), torch.tensor(hills.heights, device="cuda"))
    qd = torch.tensor(q, device="cuda")
    V = torch.empty(q.shape[1], dtype=torch.float32, device="cuda")
    dV = torch.empty((2, q.shape[1]), dtype=torch.float32, device="cuda")
    outs = {}
    for mode in (lib.ABP_EVAL_DIRECT, lib.ABP_EVAL_GRID):
        lib.bias_eval(ctx, qd, mode=mode, V=V, dVds=dV)
        torch.cuda.synchronize()
        outs[mode] = (host(V).copy(), host(dV).copy())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        lib.bias_eval(ctx, qd, mode=lib.ABP_EVAL_DIRECT, V=V, dVds=dV)
    for rep in range(3):
        lib.bias_eval(ctx, qd, mode=lib.ABP_EVAL_GRID, V=V, dVds=dV)    # eager, overwrites the outputs
        torch.cuda.synchronize()
        assert np.array_equal(host(V), outs[lib.ABP_EVAL_GRID][0])
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(V), outs[lib.ABP_EVAL_DIRECT][0])
        assert np.array_equal(host(dV), outs[lib.ABP_EVAL_DIRECT][1])
    lib.abp_sync(ctx)
