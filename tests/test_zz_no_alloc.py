"""bias_force_noalloc, the entry point that allocates nothing (its split and
chained launches use the library's fixed device workspace), against
bias_force on the same inputs: two calls in a row, the second smaller, every
output and force bitwise equal. Also the size limit."""
import numpy as np
import pytest

from paper_1609_09833_amd import workloads as W
from tests.gpu_common import device, host

pytestmark = pytest.mark.gpu


def _run(abp, fn, ctx, wk, **kw):
    dw = abp.DeviceWalkers(wk)
    s, V, dV = fn(ctx, dw, **kw)
    abp.abp_sync(ctx)
    return host(s), host(V), host(dV), host(dw.fx), host(dw.fy), host(dw.fz)


@pytest.mark.parametrize("prec", [0, 2])          # FP32-Kahan, FP64
def test_noalloc_matches_bias_force(prec):
    device()
    import torch
    from paper_1609_09833_amd import abp
    spec, hills = W.ligand_pocket_hills(seed=31, n_hills=30000)      # > 16,384 hills: workspace shapes
    ctx = abp.Context(spec, capacity=hills.n)
    abp.bias_deposit(ctx, torch.as_tensor(hills.centers, device="cuda"),
                     torch.as_tensor(hills.heights, device="cuda"))
    big = W.ligand_pocket_walkers(seed=32, n_walkers=256)             # split shape
    small = W.ligand_pocket_walkers(seed=33, n_walkers=2)             # chained shape (arrival counters)
    for name, wk in (("256 walkers", big), ("2 walkers", small)):
        print(f"noalloc prec={prec}: {name}", flush=True)
        ref = _run(abp, abp.bias_force, ctx, wk, prec=prec)
        got = _run(abp, abp.bias_force_noalloc, ctx, wk, prec=prec)
        assert np.all(np.isfinite(ref[1]))
        for k, (a, b) in enumerate(zip(ref, got)):
            assert np.array_equal(a, b), (name, k)
    ctx.close()


def test_noalloc_rejects_what_does_not_fit():
    device()
    import torch
    from paper_1609_09833_amd import abp
    spec, hills = W.ligand_pocket_hills(seed=34, n_hills=150000)     # 2,344 chunks of 64 hills per walker
    ctx = abp.Context(spec, capacity=hills.n)
    abp.bias_deposit(ctx, torch.as_tensor(hills.centers, device="cuda"),
                     torch.as_tensor(hills.heights, device="cuda"))
    wk = W.ligand_pocket_walkers(seed=35, n_walkers=1024)
    dw = abp.DeviceWalkers(wk)
    with pytest.raises(abp.AbpError) as e:                           # about 71 MB of workspace
        abp.bias_force_noalloc(ctx, dw)
    assert e.value.status == abp.ABP_E_NOMEM
    assert np.all(host(dw.fx) == 0.0)                                  # nothing was enqueued
    part = W.ligand_pocket_walkers(seed=35, n_walkers=512)           # half the walkers fit
    ref = _run(abp, abp.bias_force, ctx, part)
    got = _run(abp, abp.bias_force_noalloc, ctx, part)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    ctx.close()
