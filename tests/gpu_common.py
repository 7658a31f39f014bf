"""Helpers for the GPU tests: device selection, uploads, and per-atom CV
gradients (from the oracle's CV routines) for the force tolerance."""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")


def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def to_dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device()).contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def sample_idx(n, k):
    """k indices spread over [0, n), always including the first and last."""
    if n <= k:
        return np.arange(n)
    idx = np.unique(np.linspace(0, n - 1, k).round().astype(np.int64))
    return idx


def cv_atom_grad_abs(wk, s_oracle):
    """For each walker and CV, |d s_a / d x_j| per atom (3 components), as a dict
    global_atom -> array[ncv, 3]; computed with the oracle's CV routines."""
    out = {}
    for w in range(wk.nw):
        base = int(wk.atom_base[w])
        for a in range(wk.ncv):
            lists = []
            for t in range(2):
                b, e = int(wk.list_off[a, t, w]), int(wk.list_off[a, t, w + 1])
                lists.append(np.arange(b, e))
            kind = int(wk.kinds[a])
            pos = lambda ents: np.stack([wk.x[base + wk.list_idx[ents]], wk.y[base + wk.list_idx[ents]],
                                         wk.z[base + wk.list_idx[ents]]], axis=1).astype(np.float64)
            grads = []
            if kind == 0:
                ea, eb = lists
                _, ga, gb = oracle.com_distance(pos(ea), wk.mass[base + wk.list_idx[ea]],
                                                pos(eb), wk.mass[base + wk.list_idx[eb]])
                grads = [(ea, ga), (eb, gb)]
            elif kind == 1:
                e4 = lists[0]
                _, g4 = oracle.torsion(pos(e4))
                grads = [(e4, g4)]
            else:
                e0 = lists[0]
                ref = np.stack([wk.ref_x[e0], wk.ref_y[e0], wk.ref_z[e0]], axis=1)
                _, g0 = oracle.rmsd_off(pos(e0), ref)
                grads = [(e0, g0)]
            for ents, g in grads:
                for ent, gv in zip(ents, g):
                    j = base + int(wk.list_idx[ent])
                    arr = out.setdefault(j, np.zeros((wk.ncv, 3)))
                    arr[a] += np.abs(gv)
    return out
