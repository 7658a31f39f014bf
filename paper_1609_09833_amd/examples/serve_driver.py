"""Binding of the serving load generator (abp_serve_driver.cpp): synthetic
CV-atom positions per (walker, step) and an open-loop replay through
abp_server_submit / abp_server_poll. Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from paper_1609_09833_amd import abp  # loads libabp.so first

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libabp_serve_driver.so")


def _load():
    if not os.path.exists(PATH):
        raise ImportError(f"{PATH} not built: run __graft_entry__.build()")
    L = C.CDLL(PATH)
    P, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
    L.abp_drv_positions.argtypes = [i64, P, P, P, P, P, P, C.c_float, P, P, C.c_int]
    L.abp_drv_positions.restype = None
    L.abp_drv_replay.argtypes = [P, i32, i64, P, P, P, P, P, P, P, P, P, P, P, P, P, C.c_char_p, C.c_int]
    L.abp_drv_replay.restype = C.c_int
    return L


lib = _load()


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Engines:
    """The synthetic engines of a server's walkers: every walker's CV atoms
    (the server's order) and their base positions from a Walkers batch."""

    def __init__(self, srv, wk):
        self.n_cv = np.zeros(wk.nw, dtype=np.int32)
        atoms, base = [], []
        for w in range(wk.nw):
            a = srv.walker_atoms(w)
            b = int(wk.atom_base[w])
            self.n_cv[w] = a.size
            atoms.append(a)
            base.append(np.concatenate([wk.x[b + a], wk.y[b + a], wk.z[b + a]]).astype(np.float32))
        self.atoms = np.ascontiguousarray(np.concatenate(atoms).astype(np.int32))
        self.base = np.ascontiguousarray(np.concatenate(base))
        self.base_off = np.zeros(wk.nw, dtype=np.int64)
        self.base_off[1:] = np.cumsum(3 * self.n_cv.astype(np.int64))[:-1]

    def positions(self, walker, step, amplitude, threads=8):
        """CV-atom positions of each request, concatenated [3][n_cv] blocks, and
        each request's offset into them."""
        walker = np.ascontiguousarray(walker, dtype=np.int32)
        step = np.ascontiguousarray(step, dtype=np.int64)
        sizes = 3 * self.n_cv[walker].astype(np.int64)
        off = np.zeros(walker.size, dtype=np.int64)
        if walker.size:
            off[1:] = np.cumsum(sizes)[:-1]
        pos = np.empty(int(sizes.sum()) if walker.size else 0, dtype=np.float32)
        lib.abp_drv_positions(walker.size, _p(walker), _p(step), _p(self.base), _p(self.base_off), _p(self.n_cv),
                              _p(self.atoms), float(amplitude), _p(pos), _p(off), int(threads))
        return pos, off


def replay(srv, engines, walker, step, t_arrival, amplitude, forces=True, threads=8):
    """Open-loop replay against a started server: positions from the engines,
    each request submitted at its arrival time (seconds from the call).
    Returns per-request arrays: t_submit, t_done (the call's clock), version,
    deposit_slot, s[ncv][n], V, dVds[ncv][n], forces (concatenated [3][n_cv]
    blocks at `offset`) and the positions that were submitted."""
    walker = np.ascontiguousarray(walker, dtype=np.int32)
    step = np.ascontiguousarray(step, dtype=np.int64)
    t_arrival = np.ascontiguousarray(t_arrival, dtype=np.float64)
    n = walker.size
    pos, off = engines.positions(walker, step, amplitude, threads)
    out = {"t_submit": np.full(n, np.nan), "t_done": np.full(n, np.nan), "version": np.full(n, -1, np.int64),
           "deposit_slot": np.full(n, -2, np.int64), "s": np.full((srv.ncv, n), np.nan),
           "V": np.full(n, np.nan), "dVds": np.full((srv.ncv, n), np.nan),
           "forces": np.full(pos.size, np.nan, dtype=np.float32) if forces else None,
           "positions": pos, "offset": off}
    err = C.create_string_buffer(512)
    rc = lib.abp_drv_replay(srv.handle, srv.ncv, n, _p(walker), _p(step), _p(t_arrival), _p(pos), _p(off),
                            _p(out["t_submit"]), _p(out["t_done"]), _p(out["version"]), _p(out["deposit_slot"]),
                            _p(out["s"]), _p(out["V"]), _p(out["dVds"]), _p(out["forces"]), err, 512)
    if rc != 0:
        raise abp.AbpError(abp.ABP_E_DEVICE, err.value.decode())
    return out
