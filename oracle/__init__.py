"""FP64 CPU oracle for the bias-force path (ctypes binding of liboracle.so).

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the
benchmark's CPU-baseline leg import this package. The GPU library and its
Python binding never import it, and the two share no code: the C sources
here (abp_oracle.c / abp_oracle.h) are a separate implementation written
from the paper's definitions (arXiv:1609.09833, Supplemental Material).

Inputs are numpy arrays; float32 inputs are converted exactly to float64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "abp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ORC_OK, ORC_E_INVAL, ORC_E_INDEX, ORC_E_NONFINITE = 0, 1, 5, 6


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (FP64, no fast-math, OpenMP over queries)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-fopenmp", "-fPIC", "-shared",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Bias(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("periodic", C.c_int32 * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("kernel", C.c_int32), ("width", C.c_double * 3), ("p", C.c_int32),
                ("transform", C.c_int32), ("kT", C.c_double), ("b", C.c_double),
                ("c", C.c_double), ("grid_n", C.c_int32 * 3), ("quantize", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("ABP_ORACLE_LIB")     # a separately built copy (mutation tests)
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        L = C.CDLL(path)
        P = C.c_void_p
        i64 = C.c_int64
        L.orc_wrap.restype = C.c_double
        L.orc_wrap.argtypes = [C.c_double, C.c_double]
        L.orc_kernel_1d.restype = None
        L.orc_kernel_1d.argtypes = [C.c_int32, C.c_double, C.c_int32, C.c_double, P, P]
        L.orc_hill_sum.restype = C.c_int32
        L.orc_hill_sum.argtypes = [P, i64, P, P, i64, P, P, P, P, P]
        L.orc_transform.restype = C.c_int32
        L.orc_transform.argtypes = [P, i64, P, P, P, P, P]
        L.orc_grid_coord.restype = C.c_double
        L.orc_grid_coord.argtypes = [P, C.c_int32, i64]
        L.orc_snap_index.restype = i64
        L.orc_snap_index.argtypes = [P, C.c_int32, C.c_double]
        L.orc_snap.restype = C.c_double
        L.orc_snap.argtypes = [P, C.c_int32, C.c_double]
        L.orc_grid_nodes.restype = C.c_int32
        L.orc_grid_nodes.argtypes = [P, i64, P, P, i64, P, P]
        L.orc_grid_eval.restype = C.c_int32
        L.orc_grid_eval.argtypes = [P, P, i64, P, P, P, P]
        L.orc_com_distance.restype = C.c_int32
        L.orc_com_distance.argtypes = [i64, P, P, i64, P, P, P, P, P]
        L.orc_torsion.restype = C.c_int32
        L.orc_torsion.argtypes = [P, P, P]
        L.orc_rmsd_off.restype = C.c_int32
        L.orc_rmsd_off.argtypes = [i64, P, P, P, P]
        L.orc_bias_force.restype = C.c_int32
        L.orc_bias_force.argtypes = [P, i64, P, P, C.c_int32, P, C.c_int32, P, i64, P, P,
                                     P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def bias_struct(spec) -> _Bias:
    periodic, lo, hi, width, grid_n = spec.padded()
    b = _Bias()
    b.ndim = spec.ndim
    for i in range(3):
        b.periodic[i] = int(periodic[i])
        b.lo[i] = float(lo[i])
        b.hi[i] = float(hi[i])
        b.width[i] = float(width[i])
        b.grid_n[i] = int(grid_n[i])
    b.kernel = int(spec.kernel)
    b.p = int(spec.p)
    b.transform = int(spec.transform)
    b.kT, b.b, b.c = float(spec.kT), float(spec.b), float(spec.c)
    b.quantize = int(getattr(spec, "quantize", 0))
    return b


def _check(rc):
    if rc != ORC_OK:
        raise ValueError(f"oracle returned status {rc}")


def wrap(delta, period):
    return lib().orc_wrap(float(delta), float(period))


def kernel_1d(kernel, width, p, delta):
    v, d = C.c_double(), C.c_double()
    lib().orc_kernel_1d(int(kernel), float(width), int(p), float(delta), C.byref(v), C.byref(d))
    return v.value, d.value


def hill_sum(spec, centers, heights, q):
    """h, dh[d][nq], A0[nq], A[d][nq] for queries q[d][nq] against all given hills."""
    centers = _f64(centers).reshape(spec.ndim, -1)
    heights = _f64(heights)
    q = _f64(q).reshape(spec.ndim, -1)
    nh, nq = heights.shape[0], q.shape[1]
    h = np.empty(nq)
    dh = np.empty((spec.ndim, nq))
    A0 = np.empty(nq)
    A = np.empty((spec.ndim, nq))
    b = bias_struct(spec)
    _check(lib().orc_hill_sum(C.byref(b), nh, _ptr(centers), _ptr(heights), nq, _ptr(q),
                              _ptr(h), _ptr(dh), _ptr(A0), _ptr(A)))
    return h, dh, A0, A


def transform(spec, h, dh):
    h = _f64(h)
    dh = _f64(dh).reshape(spec.ndim, -1)
    nq = h.shape[0]
    V = np.empty(nq)
    dV = np.empty((spec.ndim, nq))
    slope = np.empty(nq)
    b = bias_struct(spec)
    _check(lib().orc_transform(C.byref(b), nq, _ptr(h), _ptr(dh), _ptr(V), _ptr(dV), _ptr(slope)))
    return V, dV, slope


def bias_eval(spec, centers, heights, q):
    """Direct-sum bias: V, dV/ds, and the tolerance scales (slope*A0, slope*A)."""
    h, dh, A0, A = hill_sum(spec, centers, heights, q)
    V, dV, slope = transform(spec, h, dh)
    return V, dV, slope * A0, slope[None, :] * A


def grid_coord(spec, axis, j):
    b = bias_struct(spec)
    return lib().orc_grid_coord(C.byref(b), int(axis), int(j))


def wt_heights(spec, centers, heights, new_centers, w0, dT):
    """Well-tempered metadynamics heights for hills deposited at new_centers:
    w = w0 exp(-V(c)/dT), V the bias of the existing hills at c (the hill-height
    factor by which WTmetaD scales the update, named after eq. Cupdate; the
    standard form of Barducci, Bussi and Parrinello, 2008)."""
    new_centers = _f64(new_centers).reshape(spec.ndim, -1)
    if np.asarray(heights).size == 0:
        V = np.zeros(new_centers.shape[1])
    else:
        V = bias_eval(spec, centers, heights, new_centers)[0]
    return np.asarray(w0, dtype=np.float64) * np.exp(-V / float(dT))


def snap_index(spec, axis, x):
    """Nearest grid node index of x on an axis (the quantised mode)."""
    return int(lib().orc_snap_index(C.byref(bias_struct(spec)), int(axis), float(x)))


def snap(spec, axis, x):
    """Coordinate of the nearest grid node of x on an axis."""
    return lib().orc_snap(C.byref(bias_struct(spec)), int(axis), float(x))


def grid_size(spec):
    n = 1
    for i in range(spec.ndim):
        n *= int(spec.grid_n[i])
    return n


def grid_nodes(spec, centers, heights, node_ids):
    """Node arrays out[len(node_ids)][2^d] for the listed linear node ids."""
    centers = _f64(centers).reshape(spec.ndim, -1)
    heights = _f64(heights)
    ids = np.ascontiguousarray(node_ids, dtype=np.int64)
    out = np.empty((ids.shape[0], 1 << spec.ndim))
    b = bias_struct(spec)
    _check(lib().orc_grid_nodes(C.byref(b), heights.shape[0], _ptr(centers), _ptr(heights),
                                ids.shape[0], _ptr(ids), _ptr(out)))
    return out


def grid_all(spec, centers, heights):
    return grid_nodes(spec, centers, heights, np.arange(grid_size(spec), dtype=np.int64))


def grid_eval(spec, H, q):
    """Hermite interpolation of node arrays H[nodes][2^d]: h, dh[d][nq], n_clamped."""
    H = _f64(H)
    q = _f64(q).reshape(spec.ndim, -1)
    nq = q.shape[1]
    h = np.empty(nq)
    dh = np.empty((spec.ndim, nq))
    ncl = C.c_int64()
    b = bias_struct(spec)
    _check(lib().orc_grid_eval(C.byref(b), _ptr(H), nq, _ptr(q), _ptr(h), _ptr(dh), C.byref(ncl)))
    return h, dh, ncl.value


def com_distance(xa, ma, xb, mb):
    xa = _f64(xa).reshape(-1, 3)
    xb = _f64(xb).reshape(-1, 3)
    ma, mb = _f64(ma), _f64(mb)
    d = C.c_double()
    ga = np.empty_like(xa)
    gb = np.empty_like(xb)
    _check(lib().orc_com_distance(xa.shape[0], _ptr(xa), _ptr(ma), xb.shape[0], _ptr(xb), _ptr(mb),
                                  C.byref(d), _ptr(ga), _ptr(gb)))
    return d.value, ga, gb


def torsion(x4):
    x4 = _f64(x4).reshape(4, 3)
    phi = C.c_double()
    g = np.empty((4, 3))
    _check(lib().orc_torsion(_ptr(x4), C.byref(phi), _ptr(g)))
    return phi.value, g


def rmsd_off(x, x0):
    x = _f64(x).reshape(-1, 3)
    x0 = _f64(x0).reshape(-1, 3)
    r = C.c_double()
    g = np.empty_like(x)
    _check(lib().orc_rmsd_off(x.shape[0], _ptr(x), _ptr(x0), C.byref(r), _ptr(g)))
    return r.value, g


def bias_force(spec, centers, heights, walkers, fx, fy, fz, use_grid=False, H=None,
               n_visible=None):
    """Oracle bias force for a Walkers batch; returns (s, V, dVds, fx, fy, fz, status).

    fx/fy/fz are the forces before the call (copied to float64 and accumulated).
    """
    centers = _f64(centers).reshape(spec.ndim, -1)
    heights = _f64(heights)
    nw, ncv = walkers.nw, walkers.ncv
    s = np.full((ncv, nw), np.nan)
    V = np.full(nw, np.nan)
    dV = np.full((ncv, nw), np.nan)
    fx, fy, fz = _f64(fx).copy(), _f64(fy).copy(), _f64(fz).copy()
    status = np.zeros(nw, dtype=np.int32)
    kinds = np.ascontiguousarray(walkers.kinds, dtype=np.int32)
    off = np.ascontiguousarray(walkers.list_off, dtype=np.int64)
    idx = np.ascontiguousarray(walkers.list_idx, dtype=np.int32)
    nvis = None if n_visible is None else np.ascontiguousarray(n_visible, dtype=np.int64)
    Hc = None if H is None else _f64(H)
    b = bias_struct(spec)
    arrs = [_f64(walkers.ref_x), _f64(walkers.ref_y), _f64(walkers.ref_z),
            np.ascontiguousarray(walkers.atom_base, dtype=np.int64),
            np.ascontiguousarray(walkers.n_atoms, dtype=np.int32),
            _f64(walkers.x), _f64(walkers.y), _f64(walkers.z), _f64(walkers.mass)]
    _check(lib().orc_bias_force(C.byref(b), heights.shape[0], _ptr(centers), _ptr(heights),
                                1 if use_grid else 0, _ptr(Hc), ncv, _ptr(kinds), nw,
                                _ptr(off), _ptr(idx), *[_ptr(a) for a in arrs], _ptr(nvis),
                                _ptr(s), _ptr(V), _ptr(dV), _ptr(fx), _ptr(fy), _ptr(fz),
                                _ptr(status)))
    return s, V, dV, fx, fy, fz, status
