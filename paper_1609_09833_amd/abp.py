"""Python binding of libabp.so (the C-ABI in include/abp.h).

Argument marshalling only: every step of the bias-force path runs in the HIP
kernels of libabp.so. PyTorch supplies device memory and streams. The
functions keep the C names (abp_create, bias_deposit, bias_eval, cv_compute,
bias_force, ...). If libabp.so is missing or fails to load, importing this
package raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # loaded first so that libabp.so binds to the same HIP runtime as torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("ABP_LIB_PATH") or os.path.join(_PKG, "libabp.so")

ABP_OK, ABP_E_INVAL, ABP_E_NOMEM, ABP_E_CAPACITY, ABP_E_DEVICE, ABP_E_INDEX, ABP_E_NONFINITE, ABP_E_BUSY = range(8)
ABP_F32, ABP_F64 = 0, 1
ABP_PREC_FP32_KAHAN, ABP_PREC_FP32_NAIVE, ABP_PREC_FP64 = 0, 1, 2
ABP_K_GAUSS, ABP_K_COMPACT = 0, 1
ABP_T_PLAIN, ABP_T_MABP = 0, 1
ABP_EVAL_DIRECT, ABP_EVAL_GRID = 0, 1
ABP_CV_COM_DIST, ABP_CV_TORSION, ABP_CV_RMSD_OFF = 0, 1, 2
ABP_SERVER_BYTES_PER_ATOM = 4           # resident device bytes per CV atom (its mass)

EXPORTED = ("abp_create", "abp_destroy", "bias_deposit", "bias_eval", "cv_compute", "bias_force",
            "bias_force_noalloc",
            "abp_set_force_shape", "abp_reserve", "abp_commit", "abp_sync", "abp_num_hills", "abp_hills_export",
            "abp_grid_export", "abp_status_str", "abp_last_error",
            "abp_server_create", "abp_server_destroy", "abp_server_add_walker", "abp_server_walker_atoms",
            "abp_server_start", "abp_server_submit", "abp_server_poll", "abp_server_stop",
            "abp_server_get_stats", "abp_server_trace")


class AbpError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{message} (status {status})")
        self.status = status


class BiasDesc(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("periodic", C.c_int32 * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("kernel", C.c_int32), ("width", C.c_double * 3), ("p", C.c_int32),
                ("transform", C.c_int32), ("kT", C.c_double), ("b", C.c_double), ("c", C.c_double),
                ("grid_n", C.c_int32 * 3), ("quantize", C.c_int32), ("capacity", C.c_int64),
                ("wt_dT", C.c_double)]


class CvDesc(C.Structure):
    _fields_ = [("ncv", C.c_int32), ("kind", C.c_int32 * 3),
                ("list_off", C.c_void_p), ("list_idx", C.c_void_p),
                ("ref_x", C.c_void_p), ("ref_y", C.c_void_p), ("ref_z", C.c_void_p)]


class WalkersDesc(C.Structure):
    _fields_ = [("nw", C.c_int64), ("atom_base", C.c_void_p), ("n_atoms", C.c_void_p),
                ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("mass", C.c_void_p),
                ("fx", C.c_void_p), ("fy", C.c_void_p), ("fz", C.c_void_p)]


class ServerDesc(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_batch", C.c_int32), ("streams", C.c_int32),
                ("deposit_every", C.c_int32), ("prec", C.c_int32), ("height0", C.c_double),
                ("height_decay", C.c_double), ("cv_kind", C.c_int32 * 3), ("max_pending", C.c_int32),
                ("eval_mode", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("batches", C.c_int64),
                ("max_batch_seen", C.c_int64), ("admissions", C.c_int64), ("evictions", C.c_int64),
                ("deposits", C.c_int64), ("peak_resident", C.c_int64), ("pool_atoms", C.c_int64),
                ("wall_seconds", C.c_double)]


# abp_server_result and abp_server_batch as numpy record types (same layout)
def _np_types():
    import numpy as np
    result = np.dtype([("request", "<i8"), ("step", "<i8"), ("version", "<i8"), ("deposit_slot", "<i8"),
                       ("walker", "<i4"), ("n_cv_atoms", "<i4"), ("t_submit", "<f8"), ("t_done", "<f8"),
                       ("s", "<f8", (3,)), ("V", "<f8"), ("dVds", "<f8", (3,))])
    batch = np.dtype([("t_formed", "<f8"), ("t_launched", "<f8"), ("t_done", "<f8"), ("requests", "<i8"),
                      ("version", "<i8"), ("slot", "<i4"), ("admitted", "<i4")])
    return result, batch


SERVER_RESULT, SERVER_BATCH = _np_types()


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libabp.so not built at {LIB_PATH}: run __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    P, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
    sigs = {
        "abp_create": ([P, C.c_int, P], i32),
        "abp_destroy": ([P], i32),
        "bias_deposit": ([P, i64, i32, P, P, P], i32),
        "bias_eval": ([P, i32, i32, i64, i32, P, i64, P, P, P], i32),
        "cv_compute": ([P, P, P, P, P], i32),
        "bias_force": ([P, i32, i32, P, P, P, P, P, P, P, P, P], i32),
        "bias_force_noalloc": ([P, i32, i32, P, P, P, P, P, P, P, P, P], i32),
        "abp_reserve": ([P, i64, P], i32),
        "abp_commit": ([P, i64, P], i32),
        "abp_sync": ([P, P], i32),
        "abp_num_hills": ([P], i64),
        "abp_hills_export": ([P, P, P, P], i32),
        "abp_grid_export": ([P, P, i64], i32),
        "abp_status_str": ([i32], C.c_char_p),
        "abp_last_error": ([], C.c_char_p),
        "abp_set_force_shape": ([P, i32], i32),
        "abp_server_create": ([P, P, P], i32),
        "abp_server_destroy": ([P], i32),
        "abp_server_add_walker": ([P, i32, P, P, P, P, P, P, P, P], i32),
        "abp_server_walker_atoms": ([P, i32, P, P], i32),
        "abp_server_start": ([P], i32),
        "abp_server_submit": ([P, i32, i64, P, P, P], i32),
        "abp_server_poll": ([P, P, i64, P, i64], i32),
        "abp_server_stop": ([P], i32),
        "abp_server_get_stats": ([P, P], i32),
        "abp_server_trace": ([P, P, i64, P], i32),
    }
    for name, (args, res) in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


lib = _load()


def _check(st):
    if st != ABP_OK:
        raise AbpError(st, lib.abp_last_error().decode() or lib.abp_status_str(st).decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dtype_code(t):
    if t.dtype == torch.float32:
        return ABP_F32
    if t.dtype == torch.float64:
        return ABP_F64
    raise TypeError(f"unsupported dtype {t.dtype}")


def _dev(t, device, dtype=None):
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(t)
    return t.to(device=device, dtype=dtype if dtype is not None else t.dtype).contiguous()


def make_desc(spec, capacity):
    """abp_bias_desc from a bias specification (an object with the fields of
    abp_bias_desc: ndim, periodic, lo, hi, kernel, width, p, transform, kT, b,
    c, grid_n) and a history capacity."""
    d = BiasDesc()
    d.ndim = int(spec.ndim)

    def pad(t, v):
        t = tuple(t)
        return t + (v,) * (3 - len(t))
    per, lo, hi = pad(spec.periodic, 0), pad(spec.lo, 0.0), pad(spec.hi, 1.0)
    width, grid_n = pad(spec.width, 1.0), pad(spec.grid_n, 0)
    for i in range(3):
        d.periodic[i] = int(per[i]) if i < d.ndim else 0
        d.lo[i], d.hi[i] = float(lo[i]), float(hi[i])
        d.width[i] = float(width[i])
        d.grid_n[i] = int(grid_n[i]) if i < d.ndim else 0
    d.kernel, d.p, d.transform = int(spec.kernel), int(spec.p), int(spec.transform)
    d.kT, d.b, d.c = float(spec.kT), float(spec.b), float(spec.c)
    d.quantize = int(getattr(spec, "quantize", 0))
    d.capacity = int(capacity)
    d.wt_dT = float(getattr(spec, "wt_dT", 0.0))
    return d


class Context:
    """An abp_ctx handle (hill history, grids, workspace on one device)."""

    def __init__(self, spec, capacity, device=0):
        self.ndim = int(spec.ndim)
        self.device = torch.device("cuda", device)
        self.desc = make_desc(spec, capacity)
        h = C.c_void_p()
        _check(lib.abp_create(C.byref(self.desc), int(device), C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _check(lib.abp_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_hills(self):
        return int(lib.abp_num_hills(self.handle))


def abp_create(spec, capacity, device=0):
    return Context(spec, capacity, device)


def abp_destroy(ctx):
    ctx.close()


def bias_deposit(ctx, centers, heights, stream=None):
    """Append hills: centers [ndim][n], heights [n] (same float dtype, device tensors)."""
    centers = _dev(centers, ctx.device)
    heights = _dev(heights, ctx.device, centers.dtype)
    n = int(heights.shape[0])
    if centers.shape != (ctx.ndim, n):
        raise ValueError(f"centers must have shape ({ctx.ndim}, {n})")
    _check(lib.bias_deposit(ctx.handle, n, _dtype_code(centers), _ptr(centers), _ptr(heights), _stream(stream)))


def bias_eval(ctx, q, mode=ABP_EVAL_DIRECT, prec=None, n_visible=-1, V=None, dVds=None, stream=None):
    """V[nq], dVds[ndim][nq] at queries q[ndim][nq] (device tensor, float32 or float64).
    prec None: FP32 + Kahan for DIRECT, the FP64 node arrays for GRID (an FP32
    precision reads the grid's FP32 mirror)."""
    if prec is None:
        prec = ABP_PREC_FP64 if mode == ABP_EVAL_GRID else ABP_PREC_FP32_KAHAN
    q = _dev(q, ctx.device)
    nq = int(q.shape[1])
    if q.shape[0] != ctx.ndim:
        raise ValueError("q must be [ndim][nq]")
    if V is None:
        V = torch.empty(nq, dtype=q.dtype, device=ctx.device)
    if dVds is None:
        dVds = torch.empty((ctx.ndim, nq), dtype=q.dtype, device=ctx.device)
    _check(lib.bias_eval(ctx.handle, int(mode), int(prec), nq, _dtype_code(q), _ptr(q), int(n_visible),
                         _ptr(V), _ptr(dVds), _stream(stream)))
    return V, dVds


class DeviceWalkers:
    """Device copies of a walker batch (SoA pools + CV lists) and the two C
    descriptors that point at them. `src` is any object with the fields of
    abp_walkers / abp_cv_desc as numpy arrays (n_atoms, atom_base, x, y, z,
    mass, kinds, list_off, list_idx, ref_x, ref_y, ref_z)."""

    def __init__(self, src, device="cuda"):
        dev = torch.device(device)
        f32, i32, i64 = torch.float32, torch.int32, torch.int64
        t = lambda a, dt: torch.as_tensor(a).to(device=dev, dtype=dt).contiguous()
        self.n_atoms = t(src.n_atoms, i32)
        self.atom_base = t(src.atom_base, i64)
        self.x, self.y, self.z = t(src.x, f32), t(src.y, f32), t(src.z, f32)
        self.mass = t(src.mass, f32)
        self.fx = torch.zeros_like(self.x)
        self.fy = torch.zeros_like(self.x)
        self.fz = torch.zeros_like(self.x)
        self.list_off = t(src.list_off, i32)
        self.list_idx = t(src.list_idx, i32)
        self.ref_x, self.ref_y, self.ref_z = t(src.ref_x, f32), t(src.ref_y, f32), t(src.ref_z, f32)
        self.kinds = [int(k) for k in src.kinds]
        self.nw = int(self.n_atoms.shape[0])
        self.ncv = len(self.kinds)

    def cv_desc(self):
        d = CvDesc()
        d.ncv = self.ncv
        for i in range(3):
            d.kind[i] = self.kinds[i] if i < self.ncv else 0
        d.list_off, d.list_idx = self.list_off.data_ptr(), self.list_idx.data_ptr()
        d.ref_x, d.ref_y, d.ref_z = self.ref_x.data_ptr(), self.ref_y.data_ptr(), self.ref_z.data_ptr()
        return d

    def walkers_desc(self):
        w = WalkersDesc()
        w.nw = self.nw
        w.atom_base, w.n_atoms = self.atom_base.data_ptr(), self.n_atoms.data_ptr()
        w.x, w.y, w.z, w.mass = self.x.data_ptr(), self.y.data_ptr(), self.z.data_ptr(), self.mass.data_ptr()
        w.fx, w.fy, w.fz = self.fx.data_ptr(), self.fy.data_ptr(), self.fz.data_ptr()
        return w


def cv_compute(ctx, walkers, s=None, stream=None):
    """CV values s[ncv][nw] (float64) of a DeviceWalkers batch."""
    if s is None:
        s = torch.full((walkers.ncv, walkers.nw), float("nan"), dtype=torch.float64, device=ctx.device)
    cv, wk = walkers.cv_desc(), walkers.walkers_desc()
    _check(lib.cv_compute(ctx.handle, C.byref(cv), C.byref(wk), _ptr(s), _stream(stream)))
    return s


def bias_force(ctx, walkers, mode=ABP_EVAL_DIRECT, prec=ABP_PREC_FP32_KAHAN, n_visible=None,
               deposit_slot=None, deposit_height=None, s=None, V=None, dVds=None, stream=None):
    """Fused CV -> bias -> chain-rule step; forces are added into walkers.fx/fy/fz.
    Returns (s[ncv][nw], V[nw], dVds[ncv][nw]) as float64 device tensors."""
    return _bias_force(lib.bias_force, ctx, walkers, mode, prec, n_visible, deposit_slot, deposit_height, s, V,
                       dVds, stream)


def bias_force_noalloc(ctx, walkers, mode=ABP_EVAL_DIRECT, prec=ABP_PREC_FP32_KAHAN, n_visible=None,
                       deposit_slot=None, deposit_height=None, s=None, V=None, dVds=None, stream=None):
    """bias_force whose workspace is the library's fixed device array (the C
    call allocates nothing; pass preallocated s, V, dVds to allocate nothing here)."""
    return _bias_force(lib.bias_force_noalloc, ctx, walkers, mode, prec, n_visible, deposit_slot, deposit_height,
                       s, V, dVds, stream)


def _bias_force(fn, ctx, walkers, mode, prec, n_visible, deposit_slot, deposit_height, s, V, dVds, stream):
    nw, ncv, dev = walkers.nw, walkers.ncv, ctx.device
    if s is None:
        s = torch.full((ncv, nw), float("nan"), dtype=torch.float64, device=dev)
    if V is None:
        V = torch.full((nw,), float("nan"), dtype=torch.float64, device=dev)
    if dVds is None:
        dVds = torch.full((ncv, nw), float("nan"), dtype=torch.float64, device=dev)
    nvis = None if n_visible is None else _dev(n_visible, dev, torch.int64)
    slot = None if deposit_slot is None else _dev(deposit_slot, dev, torch.int64)
    hgt = None if deposit_height is None else _dev(deposit_height, dev, torch.float64)
    cv, wk = walkers.cv_desc(), walkers.walkers_desc()
    _check(fn(ctx.handle, int(mode), int(prec), C.byref(cv), C.byref(wk), _ptr(nvis), _ptr(slot),
              _ptr(hgt), _ptr(s), _ptr(V), _ptr(dVds), _stream(stream)))
    return s, V, dVds


SHAPES = {"auto": 0, "fused": 1, "split": 2, "chain": 3}


def abp_set_force_shape(ctx, shape):
    """Fix bias_force's launch shape on ctx: "auto", "fused", "split" or "chain"."""
    _check(lib.abp_set_force_shape(ctx.handle, SHAPES[shape] if isinstance(shape, str) else int(shape)))


def abp_reserve(ctx, n):
    first = C.c_int64()
    _check(lib.abp_reserve(ctx.handle, int(n), C.byref(first)))
    return first.value


def abp_commit(ctx, upto, stream=None):
    _check(lib.abp_commit(ctx.handle, int(upto), _stream(stream)))


def abp_sync(ctx, stream=None):
    """Raises AbpError if the device flagged an error since the last sync."""
    _check(lib.abp_sync(ctx.handle, _stream(stream)))


def abp_num_hills(ctx):
    return ctx.num_hills


def abp_hills_export(ctx):
    import numpy as np
    n = ctx.num_hills
    cen = np.zeros((ctx.ndim, max(n, 1)), dtype=np.float64)
    hts = np.zeros(max(n, 1), dtype=np.float64)
    cnt = C.c_int64(max(n, 1))
    _check(lib.abp_hills_export(ctx.handle, cen.ctypes.data_as(C.c_void_p), hts.ctypes.data_as(C.c_void_p),
                                C.byref(cnt)))
    m = cnt.value
    return np.ascontiguousarray(cen.reshape(-1)[: ctx.ndim * m].reshape(ctx.ndim, m)), hts[:m]


def abp_grid_export(ctx):
    import numpy as np
    nodes = 1
    for i in range(ctx.ndim):
        nodes *= int(ctx.desc.grid_n[i])
    H = np.zeros((nodes, 1 << ctx.ndim), dtype=np.float64)
    _check(lib.abp_grid_export(ctx.handle, H.ctypes.data_as(C.c_void_p), H.size))
    return H


class Server:
    """An abp_server: continuous batching of bias-force requests from many
    walkers over one context's hill history. Requests carry the positions of
    a walker's CV atoms (HOST numpy arrays [3][n_cv]) and return the bias
    force on them."""

    def __init__(self, ctx, kinds, hbm_budget_bytes=1 << 30, max_batch=1024, streams=2, deposit_every=0,
                 prec=ABP_PREC_FP32_KAHAN, height0=0.0, height_decay=0.0, max_pending=4096,
                 eval_mode=ABP_EVAL_DIRECT):
        self.ctx = ctx
        d = ServerDesc()
        d.hbm_budget_bytes, d.max_batch, d.streams = int(hbm_budget_bytes), int(max_batch), int(streams)
        d.deposit_every, d.prec = int(deposit_every), int(prec)
        d.height0, d.height_decay, d.max_pending = float(height0), float(height_decay), int(max_pending)
        d.eval_mode = int(eval_mode)
        for i in range(3):
            d.cv_kind[i] = int(kinds[i]) if i < len(kinds) else 0
        self.desc = d
        self.ncv = ctx.ndim
        self._outs = {}                 # request id -> force_out array, alive until polled
        self._ncv_atoms = []
        h = C.c_void_p()
        _check(lib.abp_server_create(ctx.handle, C.byref(d), C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _check(lib.abp_server_destroy(self.handle))
            self.handle = None
            self._outs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_walker(self, mass, list_len, list_idx, ref_x=None, ref_y=None, ref_z=None):
        """Register a walker (all its atoms' masses, CV lists of walker-local
        indices); returns (walker id, number of its CV atoms)."""
        import numpy as np
        f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
        mass = f32(mass)
        ll = np.ascontiguousarray(list_len, dtype=np.int32)
        li = np.ascontiguousarray(list_idx, dtype=np.int32)
        if ll.shape != (2 * self.ncv,):
            raise ValueError("list_len must hold 2*ncv lengths")
        refs = [None if r is None else f32(r) for r in (ref_x, ref_y, ref_z)]
        p = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
        wid, ncv = C.c_int32(), C.c_int32()
        _check(lib.abp_server_add_walker(self.handle, int(mass.shape[0]), p(mass), p(ll),
                                         p(li if li.size else np.zeros(1, np.int32)), p(refs[0]), p(refs[1]),
                                         p(refs[2]), C.byref(wid), C.byref(ncv)))
        self._ncv_atoms.append(ncv.value)
        return wid.value, ncv.value

    def walker_atoms(self, walker):
        """The walker's CV atoms (walker-local indices, increasing): the order of
        submitted positions and returned forces."""
        import numpy as np
        n = C.c_int32()
        _check(lib.abp_server_walker_atoms(self.handle, int(walker), None, C.byref(n)))
        idx = np.zeros(max(n.value, 1), dtype=np.int32)
        _check(lib.abp_server_walker_atoms(self.handle, int(walker), idx.ctypes.data_as(C.c_void_p), C.byref(n)))
        return idx[: n.value]

    def start(self):
        _check(lib.abp_server_start(self.handle))

    def stop(self):
        _check(lib.abp_server_stop(self.handle))

    def submit(self, walker, step, xyz, force_out=None):
        """Submit positions xyz (float32 [3][n_cv]); force_out (float32 [3][n_cv],
        C-contiguous) receives the forces when the request is polled."""
        import numpy as np
        xyz = np.ascontiguousarray(xyz, dtype=np.float32)
        if force_out is not None and (force_out.dtype != np.float32 or not force_out.flags.c_contiguous
                                      or force_out.size < xyz.size):
            raise ValueError("force_out must be a C-contiguous float32 array as large as xyz")
        rid = C.c_int64()
        _check(lib.abp_server_submit(self.handle, int(walker), int(step), xyz.ctypes.data_as(C.c_void_p),
                                     None if force_out is None else force_out.ctypes.data_as(C.c_void_p),
                                     C.byref(rid)))
        if force_out is not None:
            self._outs[rid.value] = force_out
        return rid.value

    def poll(self, max_results=4096, wait_us=0):
        """Completed requests as a numpy record array (SERVER_RESULT fields)."""
        import numpy as np
        out = np.zeros(max(int(max_results), 1), dtype=SERVER_RESULT)
        n = C.c_int64()
        _check(lib.abp_server_poll(self.handle, out.ctypes.data_as(C.c_void_p), int(max_results), C.byref(n),
                                   int(wait_us)))
        out = out[: n.value]
        for r in out["request"]:
            self._outs.pop(int(r), None)
        return out

    def stats(self):
        s = ServerStats()
        _check(lib.abp_server_get_stats(self.handle, C.byref(s)))
        return {name: getattr(s, name) for name, _ in ServerStats._fields_}

    def trace(self, max_batches=1 << 18):
        """Batch records of the run (SERVER_BATCH fields), oldest first."""
        import numpy as np
        out = np.zeros(max(int(max_batches), 1), dtype=SERVER_BATCH)
        n = C.c_int64()
        _check(lib.abp_server_trace(self.handle, out.ctypes.data_as(C.c_void_p), int(max_batches), C.byref(n)))
        return out[: n.value]
