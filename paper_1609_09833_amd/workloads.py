"""Seeded synthetic inputs for the bias-force path.

This module is the only code shared by the GPU path's tests/benchmark and the
CPU oracle's tests. It draws random numbers (numpy PCG64) in a fixed, documented
order and returns plain arrays. It holds none of the method's arithmetic: no
kernel, sum, interpolation, collective variable or force is computed here.

The workloads follow the shapes of the paper's use of the method: two- and
three-dimensional CV spaces of torsions and distances, a few thousand to a
million deposited hills, a batch of walkers whose CV atoms are a small ligand
and a binding pocket (Results, "Timing of the implementation" and "Applications
to ligand binding"; Supplemental Material, "Convergence with S_a^p"). The
paper's own molecular systems are not reproduced.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

PI = math.pi

# Bias-descriptor enumerations (mirrors of the C-ABI values; plain integers).
KERNEL_GAUSS = 0
KERNEL_COMPACT = 1
TRANSFORM_PLAIN = 0
TRANSFORM_MABP = 1
CV_COM_DIST = 0
CV_TORSION = 1
CV_RMSD_OFF = 2

# Atom masses drawn for synthetic walkers (H, C, N, O, S; g/mol).
ATOM_MASSES = np.array([1.008, 12.011, 14.007, 15.999, 32.06])

# k_B * 300 K in kJ/mol.
KT_300K = 0.0083144626 * 300.0


@dataclass
class BiasSpec:
    """Definition of the bias (plain numbers; see include/abp.h abp_bias_desc)."""
    ndim: int
    periodic: tuple
    lo: tuple
    hi: tuple
    kernel: int = KERNEL_GAUSS
    width: tuple = (0.3, 0.3, 0.3)
    p: int = 1
    transform: int = TRANSFORM_PLAIN
    kT: float = KT_300K
    b: float = 0.9
    c: float = 0.001
    grid_n: tuple = (0, 0, 0)
    capacity: int = 0
    quantize: int = 0
    wt_dT: float = 0.0

    def padded(self):
        """Return the 3-wide tuples the C structures use."""
        def pad(t, v):
            t = tuple(t)
            return t + (v,) * (3 - len(t))
        return (pad(self.periodic, 0), pad(self.lo, 0.0), pad(self.hi, 1.0),
                pad(self.width, 1.0), pad(self.grid_n, 0))


@dataclass
class Hills:
    """Deposited hills: centers [ndim][n] float64, heights [n] float64."""
    centers: np.ndarray
    heights: np.ndarray

    @property
    def n(self) -> int:
        return int(self.heights.shape[0])


@dataclass
class Walkers:
    """A batch of walkers in SoA pools plus their CV atom lists.

    Layout (matches the C-ABI):
      n_atoms[nw] int32, atom_base[nw] int64 (offset of walker w in the pools),
      x, y, z, mass [total] float32,
      kinds[ncv] int32,
      list_off[ncv][2][nw+1] int32 CSR offsets into list_idx for (cv, slot, walker),
      list_idx[...] int32 walker-local atom indices,
      ref_x, ref_y, ref_z [len(list_idx)] float32 reference positions aligned with
      list_idx (used by RMSD_OFF lists; zeros elsewhere).
    """
    n_atoms: np.ndarray
    atom_base: np.ndarray
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    mass: np.ndarray
    kinds: np.ndarray
    list_off: np.ndarray
    list_idx: np.ndarray
    ref_x: np.ndarray
    ref_y: np.ndarray
    ref_z: np.ndarray
    extra: dict = field(default_factory=dict)

    @property
    def nw(self) -> int:
        return int(self.n_atoms.shape[0])

    @property
    def ncv(self) -> int:
        return int(self.kinds.shape[0])

    @property
    def total_atoms(self) -> int:
        return int(self.x.shape[0])


def _uniform_circle(rng, size):
    return rng.uniform(-PI, PI, size=size)


# ---------------------------------------------------------------------------
# CV-space workloads
# ---------------------------------------------------------------------------

def plain_1d(seed=0, n_hills=2000, n_queries=10000):
    """1-D periodic CV on [-pi, pi): Gaussian hills, sigma 0.35, heights U[0.1, 1.2].

    Draw order: centers, heights, queries. All float64.
    """
    rng = np.random.default_rng(seed)
    spec = BiasSpec(ndim=1, periodic=(1,), lo=(-PI,), hi=(PI,), width=(0.35,))
    centers = _uniform_circle(rng, (1, n_hills))
    heights = rng.uniform(0.1, 1.2, size=n_hills)
    q = _uniform_circle(rng, (1, n_queries))
    return spec, Hills(centers, heights), q


def lattice_1d(n_hills=2000, height=1.0, sigma=0.35, n_queries=64, seed=0):
    """n equal hills evenly spaced on the circle, plus uniform queries (no randomness in the hills)."""
    rng = np.random.default_rng(seed)
    spec = BiasSpec(ndim=1, periodic=(1,), lo=(-PI,), hi=(PI,), width=(sigma,))
    centers = (-PI + (2 * PI / n_hills) * np.arange(n_hills)).reshape(1, -1)
    heights = np.full(n_hills, float(height))
    q = _uniform_circle(rng, (1, n_queries))
    return spec, Hills(centers, heights), q


def torsion_2d(seed=0, n_hills=50000, n_queries=1 << 20, query_dtype=np.float32,
               grid_n=(256, 256)):
    """2-D periodic CV space (two torsions on [-pi, pi)^2).

    Hill k has height 1.2*exp(-k/20000) in deposit order, sigma = (0.3, 0.3).
    Queries stand for 1024 walkers x 1024 steps.
    Draw order: centers (2 x n), queries (2 x nq). Queries are rounded to
    `query_dtype` here so every consumer sees identical values.
    """
    rng = np.random.default_rng(seed)
    spec = BiasSpec(ndim=2, periodic=(1, 1), lo=(-PI, -PI), hi=(PI, PI), width=(0.3, 0.3),
                    grid_n=tuple(grid_n))
    centers = _uniform_circle(rng, (2, n_hills))
    heights = 1.2 * np.exp(-np.arange(n_hills) / 20000.0)
    q = _uniform_circle(rng, (2, n_queries)).astype(query_dtype)
    return spec, Hills(centers, heights), q


def stress_3d(seed=0, n_hills=1_000_000, n_queries=4 << 20, query_dtype=np.float32,
              grid_n=(128, 128, 128)):
    """3-D CV space: a distance (non-periodic, sigma 0.1 nm) and two torsions (sigma 0.3).

    Centers uniform on [0, 1.0] nm x [-pi, pi)^2; heights log-uniform on
    [1e-4, 1.0] kJ/mol; queries uniform on [0, 1] x [-pi, pi)^2. The grid spans
    [0, 1.2] nm on the distance axis.
    Draw order: center dim 0, center dims 1-2, log-heights, query dim 0, query dims 1-2.
    """
    rng = np.random.default_rng(seed)
    spec = BiasSpec(ndim=3, periodic=(0, 1, 1), lo=(0.0, -PI, -PI), hi=(1.2, PI, PI),
                    width=(0.1, 0.3, 0.3), grid_n=tuple(grid_n))
    c0 = rng.uniform(0.0, 1.0, size=n_hills)
    c12 = _uniform_circle(rng, (2, n_hills))
    centers = np.vstack([c0[None, :], c12])
    heights = np.exp(rng.uniform(math.log(1e-4), math.log(1.0), size=n_hills))
    q0 = rng.uniform(0.0, 1.0, size=n_queries)
    q12 = _uniform_circle(rng, (2, n_queries))
    q = np.vstack([q0[None, :], q12]).astype(query_dtype)
    return spec, Hills(centers, heights), q


# ---------------------------------------------------------------------------
# Walker (atom) workloads
# ---------------------------------------------------------------------------

def _csr(lists_per_walker):
    off = np.zeros(len(lists_per_walker) + 1, dtype=np.int64)
    for w, l in enumerate(lists_per_walker):
        off[w + 1] = off[w] + len(l)
    return off


def ligand_pocket_walkers(seed=0, n_walkers=1024, atoms_lo=2000, atoms_hi=8000, box=6.0,
                          ligand=(40, 80), pocket=(200, 600)):
    """Walkers with CV1 = COM distance(ligand, pocket) and CV2 = one ligand torsion.

    Per walker: N ~ U{atoms_lo..atoms_hi}; the ligand is a contiguous block of
    L ~ U{ligand} atoms at a random offset; the pocket is a sorted random subset
    of P ~ U{pocket} of the remaining atoms; the torsion is 4 distinct ligand
    atoms in draw order. Positions are U[0, box)^3 nm in float32, masses drawn
    from ATOM_MASSES.
    Draw order: atom counts; positions x, y, z; masses; then per walker in
    order: L, ligand offset, P, pocket subset, torsion atoms.
    """
    rng = np.random.default_rng(seed)
    n_atoms = rng.integers(atoms_lo, atoms_hi + 1, size=n_walkers).astype(np.int32)
    atom_base = np.zeros(n_walkers, dtype=np.int64)
    atom_base[1:] = np.cumsum(n_atoms[:-1].astype(np.int64))
    total = int(n_atoms.astype(np.int64).sum())
    pos = rng.uniform(0.0, box, size=(3, total)).astype(np.float32)
    mass = ATOM_MASSES[rng.integers(0, len(ATOM_MASSES), size=total)].astype(np.float32)
    lig_lists, poc_lists, tor_lists = [], [], []
    for w in range(n_walkers):
        n = int(n_atoms[w])
        L = int(rng.integers(ligand[0], ligand[1] + 1))
        off = int(rng.integers(0, n - L + 1))
        P = int(rng.integers(pocket[0], pocket[1] + 1))
        rest = np.concatenate([np.arange(0, off), np.arange(off + L, n)])
        poc = np.sort(rng.choice(rest, size=P, replace=False))
        tor = rng.choice(L, size=4, replace=False) + off
        lig_lists.append(np.arange(off, off + L, dtype=np.int32))
        poc_lists.append(poc.astype(np.int32))
        tor_lists.append(tor.astype(np.int32))
    empty = [np.zeros(0, dtype=np.int32)] * n_walkers
    kinds = np.array([CV_COM_DIST, CV_TORSION], dtype=np.int32)
    groups = [lig_lists, poc_lists, tor_lists, empty]     # (cv0,slot0) (cv0,slot1) (cv1,slot0) (cv1,slot1)
    list_off = np.zeros((2, 2, n_walkers + 1), dtype=np.int64)
    chunks = []
    base = 0
    for gi, g in enumerate(groups):
        off = _csr(g) + base
        list_off[gi // 2, gi % 2] = off
        base = int(off[-1])
        chunks.extend(g)
    list_idx = np.concatenate(chunks).astype(np.int32)
    if base >= 2 ** 31:
        raise ValueError("CV lists too long for int32 offsets")
    zeros = np.zeros(list_idx.shape[0], dtype=np.float32)
    return Walkers(n_atoms=n_atoms, atom_base=atom_base, x=pos[0].copy(), y=pos[1].copy(),
                   z=pos[2].copy(), mass=mass, kinds=kinds, list_off=list_off.astype(np.int32),
                   list_idx=list_idx, ref_x=zeros, ref_y=zeros.copy(), ref_z=zeros.copy())


def ligand_pocket_hills(seed=0, n_hills=20000):
    """Hills for the (COM distance, torsion) CV space.

    Centers U[0, 1.0] nm x U[-pi, pi); sigma = (0.1 nm, 0.3 rad); heights
    U[0.1, 1.2] kJ/mol. The grid variant spans [0, 1.5] nm x torsion, 256^2.
    Draw order: distance centers, torsion centers, heights.
    """
    rng = np.random.default_rng(seed + 1)
    spec = BiasSpec(ndim=2, periodic=(0, 1), lo=(0.0, -PI), hi=(1.5, PI), width=(0.1, 0.3),
                    grid_n=(256, 256))
    c0 = rng.uniform(0.0, 1.0, size=n_hills)
    c1 = _uniform_circle(rng, n_hills)
    heights = rng.uniform(0.1, 1.2, size=n_hills)
    return spec, Hills(np.vstack([c0, c1]), heights)


def rmsd_walkers(seed=0, n_walkers=1, n_atoms=99137, cv_atoms=4, box=5.0, ref_jitter=0.3):
    """Walkers whose CVs are two offset-RMSDs of disjoint 4-atom sets.

    This is the shape of the paper's "universal benchmark" (about 99k atoms,
    two RMSD CVs of four atoms each). Reference positions are the current
    positions plus U[-ref_jitter, ref_jitter] per coordinate.
    Draw order: positions; masses; per walker: the 2*cv_atoms atom indices
    (sorted within each CV), reference offsets.
    """
    rng = np.random.default_rng(seed)
    n_atoms_arr = np.full(n_walkers, n_atoms, dtype=np.int32)
    atom_base = (np.arange(n_walkers, dtype=np.int64) * n_atoms)
    total = n_walkers * n_atoms
    pos = rng.uniform(0.0, box, size=(3, total)).astype(np.float32)
    mass = ATOM_MASSES[rng.integers(0, len(ATOM_MASSES), size=total)].astype(np.float32)
    lists = [[], [], [], []]
    refs = [[], [], [], []]
    for w in range(n_walkers):
        sel = rng.choice(n_atoms, size=2 * cv_atoms, replace=False)
        for cv in range(2):
            idx = np.sort(sel[cv * cv_atoms:(cv + 1) * cv_atoms]).astype(np.int32)
            g = int(atom_base[w]) + idx
            jit = rng.uniform(-ref_jitter, ref_jitter, size=(3, cv_atoms))
            ref = np.vstack([pos[0][g], pos[1][g], pos[2][g]]).astype(np.float64) + jit
            lists[cv * 2].append(idx)
            refs[cv * 2].append(ref.astype(np.float32))
            lists[cv * 2 + 1].append(np.zeros(0, dtype=np.int32))
            refs[cv * 2 + 1].append(np.zeros((3, 0), dtype=np.float32))
    list_off = np.zeros((2, 2, n_walkers + 1), dtype=np.int64)
    chunks, rchunks = [], []
    base = 0
    for gi in range(4):
        off = _csr(lists[gi]) + base
        list_off[gi // 2, gi % 2] = off
        base = int(off[-1])
        chunks.extend(lists[gi])
        rchunks.extend(refs[gi])
    list_idx = np.concatenate(chunks).astype(np.int32)
    ref = np.concatenate(rchunks, axis=1) if rchunks else np.zeros((3, 0), np.float32)
    kinds = np.array([CV_RMSD_OFF, CV_RMSD_OFF], dtype=np.int32)
    return Walkers(n_atoms=n_atoms_arr, atom_base=atom_base, x=pos[0].copy(), y=pos[1].copy(),
                   z=pos[2].copy(), mass=mass, kinds=kinds, list_off=list_off.astype(np.int32),
                   list_idx=list_idx, ref_x=ref[0].copy(), ref_y=ref[1].copy(), ref_z=ref[2].copy())


def serving_schedule(seed=0, n_walkers=4096, rate=200_000.0, n_requests=200_000):
    """Open-loop Poisson arrivals to uniformly chosen walkers.

    Returns (t_arrival_seconds float64 [n], walker int32 [n]). Inter-arrival
    times are exponential with mean 1/rate.
    Draw order: inter-arrival gaps, walker ids.
    """
    rng = np.random.default_rng(seed + 7)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps)
    w = rng.integers(0, n_walkers, size=n_requests).astype(np.int32)
    return t, w


def decaying_height(k):
    """Height law 1.2*exp(-k/20000) for hill index k (a workload choice, in kJ/mol)."""
    return 1.2 * np.exp(-np.asarray(k, dtype=np.float64) / 20000.0)


# ---------------------------------------------------------------------------
# Serving workloads: many walkers, requests arriving over time
# ---------------------------------------------------------------------------

def walker_lists(wk, w):
    """CV lists of walker w in registration form: (list_len[2*ncv] int32,
    list_idx int32, ref_x, ref_y, ref_z float32), lists in (cv, slot) order."""
    lens, idx, rx, ry, rz = [], [], [], [], []
    for a in range(wk.ncv):
        for t in range(2):
            lo, hi = int(wk.list_off[a, t, w]), int(wk.list_off[a, t, w + 1])
            lens.append(hi - lo)
            idx.append(wk.list_idx[lo:hi])
            rx.append(wk.ref_x[lo:hi])
            ry.append(wk.ref_y[lo:hi])
            rz.append(wk.ref_z[lo:hi])
    cat = lambda parts, dt: np.concatenate(parts).astype(dt) if parts else np.zeros(0, dt)
    return (np.array(lens, dtype=np.int32), cat(idx, np.int32), cat(rx, np.float32), cat(ry, np.float32),
            cat(rz, np.float32))


def single_walker(wk, w, x=None, y=None, z=None):
    """Walker w of a batch as a batch of its own (lists re-based, same atom
    order); x/y/z replace its positions when given."""
    b, n = int(wk.atom_base[w]), int(wk.n_atoms[w])
    lens, idx, rx, ry, rz = walker_lists(wk, w)
    off = np.zeros((wk.ncv, 2, 2), dtype=np.int32)
    pos = 0
    for q, ln in enumerate(lens):
        off[q // 2, q % 2] = (pos, pos + int(ln))
        pos += int(ln)
    pick = lambda given, pool: (pool[b:b + n] if given is None else given).astype(np.float32).copy()
    return Walkers(n_atoms=wk.n_atoms[w:w + 1].copy(), atom_base=np.zeros(1, np.int64),
                   x=pick(x, wk.x), y=pick(y, wk.y), z=pick(z, wk.z), mass=wk.mass[b:b + n].copy(),
                   kinds=wk.kinds, list_off=off, list_idx=idx, ref_x=rx, ref_y=ry, ref_z=rz)


def serving_requests(seed=0, n_walkers=1024, rate=200_000.0, n_requests=20_000, phase=0):
    """Open-loop schedule for the serving loop: (t_arrival, walker, step).

    Arrivals and walkers as in serving_schedule. Each walker's steps count up
    by one per request from a start of 1 + U{0..phase-1} (phase = 0: start at
    1), so a deposit period of `phase` steps is met by a fraction of the
    walkers within a short window. Draw order: serving_schedule's, then the
    start offsets.
    """
    t, w = serving_schedule(seed, n_walkers, rate, n_requests)
    start = np.ones(n_walkers, dtype=np.int64)
    if phase > 0:
        start += np.random.default_rng(seed + 11).integers(0, phase, size=n_walkers)
    step = np.zeros(n_requests, dtype=np.int64)
    count = np.zeros(n_walkers, dtype=np.int64)
    for i, wi in enumerate(w):
        step[i] = start[wi] + count[wi]
        count[wi] += 1
    return t, w, step


def serving_hills(seed=0, n_hills=200_000):
    """Pre-seeded history for the serving workload: centers as in
    ligand_pocket_hills, height of hill k from decaying_height(k)."""
    spec, hills = ligand_pocket_hills(seed, n_hills)
    return spec, Hills(hills.centers, decaying_height(np.arange(n_hills)))


def _mix32(h):
    """The 'lowbias32' integer mixer (C. Wellons, 2018) on uint32 arrays."""
    h = np.asarray(h, dtype=np.uint32)
    h = h ^ (h >> np.uint32(16))
    h = h * np.uint32(0x7FEB352D)
    h = h ^ (h >> np.uint32(15))
    h = h * np.uint32(0x846CA68B)
    h = h ^ (h >> np.uint32(16))
    return h


def engine_unit(walker, step, atom, coord):
    """u in [-1, 1) (multiples of 2^-15) of the synthetic engine step for
    (walker, step, atom, coordinate); arrays broadcast, all taken mod 2^32."""
    u32 = lambda v: (np.atleast_1d(np.asarray(v, dtype=np.int64)) & 0xFFFFFFFF).astype(np.uint32)
    inner = _mix32(u32(atom) * np.uint32(0xC2B2AE3D) + u32(coord))
    mid = _mix32((u32(step) * np.uint32(0x85EBCA77)) ^ inner)
    h = _mix32((u32(walker) * np.uint32(0x9E3779B1)) ^ mid)
    k = ((h >> np.uint32(16)) & np.uint32(0xFFFF)).astype(np.float32)
    return k * np.float32(1.0 / 32768.0) - np.float32(1.0)


def engine_positions(x0, y0, z0, walker, step, atoms, amplitude):
    """Positions the synthetic engine writes for `atoms` of a walker at a step:
    x0 + amplitude * u in float32 with round-to-nearest per operation (the
    device writes the same bits). Returns copies of x0/y0/z0 with those atoms
    replaced."""
    amp = np.float32(amplitude)
    out = []
    atoms = np.unique(np.asarray(atoms, dtype=np.int64))
    for c, base in enumerate((x0, y0, z0)):
        p = np.asarray(base, dtype=np.float32).copy()
        u = engine_unit(walker, step, atoms, c)
        p[atoms] = p[atoms] + (amp * u).astype(np.float32)
        out.append(p)
    return out


def paper_grid_2d(seed=0, n_hills=20000, a_spacings=10, p=20, step=0.02, start=(1.0, 1.0)):
    """The paper's discretisation for its ligand-binding runs, in the quantised
    mode: two CVs on [0, 12] nm with 480 x 480 grid nodes, compact hills S_a^p
    with a = a_spacings node spacings (10 or 20 in the paper) and p = 20, mABP
    with c = 0.001, b = 0.9 at 300 K. Hill centres follow a Gaussian random walk
    from `start` with step sd `step` nm, reflected into [0, 12] (a stand-in for
    the visited CV values); heights 1 (one count per deposit).
    Draw order: the walk's steps.
    """
    dx = 12.0 / 479
    spec = BiasSpec(ndim=2, periodic=(0, 0), lo=(0.0, 0.0), hi=(12.0, 12.0), kernel=KERNEL_COMPACT,
                    width=(a_spacings * dx, a_spacings * dx), p=p, transform=TRANSFORM_MABP, kT=KT_300K,
                    b=0.9, c=0.001, grid_n=(480, 480), quantize=1)
    rng = np.random.default_rng(seed + 5)
    steps = rng.normal(0.0, step, (2, n_hills))
    c = np.empty((2, n_hills))
    x = np.array(start, dtype=np.float64)
    for k in range(n_hills):
        x = x + steps[:, k]
        x = np.where(x < 0.0, -x, x)
        x = np.where(x > 12.0, 24.0 - x, x)
        c[:, k] = x
    return spec, Hills(c, np.ones(n_hills))
