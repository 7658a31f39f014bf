#!/usr/bin/env python
"""Benchmark of the bias-force hot path on one MI355X.

Headline: bias evaluations per second (walker-steps/s) of the direct hill
sum in FP32 with Kahan compensation, on the 2-D torsion workload (50,000
hills, heights 1.2 exp(-k/20000), sigma 0.3; 1,048,576 queries = 1024
walkers x 1024 steps), inputs resident in HBM. One step = one bias_eval over
all queries. Printed as one JSON line, with the FP64 direct sum, the plain
FP32 sum, the grid path, the fused bias-force path and (when built) the
serving loop's latency as secondary figures, the roofline of the direct-sum
kernel, and the FP64 CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks and the figures derived from unit counts.
CU, LANES, CLOCK = 256, 64, 2.4e9
FP32_VECTOR_PEAK_TFLOPS = 157.3        # published: packed FMA on every lane every clock
FP64_VECTOR_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
VALU_LANE_OPS = CU * LANES * CLOCK     # non-packed VALU issue: 3.93e13 lane-ops/s
# Algorithmic flops per (query, hill) pair of the 2-D periodic Gaussian sum:
# per axis: difference 1, minimum image 2, scale 1, square-accumulate 2,
# gradient FMA 2; plus height multiply 1 and value add 1; the exp is not counted.
FLOPS_PER_PAIR_2D = 18
FP32_NONPACKED_PEAK_TFLOPS = VALU_LANE_OPS * 2 / 1e12   # FMA on every lane, no packed FP32: 78.6

# HBM bytes per launch of the headline kernel from rocprofv3 FETCH_SIZE (x 2,
# copy-calibrated) and WRITE_SIZE (x 1), valid only for the kernel sources
# they were taken on.
HEADLINE_TRAFFIC = {"sources_sha256": "d0bd6a969ad4991586539920b6e5d502a960f9ba454a64d35bb20db5d41036bb", "fetch_kib": 7305.6, "write_kib": 12288.0,
                    "fetch_scale": 2.0, "write_scale": 1.0}
HEADLINE_SOURCES = ("paper_1609_09833_amd/csrc/direct_sum_impl.h", "paper_1609_09833_amd/csrc/direct_sum_d2.hip",
                    "paper_1609_09833_amd/csrc/direct_sum.hip", "paper_1609_09833_amd/csrc/abp_device.h",
                    "paper_1609_09833_amd/csrc/abp_internal.h")


def sources_sha256(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def headline_traffic():
    """Measured HBM bytes per launch, or None if the kernel changed since."""
    t = HEADLINE_TRAFFIC
    if sources_sha256(HEADLINE_SOURCES) != t["sources_sha256"]:
        return None
    return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def timed(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3, wall


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo, as lscpu reports it)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


ONE_CORE_SCRIPT = """
import sys, time
import numpy as np
sys.path.insert(0, {root!r})
import oracle
from paper_1609_09833_amd import workloads as W
spec, hills, q = W.torsion_2d()
idx = np.linspace(0, q.shape[1] - 1, {n}).astype(np.int64)
t0 = time.perf_counter()
oracle.hill_sum(spec, hills.centers, hills.heights, q[:, idx])
print(time.perf_counter() - t0)
"""


def cpu_baseline(spec, hills, q, target_s=20.0):
    """The FP64 oracle on an evenly spaced sample of the queries, all host
    cores; then one core (OMP_NUM_THREADS=1, a child process) on a smaller
    sample."""
    import subprocess
    import numpy as np
    import oracle
    nq = q.shape[1]
    probe = 2048
    idx = np.linspace(0, nq - 1, probe).astype(np.int64)
    t0 = time.perf_counter()
    oracle.hill_sum(spec, hills.centers, hills.heights, q[:, idx])
    dt = time.perf_counter() - t0
    n = int(min(nq, max(probe, probe * target_s / max(dt, 1e-6))))
    idx = np.linspace(0, nq - 1, n).astype(np.int64)
    t0 = time.perf_counter()
    oracle.hill_sum(spec, hills.centers, hills.heights, q[:, idx])
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {"value": n / dt, "unit": "walker-steps/s", "cores": cores, "kind": "oracle",
           "sample": f"{n} of {nq} queries (evenly spaced) against all {hills.n} hills, FP64, {dt:.1f} s",
           "cpu_model": cpu_model()}
    n1 = max(64, int(n / cores / 2))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", ONE_CORE_SCRIPT.format(root=ROOT, n=n1)], env=env,
                           capture_output=True, text=True, timeout=300, check=True)
        dt1 = float(r.stdout.strip().splitlines()[-1])
        out["one_core"] = {"value": n1 / dt1, "unit": "walker-steps/s", "cores": 1,
                           "sample": f"{n1} of {nq} queries (evenly spaced), FP64, {dt1:.1f} s"}
    except (subprocess.SubprocessError, ValueError, IndexError) as e:
        out["one_core"] = {"error": str(e)[:200]}
    return out


def force_leg(abp, W, torch, args, stream):
    """Fused bias force on 1024 walkers of 2,000-8,000 atoms (COM distance +
    torsion), 20,000 hills: direct sum and grid, plus cv_compute alone."""
    dev = torch.device("cuda", 0)
    extra = {}
    wk = W.ligand_pocket_walkers()
    fspec, fhills = W.ligand_pocket_hills()
    fctx = abp.Context(fspec, capacity=fhills.n)
    abp.bias_deposit(fctx, torch.as_tensor(fhills.centers, device=dev), torch.as_tensor(fhills.heights, device=dev))
    dw = abp.DeviceWalkers(wk, device=dev)
    s_o = torch.empty((2, wk.nw), dtype=torch.float64, device=dev)
    V_o = torch.empty(wk.nw, dtype=torch.float64, device=dev)
    dV_o = torch.empty((2, wk.nw), dtype=torch.float64, device=dev)
    for mode, name in ((abp.ABP_EVAL_DIRECT, "bias_force_direct"), (abp.ABP_EVAL_GRID, "bias_force_grid")):
        def fstep(mode=mode):
            abp.bias_force(fctx, dw, mode=mode, s=s_o, V=V_o, dVds=dV_o)
        el4, _ = timed(fstep, args.steps, 2, stream)
        extra[name] = {"walker_steps_per_s": wk.nw * args.steps / el4, "ms_per_step": el4 / args.steps * 1e3,
                       "walkers": wk.nw, "hills": fhills.n}
        log(f"bench: {name} {wk.nw * args.steps / el4:.4e} walker-steps/s")

    def cstep():
        abp.cv_compute(fctx, dw, s=s_o)
    el5, _ = timed(cstep, args.steps, 2, stream)
    extra["cv_compute"] = {"walker_steps_per_s": wk.nw * args.steps / el5, "ms_per_step": el5 / args.steps * 1e3}
    log(f"bench: cv_compute {wk.nw * args.steps / el5:.4e} walker-steps/s")
    abp.abp_sync(fctx)
    fctx.close()
    return extra


def latency_leg(abp, W, torch, calls=200):
    """One walker of 99,137 atoms with two 4-atom offset-RMSD CVs (the shape of
    the paper's universal benchmark), mABP with compact hills (p = 20) on a
    480 x 480 grid over [0, 12] nm: latency of one bias_force call, direct sum
    at 3,000 and 100,000 hills and grid form."""
    import numpy as np
    dev = torch.device("cuda", 0)
    wk = W.rmsd_walkers(seed=2, n_walkers=1)
    spec = W.BiasSpec(ndim=2, periodic=(0, 0), lo=(0.0, 0.0), hi=(12.0, 12.0), width=(0.25, 0.25),
                      kernel=W.KERNEL_COMPACT, p=20, transform=W.TRANSFORM_MABP, kT=W.KT_300K, b=0.9, c=0.001,
                      grid_n=(480, 480))
    rng = np.random.default_rng(9)
    dw = abp.DeviceWalkers(wk, device=dev)
    s_o = torch.empty((2, 1), dtype=torch.float64, device=dev)
    V_o = torch.empty(1, dtype=torch.float64, device=dev)
    dV_o = torch.empty((2, 1), dtype=torch.float64, device=dev)
    out = {"walker": "99,137 atoms, two 4-atom RMSD_OFF CVs", "calls": calls}
    for n_hills in (3000, 100_000):
        ctx = abp.Context(spec, capacity=n_hills)
        cen = torch.as_tensor(rng.uniform(0.1, 0.4, (2, n_hills)), device=dev)
        abp.bias_deposit(ctx, cen, torch.ones(n_hills, dtype=torch.float64, device=dev))
        torch.cuda.synchronize()
        for mode, name in ((abp.ABP_EVAL_DIRECT, "direct"), (abp.ABP_EVAL_GRID, "grid")):
            def call(mode=mode):
                abp.bias_force(ctx, dw, mode=mode, s=s_o, V=V_o, dVds=dV_o)
            for _ in range(10):
                call()
            torch.cuda.synchronize()
            lat = np.empty(calls)
            for i in range(calls):
                t0 = time.perf_counter()
                call()
                torch.cuda.synchronize()
                lat[i] = time.perf_counter() - t0
            el, _ = timed(call, calls, 0, torch.cuda.current_stream())
            key = f"{name}_{n_hills}_hills"
            out[key] = {"p50_us": float(np.percentile(lat, 50) * 1e6), "p99_us": float(np.percentile(lat, 99) * 1e6),
                        "back_to_back_us": el / calls * 1e6}
            log(f"bench: single walker {key}: p50 {out[key]['p50_us']:.1f} us, back-to-back "
                f"{out[key]['back_to_back_us']:.1f} us per call")
        abp.abp_sync(ctx)
        ctx.close()
    return out


def quantised_leg(abp, W, torch, n_hills=20000, single=2000, steps=10):
    """The paper's own discretisation in the quantised mode: 480 x 480 nodes over
    [0, 12] nm, compact hills (a = 10 node spacings, p = 20), mABP; hills are
    moved to their nearest node and the force is a look-up at the node. Times
    a batched deposit, one-hill deposits (one per MD step, as in the paper),
    the look-up for 1,048,576 queries and one walker's bias_force."""
    import numpy as np
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    spec, hills = W.paper_grid_2d(seed=7, n_hills=n_hills + single)
    out = {"grid": "480 x 480 over [0, 12] nm", "a_spacings": 10, "p": 20,
           "node_updates_per_deposit": 19 * 19}
    ctx = abp.Context(spec, capacity=2 * n_hills + single)
    cen = torch.as_tensor(hills.centers, device=dev)
    hts = torch.as_tensor(hills.heights, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    first = (cen[:, :n_hills].contiguous(), hts[:n_hills].contiguous())
    abp.bias_deposit(ctx, *first)          # untimed: the context's scratch is allocated here
    torch.cuda.synchronize()
    e0.record(stream)
    abp.bias_deposit(ctx, *first)          # the same batch again, timed
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    out["batched_deposit"] = {"hills": n_hills, "ms": ms, "hills_per_s": n_hills / ms * 1e3}
    one = [(cen[:, k:k + 1].contiguous(), hts[k:k + 1].contiguous()) for k in range(n_hills, n_hills + single)]
    it = iter(one)

    def dep():
        c, h = next(it)
        abp.bias_deposit(ctx, c, h)
    el, _ = timed(dep, single - 10, 10, stream)
    out["one_hill_deposit_us"] = el / (single - 10) * 1e6
    q = torch.as_tensor(np.random.default_rng(8).uniform(0.0, 4.0, (2, 1 << 20)).astype(np.float32), device=dev)
    V = torch.empty(1 << 20, dtype=torch.float32, device=dev)
    dV = torch.empty((2, 1 << 20), dtype=torch.float32, device=dev)

    def look():
        abp.bias_eval(ctx, q, mode=abp.ABP_EVAL_GRID, V=V, dVds=dV)
    el, _ = timed(look, steps, 2, stream)
    out["look_up"] = {"queries": 1 << 20, "walker_steps_per_s": (1 << 20) * steps / el,
                      "ms_per_step": el / steps * 1e3}
    wk = W.rmsd_walkers(seed=2, n_walkers=1)
    dw = abp.DeviceWalkers(wk, device=dev)
    s_o = torch.empty((2, 1), dtype=torch.float64, device=dev)
    V_o = torch.empty(1, dtype=torch.float64, device=dev)
    dV_o = torch.empty((2, 1), dtype=torch.float64, device=dev)

    def force():
        abp.bias_force(ctx, dw, mode=abp.ABP_EVAL_GRID, s=s_o, V=V_o, dVds=dV_o)
    el, _ = timed(force, 200, 10, stream)
    out["one_walker_bias_force_us"] = el / 200 * 1e6
    abp.abp_sync(ctx)
    ctx.close()
    log(f"bench: quantised grid: batched deposit {out['batched_deposit']['hills_per_s']:.3e} hills/s, one-hill "
        f"deposit {out['one_hill_deposit_us']:.1f} us, look-up {out['look_up']['walker_steps_per_s']:.3e} "
        f"walker-steps/s, one-walker force {out['one_walker_bias_force_us']:.1f} us")
    return out


def serving_leg(abp, W, torch, window_s=1.0):
    """The serving workload: 4,096 walkers of 1,000-20,000 atoms (COM distance
    + torsion CVs, 250-690 CV atoms each), Poisson arrivals at 200,000
    requests/s to uniformly chosen walkers, each request carrying its walker's
    CV-atom positions for one step (synthetic engine: base positions plus a
    hashed displacement) and returning the forces on them; a deposit every
    500th step of a walker (heights 1.2 exp(-k/20000)); 2-D history pre-seeded
    to 0, 100,000 and 200,000 hills; walkers' resident device state (CV-atom
    masses) admitted against a budget of 2 MiB (about 28% of the walkers) or
    all resident. Requests
    are submitted and polled by the load generator in
    paper_1609_09833_amd/examples (a client of the C-ABI). Latency is arrival
    to the scheduler's observed completion, on the host clock."""
    import numpy as np
    from paper_1609_09833_amd.examples import serve_driver as D
    rate, n_walkers, period, amp = 200_000.0, 4096, 500, 2.0 ** -7
    log("bench: serving: generating 4,096 walkers of 1,000-20,000 atoms")
    wk = W.ligand_pocket_walkers(seed=11, n_walkers=n_walkers, atoms_lo=1000, atoms_hi=20000)
    spec, seed_hills = W.serving_hills(seed=11, n_hills=200_000)
    ctx = abp.Context(spec, capacity=260_000)
    dev = torch.device("cuda", 0)
    cen = torch.as_tensor(seed_hills.centers, device=dev)
    hts = torch.as_tensor(seed_hills.heights, device=dev)
    state = {"seeded": 0}

    def seed_to(n):
        k = state["seeded"]
        have = ctx.num_hills
        if n > have:
            take = n - have
            abp.bias_deposit(ctx, cen[:, k:k + take].contiguous(), hts[k:k + take].contiguous())
            state["seeded"] = k + take
        torch.cuda.synchronize()

    def server(budget, max_batch, streams, mode=abp.ABP_EVAL_DIRECT):
        srv = abp.Server(ctx, wk.kinds, hbm_budget_bytes=budget, max_batch=max_batch, streams=streams,
                         deposit_every=period, height0=1.2, height_decay=20000.0, max_pending=16384,
                         eval_mode=mode)
        for w in range(wk.nw):
            b, n = int(wk.atom_base[w]), int(wk.n_atoms[w])
            lens, idx, rx, ry, rz = W.walker_lists(wk, w)
            srv.add_walker(wk.mass[b:b + n], lens, idx)
        return srv, D.Engines(srv, wk)

    def run(srv, eng, name, n_req, seed, req_rate=rate):
        t, w, step = W.serving_requests(seed=seed, n_walkers=n_walkers, rate=req_rate, n_requests=n_req,
                                        phase=period)
        if req_rate > 1e8:
            t = np.zeros_like(t)
        srv.start()
        out = D.replay(srv, eng, w, step, t, amp, forces=True, threads=16)
        srv.stop()
        st = srv.stats()
        tr = srv.trace()
        lat = (out["t_done"] - t) * 1e6
        batch_us = (tr["t_done"] - tr["t_formed"]) * 1e6
        enqueue_us = (tr["t_launched"] - tr["t_formed"]) * 1e6
        r = {"requests": n_req, "offered_req_per_s": None if req_rate > 1e8 else req_rate,
             "completed_req_per_s": n_req / float(out["t_done"].max()),
             "p50_us": float(np.percentile(lat, 50)), "p99_us": float(np.percentile(lat, 99)),
             "p999_us": float(np.percentile(lat, 99.9)), "max_us": float(lat.max()),
             "batches": st["batches"], "mean_batch": n_req / max(st["batches"], 1), "max_batch": st["max_batch_seen"],
             "batch_formed_to_done_us": {"p50": float(np.percentile(batch_us, 50)),
                                         "p99": float(np.percentile(batch_us, 99)), "max": float(batch_us.max())},
             "batch_enqueue_us": {"p50": float(np.percentile(enqueue_us, 50)),
                                  "p99": float(np.percentile(enqueue_us, 99)), "max": float(enqueue_us.max())},
             "admissions": st["admissions"], "evictions": st["evictions"], "deposits": st["deposits"],
             "peak_resident_walkers": st["peak_resident"],
             "hills_seen": [int(out["version"].min()), int(out["version"].max())]}
        log(f"bench: serving {name}: {r['completed_req_per_s']:.4g} req/s, p50 {r['p50_us']:.1f} us, "
            f"p99 {r['p99_us']:.1f} us, p99.9 {r['p999_us']:.1f} us, mean batch {r['mean_batch']:.1f}, "
            f"evictions {r['evictions']}")
        return r

    res = {}
    n_win = int(rate * window_s)
    budget = 2 << 20
    srv, eng = server(budget, 1024, 2)     # two batches in flight
    run(srv, eng, "warm-up (not reported)", n_win // 5, 99)
    for i, hist in enumerate((0, 100_000, 200_000)):
        seed_to(hist)
        res[f"hist{hist // 1000}k_budget2MiB"] = run(srv, eng, f"{hist} hills, 2 MiB", n_win, 100 + i)
    res["hist200k_budget2MiB_saturated"] = run(srv, eng, "saturated", n_win, 110, req_rate=1e12)
    srv.close()
    srv, eng = server(1 << 30, 1024, 2)
    res["hist200k_all_resident"] = run(srv, eng, "200k hills, all resident", n_win, 120)
    srv.close()
    srv, eng = server(1 << 30, 1, 4)
    res["hist200k_plain_launches"] = run(srv, eng, "plain per-walker launches", n_win // 10, 130)
    res["hist200k_plain_launches_saturated"] = run(srv, eng, "plain saturated", n_win // 10, 131, req_rate=1e12)
    srv.close()
    # GRID evaluation: the same requests read the 256 x 256 grid (kept current
    # by the deposits' commits) instead of summing the 200k hills
    srv, eng = server(budget, 1024, 2, abp.ABP_EVAL_GRID)
    run(srv, eng, "grid warm-up (not reported)", n_win // 5, 139)
    res["hist200k_budget2MiB_grid"] = run(srv, eng, "200k hills, 2 MiB, grid", n_win, 140)
    res["hist200k_budget2MiB_grid_saturated"] = run(srv, eng, "grid saturated", n_win, 141, req_rate=1e12)
    srv.close()
    ctx.close()
    return res


def grid_leg(abp, torch, args, stream, spec, nh, cen_d, hts_d, qd, V, dV):
    """Grid form on the headline workload: accumulate the 50,000 hills into the
    256^2 FP64 grid, then interpolate at all 1,048,576 queries. A context's first
    deposit also allocates the deposit's split scratch, so the build time
    reported is a second deposit of the same 50,000 hills into the same context."""
    nq = qd.shape[1]
    extra = {}
    gctx = abp.Context(spec, capacity=2 * nh)
    times = []
    for _ in range(2):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        abp.bias_deposit(gctx, cen_d, hts_d)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    abp.abp_sync(gctx)
    extra["grid_build_ms"] = times[1]
    extra["grid_build_first_call_ms"] = times[0]
    # algorithmic work of the deposit: 2^ndim FMAs per (node, hill)
    nodes = 1
    for n in spec.grid_n[:spec.ndim]:
        nodes *= n
    dep_tflops = 2.0 * (1 << spec.ndim) * nodes * nh / (times[1] * 1e-3) / 1e12
    extra["grid_build_roofline"] = {"bound": "mfma", "achieved": dep_tflops, "peak": FP64_VECTOR_PEAK_TFLOPS,
                                    "unit": "TFLOP/s", "frac": dep_tflops / FP64_VECTOR_PEAK_TFLOPS,
                                    "note": "FP64 MFMA deposit; the timed call includes the history append "
                                            "and the split reduction"}

    for key, prec in (("grid_eval", abp.ABP_PREC_FP64), ("grid_eval_fp32_nodes", abp.ABP_PREC_FP32_KAHAN)):
        def grid_step(prec=prec):
            abp.bias_eval(gctx, qd, mode=abp.ABP_EVAL_GRID, prec=prec, V=V, dVds=dV)
        el3, _ = timed(grid_step, args.steps, 2, stream)
        extra[key] = {"walker_steps_per_s": nq * args.steps / el3, "ms_per_step": el3 / args.steps * 1e3,
                      "node_values": "FP64" if prec == abp.ABP_PREC_FP64 else "FP32 mirror",
                      "hbm_GBs_compulsory": nq * 20 * args.steps / el3 / 1e9,
                      "frac_hbm_compulsory": nq * 20 * args.steps / el3 / 1e9 / HBM_PEAK_GBS}
        log(f"bench: {key} {nq * args.steps / el3:.4e} walker-steps/s ({el3 / args.steps * 1e6:.1f} us)")
    log(f"bench: grid build {extra['grid_build_ms']:.2f} ms")
    gctx.close()
    return extra


def stress_direct_leg(abp, W, torch, n_queries=1 << 18):
    """The precision-stress direct sum: 3-D CV space (a distance and two
    torsions), 1,000,000 hills with heights log-uniform on [1e-4, 1]; the first
    n_queries of its 4,194,304 queries (the kernel's rate does not depend on
    the query count once the chip is full), FP32 + Kahan, FP32 naive and FP64."""
    spec, hills, q = W.stress_3d()
    q = q[:, :n_queries].copy()
    ctx = abp.Context(spec, capacity=hills.n)
    abp.bias_deposit(ctx, torch.as_tensor(hills.centers, device="cuda"), torch.as_tensor(hills.heights, device="cuda"))
    qd = torch.as_tensor(q, device="cuda")
    V = torch.empty(q.shape[1], dtype=torch.float32, device="cuda")
    dV = torch.empty((3, q.shape[1]), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    out = {"hills": hills.n, "queries": q.shape[1], "of_queries": 4 << 20}
    for name, prec, steps in (("fp32_kahan", abp.ABP_PREC_FP32_KAHAN, 3), ("fp32_naive", abp.ABP_PREC_FP32_NAIVE, 3),
                              ("fp64", abp.ABP_PREC_FP64, 2)):
        def fn(prec=prec):
            abp.bias_eval(ctx, qd, prec=prec, V=V, dVds=dV)
        el, _ = timed(fn, steps, 1, stream)
        pairs = q.shape[1] * hills.n * steps / el
        out[name] = {"walker_steps_per_s": q.shape[1] * steps / el, "pairs_per_s": pairs,
                     "ms_per_step": el / steps * 1e3}
        log(f"bench: stress direct {name}: {pairs:.3e} pairs/s ({q.shape[1] * steps / el:.3e} walker-steps/s "
            f"at 1M hills)")
    abp.abp_sync(ctx)
    ctx.close()
    return out


def stress_grid_leg(abp, W, torch):
    """The precision-stress grid: 1,000,000 Gaussian hills (a distance and two
    torsions) into the 128^3 FP64 grid, deposited twice into one context; the
    reported time is the second deposit (the first also allocates)."""
    spec, hills, _ = W.stress_3d(n_queries=1)
    cen = torch.as_tensor(hills.centers, device="cuda")
    hts = torch.as_tensor(hills.heights, device="cuda")
    ctx = abp.Context(spec, capacity=2 * hills.n)
    stream = torch.cuda.current_stream()
    times = []
    for _ in range(2):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        abp.bias_deposit(ctx, cen, hts)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    abp.abp_sync(ctx)
    ctx.close()
    flops = 2.0 * 8 * 128 ** 3 * hills.n
    log(f"bench: stress grid build {times[1]:.1f} ms ({flops / times[1] / 1e9:.1f} TFLOP/s of deposit FMAs)")
    return {"hills": hills.n, "grid": "128^3 x 8 FP64", "build_ms": times[1], "first_call_ms": times[0],
            "deposit_tflops": flops / times[1] / 1e9,
            "frac_fp64_peak": flops / times[1] / 1e9 / FP64_VECTOR_PEAK_TFLOPS}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--only-headline", action="store_true", help="time the headline kernel only (profiling)")
    ap.add_argument("--only", choices=("headline", "grid", "stress-grid", "stress-direct", "force", "latency",
                                       "serving", "quantised"), default=None,
                    help="run one leg only (profiling): the headline direct sum, its grid form, the "
                         "bias-force workload, single-walker latency, the quantised grid, the 128^3 "
                         "precision-stress grid build or serving")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a 1 GiB device-to-device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path has no multi-GPU form "
              "in this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1609_09833_amd import abp
    from paper_1609_09833_amd import workloads as W

    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    if args.only_headline:
        args.only = "headline"
    if args.only == "force":
        print(json.dumps({"extra": force_leg(abp, W, torch, args, stream)}), flush=True)
        return
    if args.only == "latency":
        print(json.dumps({"extra": {"single_walker_latency": latency_leg(abp, W, torch)}}), flush=True)
        return
    if args.only == "quantised":
        print(json.dumps({"extra": {"quantised_grid": quantised_leg(abp, W, torch)}}), flush=True)
        return
    if args.only == "stress-grid":
        print(json.dumps({"extra": {"stress_grid": stress_grid_leg(abp, W, torch)}}), flush=True)
        return
    if args.only == "stress-direct":
        print(json.dumps({"extra": {"stress_direct": stress_direct_leg(abp, W, torch)}}), flush=True)
        return
    if args.only == "serving":
        print(json.dumps({"extra": {"serving": serving_leg(abp, W, torch)}}), flush=True)
        return
    if args.calibrate_copy:
        n = 1 << 28                                   # 2^28 float32 = 1 GiB read + 1 GiB written per copy
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: copied 1 GiB three times")
        return
    log("bench: generating the 2-D torsion workload (50,000 hills, 1,048,576 queries)")
    spec, hills, q = W.torsion_2d()
    nq, nh = q.shape[1], hills.n
    ctx = abp.Context(spec, capacity=nh)
    cen_d = torch.as_tensor(hills.centers, device=dev)
    hts_d = torch.as_tensor(hills.heights, device=dev)
    t0 = time.perf_counter()
    abp.bias_deposit(ctx, cen_d, hts_d)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    qd = torch.as_tensor(q, device=dev)
    V = torch.empty(nq, dtype=torch.float32, device=dev)
    dV = torch.empty((2, nq), dtype=torch.float32, device=dev)
    if args.only == "grid":
        print(json.dumps({"extra": grid_leg(abp, torch, args, stream, spec, nh, cen_d, hts_d, qd, V, dV)}),
              flush=True)
        return

    def step_kahan():
        abp.bias_eval(ctx, qd, prec=abp.ABP_PREC_FP32_KAHAN, V=V, dVds=dV)

    log(f"bench: headline FP32-Kahan direct sum, {args.warmup} warmup + {args.steps} timed steps")
    el, wall = timed(step_kahan, args.steps, args.warmup, stream)
    abp.abp_sync(ctx)
    ms_step = el / args.steps * 1e3
    value = nq * args.steps / el
    pairs_s = value * nh
    achieved_tflops = pairs_s * FLOPS_PER_PAIR_2D / 1e12
    out = {
        "metric": "bias-force evals/sec (walker-steps) at 50k hills, FP32 vs FP64 plain; p99 latency",
        "value": value,
        "unit": "walker-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2-D periodic torsion CV space, direct hill sum, FP32 + Kahan, plain bias",
                   "hills": nh, "queries_per_step": nq, "walkers": 1024, "steps_per_walker": 1024,
                   "sigma": [0.3, 0.3], "heights": "1.2*exp(-k/20000)", "query_io": "f32"},
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tflops / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": headline_traffic(),
                     "kernel": "k_direct_f32<2,0,GAUSS,ISO,KAHAN,2>", "pairs_per_s": pairs_s,
                     "kernel_ms": ms_step, "flops_per_pair": FLOPS_PER_PAIR_2D,
                     "peak_no_packed_fp32": FP32_NONPACKED_PEAK_TFLOPS,
                     "frac_no_packed_fp32": achieved_tflops / FP32_NONPACKED_PEAK_TFLOPS},
    }
    log(f"bench: headline {value:.4e} walker-steps/s ({ms_step:.3f} ms/step, {pairs_s:.3e} pairs/s)")
    if args.only == "headline":
        print(json.dumps(out), flush=True)
        return

    extra = {}
    for name, prec, steps in (("fp64_direct", abp.ABP_PREC_FP64, max(2, args.steps // 4)),
                              ("fp32_naive_direct", abp.ABP_PREC_FP32_NAIVE, args.steps)):
        def fn(prec=prec):
            abp.bias_eval(ctx, qd, prec=prec, V=V, dVds=dV)
        el2, _ = timed(fn, steps, 1, stream)
        extra[name] = {"walker_steps_per_s": nq * steps / el2, "ms_per_step": el2 / steps * 1e3}
        if prec == abp.ABP_PREC_FP64:
            # the same 18 algorithmic flops per pair, against the FP64 peak
            tf = nq * steps / el2 * nh * FLOPS_PER_PAIR_2D / 1e12
            extra[name]["roofline"] = {"bound": "alu", "achieved": tf, "peak": FP64_VECTOR_PEAK_TFLOPS,
                                       "unit": "TFLOP/s", "frac": tf / FP64_VECTOR_PEAK_TFLOPS,
                                       "note": "the exponential (about 16 FP64 instructions) is not counted"}
        log(f"bench: {name} {nq * steps / el2:.4e} walker-steps/s")
    extra.update(grid_leg(abp, torch, args, stream, spec, nh, cen_d, hts_d, qd, V, dV))
    del build_s
    extra.update(force_leg(abp, W, torch, args, stream))
    extra["single_walker_latency"] = latency_leg(abp, W, torch)
    extra["quantised_grid"] = quantised_leg(abp, W, torch)
    extra["stress_grid"] = stress_grid_leg(abp, W, torch)
    extra["stress_direct"] = stress_direct_leg(abp, W, torch)
    if not args.no_serving:
        sv = serving_leg(abp, W, torch)
        head = sv["hist200k_budget2MiB"]
        out["serving"] = {"workload": "4,096 walkers of 1,000-20,000 atoms, Poisson 200k req/s, CV-atom "
                                      "positions in and forces out per request, 200k-hill history, 2 MiB "
                                      "walker budget (about 28% resident), batched",
                          "p50_us": head["p50_us"], "p99_us": head["p99_us"], "p999_us": head["p999_us"],
                          "completed_req_per_s": head["completed_req_per_s"],
                          "plain_launch_p99_us": sv["hist200k_plain_launches"]["p99_us"],
                          "plain_launch_capacity_req_per_s":
                              sv["hist200k_plain_launches_saturated"]["completed_req_per_s"],
                          "batched_capacity_req_per_s":
                              sv["hist200k_budget2MiB_saturated"]["completed_req_per_s"],
                          "grid_mode": {k: sv["hist200k_budget2MiB_grid"][k]
                                        for k in ("p50_us", "p99_us", "p999_us", "completed_req_per_s")},
                          "grid_mode_capacity_req_per_s":
                              sv["hist200k_budget2MiB_grid_saturated"]["completed_req_per_s"]}
        extra["serving"] = sv
    out["extra"] = extra
    out["valu_issue"] = {"lane_ops_per_s_peak": VALU_LANE_OPS,
                         "note": "non-packed VALU issue rate, 256 CU x 64 lanes x 2.4 GHz"}
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(spec, hills, q)
        log(f"bench: oracle {out['cpu_baseline']['value']:.4e} walker-steps/s on {out['cpu_baseline']['cores']} cores")
    del np
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
