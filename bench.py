"""Throughput of the deconvolution solve on one MI355X.

One step = one solve of G u = ubar to relative residual 1e-6 (recursive
residual normalised by ||ubar - G ubar||) over the whole batch of the
workload, inputs resident in HBM, through the C ABI.  Default workload: 16
independent 2048^2 vorticity fields with a k^-3 spectrum (4 <= k <= 512),
FP32 storage and stencil/vector arithmetic, FP64 inner products and scalars,
BiCGSTAB.  CG and Van Cittert are timed on the same batch for the
"vs Van Cittert" ratio.

Prints one JSON line.  `value` = grid points of the batch / mean time per
solve (points/s).  `roofline` prices the persistent solve kernel's
algorithmic HBM bytes against 8 TB/s.  `cpu_baseline` times the CPU FP64
oracle on a bounded sample of the same workload (rank 0, N=1).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "deconvolved grid points/s to rel. residual 1e-6; % HBM roofline; vs Van Cittert"

# Algorithmic field accesses per grid point (one access = one full-field read
# or write), the method's own count of Algorithms 1-4 with every vector read or
# written once per pass: per pass 4 (VC), 5 (SD), 8 (CG), 15 (BiCGSTAB), plus
# init and the exit true residual: VC 4n + 5, SD 5n + 5, CG 8n + 6, BiCGSTAB
# 15n + 6.  Halo re-reads are not counted.  The roofline fraction is priced on
# these counts.
def accesses(solver: str, iters: int) -> int:
    per_pass, fixed = {"vc": (4, 5), "sd": (5, 5), "cg": (8, 6), "bicgstab": (15, 6)}[solver]
    return per_pass * max(iters, 0) + fixed


# The accesses the fused kernels actually make: the first CG pass does not
# re-read p0 = r0 and the first BiCGSTAB pass does not read p0 = q0 = 0, and
# the CG init writes no separate p0 (the counts above minus 2).  Reported
# beside the method's count.
def kernel_accesses(solver: str, iters: int) -> int:
    if iters <= 0:
        return 5 if solver != "bicgstab" else 6
    if solver == "vc":
        return 3 + 4 * iters + 2
    if solver == "cg":
        return 3 + 7 + 8 * (iters - 1) + 2
    if solver == "bicgstab":
        return 4 + 13 + 15 * (iters - 1) + 2
    if solver == "sd":
        return 3 + 5 * iters + 2
    raise ValueError(solver)


WORKLOADS = {
    "c2": dict(desc="2D periodic 2048^2 x 16 fields, E(k)~k^-3 on 4<=k<=512, trapezoidal filter, "
                    "BiCGSTAB to rel. residual 1e-6 (FP32 storage/stencil/updates, FP64 dots/scalars)",
               cfg=2, ndim=2, n=2048, count=16, key="2048sq_x16"),
    "c4": dict(desc="uneven batch of 200 scalar fields in one persistent launch: 2D n=64*U{4..32} (k^-3 on 4<=k<=n/4) "
                    "and 3D n=16*U{4..12} (k^-5/3 on 2<=k<=0.3125n) with probability 1/2, BiCGSTAB to rel. residual "
                    "1e-6 (FP32 storage, FP64 dots/scalars), launch autotuned before timing",
               cfg=4, count=200, key="uneven200", batch=True),
    "c5": dict(desc="learned warm start: 2D CNN trained on the GPU (Adam) on 4096 seeded (ubar, u) pairs of "
                    "periodic 512^2 k^-3 fields (4<=k<=128), evaluated on 64 held-out 1024^2 fields (k^-3 on "
                    "4<=k<=256): BiCGSTAB to rel. residual 1e-6 from the guarded CNN start (network forward "
                    "included) vs the ubar and zero starts and Van Cittert; trapezoidal filter (value) and the "
                    "paper's differential filter at gamma = 0.1",
               cfg=5, count=64, n=1024, key="warmstart64", warm=True),
    "c5fwd": dict(desc="the warm-start network's 2D inference (k_fwd2d_fused: six layers, 37.4 k MAC per point, bf16 "
                       "MFMA for the 32->32 layers) on the 64 held-out 1024^2 evaluation fields",
                  cfg=5, count=64, n=1024, key="cnn_forward_1024sq_x64", forward=True),
    "c3": dict(desc="3D periodic 256^3 x 3 velocity components, E(k)~k^-5/3 on 2<=k<=80, divergence-free, "
                    "BiCGSTAB per component to rel. residual 1e-6 (FP32 storage, FP64 dots/scalars)",
               cfg=3, ndim=3, n=256, count=3, key="256cube_x3"),
    "germano2d": dict(desc="the paper's differential filter G = (I - delta^2 lap)^-1 (gamma = 0.01, kappa ~2e4) on "
                           "2D periodic 2048^2 x 16 fields, E(k)~k^-3 on 4<=k<=512, solved to 99 % residual reduction "
                           "(rel. residual 1e-2, the Table 1 criterion); FFT of ubar, solve on Fourier coefficients, "
                           "inverse FFT (FP32 storage, FP64 dots/scalars)",
                      cfg=2, ndim=2, n=2048, count=16, key="germano_2048sq_x16", germano=True, gamma=0.01, tol=1e-2),
    "germano3d": dict(desc="the paper's differential filter (gamma = 0.01) on a 3D periodic 256^3 x 3 velocity, "
                           "E(k)~k^-5/3 on 2<=k<=80, to 99 % residual reduction (FP32 storage, FP64 dots/scalars)",
                      cfg=3, ndim=3, n=256, count=3, key="germano_256cube_x3", germano=True, gamma=0.01, tol=1e-2),
    "table1": dict(desc="Table 1's setting (resolution inferred from the paper's per-iteration times): one 2D "
                        "256^2 k^-3 field and one 3D 64^3 k^-5/3 velocity component, the paper's differential filter "
                        "at gamma = 0.1, all four solvers to 99 % residual reduction (FP64)",
                   key="table1", table1=True),
    "closure3d": dict(desc="approximate-deconvolution closure stress tau_ij = ubar_i ubar_j - G(u*_i u*_j), 6 pairs, "
                           "from one 3D 256^3 divergence-free velocity (E(k)~k^-5/3 on 2<=k<=80), u* = BiCGSTAB "
                           "deconvolution of ubar to rel. residual 1e-6 (FP32)",
                      cfg=3, ndim=3, n=256, count=3, key="closure_256cube", closure=True),
    "closure2d": dict(desc="approximate-deconvolution closure stress, 3 pairs, from eight 2D 2048^2 velocities "
                           "(16 k^-3 fields on 4<=k<=512 as components), u* = BiCGSTAB deconvolution to rel. "
                           "residual 1e-6 (FP32)",
                      cfg=2, ndim=2, n=2048, count=16, key="closure_2048sq_x8", closure=True),
}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_solve_kernel_bicgstab.txt")
CLOSURE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_closure_kernel.txt")


SOLVE_SOURCES = ["gd_device.h", "gd_kernels.h", "gd_ops.h", "gd_internal.h", "gd_inst.inc", "gd_api.hip",
                 "gd_tune.hip"] + [f"gd_inst_{t}_{s}.hip" for t in ("f32", "f64") for s in ("vc", "cg", "bicgstab", "sd")]
CLOSURE_SOURCES = ["gd_closure.hip"]


def kernel_source_hash(sources=None) -> str:
    """sha256 over a kernel's sources (by default the persistent solve
    kernel's), the build script and the C header."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1707_09177_amd", "csrc")
    files = [os.path.join(csrc, f) for f in (sources or SOLVE_SOURCES)]
    files += [os.path.join(csrc, "build.py"), os.path.join(ROOT, "include", "gdecon.h")]
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.relpath(f, ROOT).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(key: str, path: str = TRAFFIC_FILE, sources=None):
    """HBM bytes per launch of a kernel (the BiCGSTAB solve kernel by default)
    from a committed FETCH_SIZE / WRITE_SIZE summary, or None when the kernel
    sources have changed since those counters were taken (or no figure exists)."""
    try:
        with open(path) as fh:
            kv = dict(line.split(" = ", 1) for line in fh.read().splitlines() if " = " in line)
    except OSError:
        return None
    if kv.get("kernel_sources_sha256", "").strip() != kernel_source_hash(sources):
        return None
    v = kv.get(f"traffic_bytes[{key}]")
    return float(v) if v is not None else None


def copy_bandwidth(torch, nbytes=1 << 30, reps=5) -> float:
    """GB/s of a plain device-to-device copy (read + write), HIP events on the
    current stream; the practical HBM ceiling beside the 8 TB/s vendor peak."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(reps):
        dst.copy_(src)
    b.record(stream)
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    return gbs


def traffic_rate(traffic, ms):
    """The measured-traffic roofline figure: HBM bytes per launch (rocprofv3
    FETCH_SIZE + WRITE_SIZE, committed under profiles/) over the launch's
    time, and its fraction of the HBM peak; None where no traffic figure
    matches the current sources."""
    if not traffic or not ms:
        return None, None
    gbs = traffic / (ms * 1e-3) / 1e9
    return gbs, gbs / HBM_PEAK_GBS


def add_traffic_rate(roof: dict, ms) -> dict:
    roof["traffic_GBs"], roof["traffic_frac"] = traffic_rate(roof.get("traffic"), ms)
    return roof


def add_copy_ceiling(roof: dict, torch) -> dict:
    """Measured copy bandwidth and the kernel's fraction of it, next to the
    vendor-peak fraction (measured after the timed region)."""
    c = copy_bandwidth(torch)
    roof["copy_GBs"] = c
    roof["frac_of_copy"] = roof["achieved"] / c
    return roof


def make_inputs(w, torch, gd, dev):
    from paper_1707_09177_amd import synth
    u = synth.config_fields(w["cfg"], n=w["n"], count=w["count"], dtype=np.float32)
    ut = torch.from_numpy(u).to(dev)
    ubar = gd.filter_apply(ut, ndim=w["ndim"])   # ubar = G u on the GPU
    torch.cuda.synchronize()
    return u, ubar


def make_batch_inputs(w, torch, gd, dev):
    from concurrent.futures import ThreadPoolExecutor

    from paper_1707_09177_amd import synth
    sizes = synth.batch_instances(count=w["count"])
    # the fields are drawn on the host's cores (numpy's FFT runs outside the GIL)
    with ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1))) as ex:
        fields = list(ex.map(lambda a: synth.batch_field(a[1][0], a[1][1], a[0], dtype=np.float32), enumerate(sizes)))
    shapes, ubars, us = [], [], []
    for i, (nd, n) in enumerate(sizes):
        u = fields[i]
        ut = torch.from_numpy(u).to(dev)
        ubars.append(gd.filter_apply(ut, ndim=nd))
        shapes.append(tuple(u.shape))
        us.append(u)
    torch.cuda.synchronize()
    return sizes, shapes, us, ubars


def time_batch(gd, torch, shapes, ubars, solver, steps, warmup, tol=1e-6, max_iter=500, tune=True):
    b = gd.BatchDeconvolver(shapes, ubars[0].dtype, solver)
    outs = [torch.empty_like(x) for x in ubars]
    tune = b.autotune(ubars, outs) if tune else None   # first-call tuning, outside the timed region
    for _ in range(warmup):
        b.solve(ubars, max_iter, tol, outs=outs)
    torch.cuda.synchronize()
    info = b.solve(ubars, max_iter, tol, outs=outs).info()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, e in evs:
        a.record(stream)
        b.solve(ubars, max_iter, tol, outs=outs)
        e.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    ms = [a.elapsed_time(e) for a, e in evs]
    return dict(info=info, ms_events=float(np.mean(ms)), ms_min=float(np.min(ms)), wall_ms=wall * 1e3, tune=tune)


def time_batch_graph(gd, torch, shapes, ubars, solver, steps, warmup, tol=1e-6, max_iter=500, tune=True):
    """The uneven batch as one captured HIP graph (instance-table kernels, the
    barrier-state prep and the persistent solve), timed as graph replays with
    HIP events on the stream they run on.  Tuning is first-call work, outside
    the graph and the timed region."""
    b = gd.BatchDeconvolver(shapes, ubars[0].dtype, solver)
    outs = [torch.empty_like(x) for x in ubars]
    tune = b.autotune(ubars, outs) if tune else None
    res = b.solve(ubars, max_iter, tol, outs=outs)
    torch.cuda.synchronize()
    eager_info = res.info()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.solve(ubars, max_iter, tol, outs=outs)
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, e in evs:
        a.record(stream)
        g.replay()
        e.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    ms = [a.elapsed_time(e) for a, e in evs]
    info = res.info()
    same = [(i["iters"], i["status"]) for i in info] == [(i["iters"], i["status"]) for i in eager_info]
    del g
    return dict(info=info, ms_events=float(np.mean(ms)), ms_min=float(np.min(ms)), wall_ms=wall * 1e3, tune=tune,
                replays_match_eager=same)


def cpu_baseline_batch(sizes, us, tol=1e-6, budget_s=20.0):
    """FP64 oracle on a seeded subset of the batch (smallest instances first,
    until about `budget_s` of CPU time), scaled by point count."""
    import oracle
    order = sorted(range(len(sizes)), key=lambda i: us[i].size)
    pts, dt, done = 0, 0.0, []
    for i in order:
        nd = sizes[i][0]
        ub = oracle.filter(us[i].astype(np.float64), nd).astype(np.float32).astype(np.float64)
        t0 = time.perf_counter()
        _, infos, _ = oracle.solve("bicgstab", ub, nd, 500, tol=tol)
        dt += time.perf_counter() - t0
        pts += us[i].size
        done.append(f"{nd}D n={sizes[i][1]}:{infos[0]['iters']}")
        if dt > budget_s:
            break
    return dict(value=pts / dt, unit="points/s", cores=1, kind="oracle", cpu_model=cpu_model(), nproc=os.cpu_count(),
                sample=f"{len(done)} of {len(sizes)} instances, smallest first ({', '.join(done[:6])}"
                       f"{', ...' if len(done) > 6 else ''}), FP64 oracle BiCGSTAB to 1e-6, single thread, "
                       f"{dt:.1f} s, scaled by point count")


def batch_result(gd, torch, shapes, ubars, s, steps, warmup, tune, npts, itemsize, graph=True):
    """One solver on the uneven batch, timed as replays of a captured graph
    (or, for counter collection, as eager calls)."""
    if graph:
        r = time_batch_graph(gd, torch, shapes, ubars, s, steps, warmup, tune=tune)
    else:
        r = dict(time_batch(gd, torch, shapes, ubars, s, steps, warmup, tune=tune), replays_match_eager=None)
    iters = [i["iters"] for i in r["info"]]
    st = sorted({i["status_name"] for i in r["info"]})
    worst_true = max(i["r_true"] / i["r_ref"] for i in r["info"])
    algo = sum(int(np.prod(sh)) * itemsize * accesses(s, it) for sh, it in zip(shapes, iters))
    kern = sum(int(np.prod(sh)) * itemsize * kernel_accesses(s, it) for sh, it in zip(shapes, iters))
    gbs = algo / (r["ms_events"] * 1e-3) / 1e9
    return dict(ms=r["ms_events"], ms_min=r["ms_min"], wall_ms=r["wall_ms"],
                timed_as="hipGraph replays" if graph else "eager calls",
                replays_match_eager=r["replays_match_eager"],
                iters_min=min(iters), iters_max=max(iters), status=st,
                replaced=sum(i["replaced"] for i in r["info"]),
                worst_true_rel_residual=worst_true, points_per_s=npts / (r["ms_events"] * 1e-3),
                algorithmic_bytes=algo, algorithmic_GBs=gbs, hbm_frac=gbs / HBM_PEAK_GBS,
                kernel_bytes=kern, kernel_hbm_frac=kern / (r["ms_events"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                tune=r["tune"])


def main_batch(args, w, torch, gd, dev):
    sizes, shapes, us, ubars = make_batch_inputs(w, torch, gd, dev)
    npts = int(sum(int(np.prod(s)) for s in shapes))
    itemsize = ubars[0].element_size()
    solvers = [x for x in args.solvers.split(",") if x != "vcb"]   # uneven batches: the persistent solvers
    if args.tune_only:
        for s in solvers:
            b = gd.BatchDeconvolver(shapes, ubars[0].dtype, s)
            print(json.dumps({"solver": s, "tune": b.autotune(ubars, [torch.empty_like(x) for x in ubars])}))
        return
    results = {}
    for s in solvers:
        results[s] = batch_result(gd, torch, shapes, ubars, s,
                                  args.steps if s == "bicgstab" else max(3, args.steps // 2), args.warmup,
                                  not args.no_tune, npts, itemsize, graph=not args.no_graph)
    main_s = "bicgstab" if "bicgstab" in results else list(results)[0]
    m = results[main_s]
    out = {
        "metric": METRIC, "value": m["points_per_s"], "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": m["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w["desc"], "instances": len(shapes),
                   "instances_2d": sum(1 for s in sizes if s[0] == 2), "points": npts, "solver": main_s,
                   "tol": 1e-6},
        "roofline": add_copy_ceiling(add_traffic_rate({"bound": "hbm", "achieved": m["algorithmic_GBs"],
                                                       "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": m["hbm_frac"],
                     "traffic": measured_traffic(w["key"]) if main_s == "bicgstab" else None,
                     "kernel": f"solve_kernel<float,{main_s}> (one persistent launch per batch solve, "
                               f"captured with its table and prep kernels in one graph)",
                     "bytes_per_launch": m["algorithmic_bytes"]}, m["ms"]), torch),
        "solvers": results,
    }
    if "vc" in results and main_s != "vc":
        out["vs_vancittert"] = results["vc"]["ms"] / m["ms"]
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_batch(sizes, us)
    print(json.dumps(out))


def closure_accesses(ndim: int) -> int:
    """Field accesses per point of the closure kernel: read ndim components of
    ubar and of u*, write ndim (ndim + 1) / 2 stress components."""
    return 2 * ndim + ndim * (ndim + 1) // 2


def closure_measure(w, torch, gd, dev, steps, warmup, tune):
    """Deconvolve the filtered velocity (BiCGSTAB to 1e-6), then time the
    closure stress kernel and the whole chain (solve of every component +
    closure).  Returns the timings, the algorithmic bytes and the tensors."""
    nd = w["ndim"]
    u32, ubar = make_inputs(w, torch, gd, dev)
    del u32
    vel = ubar.view(-1, nd, *ubar.shape[1:])                 # (fields, components, grid)
    d = gd.Deconvolver(ubar.shape, nd, ubar.dtype, "bicgstab")
    ustar = torch.empty_like(ubar)
    if tune:
        gd.autotune("bicgstab", ubar, ndim=nd, out=ustar)
    info = d.solve(ubar, 500, 1e-6, out=ustar).info()
    us = ustar.view_as(vel)
    tau = gd.closure_stress(vel, us, nd)
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in evs:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        ms = [a.elapsed_time(b) for a, b in evs]
        return float(np.mean(ms)), float(np.min(ms))

    ms_cl, ms_cl_min = timed(lambda: gd.closure_stress(vel, us, nd, out=tau), steps)
    ms_chain, _ = timed(lambda: (d.solve(ubar, 500, 1e-6, out=ustar), gd.closure_stress(vel, us, nd, out=tau)),
                        max(3, steps // 4))
    npts = int(np.prod(vel.shape[2:])) * vel.shape[0]             # grid points of the velocity batch
    algo = npts * ubar.element_size() * closure_accesses(nd)
    gbs = algo / (ms_cl * 1e-3) / 1e9
    return dict(ms_cl=ms_cl, ms_cl_min=ms_cl_min, ms_chain=ms_chain, npts=npts, algo=algo, gbs=gbs, info=info,
                vel=vel, us=us)


def main_closure(args, w, torch, gd, dev):
    """Deconvolve the filtered velocity, then time the closure stress kernel
    (and the whole chain: solve of every component + closure)."""
    nd = w["ndim"]
    r = closure_measure(w, torch, gd, dev, args.steps, args.warmup, not args.no_tune)
    ms_cl, ms_cl_min, ms_chain, npts, algo, gbs, info, vel, us = (
        r[k] for k in ("ms_cl", "ms_cl_min", "ms_chain", "npts", "algo", "gbs", "info", "vel", "us"))
    out = {
        "metric": "closure-stress grid points/s (all tau_ij pairs); % HBM roofline", "value": npts / (ms_cl * 1e-3),
        "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_cl,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w["desc"], "velocity_fields": vel.shape[0], "grid": [w["n"]] * nd, "points": npts,
                   "pairs": nd * (nd + 1) // 2},
        "roofline": add_copy_ceiling(add_traffic_rate({"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
                                                       "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                     "traffic": measured_traffic(w["key"], CLOSURE_TRAFFIC_FILE, CLOSURE_SOURCES), "kernel": f"k_closure<float,{nd}>",
                     "bytes_per_launch": algo}, ms_cl), torch),
        "closure_ms_min": ms_cl_min,
        "chain": {"ms": ms_chain, "points_per_s": npts / (ms_chain * 1e-3),
                  "solve_iters": sorted({i["iters"] for i in info}),
                  "status": sorted({i["status_name"] for i in info}),
                  "closure_share": ms_cl / ms_chain},
    }
    if not args.no_cpu:
        import oracle
        ub64 = vel.double().cpu().numpy()
        us64 = us.double().cpu().numpy()
        k = 1 if nd == 3 else 2                                  # velocity fields in the sample
        t0 = time.perf_counter()
        oracle.closure_stress(ub64[:k], us64[:k], nd)
        dt = time.perf_counter() - t0
        pts = int(np.prod(vel.shape[2:])) * k
        out["cpu_baseline"] = dict(value=pts / dt, unit="points/s", cores=1, kind="oracle",
                                   sample=f"{k} of {vel.shape[0]} velocity fields, FP64 oracle closure stress "
                                          f"(numpy products + C filter), single thread, {dt:.2f} s")
    print(json.dumps(out))


def germano_inputs(w, torch, gd, dev):
    """The workload's fields (FP32, host) and their differential-filter images (device)."""
    from paper_1707_09177_amd import synth
    u = synth.config_fields(w["cfg"], n=w["n"], count=w["count"], dtype=np.float32)
    ut = torch.from_numpy(u).to(dev)
    ubar = gd.germano_filter(ut, w["gamma"], ndim=w["ndim"])
    torch.cuda.synchronize()
    del ut
    return u, ubar


def germano_result(gd, torch, ubar, w, s, steps, warmup, tune, dev):
    """One solver with the differential filter, whole call (forward FFT, solve
    on the coefficients, inverse FFT) to the workload's tolerance: time,
    passes, and the call's algorithmic bytes per second."""
    nd, gamma, tol = w["ndim"], w["gamma"], w["tol"]
    npts = int(ubar.numel())
    stream = torch.cuda.current_stream()
    d = gd.GermanoDeconvolver(ubar.shape, nd, ubar.dtype, s, gamma, device=dev)
    out = torch.empty_like(ubar)
    tuned = d.autotune(ubar, out) if tune else None   # untimed
    reps = steps if s == "bicgstab" else max(2, steps // (10 if s in ("vc", "sd") else 2))
    for _ in range(warmup):
        d.solve(ubar, 5000, tol, out=out)
    torch.cuda.synchronize()
    info = d.solve(ubar, 5000, tol, out=out).info()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    for a, b in evs:
        a.record(stream)
        d.solve(ubar, 5000, tol, out=out)
        b.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    iters = [i["iters"] for i in info]
    # the stored half spectrum the solve kernel sweeps: 2 (n_x/2 + 1) reals per row, padded to 16 bytes
    nxs = (2 * (w["n"] // 2 + 1) + 3) // 4 * 4
    spec_pts = npts // w["n"] * nxs
    algo = spec_pts * 4 * accesses(s, max(iters))
    # whole call: forward FFT (real rows in, spectrum out, then each column axis
    # read and written), the solve on the spectrum, and the inverse FFT in reverse
    call_bytes = algo + 2 * npts * 4 + (6 if nd == 2 else 10) * spec_pts * 4
    launch = gd.last_launch()
    return dict(ms=ms, iters=sorted(set(iters)), status=sorted({i["status_name"] for i in info}),
                worst_true_rel_residual=max(i["r_true"] / i["r_ref"] for i in info),
                points_per_s=npts / (ms * 1e-3), solve_kernel_bytes=algo, call_bytes=call_bytes,
                call_GBs=call_bytes / (ms * 1e-3) / 1e9, call_hbm_frac=call_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                launch=launch, tune=tuned)


def main_germano(args, w, torch, gd, dev):
    """Time Algorithms 1-4 with the paper's differential filter to 99 % residual
    reduction (whole call: forward FFT, solve on the coefficients, inverse FFT)."""
    nd, gamma, tol = w["ndim"], w["gamma"], w["tol"]
    u, ubar = germano_inputs(w, torch, gd, dev)
    npts = int(ubar.numel())
    stream = torch.cuda.current_stream()
    if args.tune_only:
        for s in args.solvers.split(","):
            d = gd.GermanoDeconvolver(ubar.shape, nd, ubar.dtype, s, gamma, device=dev)
            print(json.dumps({"solver": s, "tune": d.autotune(ubar)}))
        return
    results = {s: germano_result(gd, torch, ubar, w, s, args.steps, args.warmup, not args.no_tune, dev)
               for s in args.solvers.split(",")}
    # the paper's spectral assessment (its N = 5 comparison): the highest shell up to
    # which the recovered energy spectrum keeps at least half of the true one
    kpow = -2.0 if nd == 2 else 0.0          # 2D fields are vorticities: kinetic energy is |w_hat|^2 / k^2
    e_true = gd.energy_spectrum(torch.from_numpy(u).to(dev), nd, kpow).sum(0)

    def k_half(x):
        e = gd.energy_spectrum(x, nd, kpow).sum(0)
        bad = ((e / e_true.clamp_min(1e-300)) < 0.5).nonzero()
        bad = bad[bad > 0]
        return int(bad[0].item()) - 1 if bad.numel() else int(e.numel()) - 1
    recovery = {"filtered": k_half(ubar)}
    t0 = time.perf_counter()
    for s in args.solvers.split(","):
        d = gd.GermanoDeconvolver(ubar.shape, nd, ubar.dtype, s, gamma, device=dev)
        recovery[s] = k_half(d.solve(ubar, 5, 0.0).u)
        del d
    torch.cuda.synchronize()
    diag_ms = {}
    for name, fn in (("energy_spectrum", lambda: gd.energy_spectrum(ubar, nd, kpow)),
                     ("pdf_counts", lambda: gd.pdf_counts(ubar, -6.0, 6.0, 512, ndim=nd))):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(5):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        diag_ms[name] = a.elapsed_time(b) / 5
    main_s = "bicgstab" if "bicgstab" in results else list(results)[0]
    m = results[main_s]
    out = {
        "metric": "deconvolved grid points/s to 99 % residual reduction, the paper's differential filter",
        "value": m["points_per_s"], "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": m["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["desc"], "fields": w["count"], "grid": [w["n"]] * nd, "points": npts,
                   "solver": main_s, "gamma": gamma, "tol": tol},
        "roofline": {"bound": "hbm", "achieved": m["call_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": m["call_GBs"] / HBM_PEAK_GBS, "traffic": None,
                     "kernel": f"solve_kernel<float,{main_s},spectral> with its forward and inverse FFTs (whole call)",
                     "bytes_per_launch": m["call_bytes"]},
        "solvers": results,
    }
    if "vc" in results and main_s != "vc":
        out["vs_vancittert"] = results["vc"]["ms"] / m["ms"]
    if "cg" in results and "vc" in results:
        out["cg_vs_vancittert"] = results["vc"]["ms"] / results["cg"]["ms"]
    out["spectral_recovery_N5"] = {"k_half_true": recovery, "kpow": kpow,
                                   "meaning": "highest shell up to which the recovered energy spectrum after 5 "
                                              "passes keeps at least half of the true one (all fields summed)"}
    out["diagnostics_ms"] = diag_ms
    # algorithmic bytes: the PDF reads the fields once; the spectrum is the forward
    # FFT (without the solve's scaling) plus one read of the stored spectrum
    spec_b = npts // w["n"] * ((2 * (w["n"] // 2 + 1) + 3) // 4 * 4) * 4
    spec_call = npts * 4 + spec_b + (2 if nd == 2 else 4) * spec_b + spec_b
    out["diagnostics_GBs"] = {"pdf_counts": npts * 4 / (diag_ms["pdf_counts"] * 1e-3) / 1e9,
                              "energy_spectrum": spec_call / (diag_ms["energy_spectrum"] * 1e-3) / 1e9}
    if not args.no_cpu:
        import oracle
        ub = ubar[:1].double().cpu().numpy()
        t0 = time.perf_counter()
        _, infos, _ = oracle.solve(main_s, ub, nd, 5000, tol=tol, gamma=gamma)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = dict(value=ub.size / dt, unit="points/s", cores=1, kind="oracle",
                                   sample=f"1 of {w['count']} fields, FP64 oracle {main_s} with the FFT filter "
                                          f"(numpy), single thread, {dt:.1f} s, iters {infos[0]['iters']}")
    print(json.dumps(out))


# Table 1 of the paper (CPU seconds), quoted as context: per iteration and to 99 % recovery
PAPER_TABLE1 = {"vc": (1.5156e-2, 6.9661e-2, 1.1064, 6.6178), "sd": (1.5625e-2, 7.6068e-2, 0.6719, 3.9555),
                "cg": (1.6093e-2, 8.3464e-2, 0.2414, 1.2520), "bicgstab": (3.0625e-2, 16.3724e-2, 0.2450, 1.3098)}


def main_table1(args, w, torch, gd, dev):
    """The paper's Table 1 experiment on the GPU: passes and time to 99 %
    residual reduction for each solver, 2D and 3D, differential filter."""
    from paper_1707_09177_amd import synth
    cases = {"2d": (2, synth.config_fields(2, n=256, count=1)), "3d": (3, synth.config_fields(3, n=64, count=1))}
    stream = torch.cuda.current_stream()
    rows = {}
    for tag, (nd, u) in cases.items():
        ub = gd.germano_filter(torch.from_numpy(u).to(dev), 0.1, ndim=nd)
        for s in ("vc", "sd", "cg", "bicgstab"):
            d = gd.GermanoDeconvolver(ub.shape, nd, ub.dtype, s, 0.1, device=dev)
            out = torch.empty_like(ub)
            for _ in range(args.warmup):
                d.solve(ub, 5000, 1e-2, out=out)
            info = d.solve(ub, 5000, 1e-2, out=out).info()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(args.steps):
                d.solve(ub, 5000, 1e-2, out=out)
            b.record(stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / args.steps
            it = info[0]["iters"]
            paper = PAPER_TABLE1[s]
            rows[f"{tag}_{s}"] = dict(passes=it, ms=ms, ms_per_pass=ms / max(it, 1), status=info[0]["status_name"],
                                      paper_passes=round(paper[2 + (nd == 3)] / paper[nd == 3]),
                                      paper_cpu_s=paper[2 + (nd == 3)])
    npts2 = 256 * 256
    m = rows["2d_bicgstab"]
    out = {
        "metric": "deconvolved grid points/s to 99 % residual reduction, Table 1 setting", "value": npts2 / (m["ms"] * 1e-3),
        "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": m["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w["desc"], "gamma": 0.1, "tol": 1e-2},
        "table1": rows,
        "speedup_over_vc": {tag: {s: rows[f"{tag}_vc"]["ms"] / rows[f"{tag}_{s}"]["ms"] for s in ("sd", "cg", "bicgstab")}
                            for tag in ("2d", "3d")},
        "paper_speedup_over_vc": {tag: {s: PAPER_TABLE1["vc"][2 + i] / PAPER_TABLE1[s][2 + i] for s in ("sd", "cg", "bicgstab")}
                                  for i, tag in enumerate(("2d", "3d"))},
    }
    print(json.dumps(out))


def event_ms(torch, fn, reps):
    """Mean ms of fn() over reps calls (one untimed call first), HIP events
    on the current stream."""
    stream = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, e in evs:
        a.record(stream)
        fn()
        e.record(stream)
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(e) for a, e in evs]))


def train_warm_start(gd, torch, ub, u, ndim, steps, batch, smooth, lr=1e-3, seed=0):
    """Adam on the pairs (ub[i], u[i]) in shuffled minibatches (a seeded
    permutation per epoch); the learning rate drops 10x for the last third.
    Returns the network and a training record."""
    from paper_1707_09177_amd import synth
    net = gd.WarmStart(synth.cnn_init_params(seed, ndim=ndim), lr=lr, ndim=ndim, smooth=smooth)
    g = torch.Generator(device="cpu").manual_seed(1707 + seed)
    count = ub.shape[0]
    perm, pos = torch.randperm(count, generator=g), 0
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        if pos + batch > count:
            perm, pos = torch.randperm(count, generator=g), 0
        idx = perm[pos:pos + batch].to(ub.device)
        pos += batch
        loss = net.train_step(ub.index_select(0, idx), u.index_select(0, idx))
        if k == (2 * steps) // 3:
            net.set_lr(lr / 10)
        if k % max(1, steps // 8) == 0 or k == steps - 1:
            losses.append(float(loss.item()))
            print(f"train {ndim}D: step {k + 1}/{steps} loss {losses[-1]:.3e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return net, {"steps": steps, "batch": batch, "fields": int(count), "grid": list(ub.shape[1:]), "smooth": smooth,
                 "seconds": time.perf_counter() - t0, "loss": losses}


def warm_starts(gd, torch, net, ubar, make_solver, reps, solvers=("bicgstab", "vc"), band_in_solve=False):
    """BiCGSTAB to rel. residual 1e-6 from the ubar, zero and network starts
    (the network's start guarded: a field whose predicted start is no better
    than ubar starts from ubar), and Van Cittert from ubar, on the same
    fields.  The network start is timed as forward pass + band projection +
    solve, and each part on its own; `cnn_unprojected` is the same network
    without the band projection.  band_in_solve: the solver projects a warm
    start itself (the differential filter's, on its Fourier coefficients), so
    the network's output goes to it unprojected."""
    res = {}
    d = make_solver("bicgstab")
    out = torch.empty_like(ubar)
    for start in ("ubar", "zero"):
        ms = event_ms(torch, lambda: d.solve(ubar, 500, 1e-6, init=start, out=out), reps)
        inf = d.solve(ubar, 500, 1e-6, init=start, out=out).info()
        res[start] = dict(ms=ms, iters_mean=float(np.mean([i["iters"] for i in inf])),
                          iters=sorted({i["iters"] for i in inf}), status=sorted({i["status_name"] for i in inf}),
                          worst_true_rel_residual=max(i["r_true"] / i["r_ref"] for i in inf))
    u0 = torch.empty_like(ubar)
    nd = net.ndim

    def record(inf, **kw):
        given = [i for i in inf if i["start"] == "given"]
        return dict(iters_mean=float(np.mean([i["iters"] for i in inf])), iters=sorted({i["iters"] for i in inf}),
                    status=sorted({i["status_name"] for i in inf}),
                    fallbacks=sum(1 for i in inf if i["start"] == "ubar"),
                    worst_true_rel_residual=max(i["r_true"] / i["r_ref"] for i in inf),
                    r0_over_ref_mean=float(np.mean([i["r0"] / i["r_ref"] for i in given])) if given else None, **kw)

    ms_fwd = event_ms(torch, lambda: net.forward(ubar, out=u0, band=False), reps)
    net.forward(ubar, out=u0, band=False)
    if not band_in_solve:
        out.copy_(u0)
        res["cnn_unprojected"] = record(d.solve(ubar, 500, 1e-6, init="warm", out=out).info())
        bwork = torch.empty(int(gd.load().band_project_workspace_bytes(gd.make_grid(ubar.shape, nd, ubar.dtype))),
                            dtype=torch.uint8, device=ubar.device)
        ms_band = event_ms(torch, lambda: (out.copy_(u0), gd.band_project(ubar, out, nd, work=bwork)), reps) - \
            event_ms(torch, lambda: out.copy_(u0), reps)
    else:
        out.copy_(u0)
        res["cnn_unprojected"] = record(d.solve(ubar, 500, 1e-6, init="given", out=out).info())
        ms_band = 0.0  # inside the solve
    net.forward(ubar, out=u0, band=not band_in_solve)

    def solve_from_u0():
        out.copy_(u0)
        d.solve(ubar, 500, 1e-6, init="warm", out=out)
    ms_solve = event_ms(torch, solve_from_u0, reps) - event_ms(torch, lambda: out.copy_(u0), reps)
    ms_total = event_ms(torch, lambda: (net.forward(ubar, out=out, band=not band_in_solve),
                                        d.solve(ubar, 500, 1e-6, init="warm", out=out)), reps)
    net.forward(ubar, out=out, band=not band_in_solve)
    res["cnn"] = record(d.solve(ubar, 500, 1e-6, init="warm", out=out).info(), ms=ms_total, ms_forward=ms_fwd,
                        ms_band_project=ms_band, ms_solve=ms_solve)
    if "vc" in solvers:
        dv = make_solver("vc")
        ms = event_ms(torch, lambda: dv.solve(ubar, 20000, 1e-6, out=out), max(2, reps // 4))
        inf = dv.solve(ubar, 20000, 1e-6, out=out).info()
        res["vc"] = dict(ms=ms, iters_mean=float(np.mean([i["iters"] for i in inf])),
                         status=sorted({i["status_name"] for i in inf}))
    res["cnn_vs_ubar_passes"] = res["ubar"]["iters_mean"] / res["cnn"]["iters_mean"]
    res["cnn_vs_zero_passes"] = res["zero"]["iters_mean"] / res["cnn"]["iters_mean"]
    res["cnn_vs_ubar_time"] = res["ubar"]["ms"] / res["cnn"]["ms"]
    res["cnn_vs_zero_time"] = res["zero"]["ms"] / res["cnn"]["ms"]
    if "vc" in res:
        res["cnn_vs_vc_time"] = res["vc"]["ms"] / res["cnn"]["ms"]
    return res


def main_warm(args, w, torch, gd, dev):
    """Config 5: the warm-start network trained on the GPU on 4096 seeded
    (ubar, u) pairs of periodic 512^2 k^-3 fields, evaluated on 64 held-out
    1024^2 fields; with the trapezoidal filter (the path's G) and with the
    paper's differential filter at gamma = 0.1 (its Table 1 setting, where
    the plain solve needs many passes); plus the 3D network on 128^3."""
    from paper_1707_09177_amd import synth
    U = torch.from_numpy(synth.training_fields(args.train_fields, n=512)).to(dev)
    ev = torch.from_numpy(np.stack([synth.field_2d(w["n"], synth.spectrum_kraichnan, 4.0, w["n"] / 4.0,
                                                   synth.rng_for(5, 50000 + i), np.float32)
                                    for i in range(w["count"])])).to(dev)
    npts = int(ev.numel())
    out = {"metric": METRIC, "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+bf16",
           "data": "synthetic"}
    regimes = {}
    # the path's filter: G = the trapezoidal stencil
    ubt = gd.filter_apply(U, ndim=2)
    net, rec = train_warm_start(gd, torch, ubt, U, 2, args.train_steps, 8, args.smooth)
    del ubt
    ubar = gd.filter_apply(ev, ndim=2)
    regimes["trapezoidal"] = dict(training=rec, starts=warm_starts(
        gd, torch, net, ubar, lambda s: gd.Deconvolver(ubar.shape, 2, ubar.dtype, s), args.steps))
    del net, ubar
    # the paper's filter G = (I - delta^2 lap)^-1, gamma = 0.1
    gamma = 0.1
    ubt = gd.germano_filter(U, gamma, ndim=2)
    net, rec = train_warm_start(gd, torch, ubt, U, 2, args.train_steps, 8, args.smooth, seed=1)
    del ubt, U
    ubar = gd.germano_filter(ev, gamma, ndim=2)
    regimes["differential_gamma0.1"] = dict(training=rec, starts=warm_starts(
        gd, torch, net, ubar, lambda s: gd.GermanoDeconvolver(ubar.shape, 2, ubar.dtype, s, gamma, device=dev),
        args.steps, band_in_solve=True))
    del net, ubar
    m = regimes["trapezoidal"]["starts"]["cnn"]
    out.update(value=npts / (m["ms"] * 1e-3), ms_per_step=m["ms"],
               config={"workload": w["desc"], "fields": w["count"], "grid": [w["n"], w["n"]], "points": npts,
                       "solver": "bicgstab", "tol": 1e-6, "train_fields": args.train_fields,
                       "train_steps": args.train_steps, "train_batch": 8, "smooth": args.smooth},
               warmstart=regimes, warmstart_3d=warm_3d(gd, torch, dev, synth, args))
    print(json.dumps(out))


# model flops per point of the 2D network: 2 x (9 + 4 x 9 x 32 + 9) x 32 MACs
CNN2D_FLOP_PER_POINT = 2 * (9 * 32 + 4 * 9 * 32 * 32 + 9 * 32)
MFMA_BF16_PEAK_TFLOPS = 2500.0


def forward_result(w, torch, gd, dev, steps, warmup):
    """Time the network's 2D forward call on the c5 evaluation batch: ms,
    points and model TFLOP/s."""
    from paper_1707_09177_amd import synth
    ev = torch.from_numpy(np.stack([synth.field_2d(w["n"], synth.spectrum_kraichnan, 4.0, w["n"] / 4.0,
                                                   synth.rng_for(5, 50000 + i), np.float32)
                                    for i in range(w["count"])])).to(dev)
    ubar = gd.filter_apply(ev, ndim=2)
    del ev
    net = gd.WarmStart(synth.cnn_init_params(0))
    u0 = torch.empty_like(ubar)
    for _ in range(warmup):
        net.forward(ubar, out=u0, band=False)
    ms = event_ms(torch, lambda: net.forward(ubar, out=u0, band=False), steps)
    npts = int(ubar.numel())
    return ms, npts, CNN2D_FLOP_PER_POINT * npts / (ms * 1e-3) / 1e12


def main_forward(args, w, torch, gd, dev):
    """The network's 2D forward pass alone (untrained weights: the cost does
    not depend on them), without the band projection, on the c5 evaluation
    batch.  roofline: model flops per launch / the fused kernel's duration,
    against the dense bf16 matrix-core peak."""
    ms, npts, tflops = forward_result(w, torch, gd, dev, args.steps, args.warmup)
    print(json.dumps({"metric": "warm-start network forward points/s; % bf16 MFMA peak", "value": npts / (ms * 1e-3),
                      "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
                      "data": "synthetic", "config": {"workload": w["desc"], "fields": w["count"],
                                                      "grid": [w["n"], w["n"]], "points": npts},
                      "roofline": {"bound": "mfma", "achieved": tflops, "peak": MFMA_BF16_PEAK_TFLOPS,
                                   "unit": "TFLOP/s", "frac": tflops / MFMA_BF16_PEAK_TFLOPS, "traffic": None,
                                   "flop_per_point": CNN2D_FLOP_PER_POINT,
                                   "note": "whole forward call (RMS, fused layers, G, u0 = ubar + s y); the fused "
                                           "kernel's own share is in profiles/"}}))


def warm_3d(gd, torch, dev, synth, args, n_train=64, n_eval=128, count_eval=8):
    """3D network: trained on 64^3 k^-5/3 fields, evaluated on held-out
    128^3 fields (k^-5/3 on 2 <= k <= 40): BiCGSTAB passes and time from the
    ubar, zero and network starts, trapezoidal filter."""
    U = torch.from_numpy(np.stack(synth.training_pairs_3d(64, n=n_train))).to(dev)
    ubt = gd.filter_apply(U, ndim=3)
    net, rec = train_warm_start(gd, torch, ubt, U, 3, max(1, args.train_steps // 3), 4, args.smooth)
    del U, ubt
    ev = np.stack([synth.scalar_3d(n_eval, synth.spectrum_kolmogorov, 2.0, 0.3125 * n_eval,
                                   synth.rng_for(6, 60000 + i), np.float32) for i in range(count_eval)])
    ubar = gd.filter_apply(torch.from_numpy(ev).to(dev), ndim=3)
    res = warm_starts(gd, torch, net, ubar, lambda s: gd.Deconvolver(ubar.shape, 3, ubar.dtype, s), args.steps)
    return {"training": rec, "eval": f"{count_eval} x {n_eval}^3", "starts": res}


def time_solver(gd, torch, ubar, w, solver, steps, warmup, tol=1e-6, max_iter=500, tune=True):
    out = torch.empty_like(ubar)
    if solver == "vcb":  # Van Cittert with several passes per sweep
        d = gd.BlockedVanCittert(ubar.shape, w["ndim"], ubar.dtype)
        tuned = None
    else:
        d = gd.Deconvolver(ubar.shape, w["ndim"], ubar.dtype, solver)
        tuned = gd.autotune(solver, ubar, ndim=w["ndim"], out=out) if tune else None   # first-call tuning, untimed
    for _ in range(warmup):
        d.solve(ubar, max_iter, tol, out=out)
    torch.cuda.synchronize()
    info = d.solve(ubar, max_iter, tol, out=out).info()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        d.solve(ubar, max_iter, tol, out=out)
        b.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    ms = [a.elapsed_time(b) for a, b in evs]
    return dict(info=info, ms_events=float(np.mean(ms)), ms_min=float(np.min(ms)), wall_ms=wall * 1e3, u=out,
                tune=tuned, launch=gd.last_launch() if solver != "vcb" else None)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, u32, tol=1e-6, fields_1t=4, fields_all=16):
    """The FP64 oracle's BiCGSTAB on a sample of the workload's fields: on one
    thread (serial compensated sums), then on every core the host offers
    (OpenMP over points, fixed-chunk compensated sums, the same result for
    any thread count).  `value` is the all-core rate."""
    import oracle
    nd = w["ndim"]
    procs = oracle.host_procs()

    def run(nfields, threads):
        fields = u32[:nfields].astype(np.float64)
        ub = oracle.filter(fields, nd).astype(np.float32).astype(np.float64)
        used = oracle.set_threads(threads)
        try:
            t0 = time.perf_counter()
            _, infos, _ = oracle.solve("bicgstab", ub, nd, 500, tol=tol,
                                       sum_mode=oracle.SUM_CHUNKED if used > 1 else 0)
            dt = time.perf_counter() - t0
        finally:
            oracle.set_threads(1)
        return fields.size / dt, dt, used, [i["iters"] for i in infos], len(fields)

    v1, dt1, _, it1, n1 = run(min(fields_1t, len(u32)), 1)
    va, dta, used, ita, na = run(min(fields_all, len(u32)), procs)
    grid = "x".join(str(s) for s in u32.shape[1:])
    return dict(value=va, unit="points/s", cores=used, kind="oracle",
                sample=f"{na} of {w['count']} fields ({grid}), FP64 oracle BiCGSTAB to 1e-6, {used} threads "
                       f"(every logical CPU of the host), {dta:.1f} s, iters {ita}",
                cpu_model=cpu_model(), nproc=os.cpu_count(),
                single_thread=dict(value=v1, unit="points/s", cores=1,
                                   sample=f"{n1} of {w['count']} fields ({grid}), one thread, {dt1:.1f} s, "
                                          f"iters {it1}"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-graph", action="store_true",
                    help="uneven batch: time eager calls instead of graph replays (for counter collection)")
    ap.add_argument("--no-extra", action="store_true",
                    help="default workload: skip the 3 x 256^3 and uneven-batch keys")
    ap.add_argument("--no-tune", action="store_true",
                    help="do not run the autotuner (choices come from the GD_TUNE_CACHE file when it is set, "
                         "else the defaults)")
    ap.add_argument("--tune-only", action="store_true",
                    help="run the autotuner for the workload's solvers and exit (with GD_TUNE_CACHE set, the "
                         "choices are saved for later --no-tune runs, e.g. under a profiler)")
    ap.add_argument("--solvers", default="bicgstab,cg,vc,vcb",
                    help="vcb: Van Cittert with several passes per sweep (same iterates, less traffic)")
    ap.add_argument("--train-steps", type=int, default=16384,
                    help="warm-start workload: Adam steps (batches of 8 fields: 32 passes over 4096 fields, "
                         "about 100 s per 2D network; 8192 steps left the differential start at the plain "
                         "start's wall-clock, 16384 beat it)")
    ap.add_argument("--train-fields", type=int, default=4096, help="warm-start workload: 512^2 training fields")
    ap.add_argument("--smooth", type=int, default=1,
                    help="warm-start workload: applications of G to the network's output (1 measured best: with the "
                         "band projection the start needed 4 BiCGSTAB passes at 1 and at 2, at a lower r0 with 1)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 1 GiB device copy (x5): the reference kernel that scales "
                         "FETCH_SIZE / WRITE_SIZE counter readings to bytes")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(fields shard across GPUs with no communication; see DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calib:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes_read": src.numel() * 4, "copy_calib_bytes_written": dst.numel() * 4,
                          "launches": 5}))
        return
    from paper_1707_09177_amd import gdecon as gd
    gd.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = WORKLOADS[args.workload]
    if w.get("batch"):
        return main_batch(args, w, torch, gd, dev)
    if w.get("warm"):
        return main_warm(args, w, torch, gd, dev)
    if w.get("forward"):
        return main_forward(args, w, torch, gd, dev)
    if w.get("closure"):
        return main_closure(args, w, torch, gd, dev)
    if w.get("table1"):
        return main_table1(args, w, torch, gd, dev)
    if w.get("germano"):
        if args.solvers == "bicgstab,cg,vc,vcb":
            args.solvers = "bicgstab,cg,sd,vc"
        return main_germano(args, w, torch, gd, dev)
    u32, ubar = make_inputs(w, torch, gd, dev)
    if args.tune_only:
        for s in [x for x in args.solvers.split(",") if x != "vcb"]:   # vcb has no launch choices
            print(json.dumps({"solver": s, "tune": gd.autotune(s, ubar, ndim=w["ndim"])}))
        return
    npts = int(ubar.numel())
    itemsize = ubar.element_size()

    results = {}
    for s in args.solvers.split(","):
        results[s] = uniform_result(gd, torch, ubar, w, s, args.steps if s == "bicgstab" else max(3, args.steps // 2),
                                    args.warmup, not args.no_tune, npts, itemsize)
    main_s = "bicgstab" if "bicgstab" in results else list(results)[0]
    m = results[main_s]
    if "CONVERGED" not in m["status"] or len(m["status"]) != 1:
        print(f"warning: {main_s} did not converge on every field: {m['status']}", file=sys.stderr)

    out = {
        "metric": METRIC,
        "value": m["points_per_s"],
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["desc"], "fields": w["count"], "grid": [w["n"]] * w["ndim"],
                   "points": npts, "solver": main_s, "tol": 1e-6},
        "roofline": add_copy_ceiling(add_traffic_rate({"bound": "hbm", "achieved": m["algorithmic_GBs"],
                                                       "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": m["hbm_frac"],
                     "traffic": measured_traffic(w["key"]) if main_s == "bicgstab" else None,
                     "kernel": f"solve_kernel<float,{main_s}> (one persistent launch per solve)",
                     "bytes_per_launch": npts * itemsize * m["accesses_per_point"],
                     "accesses_per_point": m["accesses_per_point"],
                     "kernel_accesses_per_point": m["kernel_accesses_per_point"],
                     "kernel_frac": m["kernel_hbm_frac"]}, m["ms"]), torch),
        "iterations": m["iters"][0] if len(set(m["iters"])) == 1 else m["iters"],
        "solvers": {k: {kk: vv for kk, vv in v.items()} for k, v in results.items()},
    }
    if "vc" in results and main_s != "vc":
        out["vs_vancittert"] = results["vc"]["ms"] / m["ms"]
    if "vcb" in results and main_s != "vcb":
        out["vs_vancittert_blocked"] = results["vcb"]["ms"] / m["ms"]
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, u32)
    if args.workload == "c2" and not args.no_extra:
        # the other headline workloads in the same run: 3 x 256^3 BiCGSTAB and
        # the 200-instance uneven batch as graph replays
        del ubar, u32
        torch.cuda.empty_cache()
        out["c3"] = extra_uniform(args, WORKLOADS["c3"], torch, gd, dev)
        torch.cuda.empty_cache()
        out["c4"] = extra_batch(args, WORKLOADS["c4"], torch, gd, dev)
        torch.cuda.empty_cache()
        out["germano2d"] = extra_germano(args, WORKLOADS["germano2d"], torch, gd, dev)
        torch.cuda.empty_cache()
        out["c5fwd"] = extra_forward(args, WORKLOADS["c5fwd"], torch, gd, dev)
        torch.cuda.empty_cache()
        out["closure3d"] = extra_closure(args, WORKLOADS["closure3d"], torch, gd, dev)
    print(json.dumps(out))


def uniform_result(gd, torch, ubar, w, s, steps, warmup, tune, npts, itemsize):
    """One solver on a uniform batch: time, passes, and its algorithmic bytes
    priced against the HBM peak (the method's access count, and beside it the
    count the fused kernel actually makes)."""
    r = time_solver(gd, torch, ubar, w, s, steps, warmup, tune=tune)
    iters = [i["iters"] for i in r["info"]]
    st = {i["status_name"] for i in r["info"]}
    worst_true = max(i["r_true"] / i["r_ref"] for i in r["info"])
    base = "vc" if s == "vcb" else s   # vcb: the one-pass solve's accesses, for comparison
    acc = accesses(base, max(iters))
    kacc = kernel_accesses(base, max(iters))
    sec = r["ms_events"] * 1e-3
    gbs = npts * itemsize * acc / sec / 1e9
    return dict(ms=r["ms_events"], ms_min=r["ms_min"], wall_ms=r["wall_ms"], iters=iters,
                status=sorted(st), worst_true_rel_residual=worst_true,
                replaced=sum(i.get("replaced", 0) for i in r["info"]),
                points_per_s=npts / sec, accesses_per_point=acc, kernel_accesses_per_point=kacc,
                algorithmic_GBs=gbs, hbm_frac=gbs / HBM_PEAK_GBS,
                kernel_hbm_frac=npts * itemsize * kacc / sec / 1e9 / HBM_PEAK_GBS,
                tune=r["tune"], launch=r["launch"])


def extra_uniform(args, w, torch, gd, dev, others=("cg", "vc")):
    """BiCGSTAB on a second uniform workload, reported as an extra key, with
    CG and Van Cittert on the same fields for the "vs Van Cittert" ratio."""
    u32, ubar = make_inputs(w, torch, gd, dev)
    npts, itemsize = int(ubar.numel()), ubar.element_size()
    r = uniform_result(gd, torch, ubar, w, "bicgstab", args.steps, args.warmup, not args.no_tune, npts, itemsize)
    rest = {s: uniform_result(gd, torch, ubar, w, s, max(5, args.steps // 2), args.warmup, not args.no_tune, npts,
                              itemsize) for s in others}
    del ubar, u32
    traffic = measured_traffic(w["key"])
    out = {"workload": w["desc"], "points": npts, "solver": "bicgstab", "points_per_s": r["points_per_s"],
           "ms": r["ms"], "hbm_frac": r["hbm_frac"], "traffic": traffic,
           "traffic_frac": traffic_rate(traffic, r["ms"])[1], **r}
    out["others"] = {s: {k: v[k] for k in ("ms", "iters", "status", "worst_true_rel_residual", "hbm_frac", "tune",
                                            "launch")} for s, v in rest.items()}
    if "vc" in rest:
        out["vs_vancittert"] = rest["vc"]["ms"] / r["ms"]
        if "cg" in rest:
            out["cg_vs_vancittert"] = rest["vc"]["ms"] / rest["cg"]["ms"]
    return out


def extra_batch(args, w, torch, gd, dev):
    """BiCGSTAB on the uneven batch, one captured graph per solve, reported as
    an extra key."""
    sizes, shapes, us, ubars = make_batch_inputs(w, torch, gd, dev)
    npts = int(sum(int(np.prod(s)) for s in shapes))
    r = batch_result(gd, torch, shapes, ubars, "bicgstab", max(5, args.steps // 2), args.warmup, not args.no_tune,
                     npts, ubars[0].element_size(), graph=not args.no_graph)
    del ubars, us
    traffic = measured_traffic(w["key"])
    return {"workload": w["desc"], "instances": len(shapes), "instances_2d": sum(1 for s in sizes if s[0] == 2),
            "points": npts, "solver": "bicgstab", "points_per_s": r["points_per_s"], "ms": r["ms"],
            "hbm_frac": r["hbm_frac"], "traffic": traffic, "traffic_frac": traffic_rate(traffic, r["ms"])[1], **r}


def extra_germano(args, w, torch, gd, dev):
    """BiCGSTAB and Van Cittert with the paper's differential filter (whole
    call), reported as an extra key."""
    _, ubar = germano_inputs(w, torch, gd, dev)
    r = {s: germano_result(gd, torch, ubar, w, s, max(5, args.steps // 2), args.warmup, not args.no_tune, dev)
         for s in ("bicgstab", "vc")}
    del ubar
    return {"workload": w["desc"], "solvers": r, "ms": r["bicgstab"]["ms"],
            "call_hbm_frac": r["bicgstab"]["call_hbm_frac"], "vs_vancittert": r["vc"]["ms"] / r["bicgstab"]["ms"]}


def extra_closure(args, w, torch, gd, dev):
    """The closure stress kernel after the velocity's deconvolution, reported
    as an extra key."""
    r = closure_measure(w, torch, gd, dev, args.steps, args.warmup, not args.no_tune)
    traffic = measured_traffic(w["key"], CLOSURE_TRAFFIC_FILE, CLOSURE_SOURCES)
    out = {"workload": w["desc"], "points": r["npts"], "ms": r["ms_cl"], "algorithmic_GBs": r["gbs"],
           "hbm_frac": r["gbs"] / HBM_PEAK_GBS, "traffic": traffic, "traffic_frac": traffic_rate(traffic, r["ms_cl"])[1],
           "chain_ms": r["ms_chain"], "closure_share": r["ms_cl"] / r["ms_chain"],
           "solve_iters": sorted({i["iters"] for i in r["info"]})}
    del r
    return out


def extra_forward(args, w, torch, gd, dev):
    """The warm-start network's 2D forward call, reported as an extra key."""
    ms, npts, tflops = forward_result(w, torch, gd, dev, max(10, args.steps), args.warmup)
    return {"workload": w["desc"], "points": npts, "ms": ms, "tflops": tflops,
            "mfma_frac": tflops / MFMA_BF16_PEAK_TFLOPS, "peak_tflops": MFMA_BF16_PEAK_TFLOPS}


if __name__ == "__main__":
    main()
