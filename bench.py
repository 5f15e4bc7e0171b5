#!/usr/bin/env python3
"""MLUPS and HBM roofline of the sparse D3Q19 LBGK step on one MI355X.

Headline workload (the branching-artery configuration): a Murray's-law tree of
depth 8 (256 outlets), root radius 40 lu, branch angles uniform in 25-45
degrees, seeded, voxelised in a 768^3 box with the segment length/radius
ratio chosen so the tree fits the box; Bouzidi walls with a wall fraction q
uniform in (0, 1] per link; tau = 0.55; steady parabolic velocity inlet (peak
0.01) at the root; pressure outlets at rho = 1.  Inputs are synthetic and
seeded.

Batched forms, in the same run: the self-coupled arterial-venous pair (64
outlet-to-inlet pairs exchanging boundary values on the device every step,
pulsatile 3-harmonic inlet) and the ensemble of 32 uneven trees (0.5-8 M
sites each, own tau and inlet waveform each), every domain of a workload in
the same launches, in FP32 and FP64 at a fixed layout and schedule.

One timed step is one lattice update of every fluid site (all kernels of the
path: gather, boundary links, collision, store, iolet reductions, coupling,
boundary update).  MLUPS = sites * steps / time / 1e6, timed with HIP events
recorded on the stream the library launches on, inputs resident in HBM.

Printed: one JSON line (rank 0, N = 1) with the FP32 offset-storage figure of
the branching artery as ``value``; its FP64 and FP16 forms under ``variants``
(each with its error against the FP64 GPU run); the batched workloads under
``batched``; ``parity`` of the FP64 GPU path against the FP64 CPU oracle at
full size, from rest and from a developed state; ``roofline`` for the dominant
kernel (the fused FP32 step) on the algorithmic bytes per site of the
method's two-lattice form (2 x 19 populations + 18 int32 pull indices),
against the published 8 TB/s and a measured streaming-copy ceiling;
``cpu_baseline`` for the oracle timed on this host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
DRIVES = {0: "launch", 1: "graph"}
STORE_BYTES = {"f64": 8, "f32": 4, "f16": 2, "f16w": 2, "f16sr": 2}
TAU = 0.55
U_IN = 0.01
METRIC = "MLUPS + achieved HBM GB/s (% peak), FP64 vs FP32 at stated error, 1 GPU"
# the machine's CPU share for one GPU: worker pools and the oracle's threads stay
# within it whatever the host reports
CPU_SHARE = 16


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def bytes_per_site(prec, aa=False, near=0.0):
    """HBM bytes of one site update: 19 populations read and written, plus 18
    pull indices (two-lattice pull) or, averaged over an even and an odd step
    of the in-place scheme, 9; an index is 2 bytes for the fraction `near` of
    sites addressed through int16 deltas, else 4.  With near = 0 this is the
    algorithmic figure of the method (376 / 224 / 148 B two-lattice, 340 /
    188 / 112 B in place, FP64 / FP32 / FP16)."""
    return 2 * 19 * STORE_BYTES[prec] + (9 if aa else 18) * (4.0 - 2.0 * near)


def _code_only(text):
    """Source text without comments and blank lines (a comment edit does not
    change the kernels)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def kernel_source_hash(read=None):
    """Hash of the library code: the kernels, the layout structs they read and
    the host code that orders the sites and builds the schedule."""
    h = hashlib.sha256()
    for name in ("hl_kernels.hip", "hl_internal.h", "hl_api.cpp", "hl_host.h", "hl_layout.cpp"):
        if read is None:
            with open(os.path.join(ROOT, "paper_2010_04144_amd", "csrc", name)) as fh:
                text = fh.read()
        else:
            text = read(name)
        h.update(_code_only(text).encode())
    return h.hexdigest()[:16]


def traffic_from_profile(prec, layout, block, sched):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, when it was taken from the same kernel sources, layout and
    schedule; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_branching_artery.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    for e in t.get("entries", []):
        if (e.get("prec"), e.get("layout_flags"), e.get("block"), e.get("sched_flags")) == (prec, layout, block, sched):
            return e.get("bytes_per_launch")
    return None


def cpu_threads():
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(avail, CPU_SHARE)), avail


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_quota():
    """CPUs' worth of time the cgroup grants this process (cpu.max), or None
    when it sets no limit."""
    for path in ("/sys/fs/cgroup/cpu.max",):
        try:
            with open(path) as fh:
                quota, period = fh.read().split()[:2]
            if quota != "max":
                return round(int(quota) / int(period), 2)
        except (OSError, ValueError):
            pass
    try:
        with open("/sys/fs/cgroup/cpu/cpu.cfs_quota_us") as fh:
            q = int(fh.read())
        with open("/sys/fs/cgroup/cpu/cpu.cfs_period_us") as fh:
            per = int(fh.read())
        if q > 0:
            return round(q / per, 2)
    except (OSError, ValueError):
        pass
    return None


def rel_err(a, b, scale, floor=0.0, record=None, name=None):
    """max |a - b| over the largest |scale|, or `floor` when that is smaller;
    with `record`, also stores the absolute difference and the signal size
    under `name`."""
    sig = float(np.max(np.abs(scale))) if np.size(scale) else 0.0
    s = max(sig, floor)
    d = float(np.max(np.abs(a - b))) if np.size(a) else 0.0
    if record is not None:
        record[name] = {"abs": d, "signal": sig, "floor": floor}
    return d / s if s > 0 else d


# --------------------------------------------------------------------------
# contexts
# --------------------------------------------------------------------------
def make_ctx(hl, geo, prec, torch, order=0):
    ctx = hl.Context(0, prec, order=order)
    d = ctx.add_domain()
    ctx.load_geometry(d, geo)
    ctx.set_tau(d, TAU)
    ctx.set_wall_mode(d, hl.HL_WALL_BOUZIDI)
    ctx.set_inlet_velocity(d, 0, U_IN)
    ctx.set_stream(torch.cuda.current_stream())
    ctx.commit()
    return ctx


def make_workload_ctx(hl, wl, prec, torch, order):
    ctx = hl.Context(0, prec, order=order)
    for d, dm in enumerate(wl.domains):
        ctx.add_domain()
        ctx.load_geometry(d, dm.geo)
        ctx.set_tau(d, dm.tau)
        ctx.set_wall_mode(d, hl.HL_WALL_BOUZIDI if dm.bouzidi else hl.HL_WALL_SBB)
        for k, (a0, a, b, T) in dm.inlets.items():
            ctx.set_inlet_velocity(d, k, a0, a, b, T)
        for k, (r0, a, b, T) in dm.outlets.items():
            ctx.set_outlet_density(d, k, r0, a, b, T)
    for pr in wl.pairs:
        ctx.couple(*pr)
    ctx.set_coupling_mode(wl.mode)
    ctx.set_stream(torch.cuda.current_stream())
    log(f"{len(wl.domains)} domains loaded ({prec}); planning the layout")
    ctx.commit()
    return ctx


def measure(ctx, torch, steps):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    ctx.step(steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.sync()
    return e0.elapsed_time(e1), wall


# --------------------------------------------------------------------------
# the branching artery
# --------------------------------------------------------------------------
def choose_layout(hl, torch, geo, prec, layouts, autotune_ms, probe_steps, schedule=None, drives=None):
    """Layout search (site order and streaming scheme, fixed at context
    creation) around the library's own schedule autotuner (work-group size,
    fused or split launches, XCD order), or a fixed schedule (block, flags);
    then the step drive (plain launches or graph replay) of the fastest.
    Returns (layout, drive, context)."""
    if drives is None:
        drives = (hl.HL_DRIVE_GRAPH, hl.HL_DRIVE_LAUNCH)
    best = None
    for order in layouts:
        ctx = make_ctx(hl, geo, prec, torch, order)
        if schedule is not None:
            ctx.set_schedule(*schedule)
        elif autotune_ms > 0:
            ctx.autotune(autotune_ms)
            n, b, r, sp = ctx.autotune_report()
            log(f"{prec} layout {order}: autotune kept {ctx.schedule()} of {n} candidates, "
                f"median {b * 1e3:.1f} us/step (runner-up {r * 1e3:.1f}), spread {100 * sp:.1f} %")
        for drive in drives:
            # warm-up long enough to capture and instantiate the graph (16 steps per replay)
            ctx.set_drive(drive)
            ctx.step(48)
            ms, _ = measure(ctx, torch, probe_steps)
            log(f"{prec} layout {order}: schedule {ctx.schedule()}, drive {DRIVES[drive]}, "
                f"{geo.n * probe_steps / (ms * 1e-3) / 1e6:.0f} MLUPS")
            if best is None or ms < best[0]:
                if best is not None and best[3] is not ctx:
                    best[3].close()
                best = (ms, order, drive, ctx)
        if best[3] is not ctx:
            ctx.close()
    _, order, drive, ctx = best
    ctx.set_drive(drive)
    return order, drive, ctx


def run_precision(hl, torch, geo, prec, steps, warmup, kernel_steps, autotune_ms, layouts, probe_steps,
                  schedule=None, drives=None):
    """Returns (result dict, context after the run)."""
    order, drive, ctx = choose_layout(hl, torch, geo, prec, layouts, autotune_ms, probe_steps, schedule, drives)
    tune = None
    try:
        n_c, b, r, sp = ctx.autotune_report()
        tune = {"candidates": n_c, "median_ms": round(b, 5), "runner_up_ms": round(r, 5), "spread": round(sp, 4)}
    except Exception:
        pass
    ctx.step(warmup)
    ctx.sync()
    t_start = ctx.t
    ms, wall = measure(ctx, torch, steps)
    kb, kn = ctx.time_kernels(kernel_steps)
    info = ctx.info()
    sched = ctx.schedule()
    n = geo.n
    mlups = n * steps / (ms * 1e-3) / 1e6
    aa = bool(order & hl.HL_SCHEME_AA)
    near = info["n_near"] / info["n_sites"]
    B_alg = bytes_per_site(prec, aa)
    B_i16 = round(bytes_per_site(prec, aa, near), 2)
    res = {
        "mlups": round(mlups, 1),
        "ms_per_step": round(ms / steps, 5),
        "wall_s": round(wall, 3),
        "bytes_per_site": B_alg,
        "alg_GBps": round(mlups * 1e6 * B_alg / 1e9, 1),
        "alg_frac_peak": round(mlups * 1e6 * B_alg / 1e9 / PEAK_HBM_GBS, 4),
        "bytes_per_site_int16": B_i16,
        "near_fraction": round(near, 4),
        "bulk_kernel_ms": round(kb, 5),
        "boundary_kernel_ms": round(kn, 5),
        "n_bulk": info["n_bulk"],
        "n_boundary": info["n_boundary"],
        "layout_flags": order,
        "scheme": "in-place AA" if aa else "two-lattice pull",
        "block": sched[0],
        "sched_flags": sched[1],
        "drive": DRIVES[drive],
        "autotune": tune,
        "steps_timed_from": t_start,
        "device_GB": round(info["device_bytes"] / 1e9, 2),
    }
    log(prec, json.dumps(res))
    return res, ctx


def parity_developed(hl, ctx, geo, threads, t_dev, steps=3):
    """Full-size parity from a developed state: the FP64 context is advanced to
    step t_dev, its populations go into the oracle, both take `steps` more
    steps, and every output is compared."""
    import oracle
    ctx.step(max(0, t_dev - ctx.t))
    f_dev = ctx.populations(0)
    mu_dev, _ = ctx.iolet_stats(0)
    t0 = ctx.t
    sysm = oracle.System(1)
    sysm.set_geometry(0, geo)
    sysm.set_params(0, TAU, oracle.BOUZIDI)
    io = geo.iolets[0]
    sysm.set_iolet(0, 0, oracle.INLET, io.centre, io.normal, io.radius, U_IN)
    sysm.init()
    sysm.set_f(0, f_dev)
    del f_dev
    sysm.step(steps, threads)
    ctx.step(steps)
    res = _compare(ctx, sysm)
    res.update({"from_step": t0, "steps": steps, "outlet_mean_u_min": float(np.abs(mu_dev[1:]).min()),
                "inlet_mean_u": float(mu_dev[0])})
    return res


def _compare(ctx, sysm, dom=0):
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    detail = {}
    rho_r, u_r = sysm.moments(dom)
    out = {"e_u": rel_err(ctx.velocity(dom), u_r, u_r, 1e-4, detail, "u"),
           "e_rho": rel_err(ctx.density(dom), rho_r, rho_r - 1.0, 1e-2, detail, "rho")}
    del rho_r, u_r
    f_r = sysm.f(dom)
    out["e_f"] = rel_err(ctx.populations(dom), f_r, f_r - w[:, None], 1e-3, detail, "f")
    del f_r
    w_r = sysm.wss(dom)
    out["e_wss"] = rel_err(ctx.wss(dom), w_r, w_r, 1e-6, detail, "wss")
    mu_r, mp_r, _ = sysm.iolet_stats(dom)
    mu, mp = ctx.iolet_stats(dom)
    out["e_iolet_u"] = rel_err(mu, mu_r, mu_r, 1e-4, detail, "iolet_u")
    out["e_iolet_p"] = rel_err(mp, mp_r, mp_r, 1e-2 / 3, detail, "iolet_p")
    out["detail"] = detail
    out["tolerance"] = 1e-12
    out["pass"] = all(v <= 1e-12 for k, v in out.items() if k.startswith("e_"))
    return out


def cpu_baseline_and_parity(hl, torch, geo, threads, avail, steps_all, steps_single, order):
    """The FP64 oracle as it stands, on the same workload: 1 untimed and
    `steps_all` timed steps on `threads` OpenMP threads, then `steps_single`
    timed steps on one thread; then the FP64 GPU path runs the same number of
    steps from rest and every output is compared (full-size parity from rest)."""
    import oracle
    sysm = oracle.System(1)
    sysm.set_geometry(0, geo)
    sysm.set_params(0, TAU, oracle.BOUZIDI)
    io = geo.iolets[0]
    sysm.set_iolet(0, 0, oracle.INLET, io.centre, io.normal, io.radius, U_IN)
    sysm.init()
    sysm.step(1, threads)
    t0 = time.perf_counter()
    sysm.step(steps_all, threads)
    t_all = time.perf_counter() - t0
    log(f"oracle: {steps_all} steps in {t_all:.1f} s on {threads} threads")
    t0 = time.perf_counter()
    sysm.step(steps_single, 1)
    t_one = time.perf_counter() - t0
    log(f"oracle: {steps_single} steps in {t_one:.1f} s on 1 thread")
    total = 1 + steps_all + steps_single
    ctx = make_ctx(hl, geo, "f64", torch, order)
    ctx.step(total)
    par = _compare(ctx, sysm)
    ctx.close()
    del sysm
    par.update({"steps": total, "layout_flags": order})
    model = cpu_model()
    cpu = {
        "value": round(geo.n * steps_all / t_all / 1e6, 3),
        "unit": "MLUPS",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"the same workload ({geo.n} sites), FP64, OpenMP over sites: {steps_all} timed steps on "
                   f"{threads} threads after 1 untimed step"),
        "single_thread": {"value": round(geo.n * steps_single / t_one / 1e6, 4), "unit": "MLUPS", "cores": 1,
                          "sample": f"{steps_single} timed steps on 1 thread, after the threaded run"},
        "cpu_model": model,
        "nproc": avail,
        "os_cpu_count": os.cpu_count(),
        "cgroup_cpu_quota": cpu_quota(),
        "threads_rule": f"all CPUs this process may run on, at most {CPU_SHARE} (the host's share for one GPU)",
    }
    return cpu, par


# --------------------------------------------------------------------------
# batched workloads
# --------------------------------------------------------------------------
def run_batched(hl, torch, name, wl, precs, steps, warmup, layout, schedule, drive, long_run=(None, 0)):
    """Every domain of the workload in one context, per precision: MLUPS over
    `steps` timed steps.  long_run = (precision, total steps): that context
    then runs on to the total, logging the root means of the first two
    domains every tenth of the way."""
    n = sum(d.geo.n for d in wl.domains)
    out = {"sites": n, "domains": len(wl.domains), "pairs": len(wl.pairs)}
    for prec in precs:
        t0 = time.perf_counter()
        ctx = make_workload_ctx(hl, wl, prec, torch, layout)
        ctx.set_schedule(*schedule)
        ctx.set_drive(drive)
        ctx.commit()
        t_commit = time.perf_counter() - t0
        log(f"{name} {prec}: {n} sites committed in {t_commit:.1f} s")
        ctx.step(warmup)
        ms, _ = measure(ctx, torch, steps)
        info = ctx.info()
        mlups = n * steps / (ms * 1e-3) / 1e6
        aa = bool(layout & hl.HL_SCHEME_AA)
        B = bytes_per_site(prec, aa)
        r = {"mlups": round(mlups, 1), "ms_per_step": round(ms / steps, 5), "bytes_per_site": B,
             "alg_GBps": round(mlups * 1e6 * B / 1e9, 1),
             "alg_frac_peak": round(mlups * 1e6 * B / 1e9 / PEAK_HBM_GBS, 4),
             "bytes_per_site_int16": round(bytes_per_site(prec, aa, info["n_near"] / info["n_sites"]), 2),
             "device_GB": round(info["device_bytes"] / 1e9, 2), "layout_flags": layout,
             "block": schedule[0], "sched_flags": schedule[1], "drive": DRIVES[drive], "t": ctx.t,
             "setup_s": round(t_commit, 1)}
        if wl.pairs:
            mu, _ = ctx.iolet_stats(0)
            r["mean_u_arterial_root"] = float(mu[0])
        if prec == long_run[0] and long_run[1] > ctx.t:
            series, chunk = [], max(1, long_run[1] // 10)
            t1 = time.perf_counter()
            while ctx.t < long_run[1]:
                ctx.step(min(chunk, long_run[1] - ctx.t))
                roots = [float(ctx.iolet_stats(d)[0][0]) for d in range(min(2, len(wl.domains)))]
                series.append([ctx.t] + roots)
                log(f"{name} {prec}: step {ctx.t}, root mean velocities {roots}")
            r["long_run"] = {"steps": ctx.t, "wall_s": round(time.perf_counter() - t1, 1),
                             "root_mean_u": series, "columns": ["t"] + [f"domain {d} iolet 0"
                                                                      for d in range(len(series[0]) - 1)]}
        ctx.close()
        out[prec] = r
        log(name, prec, json.dumps(r))
    return out


def copy_ceiling(hl, torch, nbytes=2 << 30, reps=20):
    """Measured HBM ceiling in GB/s (read + write): the library's streaming
    copy of 2 GiB, one 16-byte element per lane with non-temporal loads and
    stores, timed with HIP events on the current stream."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(7)
    dst = torch.empty_like(src)
    gbps = hl.hl_copy_bandwidth(dst, src, nbytes, reps=reps, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()
    return round(gbps, 1)


def copy_calibration(torch):
    """A plain device copy of known size for scaling the HBM byte counters."""
    nbytes = 1 << 30
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 3}), flush=True)


def run_coupled_full(hl, torch, args, wl):
    """The coupled pair at its stated size: an arterial tree of about 60 M
    sites (segment length / radius fitted), the venous tree with radii x1.5,
    64 pairs; FP32 and FP64, one line."""
    batched = run_batched(hl, torch, "coupled pair (stated size)", wl, args.precisions.split(","), args.steps,
                          args.warmup, args.batched_layout, _sched(args.batched_schedule), _drive(hl, args),
                          long_run=("f32", args.coupled_steps))
    head = "f32" if "f32" in batched else args.precisions.split(",")[0]
    line = {
        "metric": METRIC, "value": batched[head]["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": batched[head]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": head, "data": "synthetic",
        "config": {"workload": "self-coupled arterial-venous pair at the stated size: Murray trees of depth 6, "
                               "root radius 48, veins x1.5, 64 pairs",
                   "domain_sites": [d.geo.n for d in wl.domains], "segment_length_over_radius": wl.meta["lam"],
                   "lattice_elements_19N": 19 * batched["sites"]},
        "batched": {"coupled_pair": batched},
    }
    if args.coupled_parity > 0:
        threads, _ = cpu_threads()
        line["parity"] = {"developed": coupled_parity_developed(hl, torch, wl, args.coupled_parity, threads)}
    print(json.dumps(line), flush=True)


def coupled_parity_developed(hl, torch, wl, t_dev, threads, steps=3, layout=40, schedule=(256, 11)):
    """Parity of a coupled workload from a developed state: an FP64 context
    of all its domains runs to step t_dev; its populations, its step counter
    and the coupled values its last step used go into the oracle; both take
    `steps` more steps and every output of every domain is compared."""
    import oracle
    t0 = time.perf_counter()
    ctx = make_workload_ctx(hl, wl, "f64", torch, layout)
    ctx.set_schedule(*schedule)
    chunk = 2000
    while ctx.t < t_dev:
        ctx.step(min(chunk, t_dev - ctx.t))
        ctx.sync()
        log(f"coupled parity: FP64 context at step {ctx.t}")
    t = ctx.t
    roots = [float(ctx.iolet_stats(d)[0][0]) for d in range(len(wl.domains))]
    log(f"coupled parity: FP64 context at step {t} ({time.perf_counter() - t0:.1f} s), root mean velocities {roots}")
    sysm = oracle.System(len(wl.domains))
    for d, dm in enumerate(wl.domains):
        sysm.set_geometry(d, dm.geo)
        sysm.set_params(d, dm.tau, oracle.BOUZIDI if dm.bouzidi else oracle.SBB)
        for k, io in enumerate(dm.geo.iolets):
            if io.kind == "inlet" and k in dm.inlets:
                a0, a, b, T = dm.inlets[k]
                sysm.set_iolet(d, k, oracle.INLET, io.centre, io.normal, io.radius, a0, a, b, T)
            if io.kind == "outlet" and k in dm.outlets:
                r0, a, b, T = dm.outlets[k]
                sysm.set_iolet(d, k, oracle.OUTLET, io.centre, io.normal, io.radius, r0, a, b, T)
    for pr in wl.pairs:
        sysm.couple(*pr)
    sysm.set_coupling_mode(wl.mode)
    sysm.init()
    sysm.set_time(t)
    for d in range(len(wl.domains)):
        sysm.set_f(d, ctx.populations(d))
        for k, v in enumerate(ctx.iolet_bc(d, which=1)):
            sysm.set_held(d, k, v)
    log(f"coupled parity: oracle loaded ({time.perf_counter() - t0:.1f} s)")
    t1 = time.perf_counter()
    for k in range(steps):
        sysm.step(1, threads)
        log(f"coupled parity: oracle step {k + 1} of {steps} done ({time.perf_counter() - t1:.1f} s on {threads} threads)")
    ctx.step(steps)
    res = {"from_step": t, "steps": steps, "root_mean_u": roots, "tolerance": 1e-12}
    for d in range(len(wl.domains)):
        res[f"domain {d}"] = _compare(ctx, sysm, d)
        res[f"domain {d}"]["boundary_values"] = float(np.abs(ctx.iolet_bc(d, which=1) - sysm.last_bc(d)).max())
    res["pass"] = all(res[f"domain {d}"]["pass"] for d in range(len(wl.domains)))
    ctx.close()
    del sysm
    log(f"coupled parity: {json.dumps(res)}")
    return res


def _sched(text):
    b, f = (int(v) for v in text.split(":"))
    return b, f


def _drive(hl, args):
    return hl.HL_DRIVE_GRAPH if args.batched_drive == "graph" else hl.HL_DRIVE_LAUNCH


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--box", type=int, default=768)
    ap.add_argument("--precisions", default="f64,f32,f16")
    ap.add_argument("--kernel-steps", type=int, default=50)
    ap.add_argument("--autotune-ms", type=int, default=400)
    ap.add_argument("--layouts", default="40,56",
                    help="hl_create layout flags to search (HL_ORDER_* | HL_SCHEME_AA)")
    ap.add_argument("--probe-steps", type=int, default=200)
    ap.add_argument("--schedule", default="",
                    help="fixed schedule BLOCK:FLAGS (HL_SCHED_* bits) instead of the autotuner")
    ap.add_argument("--drive", default="", choices=["", "launch", "graph"],
                    help="fixed step drive instead of timing both")
    ap.add_argument("--cpu-steps", type=int, default=20, help="timed oracle steps on all of the CPU share")
    ap.add_argument("--cpu-single-steps", type=int, default=2, help="timed oracle steps on one thread")
    ap.add_argument("--developed-steps", type=int, default=2000,
                    help="FP64 steps before the developed-state parity check")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline and full-size parity")
    ap.add_argument("--no-batched", action="store_true", help="skip the coupled pair and the ensemble")
    ap.add_argument("--batched-layout", type=int, default=40)
    ap.add_argument("--batched-schedule", default="256:11", help="BLOCK:FLAGS of the batched runs")
    ap.add_argument("--batched-drive", default="launch", choices=["launch", "graph"])
    ap.add_argument("--batched-precisions", default="f32,f64")
    ap.add_argument("--copy-calibration", action="store_true", help="only run a 1 GiB device copy")
    ap.add_argument("--coupled-parity", type=int, default=0,
                    help="coupled-full: FP64 parity against the oracle from this step on (3 steps)")
    ap.add_argument("--coupled-steps", type=int, default=0,
                    help="coupled-full: run the FP32 context on to this many steps, logging the root means")
    ap.add_argument("--workload", default="artery", choices=["artery", "coupled-full"],
                    help="artery: the default line; coupled-full: the coupled pair at its stated size only")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(the step shards by domain or by contiguous site ranges, not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        import torch
        copy_calibration(torch)
        return
    import synth
    workers, _ = cpu_threads()

    # every geometry is built before anything touches the GPU (the workers are
    # forked processes)
    t0 = time.perf_counter()
    if args.workload == "coupled-full":
        lam = synth.workloads.coupled_lambda()
        log(f"coupled pair at the stated size: lambda {lam:.3f}")
        wl = synth.workloads.coupled_pair(lam=lam, progress=log, workers=workers, job_progress=log)
        log(f"geometry {time.perf_counter() - t0:.1f} s")
    else:
        geo = synth.branching_artery(box=args.box)
        log(f"branching artery: {geo.n} sites, fill {geo.meta['fill']:.4f}, lambda {geo.meta['lam']:.3f}, "
            f"{len(geo.iolets)} iolets, {geo.q.size} wall links ({time.perf_counter() - t0:.1f} s)")
        batched_wl = {}
        if not args.no_batched:
            t1 = time.perf_counter()
            batched_wl["coupled_pair"] = synth.workloads.coupled_pair(workers=workers)
            batched_wl["ensemble"] = synth.workloads.ensemble(workers=workers)
            log(f"batched geometry: {sum(d.geo.n for d in batched_wl['coupled_pair'].domains)} + "
                f"{sum(d.geo.n for d in batched_wl['ensemble'].domains)} sites ({time.perf_counter() - t1:.1f} s)")

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    import paper_2010_04144_amd as hl
    if args.workload == "coupled-full":
        run_coupled_full(hl, torch, args, wl)
        return

    precs = [p.strip() for p in args.precisions.split(",") if p.strip()]
    layouts = [int(v) for v in args.layouts.split(",") if v.strip()]
    schedule = _sched(args.schedule) if args.schedule else None
    drives = {"launch": (hl.HL_DRIVE_LAUNCH,), "graph": (hl.HL_DRIVE_GRAPH,)}.get(args.drive)
    runs, fields, ctx64 = {}, {}, None
    for p in precs:
        res, ctx = run_precision(hl, torch, geo, p, args.steps, args.warmup, args.kernel_steps, args.autotune_ms,
                                 layouts, args.probe_steps, schedule, drives)
        runs[p] = res
        fields[p] = (ctx.velocity(0), ctx.density(0), ctx.t)
        if p == "f64" and not args.no_cpu:
            ctx64 = ctx
        else:
            ctx.close()
    if "f64" in fields:
        u64, r64, t64 = fields["f64"]
        for p in precs:
            u, r, t = fields[p]
            if p != "f64" and t == t64:
                runs[p]["error_vs_f64"] = {"e_u": rel_err(u, u64, u64, 1e-4), "e_rho": rel_err(r, r64, r64 - 1.0, 1e-2),
                                           "after_steps": t}
    del fields

    threads, avail = cpu_threads()
    parity, cpu = {}, None
    if ctx64 is not None:
        parity["developed"] = parity_developed(hl, ctx64, geo, threads, args.developed_steps)
        log("full-size parity, developed state", json.dumps(parity["developed"]))
        ctx64.close()

    batched = {}
    if not args.no_batched:
        for name, wl in batched_wl.items():
            batched[name] = run_batched(hl, torch, name, wl, args.batched_precisions.split(","), args.steps,
                                        args.warmup, args.batched_layout, _sched(args.batched_schedule),
                                        _drive(hl, args))
            wl.domains.clear()

    if not args.no_cpu:
        cpu, parity["from_rest"] = cpu_baseline_and_parity(hl, torch, geo, threads, avail, args.cpu_steps,
                                                           args.cpu_single_steps,
                                                           runs.get("f64", {}).get("layout_flags", 40))
        log("full-size parity from rest", json.dumps(parity["from_rest"]))

    ceiling = copy_ceiling(hl, torch)
    head = "f32" if "f32" in runs else precs[0]
    r = runs[head]
    fused = bool(r["sched_flags"] & hl.HL_SCHED_FUSED)
    k_ms = r["boundary_kernel_ms"] if fused else r["bulk_kernel_ms"]
    k_sites = geo.n if fused else r["n_bulk"]
    B = r["bytes_per_site"]
    achieved = round(k_sites * B / (k_ms * 1e-3) / 1e9, 1)
    kname = ("k_aa" if r["scheme"].startswith("in-place") else "k_step") + (" fused" if fused else " bulk")
    traffic = traffic_from_profile(head, r["layout_flags"], r["block"], r["sched_flags"])
    line = {
        "metric": METRIC,
        "value": r["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic",
        "config": {
            "workload": "branching artery: Murray tree depth 8, root radius 40 lu, 768^3 box, Bouzidi walls, tau 0.55",
            "sites": geo.n,
            "fill": round(geo.meta["fill"], 5),
            "box": args.box,
            "segment_length_over_radius": round(geo.meta["lam"], 4),
            "iolets": len(geo.iolets),
            "storage": {"f64": "FP64", "f32": "FP32 offset f - w rho0", "f16": "FP16 offset f - w rho0",
                        "f16w": "FP16 (f - w rho0) / w", "f16sr": "FP16 offset, stochastic rounding"}[head],
            "arithmetic": "FP64" if head == "f64" else "FP32",
            "scheme": r["scheme"] + f", pull table: int16 deltas for {100 * r['near_fraction']:.1f} % of sites, "
                                    "int32 indices for the rest",
            "layout_flags": r["layout_flags"],
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kname + " (" + head + ")",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            "bytes_per_site": B,
            "bytes_basis": "algorithmic: 2 x 19 populations + 18 int32 pull indices per site",
            "sites_per_launch": k_sites,
            "kernel_ms": k_ms,
            "traffic_over_algorithmic": round(traffic / (B * k_sites), 3) if traffic else None,
            "bytes_per_site_int16": r["bytes_per_site_int16"],
            "achieved_on_int16_bytes": round(k_sites * r["bytes_per_site_int16"] / (k_ms * 1e-3) / 1e9, 1),
            "copy_ceiling": ceiling,
            "frac_of_copy_ceiling": round(achieved / ceiling, 4),
        },
        "variants": runs,
        "batched": batched,
        "parity": parity,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
