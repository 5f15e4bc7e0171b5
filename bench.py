#!/usr/bin/env python3
"""MLUPS and HBM roofline of the sparse D3Q19 LBGK step on one MI355X.

Workload (the branching-artery configuration): a Murray's-law tree of depth 8
(256 outlets), root radius 40 lu, branch angles uniform in 25-45 degrees,
seeded, voxelised in a 768^3 box with the segment length/radius ratio chosen
so the tree fits the box; Bouzidi walls with a wall fraction q uniform in
(0, 1] per link; tau = 0.55; steady parabolic velocity inlet (peak 0.01) at
the root; pressure outlets at rho = 1.  Inputs are synthetic and seeded.

One timed step is one lattice update of every fluid site (all kernels of the
path: gather, boundary links, collision, store, iolet reductions, boundary
update).  MLUPS = sites * steps / time / 1e6, timed with HIP events recorded
on the stream the library launches on, inputs resident in HBM.

Printed: one JSON line (rank 0, N = 1) with the FP32 offset-storage figure as
``value`` and the FP64 and FP16 forms under ``variants``, each with its error
against the FP64 GPU run (itself checked against the FP64 CPU oracle at full
size under ``parity``); ``roofline`` for the dominant kernel (the fused step)
against the published 8 TB/s and against a measured streaming-copy ceiling;
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


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def bytes_per_site(prec, aa=False, near=0.0):
    """Algorithmic HBM bytes of one site update: 19 populations read and
    written, plus 18 pull indices (two-lattice pull) or, averaged over an even
    and an odd step of the in-place scheme, 9; an index is 2 bytes for the
    fraction `near` of sites addressed through int16 deltas, else 4."""
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
        for drive in drives:
            ctx.set_drive(drive)
            ctx.step(4)
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
    order, drive, ctx = choose_layout(hl, torch, geo, prec, layouts, autotune_ms, probe_steps, schedule, drives)
    ctx.step(warmup)
    ctx.sync()
    t_start = ctx.t
    ms, wall = measure(ctx, torch, steps)
    kb, kn = ctx.time_kernels(kernel_steps)
    info = ctx.info()
    u = ctx.velocity(0)
    rho = ctx.density(0)
    sched = ctx.schedule()
    t_end = ctx.t
    ctx.close()
    n = geo.n
    mlups = n * steps / (ms * 1e-3) / 1e6
    aa = bool(order & hl.HL_SCHEME_AA)
    near = info["n_near"] / info["n_sites"]
    B = round(bytes_per_site(prec, aa, near), 2)
    bulk_bytes = info["n_bulk"] * B
    res = {
        "mlups": round(mlups, 1),
        "ms_per_step": round(ms / steps, 5),
        "wall_s": round(wall, 3),
        "alg_GBps": round(mlups * 1e6 * B / 1e9, 1),
        "alg_frac_peak": round(mlups * 1e6 * B / 1e9 / PEAK_HBM_GBS, 4),
        "bulk_kernel_ms": round(kb, 5),
        "boundary_kernel_ms": round(kn, 5),
        "bulk_kernel_GBps": round(bulk_bytes / (kb * 1e-3) / 1e9, 1) if kb > 0.01 else None,
        "bytes_per_site": B,
        "near_fraction": round(near, 4),
        "n_bulk": info["n_bulk"],
        "n_boundary": info["n_boundary"],
        "layout_flags": order,
        "scheme": "in-place AA" if aa else "two-lattice pull",
        "block": sched[0],
        "sched_flags": sched[1],
        "drive": DRIVES[drive],
        "steps_timed_from": t_start,
    }
    log(prec, json.dumps(res))
    return res, u, rho, t_end, order


def rel_err(a, b, scale):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(scale)))


def cpu_baseline_and_parity(hl, torch, geo, seconds, threads, order=0):
    """Time the FP64 oracle on this host's cores over a bounded number of
    steps of the same workload, then run the FP64 GPU path for the same
    steps and compare."""
    import oracle
    sysm = oracle.System(1)
    sysm.set_geometry(0, geo)
    sysm.set_params(0, TAU, oracle.BOUZIDI)
    io = geo.iolets[0]
    sysm.set_iolet(0, 0, oracle.INLET, io.centre, io.normal, io.radius, U_IN)
    sysm.init()
    t0 = time.perf_counter()
    sysm.step(1, threads)
    t1 = time.perf_counter() - t0
    k = max(1, int(seconds / max(t1, 1e-3)) - 1)
    t0 = time.perf_counter()
    sysm.step(k, threads)
    tk = time.perf_counter() - t0
    steps = k + 1
    mlups = geo.n * k / tk / 1e6
    log(f"oracle: {steps} steps, {tk:.1f} s timed for {k} steps, {mlups:.2f} MLUPS on {threads} threads")
    rho_r, u_r = sysm.moments(0)
    f_r = sysm.f(0)
    mu_r, _, _ = sysm.iolet_stats(0)
    del sysm
    ctx = make_ctx(hl, geo, "f64", torch, order)
    ctx.step(steps)
    u = ctx.velocity(0)
    rho = ctx.density(0)
    f = ctx.populations(0)
    mu, _ = ctx.iolet_stats(0)
    ctx.close()
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    par = {
        "steps": steps,
        "layout_flags": order,
        "e_u": rel_err(u, u_r, u_r),
        "e_rho": rel_err(rho, rho_r, rho_r - 1.0),
        "e_f": rel_err(f, f_r, f_r - w[:, None]),
        "e_iolet_u": rel_err(mu, mu_r, mu_r),
        "tolerance": 1e-12,
    }
    par["pass"] = all(par[k2] <= 1e-12 for k2 in ("e_u", "e_rho", "e_f", "e_iolet_u"))
    log("full-size parity", json.dumps(par))
    cpu = {
        "value": round(mlups, 3),
        "unit": "MLUPS",
        "cores": threads,
        "kind": "oracle",
        "sample": f"the same workload ({geo.n} sites), {k} timed steps after 1 untimed step, FP64, OpenMP over sites",
    }
    return cpu, par


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


def run_multi(hl, torch, args):
    """Multi-domain workloads (one context, every domain in the same launches):
    the coupled arterial-venous pair or the ensemble of uneven trees."""
    import synth
    t0 = time.perf_counter()
    if args.workload == "coupled":
        wl = synth.workloads.coupled_pair(lam=args.lam, progress=log)
    else:
        wl = synth.workloads.ensemble(progress=log)
    n = sum(d.geo.n for d in wl.domains)
    log(f"{wl.name}: {len(wl.domains)} domains, {n} sites, {len(wl.pairs)} coupled pairs "
        f"({time.perf_counter() - t0:.1f} s)")
    layouts = [int(v) for v in args.layouts.split(",") if v.strip()]
    out = {}
    for prec in [p.strip() for p in args.precisions.split(",") if p.strip()]:
        best = None
        for order in layouts:
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
            ctx.set_stream(torch.cuda.current_stream())
            ctx.commit()
            if args.autotune_ms > 0:
                ctx.autotune(args.autotune_ms)
            for drive in (hl.HL_DRIVE_GRAPH, hl.HL_DRIVE_LAUNCH):
                ctx.set_drive(drive)
                ctx.step(4)
                ms, _ = measure(ctx, torch, args.probe_steps)
                log(f"{prec} layout {order}: schedule {ctx.schedule()}, drive {DRIVES[drive]}, "
                    f"{n * args.probe_steps / (ms * 1e-3) / 1e6:.0f} MLUPS")
                if best is None or ms < best[0]:
                    if best is not None and best[2] is not ctx:
                        best[2].close()
                    best = (ms, order, ctx, drive)
            if best[2] is not ctx:
                ctx.close()
        _, order, ctx, drive = best
        ctx.set_drive(drive)
        ctx.step(args.warmup)
        ms, wall = measure(ctx, torch, args.steps)
        mlups = n * args.steps / (ms * 1e-3) / 1e6
        info = ctx.info()
        aa = bool(order & hl.HL_SCHEME_AA)
        B = bytes_per_site(prec, aa, info["n_near"] / info["n_sites"])
        out[prec] = {"mlups": round(mlups, 1), "ms_per_step": round(ms / args.steps, 5), "layout_flags": order,
                     "schedule": list(ctx.schedule()), "drive": DRIVES[drive], "bytes_per_site": round(B, 2),
                     "alg_GBps": round(mlups * 1e6 * B / 1e9, 1),
                     "device_GB": round(info["device_bytes"] / 1e9, 2), "t": ctx.t}
        if wl.pairs:
            mu, _ = ctx.iolet_stats(0)
            mv, _ = ctx.iolet_stats(1)
            out[prec]["mean_u_arterial_root"] = float(mu[0])
            out[prec]["mean_u_venous_root"] = float(mv[0])
        log(prec, json.dumps(out[prec]))
        ctx.close()
    head = "f32" if "f32" in out else next(iter(out))
    line = {
        "metric": "MLUPS + achieved HBM GB/s (% peak), FP64 vs FP32 at stated error, 1 GPU",
        "value": out[head]["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": out[head]["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": head, "data": "synthetic",
        "config": {"workload": wl.name, "sites": n, "domains": len(wl.domains), "pairs": len(wl.pairs),
                   "domain_sites": [d.geo.n for d in wl.domains] if len(wl.domains) <= 64 else None,
                   "meta": {k: v for k, v in wl.meta.items() if k != "targets"}},
        "variants": out,
    }
    print(json.dumps(line), flush=True)


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


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--box", type=int, default=768)
    ap.add_argument("--precisions", default="f64,f32,f16")
    ap.add_argument("--kernel-steps", type=int, default=50)
    ap.add_argument("--autotune-ms", type=int, default=400)
    ap.add_argument("--layouts", default="8,24,40,56",
                    help="hl_create layout flags to search (HL_ORDER_* | HL_SCHEME_AA)")
    ap.add_argument("--probe-steps", type=int, default=200)
    ap.add_argument("--schedule", default="",
                    help="fixed schedule BLOCK:FLAGS (HL_SCHED_* bits) instead of the autotuner")
    ap.add_argument("--drive", default="", choices=["", "launch", "graph"],
                    help="fixed step drive instead of timing both")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline and full-size parity")
    ap.add_argument("--copy-calibration", action="store_true", help="only run a 1 GiB device copy")
    ap.add_argument("--workload", default="artery", choices=["artery", "coupled", "ensemble"],
                    help="artery: the branching-artery line (default); coupled / ensemble: multi-domain workloads")
    ap.add_argument("--lam", type=float, default=8.0, help="segment length / radius of the coupled trees")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(the step shards by domain or by contiguous site ranges, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        copy_calibration(torch)
        return
    import paper_2010_04144_amd as hl
    import synth

    if args.workload != "artery":
        run_multi(hl, torch, args)
        return
    t0 = time.perf_counter()
    geo = synth.branching_artery(box=args.box)
    log(f"geometry: {geo.n} sites, fill {geo.meta['fill']:.4f}, lambda {geo.meta['lam']:.3f}, "
        f"{len(geo.iolets)} iolets, {geo.q.size} wall links ({time.perf_counter() - t0:.1f} s)")

    precs = [p.strip() for p in args.precisions.split(",") if p.strip()]
    layouts = [int(v) for v in args.layouts.split(",") if v.strip()]
    schedule = tuple(int(v) for v in args.schedule.split(":")) if args.schedule else None
    drives = {"launch": (hl.HL_DRIVE_LAUNCH,), "graph": (hl.HL_DRIVE_GRAPH,)}.get(args.drive)
    runs, fields, tends, chosen = {}, {}, {}, {}
    for p in precs:
        res, u, rho, t_end, order = run_precision(hl, torch, geo, p, args.steps, args.warmup, args.kernel_steps,
                                                  args.autotune_ms, layouts, args.probe_steps, schedule, drives)
        runs[p] = res
        fields[p] = (u, rho)
        tends[p] = t_end
        chosen[p] = order
    if "f64" in fields:
        u64, r64 = fields["f64"]
        for p in precs:
            if p == "f64":
                continue
            u, r = fields[p]
            if tends[p] != tends["f64"]:
                continue
            runs[p]["error_vs_f64"] = {"e_u": rel_err(u, u64, u64), "e_rho": rel_err(r, r64, r64 - 1.0),
                                       "after_steps": tends[p]}

    cpu, parity = None, None
    if not args.no_cpu:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        cpu, parity = cpu_baseline_and_parity(hl, torch, geo, args.cpu_seconds, threads, chosen.get("f64", 0))

    ceiling = copy_ceiling(hl, torch)
    head = "f32" if "f32" in runs else precs[0]
    r = runs[head]
    B = r["bytes_per_site"]
    fused = bool(r["sched_flags"] & hl.HL_SCHED_FUSED)
    k_ms = r["boundary_kernel_ms"] if fused else r["bulk_kernel_ms"]
    k_sites = geo.n if fused else r["n_bulk"]
    achieved = round(k_sites * B / (k_ms * 1e-3) / 1e9, 1)
    kname = ("k_aa" if r["scheme"].startswith("in-place") else "k_step") + (" fused" if fused else " bulk")
    traffic = traffic_from_profile(head, r["layout_flags"], r["block"], r["sched_flags"])
    line = {
        "metric": "MLUPS + achieved HBM GB/s (% peak), FP64 vs FP32 at stated error, 1 GPU",
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
            "copy_ceiling": ceiling,
            "frac_of_copy_ceiling": round(achieved / ceiling, 4),
            "bytes_per_site": B,
            "sites_per_launch": k_sites,
            "kernel_ms": k_ms,
        },
        "variants": runs,
        "parity": parity,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
