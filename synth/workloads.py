"""Seeded workload descriptions: geometry plus the physical settings of each
configuration (relaxation time, inlet waveforms, outlet densities, body
force, coupling pairs).  Only inputs live here; no lattice arithmetic.

The random numbers a configuration needs (wall fractions, pressure-drop
factors, per-tree relaxation times, waveform coefficients) are drawn here
with NumPy's PCG64 from fixed seeds and passed to both the oracle and the
library as inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .geometry import cylinder
from .trees import tree_geometry

MASTER_SEED = 20100414


@dataclass
class DomainSpec:
    geo: object
    tau: float
    bouzidi: bool = False
    F0: tuple = (0.0, 0.0, 0.0)
    omega: float = 0.0
    inlets: dict = field(default_factory=dict)     # k -> (a0, a, b, period)
    outlets: dict = field(default_factory=dict)    # k -> (rho, a, b, period)


@dataclass
class Workload:
    name: str
    domains: list
    pairs: list = field(default_factory=list)      # (dom_a, outlet, dom_b, inlet, s_vel, dp_ratio)
    mode: int = 0
    steps: int = 0
    meta: dict = field(default_factory=dict)


def womersley(alpha=10.0, radius=32.0, length=1024, tau=0.8, u_centre=0.01):
    """Periodic straight pipe driven by a uniform force G0 cos(w t) along the
    axis, w = alpha^2 nu / R^2; G0 is chosen so that the analytic centreline
    amplitude is u_centre.  Five periods."""
    from scipy.special import jv
    nu = (tau - 0.5) / 3.0
    omega = alpha ** 2 * nu / radius ** 2
    i32 = np.exp(1j * 3 * np.pi / 4)
    amp = abs((1.0 / (1j * omega)) * (1.0 - 1.0 / jv(0, i32 * alpha)))
    G0 = u_centre / amp
    n = int(np.ceil(2 * radius)) + 2
    geo = cylinder(nx=n, ny=n, nz=length, radius=radius, ends="periodic")
    period = 2 * np.pi / omega
    d = DomainSpec(geo, tau, F0=(0.0, 0.0, G0), omega=omega)
    return Workload(f"womersley alpha {alpha:g}", [d], steps=int(round(5 * period)),
                    meta=dict(alpha=alpha, radius=radius, omega=omega, G0=G0, period=period, nu=nu,
                              axis=geo.meta["axis"]))


def womersley_profile(r, t, meta):
    """Womersley's (1955) velocity for the force G0 cos(w t)."""
    from scipy.special import jv
    i32 = np.exp(1j * 3 * np.pi / 4)
    a, R, w, G0 = meta["alpha"], meta["radius"], meta["omega"], meta["G0"]
    return np.real(G0 / (1j * w) * (1 - jv(0, i32 * a * r / R) / jv(0, i32 * a)) * np.exp(1j * w * t))


def pulsatile(rng, mean=0.01, spread=0.003, harmonics=3, period=None):
    a = rng.uniform(-spread, spread, harmonics)
    b = rng.uniform(-spread, spread, harmonics)
    T = float(rng.uniform(1000, 4000)) if period is None else float(period)
    peak = mean + np.sum(np.abs(a) + np.abs(b))
    if np.sqrt(3) * peak >= 0.1:          # keep Ma = sqrt(3) U below 0.1
        s = (0.1 / np.sqrt(3) * 0.99 - mean) / np.sum(np.abs(a) + np.abs(b))
        a, b = a * s, b * s
    return (mean, tuple(a), tuple(b), T)


_JOB_PROGRESS = None  # progress(msg) of the tree jobs, set before the workers fork


def _tree_job(job):
    depth, r0, seed, kw = job
    return tree_geometry(depth, r0, seed, progress=_JOB_PROGRESS, **kw)


def build_trees(jobs, workers=1, progress=None, job_progress=None):
    """tree_geometry(depth, r0, seed, **kw) for every (depth, r0, seed, kw) in
    jobs, in that order; with workers > 1 in forked worker processes (largest
    trees first), which must happen before the calling process touches a
    GPU.  The result does not depend on the number of workers.  progress(msg)
    is called after each tree; job_progress(msg), inside the job, as a tree
    is built."""
    global _JOB_PROGRESS
    _JOB_PROGRESS = job_progress
    if workers <= 1 or len(jobs) <= 1:
        out = []
        for j in jobs:
            out.append(_tree_job(j))
            if progress is not None:
                progress(f"tree {len(out)}/{len(jobs)}: {out[-1].n} sites")
        return out
    import multiprocessing as mp
    order = sorted(range(len(jobs)), key=lambda k: -(jobs[k][1] ** 3) * jobs[k][3].get("radius_scale", 1.0) ** 2)
    out = [None] * len(jobs)
    with mp.get_context("fork").Pool(min(workers, len(jobs))) as pool:
        for k, geo in zip(order, pool.imap(_tree_job, [jobs[k] for k in order], chunksize=1)):
            out[k] = geo
            if progress is not None:
                progress(f"tree {sum(g is not None for g in out)}/{len(jobs)}: {geo.n} sites")
    return out


def coupled_lambda(depth=6, r0=48.0, seed=MASTER_SEED + 4, arterial_sites=60e6):
    """Segment length / radius ratio for which the arterial tree of the
    coupled pair holds about `arterial_sites` sites.  The segments' volume
    grows linearly with it and the joints' does not, so two probe trees of the
    same shape at half the radius (1/8 of the volume) fix a line n(lambda)."""
    n8 = tree_geometry(depth, r0 / 2.0, seed, lam=8.0).n * 8.0
    n16 = tree_geometry(depth, r0 / 2.0, seed, lam=16.0).n * 8.0
    slope = (n16 - n8) / 8.0
    return float(8.0 + (arterial_sites - n8) / slope)


def coupled_pair(depth=6, r0=48.0, lam=None, vein_scale=1.5, seed=MASTER_SEED + 4, period=4000.0,
                 tau=0.8, steps=20000, progress=None, workers=1, job_progress=None):
    """Arterial tree (root velocity inlet, leaf pressure outlets) coupled 1:1
    at every leaf to the mirrored venous tree of the same seeded topology with
    radii scaled by vein_scale (leaf velocity inlets, root pressure outlet).
    s_i = A_artery / A_vein (Eq. (2) with one vein per outlet), dP_i/P0 drawn
    uniformly from [0.3, 0.7) (Sec. 3).  Pulsatile 3-harmonic root inlet."""
    rng = np.random.default_rng(seed)
    if lam is None:
        lam = 8.0
    art, ven = build_trees([(depth, r0, seed, dict(lam=lam)),
                            (depth, r0, seed, dict(lam=lam, radius_scale=vein_scale, mirror=True, venous=True))],
                           workers=workers, job_progress=job_progress)
    if progress is not None:
        progress(f"arterial tree: {art.n} sites; venous tree: {ven.n} sites")
    inlet = pulsatile(rng, period=period)
    a = DomainSpec(art, tau, bouzidi=True, inlets={0: inlet})
    v = DomainSpec(ven, tau, bouzidi=True, outlets={0: (1.0, (), (), 1.0)})
    pairs = []
    area_a = _iolet_areas(art)
    area_v = _iolet_areas(ven)
    for k in range(1, len(art.iolets)):
        dp = float(rng.uniform(0.3, 0.7))
        pairs.append((0, k, 1, k, float(area_a[k] / area_v[k]), dp))
    for k in range(1, len(art.iolets)):
        a.outlets[k] = (1.0, (), (), 1.0)
    return Workload("coupled arterial-venous pair", [a, v], pairs=pairs, steps=steps,
                    meta=dict(depth=depth, r0=r0, lam=lam, vein_scale=vein_scale))


def _iolet_areas(geo):
    """Number of sites bordering each iolet (the boundary 'area')."""
    codes = geo.nbr[1:]
    out = np.zeros(len(geo.iolets), np.int64)
    for k in range(len(geo.iolets)):
        out[k] = int(np.count_nonzero((codes == -2 - k).any(axis=0)))
    return out


def ensemble(count=32, lo=5e5, hi=8e6, depth=6, lam=8.0, seed=MASTER_SEED + 5, steps=2000, progress=None,
             workers=1):
    """count trees with site counts log-uniform in [lo, hi] (root radius scaled
    to hit each target), each with its own tau in [0.52, 0.9] and a seeded
    3-harmonic inlet waveform with period in [1000, 4000].  progress(msg) is
    called after each tree."""
    rng = np.random.default_rng(seed)
    targets = np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))
    jobs = [(depth, float((nt / ((depth + 1) * np.pi * lam)) ** (1.0 / 3.0)), seed + 100 + m, dict(lam=lam))
            for m, nt in enumerate(targets)]
    geos = build_trees(jobs, workers=workers, progress=progress)
    doms = []
    for m, geo in enumerate(geos):
        tau = float(rng.uniform(0.52, 0.9))
        inlet = pulsatile(rng)
        outs = {k: (1.0, (), (), 1.0) for k in range(1, len(geo.iolets))}
        doms.append(DomainSpec(geo, tau, bouzidi=True, inlets={0: inlet}, outlets=outs))
    return Workload("ensemble of uneven trees", doms, steps=steps, meta=dict(targets=targets.tolist()))
