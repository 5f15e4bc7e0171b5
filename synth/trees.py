"""Seeded synthetic vascular trees (Murray's-law bifurcating networks).

Stand-ins for the patient geometries of the paper (the circle-of-Willis set of
Sec. 2.2 and the arterial / venous leg trees of Sec. 3.3), which are not
available.  A tree of depth ``D`` has ``2**D`` leaves; a child has radius
``r * 2**(-1/3)`` (symmetric Murray's law) and length ``lam * r``.  Each child
leaves its parent at an angle drawn uniformly from ``angle`` degrees, in a
bifurcation plane that turns by 90 +- 30 degrees from one generation to the
next.  Open ends are cut flat, perpendicular to the centreline, as the tip
clipping of Sec. 3.1 does for the real anatomy.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .geometry import INLET, OUTLET, Iolet, build_site_list


@dataclass
class Segment:
    p0: np.ndarray
    p1: np.ndarray
    r: float
    parent: int
    children: tuple
    gen: int


def _rot(v, axis, ang):
    axis = axis / np.linalg.norm(axis)
    c, s = np.cos(ang), np.sin(ang)
    return v * c + np.cross(axis, v) * s + axis * np.dot(axis, v) * (1 - c)


def tree_topology(depth, seed, angle=(25.0, 45.0), twist=(60.0, 120.0)):
    """Unit-free tree: per segment a direction, generation and parent.  All
    random draws happen here, in breadth-first order, so the shape does not
    depend on the length or radius scale chosen later."""
    rng = np.random.default_rng(seed)
    dirs = [np.array([0.0, 0.0, 1.0])]
    planes = [np.array([1.0, 0.0, 0.0])]
    gens, parents, children = [0], [-1], [[]]
    frontier = [0]
    for g in range(depth):
        nxt = []
        for s in frontier:
            d, k = dirs[s], planes[s]
            ta, tb = np.radians(rng.uniform(*angle, size=2))
            tw = np.radians(rng.uniform(*twist, size=2))
            for sign, th, t2 in ((1.0, ta, tw[0]), (-1.0, tb, tw[1])):
                cd = _rot(d, k, sign * th)
                ck = _rot(k, cd, t2)
                ck = ck - np.dot(ck, cd) * cd
                ck /= np.linalg.norm(ck)
                dirs.append(cd / np.linalg.norm(cd))
                planes.append(ck)
                gens.append(g + 1)
                parents.append(s)
                children.append([])
                children[s].append(len(dirs) - 1)
                nxt.append(len(dirs) - 1)
        frontier = nxt
    return dirs, gens, parents, children


def tree_segments(depth, r0, lam, seed, radius_scale=1.0, mirror=False, **kw):
    dirs, gens, parents, children = tree_topology(depth, seed, **kw)
    segs = []
    for s in range(len(dirs)):
        r_geo = r0 * 2.0 ** (-gens[s] / 3.0)          # length follows the arterial radius
        L = lam * r_geo
        p0 = np.zeros(3) if parents[s] < 0 else segs[parents[s]].p1.copy()
        d = dirs[s].copy()
        if mirror:
            d[0] = -d[0]
        segs.append(Segment(p0, p0 + L * d, r_geo * radius_scale, parents[s], tuple(children[s]), gens[s]))
    return segs


def _extent(segs):
    lo = np.min([np.minimum(s.p0, s.p1) - s.r for s in segs], axis=0)
    hi = np.max([np.maximum(s.p0, s.p1) + s.r for s in segs], axis=0)
    return lo, hi


def fit_lambda(depth, r0, seed, box, margin=4, radius_scale=1.0, lo=1.0, hi=60.0, **kw):
    """Largest length/radius ratio for which the tree fits in ``box``^3."""
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        a, b = _extent(tree_segments(depth, r0, mid, seed, radius_scale, **kw))
        if np.all(b - a <= box - 2 * margin - 2):
            lo = mid
        else:
            hi = mid
    return lo


def _voxelise(segs, dims, chunk=32, progress=None):
    """Integer voxels inside the union of the segments (flat ends at open
    ends, a sphere of the parent's radius at every internal joint).
    progress(msg), when given, is called after every 16 segments."""
    parts = []
    nx, ny, nz = dims
    half_diag = 0.5 * chunk * np.sqrt(3.0)
    for k_seg, s in enumerate(segs):
        a = s.p1 - s.p0
        L = np.linalg.norm(a)
        a = a / L
        cap = len(s.children) > 0
        lo = np.floor(np.minimum(s.p0, s.p1) - s.r - 1).astype(np.int64)
        hi = np.ceil(np.maximum(s.p0, s.p1) + s.r + 1).astype(np.int64)
        lo = np.maximum(lo, 0)
        hi = np.minimum(hi, np.array(dims) - 1)
        r2 = s.r * s.r
        for cz in range(lo[2], hi[2] + 1, chunk):
            for cy in range(lo[1], hi[1] + 1, chunk):
                for cx in range(lo[0], hi[0] + 1, chunk):
                    c0 = np.array([cx, cy, cz], np.float64)
                    c1 = np.minimum(c0 + chunk - 1, hi)
                    mid = 0.5 * (c0 + c1)
                    rel = mid - s.p0
                    t = np.clip(rel @ a, 0.0, L)
                    if np.linalg.norm(rel - t * a) > s.r + half_diag + 1:
                        continue
                    gz, gy, gx = np.meshgrid(np.arange(cz, int(c1[2]) + 1), np.arange(cy, int(c1[1]) + 1),
                                             np.arange(cx, int(c1[0]) + 1), indexing="ij")
                    vx, vy, vz = gx.ravel(), gy.ravel(), gz.ravel()
                    rx, ry, rz = vx - s.p0[0], vy - s.p0[1], vz - s.p0[2]
                    tt = rx * a[0] + ry * a[1] + rz * a[2]
                    lat2 = rx * rx + ry * ry + rz * rz - tt * tt
                    m = (tt >= 0) & (tt <= L) & (lat2 < r2)
                    if cap:
                        ex, ey, ez = vx - s.p1[0], vy - s.p1[1], vz - s.p1[2]
                        m |= ex * ex + ey * ey + ez * ez < r2
                    if m.any():
                        parts.append(((vz[m].astype(np.int64) * ny + vy[m]) * nx + vx[m]))
        if progress is not None and ((k_seg + 1) % 16 == 0 or k_seg + 1 == len(segs)):
            progress(f"voxelised {k_seg + 1}/{len(segs)} segments")
    lin = np.unique(np.concatenate(parts)) if parts else np.zeros(0, np.int64)
    x = lin % nx
    y = (lin // nx) % ny
    z = lin // (nx * ny)
    return x, y, z


def tree_geometry(depth, r0, seed, lam=None, box=None, margin=4, radius_scale=1.0,
                  mirror=False, venous=False, q="random", q_seed=None, progress=None, **kw):
    """Voxelised tree.  Arterial trees have one velocity inlet at the root and
    a pressure outlet at every leaf; ``venous`` trees are the reverse (one
    inlet per leaf, a pressure outlet at the root).  Iolet 0 is the root,
    iolets 1.. are the leaves in breadth-first order.  progress(msg), when
    given, reports the voxelisation and the neighbour table as they go."""
    if lam is None:
        lam = fit_lambda(depth, r0, seed, box, margin, radius_scale, **kw)
    segs = tree_segments(depth, r0, lam, seed, radius_scale, mirror, **kw)
    lo, hi = _extent(segs)
    shift = margin - lo
    for s in segs:
        s.p0 = s.p0 + shift
        s.p1 = s.p1 + shift
    ext = np.ceil(hi - lo).astype(np.int64) + 2 * margin
    dims = (int(box),) * 3 if box else tuple(int(v) for v in ext)
    x, y, z = _voxelise(segs, dims, progress=progress)
    root = segs[0]
    ra = (root.p1 - root.p0) / np.linalg.norm(root.p1 - root.p0)
    iolets = [Iolet(OUTLET if venous else INLET, root.p0.copy(), (-ra if venous else ra), root.r)]
    leaves = [s for s in segs if not s.children]
    for s in leaves:
        a = (s.p1 - s.p0) / np.linalg.norm(s.p1 - s.p0)
        iolets.append(Iolet(INLET if venous else OUTLET, s.p1.copy(), (-a if venous else a), s.r))
    g = build_site_list(x, y, z, dims, (False, False, False), iolets,
                        meta=dict(kind="tree", depth=depth, r0=r0, lam=float(lam), seed=seed,
                                  radius_scale=radius_scale, venous=venous, n_leaves=len(leaves),
                                  fill=float(x.size) / float(np.prod(dims))), progress=progress)
    if q == "random":
        g = g.with_q("random", seed=seed + 7 if q_seed is None else q_seed)
    return g


def branching_artery(box=768, depth=8, r0=40.0, seed=20100414 + 2):
    """Branching artery of depth 8, root radius 40, seeded, in a box^3 grid,
    with random Bouzidi wall fractions."""
    return tree_geometry(depth, r0, seed, box=box)


def coupled_pair(depth=6, r0=48.0, seed=20100414 + 4, lam=None, box=None, vein_scale=1.5):
    """Arterial tree plus a mirrored venous tree of the same seeded topology
    with radii scaled by ``vein_scale``.  Returns (artery, vein)."""
    if lam is None:
        lam = fit_lambda(depth, r0, seed, box) if box else 8.0
    art = tree_geometry(depth, r0, seed, lam=lam)
    ven = tree_geometry(depth, r0, seed, lam=lam, radius_scale=vein_scale, mirror=True, venous=True)
    return art, ven


def ensemble(count=32, lo=5e5, hi=8e6, depth=6, lam=8.0, seed=20100414 + 5):
    """``count`` trees whose site counts are log-uniform in [lo, hi]; the root
    radius of each is scaled to hit its target.  Returns (geometries, targets)."""
    rng = np.random.default_rng(seed)
    targets = np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))
    geos = []
    for m, nt in enumerate(targets):
        r0 = (nt / ((depth + 1) * np.pi * lam)) ** (1.0 / 3.0)
        geos.append(tree_geometry(depth, float(r0), seed + 100 + m, lam=lam))
    return geos, targets
