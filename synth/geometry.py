"""Seeded synthetic vascular geometries as sparse D3Q19 site lists.

This module only builds *inputs*: it voxelises shapes, numbers the fluid
voxels and writes, for every site and lattice direction, the index of the
neighbouring fluid site or a boundary code.  It holds none of the lattice
Boltzmann arithmetic, so both the CPU oracle and the GPU library can consume
what it produces without sharing any of the method.

Site-list interface (the same one the C library's ``hl_load_sites`` takes):

* ``coords``  int32 [3][n]   integer voxel coordinates (x, y, z) of each site.
* ``nbr``     int32 [19][n]  ``nbr[i][s]`` is the site at ``x_s + c_i`` when that
  voxel is fluid; ``-1`` when it is solid wall; ``-2-k`` when it lies beyond the
  cut plane of inlet/outlet ("iolet") ``k``.  ``nbr[0][s] == s``.
* wall-distance fractions ``(q_site, q_dir, q)``: for a wall link ``(s, i)`` the
  wall sits at ``x_s + q c_i`` with ``q`` in (0, 1].  Links without an entry are
  halfway links (``q = 1/2``).

The direction order is: rest; +x, -x, +y, -y, +z, -z; then the twelve edge
directions in opposite pairs (+x+y, -x-y), (+x-y, -x+y), (+x+z, -x-z),
(+x-z, -x+z), (+y+z, -y-z), (+y-z, -y+z).  The paper does not fix an ordering
(Sec. 2 names only the D3Q19 velocity set), so the interface does.

Sizes of the tree workloads follow the arterial and venous trees the paper
simulates (Sec. 3.3): Murray's-law bifurcating trees with flat cuts
perpendicular to the centreline at every open end (Sec. 3.1 describes that
tip clipping for the real anatomy).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Direction table of the interface: rest, faces, edges, opposite pairs adjacent.
DIRS = np.array(
    [
        (0, 0, 0),
        (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
        (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
        (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
        (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1),
    ],
    dtype=np.int64,
)
NDIR = 19
WALL = -1
INLET, OUTLET = "inlet", "outlet"


def iolet_code(k: int) -> int:
    """Neighbour code of a link that ends beyond the cut plane of iolet ``k``."""
    return -2 - int(k)


@dataclass
class Iolet:
    """One open boundary.  ``normal`` points into the fluid for an inlet and out
    of the fluid for an outlet; ``centre`` lies on the cut plane."""

    kind: str
    centre: np.ndarray
    normal: np.ndarray
    radius: float

    def outward(self) -> np.ndarray:
        n = np.asarray(self.normal, dtype=np.float64)
        return -n if self.kind == INLET else n


@dataclass
class Geometry:
    coords: np.ndarray            # int32 [3, n]
    nbr: np.ndarray               # int32 [19, n]
    iolets: list                  # list[Iolet]
    dims: tuple                   # box size (nx, ny, nz)
    q_site: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))
    q_dir: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int8))
    q: np.ndarray = field(default_factory=lambda: np.zeros(0, np.float32))
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.coords.shape[1])

    def dense_q(self) -> np.ndarray:
        """float64 [19, n] wall fractions, 0.5 where no entry was given."""
        out = np.full((NDIR, self.n), 0.5)
        if self.q.size:
            out[self.q_dir.astype(np.int64), self.q_site] = self.q.astype(np.float64)
        return out

    def wall_links(self):
        """(site, dir) arrays of every wall link."""
        d, s = np.nonzero(self.nbr == WALL)
        return s.astype(np.int64), d.astype(np.int8)

    def with_q(self, mode: str, seed: int = 0, axis_xy=None, radius=None) -> "Geometry":
        """Attach wall fractions: ``half`` (none), ``random`` (q = 1 - U[0,1),
        seeded, drawn in (dir, site) order) or ``cylinder`` (exact ray / circle
        intersection for a z-aligned cylinder of given axis and radius)."""
        s, d = self.wall_links()
        order = np.lexsort((s, d))
        s, d = s[order], d[order]
        if mode == "half":
            q = np.zeros(0, np.float32)
            s, d = s[:0], d[:0]
        elif mode == "random":
            rng = np.random.default_rng(seed)
            q = (1.0 - rng.random(s.size)).astype(np.float32)
        elif mode == "cylinder":
            q = _cylinder_q(self.coords[:, s], DIRS[d], axis_xy, radius).astype(np.float32)
        else:
            raise ValueError(mode)
        g = Geometry(self.coords, self.nbr, self.iolets, self.dims, s, d, q, dict(self.meta))
        g.meta["q_mode"] = mode
        return g


def _cylinder_q(xyz, c, axis_xy, radius):
    px = xyz[0].astype(np.float64) - axis_xy[0]
    py = xyz[1].astype(np.float64) - axis_xy[1]
    dx = c[:, 0].astype(np.float64)
    dy = c[:, 1].astype(np.float64)
    a = dx * dx + dy * dy
    b = px * dx + py * dy
    cc = px * px + py * py - radius * radius
    q = np.full(px.shape, 0.5)
    ok = a > 0
    disc = np.maximum(b[ok] ** 2 - a[ok] * cc[ok], 0.0)
    t = (-b[ok] + np.sqrt(disc)) / a[ok]
    q[ok] = np.clip(t, 1e-6, 1.0)
    return q


# ---------------------------------------------------------------------------
# neighbour-table construction
# ---------------------------------------------------------------------------
class _BrickIndex:
    """Voxel -> site lookup through 8^3 bricks: a dense brick grid plus one
    512-entry table per non-empty brick (the block structure of Sec. 2.2)."""

    def __init__(self, x, y, z, dims):
        self.dims = tuple(int(v) for v in dims)
        nbx, nby, nbz = ((d + 7) // 8 for d in self.dims)
        self.nb = (nbx, nby, nbz)
        bid = ((z >> 3).astype(np.int64) * nby + (y >> 3)) * nbx + (x >> 3)
        ubid, inv = np.unique(bid, return_inverse=True)
        self.grid = np.full(nbx * nby * nbz, -1, np.int32)
        self.grid[ubid] = np.arange(ubid.size, dtype=np.int32)
        self.table = np.full((ubid.size, 512), -1, np.int32)
        local = (((z & 7) * 8 + (y & 7)) * 8 + (x & 7)).astype(np.int64)
        self.table[inv, local] = np.arange(x.size, dtype=np.int32)

    def lookup(self, x, y, z):
        nx, ny, nz = self.dims
        nbx, nby, _ = self.nb
        inside = (x >= 0) & (x < nx) & (y >= 0) & (y < ny) & (z >= 0) & (z < nz)
        out = np.full(x.shape, -1, np.int32)
        xi, yi, zi = x[inside], y[inside], z[inside]
        slot = self.grid[((zi >> 3).astype(np.int64) * nby + (yi >> 3)) * nbx + (xi >> 3)]
        hit = slot >= 0
        local = (((zi & 7) * 8 + (yi & 7)) * 8 + (xi & 7)).astype(np.int64)
        res = np.full(xi.shape, -1, np.int32)
        res[hit] = self.table[slot[hit], local[hit]]
        out[inside] = res
        return out


_OFF = 1 << 19


def _key(x, y, z):
    return ((z.astype(np.int64) + _OFF) << 42) | ((y.astype(np.int64) + _OFF) << 21) | (x.astype(np.int64) + _OFF)


class _SlabIndex:
    """Voxels that lie just beyond the cut plane of an iolet are labelled with
    that iolet: a link ending there is an iolet link, otherwise a wall link."""

    def __init__(self, iolets, depth=1.5, margin=1.5):
        keys, labels = [], []
        for k, io in enumerate(iolets):
            c = np.asarray(io.centre, np.float64)
            o = io.outward()
            o = o / np.linalg.norm(o)
            rr = io.radius + margin
            ext = rr + depth + 1
            lo = np.floor(c - ext).astype(np.int64)
            hi = np.ceil(c + ext).astype(np.int64)
            gx, gy, gz = np.meshgrid(
                np.arange(lo[0], hi[0] + 1), np.arange(lo[1], hi[1] + 1),
                np.arange(lo[2], hi[2] + 1), indexing="ij")
            v = np.stack([gx.ravel(), gy.ravel(), gz.ravel()]).astype(np.float64)
            rel = v - c[:, None]
            t = o @ rel
            lat2 = (rel * rel).sum(0) - t * t
            m = (t > 0) & (t <= depth) & (lat2 < rr * rr)
            vv = v[:, m].astype(np.int64)
            keys.append(_key(vv[0], vv[1], vv[2]))
            labels.append(np.full(vv.shape[1], k, np.int32))
        if keys:
            keys = np.concatenate(keys)
            labels = np.concatenate(labels)
            order = np.argsort(keys, kind="stable")
            keys, labels = keys[order], labels[order]
            # a voxel claimed by two slabs keeps the lower iolet index
            first = np.ones(keys.size, bool)
            first[1:] = keys[1:] != keys[:-1]
            self.keys, self.labels = keys[first], labels[first]
        else:
            self.keys = np.zeros(0, np.int64)
            self.labels = np.zeros(0, np.int32)

    def classify(self, x, y, z):
        out = np.full(x.shape, WALL, np.int32)
        if self.keys.size == 0 or x.size == 0:
            return out
        k = _key(x, y, z)
        pos = np.searchsorted(self.keys, k)
        pos = np.minimum(pos, self.keys.size - 1)
        hit = self.keys[pos] == k
        out[hit] = -2 - self.labels[pos[hit]]
        return out


def build_site_list(x, y, z, dims, periodic=(False, False, False), iolets=(), meta=None, progress=None):
    """Number fluid voxels (in the given order) and build the neighbour table.
    progress(msg), when given, is called after every sixth direction."""
    x = np.ascontiguousarray(x, dtype=np.int64)
    y = np.ascontiguousarray(y, dtype=np.int64)
    z = np.ascontiguousarray(z, dtype=np.int64)
    n = x.size
    if n >= 2**31 - 1:
        raise ValueError("site count exceeds the int32 index range")
    dims = tuple(int(d) for d in dims)
    idx = _BrickIndex(x, y, z, dims)
    slabs = _SlabIndex(list(iolets))
    nbr = np.empty((NDIR, n), np.int32)
    nbr[0] = np.arange(n, dtype=np.int32)
    for i in range(1, NDIR):
        cx, cy, cz = DIRS[i]
        xx, yy, zz = x + cx, y + cy, z + cz
        if periodic[0]:
            xx %= dims[0]
        if periodic[1]:
            yy %= dims[1]
        if periodic[2]:
            zz %= dims[2]
        j = idx.lookup(xx, yy, zz)
        miss = np.flatnonzero(j < 0)
        if miss.size:
            j[miss] = slabs.classify(xx[miss], yy[miss], zz[miss])
        nbr[i] = j
        if progress is not None and i % 6 == 0:
            progress(f"neighbour table: {i}/{NDIR - 1} directions of {n} sites")
    _one_iolet_per_site(nbr)
    coords = np.stack([x, y, z]).astype(np.int32)
    return Geometry(coords, nbr, list(iolets), dims, meta=dict(meta or {}))


def _one_iolet_per_site(nbr):
    """A site may border one iolet only: links of a site to any iolet other
    than the lowest-numbered one it touches become wall links."""
    codes = np.where(nbr[1:] <= -2, nbr[1:], np.iinfo(np.int32).min)
    top = codes.max(axis=0)                   # -2-k of the lowest k touched
    clash = (nbr[1:] <= -2) & (nbr[1:] != top[None, :])
    if clash.any():
        sub = nbr[1:]
        sub[clash] = WALL


# ---------------------------------------------------------------------------
# simple shapes
# ---------------------------------------------------------------------------
def cylinder(nx=20, ny=20, nz=64, radius=8.0, axis=None, ends="iolets", q="half", seed=0):
    """Straight z-aligned cylinder, fluid iff (x-ax)^2 + (y-ay)^2 < R^2.

    ``ends``: ``"iolets"`` (velocity inlet below z=0, pressure outlet above
    z=nz-1), ``"periodic"`` (wraps in z) or ``"closed"`` (solid end caps)."""
    ax = (nx - 1) / 2.0 if axis is None else axis[0]
    ay = (ny - 1) / 2.0 if axis is None else axis[1]
    gx, gy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    inside = (gx - ax) ** 2 + (gy - ay) ** 2 < radius * radius
    sx, sy = gx[inside].astype(np.int64), gy[inside].astype(np.int64)   # row-major: x fastest
    m = sx.size
    z = np.repeat(np.arange(nz, dtype=np.int64), m)
    x = np.tile(sx, nz)
    y = np.tile(sy, nz)
    iolets = []
    if ends == "iolets":
        iolets = [
            Iolet(INLET, np.array([ax, ay, -0.5]), np.array([0.0, 0.0, 1.0]), float(radius)),
            Iolet(OUTLET, np.array([ax, ay, nz - 0.5]), np.array([0.0, 0.0, 1.0]), float(radius)),
        ]
    periodic = (False, False, ends == "periodic")
    g = build_site_list(x, y, z, (nx, ny, nz), periodic, iolets,
                        meta=dict(kind="cylinder", radius=radius, axis=(ax, ay), ends=ends,
                                  sites_per_slice=int(m)))
    if q == "half":
        return g
    return g.with_q(q, seed=seed, axis_xy=(ax, ay), radius=radius)


def channel(nx=2, ny=8, nz=2, walls="y"):
    """Plane channel: periodic in x and z, flat walls below y=0 and above y=ny-1."""
    gz, gy, gx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    g = build_site_list(gx.ravel(), gy.ravel(), gz.ravel(), (nx, ny, nz), (True, False, True), (),
                        meta=dict(kind="channel"))
    return g


def box(nx, ny, nz, periodic=(True, True, True), solid=None):
    """Every voxel of an nx*ny*nz box that ``solid`` (boolean [nz,ny,nx]) does not mark."""
    gz, gy, gx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    keep = np.ones(gx.shape, bool) if solid is None else ~solid
    return build_site_list(gx[keep], gy[keep], gz[keep], (nx, ny, nz), periodic, (),
                           meta=dict(kind="box"))


def tubes(count=1, radius=4.0, length=24, gap=3, q="half", seed=0):
    """``count`` parallel z-aligned tubes side by side along x in one domain.
    Iolets: inlets 0..count-1 below z=0, then outlets count..2*count-1 above
    z=length-1 (tube order).  Used for small coupled layouts such as the 1:3
    arterial/venous test of Sec. 3."""
    w = int(np.ceil(2 * radius)) + 2
    ny = w
    nx = count * w + (count - 1) * gap
    ay = (ny - 1) / 2.0
    xs, ys = [], []
    axes = []
    for t in range(count):
        ax = t * (w + gap) + (w - 1) / 2.0
        axes.append(ax)
        gx, gy = np.meshgrid(np.arange(t * (w + gap), t * (w + gap) + w), np.arange(ny), indexing="xy")
        m = (gx - ax) ** 2 + (gy - ay) ** 2 < radius * radius
        xs.append(gx[m])
        ys.append(gy[m])
    # one z-slice: order sites by (y, x) so x runs fastest across all tubes
    sx = np.concatenate(xs).astype(np.int64)
    sy = np.concatenate(ys).astype(np.int64)
    o = np.lexsort((sx, sy))
    sx, sy = sx[o], sy[o]
    m = sx.size
    z = np.repeat(np.arange(length, dtype=np.int64), m)
    x = np.tile(sx, length)
    y = np.tile(sy, length)
    iolets = [Iolet(INLET, np.array([ax, ay, -0.5]), np.array([0.0, 0.0, 1.0]), float(radius)) for ax in axes]
    iolets += [Iolet(OUTLET, np.array([ax, ay, length - 0.5]), np.array([0.0, 0.0, 1.0]), float(radius))
               for ax in axes]
    g = build_site_list(x, y, z, (nx, ny, length), (False, False, False), iolets,
                        meta=dict(kind="tubes", count=count, radius=radius, length=length))
    if q == "random":
        g = g.with_q("random", seed=seed)
    return g


def long_pipe(nx, ny, radius, nz, q="half"):
    """z-periodic straight pipe of nz slices, fluid iff (x-ax)^2 + (y-ay)^2 <
    R^2, built without a dense grid: the neighbour table of the middle slice
    of a 3-slice periodic cylinder is repeated along z (sites numbered slice by
    slice, the same in-slice order as ``cylinder``).  ``q``: ``half`` or
    ``cylinder`` (exact ray / circle wall fractions, the same in every slice).
    For site lists whose element count 19 n exceeds 2^31."""
    base = cylinder(nx=nx, ny=ny, nz=3, radius=radius, ends="periodic", q=q)
    S = base.meta["sites_per_slice"]
    n = S * nz
    if n >= 2**31 - 1:
        raise ValueError("site count exceeds the int32 index range")
    mid = base.nbr[:, S:2 * S].astype(np.int64)
    nbr = np.empty((NDIR, n), np.int32)
    z = np.arange(nz, dtype=np.int64)
    for i in range(NDIR):
        cz = int(DIRS[i, 2])
        row = mid[i]
        wall = row < 0
        kp = np.where(wall, 0, row - (1 + cz) * S)        # in-slice index of the neighbour
        zz = (z + cz) % nz
        out = nbr[i].reshape(nz, S)
        for z0 in range(0, nz, 4096):
            z1 = min(nz, z0 + 4096)
            blk = zz[z0:z1, None] * S + kp[None, :]
            blk[:, wall] = -1
            out[z0:z1] = blk
    coords = np.empty((3, n), np.int32)
    coords[0] = np.tile(base.coords[0, :S], nz)
    coords[1] = np.tile(base.coords[1, :S], nz)
    coords[2] = np.repeat(np.arange(nz, dtype=np.int32), S)
    g = Geometry(coords, nbr, [], (nx, ny, nz),
                 meta=dict(kind="long pipe", radius=radius, axis=base.meta["axis"], ends="periodic",
                           sites_per_slice=int(S), slices=int(nz)))
    if q != "half":
        sel = (base.q_site >= S) & (base.q_site < 2 * S)
        ks, kd, kq = base.q_site[sel] - S, base.q_dir[sel], base.q[sel]
        m = ks.size
        g.q_site = (np.arange(nz, dtype=np.int64)[:, None] * S + ks[None, :]).ravel()
        g.q_dir = np.tile(kd, nz)
        g.q = np.tile(kq, nz)
        assert g.q_site.size == m * nz
    return g
