"""ctypes wrapper of the plain FP64 CPU oracle (``lbgk_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library.  See the C file's
header for what each step computes and which passage or textbook form it
follows.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB_OVERRIDE names another build of lbgk_oracle.c to load instead (the
# mutation check of the pins builds deliberately broken copies on the CPU)
_LIB_PATH = os.environ.get("ORACLE_LIB_OVERRIDE") or os.path.join(_HERE, "liblbgk_oracle.so")
_lib = None

INLET, OUTLET = 0, 1
SBB, BOUZIDI = 0, 1
ALTERNATE, BOTH, VEL = 0, 1, 2   # VEL: velocity-reverse coupling (a bit, combines with BOTH)

_P = ct.c_void_p
_D = ct.POINTER(ct.c_double)
_I32 = ct.POINTER(ct.c_int32)
_I64 = ct.POINTER(ct.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        if os.environ.get("ORACLE_LIB_OVERRIDE"):
            raise FileNotFoundError(_LIB_PATH)
        from . import build as _b
        _b.build()
    lib = ct.CDLL(_LIB_PATH)
    sig = {
        "or_lattice": (None, [_I32, _D]),
        "or_feq": (None, [ct.c_double, _D, _D]),
        "or_moments_site": (None, [_D, _D, _D, _D]),
        "or_collide_site": (None, [_D, _D, ct.c_double, _D]),
        "or_create": (_P, [ct.c_int]),
        "or_destroy": (None, [_P]),
        "or_set_sites": (ct.c_int, [_P, ct.c_int, ct.c_int64, _I32, _I32, ct.c_int]),
        "or_set_q": (ct.c_int, [_P, ct.c_int, ct.c_int64, _I64, ct.POINTER(ct.c_int8), ct.POINTER(ct.c_float)]),
        "or_set_wall_normals": (ct.c_int, [_P, ct.c_int, _D]),
        "or_set_params": (ct.c_int, [_P, ct.c_int, ct.c_double, ct.c_int]),
        "or_set_force": (ct.c_int, [_P, ct.c_int, _D, ct.c_double]),
        "or_set_iolet": (ct.c_int, [_P, ct.c_int, ct.c_int, ct.c_int, _D, _D, ct.c_double,
                                    ct.c_double, ct.c_int, _D, _D, ct.c_double]),
        "or_couple": (ct.c_int, [_P, ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_double, ct.c_double]),
        "or_set_coupling_mode": (None, [_P, ct.c_int]),
        "or_init": (ct.c_int, [_P]),
        "or_set_f": (ct.c_int, [_P, ct.c_int, _D]),
        "or_set_time": (ct.c_int, [_P, ct.c_int64]),
        "or_set_held": (ct.c_int, [_P, ct.c_int, ct.c_int, ct.c_double]),
        "or_step": (ct.c_int, [_P, ct.c_int64, ct.c_int]),
        "or_time": (ct.c_int64, [_P]),
        "or_read_f": (ct.c_int, [_P, ct.c_int, _D]),
        "or_read_fpost": (ct.c_int, [_P, ct.c_int, _D]),
        "or_read_moments": (ct.c_int, [_P, ct.c_int, _D, _D]),
        "or_read_iolet_stats": (ct.c_int, [_P, ct.c_int, _D, _D, _I64]),
        "or_read_wss": (ct.c_int, [_P, ct.c_int, _D]),
        "or_read_bc": (ct.c_int, [_P, ct.c_int, _D]),
        "or_velocity_factors": (None, [ct.c_int, _D, _D, _D, ct.c_double, _D]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _d(a):
    return a.ctypes.data_as(_D)


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def lattice():
    """(c int [19,3], w float64 [19]) as the oracle defines them."""
    lib = _load()
    c = np.zeros(57, np.int32)
    w = np.zeros(19)
    lib.or_lattice(c.ctypes.data_as(_I32), _d(w))
    return c.reshape(19, 3), w


def feq(rho, u):
    lib = _load()
    u = _arr(u, np.float64)
    out = np.zeros(19)
    lib.or_feq(float(rho), _d(u), _d(out))
    return out


def moments_site(f, F=(0.0, 0.0, 0.0)):
    lib = _load()
    f = _arr(f, np.float64)
    F = _arr(F, np.float64)
    rho = np.zeros(1)
    u = np.zeros(3)
    lib.or_moments_site(_d(f), _d(F), _d(rho), _d(u))
    return float(rho[0]), u


def collide_site(f, tau, F=(0.0, 0.0, 0.0)):
    lib = _load()
    f = _arr(f, np.float64)
    F = _arr(F, np.float64)
    out = np.zeros(19)
    lib.or_collide_site(_d(f), _d(F), float(tau), _d(out))
    return out


def velocity_factors(dp, L, A, A0):
    """Eq. (2) for the veins of one arterial outlet."""
    lib = _load()
    dp, L, A = (_arr(v, np.float64) for v in (dp, L, A))
    out = np.zeros(dp.size)
    lib.or_velocity_factors(int(dp.size), _d(dp), _d(L), _d(A), float(A0), _d(out))
    return out


class System:
    """Several domains (vascular trees) advanced together, optionally coupled."""

    def __init__(self, ndom=1):
        self._lib = _load()
        self._h = self._lib.or_create(int(ndom))
        self.ndom = ndom
        self.n = [0] * ndom
        self.n_iolet = [0] * ndom
        self._keep = []

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.or_destroy(h)
            self._h = None

    def _chk(self, rc, what):
        if rc != 0:
            raise RuntimeError(f"oracle {what} failed ({rc})")

    def set_geometry(self, dom, geo):
        coords = _arr(geo.coords, np.int32)
        nbr = _arr(geo.nbr, np.int32)
        n = coords.shape[1]
        self._chk(self._lib.or_set_sites(self._h, dom, n, coords.ctypes.data_as(_I32),
                                         nbr.ctypes.data_as(_I32), len(geo.iolets)), "set_sites")
        self.n[dom] = n
        self.n_iolet[dom] = len(geo.iolets)
        if geo.q.size:
            qs = _arr(geo.q_site, np.int64)
            qd = _arr(geo.q_dir, np.int8)
            qq = _arr(geo.q, np.float32)
            self._chk(self._lib.or_set_q(self._h, dom, qs.size, qs.ctypes.data_as(_I64),
                                         qd.ctypes.data_as(ct.POINTER(ct.c_int8)),
                                         qq.ctypes.data_as(ct.POINTER(ct.c_float))), "set_q")
        for k, io in enumerate(geo.iolets):
            kind = INLET if io.kind == "inlet" else OUTLET
            self.set_iolet(dom, k, kind, io.centre, io.normal, io.radius,
                           a0=(0.0 if kind == INLET else 1.0))

    def set_wall_normals(self, dom, wn):
        wn = None if wn is None else _arr(wn, np.float64)
        self._keep.append(wn)
        self._lib.or_set_wall_normals(self._h, dom, None if wn is None else _d(wn))

    def set_params(self, dom, tau, wall_mode=SBB):
        self._lib.or_set_params(self._h, dom, float(tau), int(wall_mode))

    def set_force(self, dom, F0, omega=0.0):
        F0 = _arr(F0, np.float64)
        self._lib.or_set_force(self._h, dom, _d(F0), float(omega))

    def set_iolet(self, dom, k, kind, centre, normal, radius, a0, a=(), b=(), period=1.0):
        """Iolet k: kind, plane centre, normal (into the fluid for an inlet, out
        of it for an outlet), radius, and the series
        a0 + sum_m a_m cos(2 pi m t/T) + b_m sin(2 pi m t/T) giving the inlet
        peak velocity or the outlet density at step t."""
        c = _arr(centre, np.float64)
        nr = _arr(normal, np.float64)
        nh = len(a)
        assert len(b) == nh
        aa = _arr(a, np.float64) if nh else np.zeros(1)
        bb = _arr(b, np.float64) if nh else np.zeros(1)
        self._chk(self._lib.or_set_iolet(self._h, dom, k, kind, _d(c), _d(nr), float(radius), float(a0),
                                         int(nh), _d(aa), _d(bb), float(period)), "set_iolet")

    def couple(self, da, ka, db, kb, s, delta):
        self._chk(self._lib.or_couple(self._h, da, ka, db, kb, float(s), float(delta)), "couple")

    def set_coupling_mode(self, mode):
        self._lib.or_set_coupling_mode(self._h, int(mode))

    def init(self):
        self._chk(self._lib.or_init(self._h), "init")

    def set_f(self, dom, f):
        f = _arr(f, np.float64)
        assert f.shape == (19, self.n[dom])
        self._chk(self._lib.or_set_f(self._h, dom, _d(f)), "set_f")

    def set_time(self, t):
        """Step counter of an injected state (waveform phase, exchange half)."""
        self._chk(self._lib.or_set_time(self._h, int(t)), "set_time")

    def set_held(self, dom, k, v):
        """Held coupled value of iolet k of an injected state."""
        self._chk(self._lib.or_set_held(self._h, dom, int(k), float(v)), "set_held")

    def step(self, nsteps, threads=1):
        self._chk(self._lib.or_step(self._h, int(nsteps), int(threads)), "step")

    @property
    def t(self):
        return int(self._lib.or_time(self._h))

    def f(self, dom=0):
        out = np.zeros((19, self.n[dom]))
        self._lib.or_read_f(self._h, dom, _d(out))
        return out

    def fpost(self, dom=0):
        out = np.zeros((19, self.n[dom]))
        self._lib.or_read_fpost(self._h, dom, _d(out))
        return out

    def moments(self, dom=0):
        rho = np.zeros(self.n[dom])
        u = np.zeros((3, self.n[dom]))
        self._lib.or_read_moments(self._h, dom, _d(rho), _d(u))
        return rho, u

    def iolet_stats(self, dom=0):
        k = max(self.n_iolet[dom], 1)
        mu, mp = np.zeros(k), np.zeros(k)
        area = np.zeros(k, np.int64)
        self._lib.or_read_iolet_stats(self._h, dom, _d(mu), _d(mp), area.ctypes.data_as(_I64))
        m = self.n_iolet[dom]
        return mu[:m], mp[:m], area[:m]

    def wss(self, dom=0):
        out = np.zeros(self.n[dom])
        self._lib.or_read_wss(self._h, dom, _d(out))
        return out

    def last_bc(self, dom=0):
        out = np.zeros(max(self.n_iolet[dom], 1))
        self._lib.or_read_bc(self._h, dom, _d(out))
        return out[: self.n_iolet[dom]]
