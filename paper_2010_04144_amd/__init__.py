"""MI355X (gfx950) sparse D3Q19 LBGK library: Python binding.

The binding marshals numpy arrays (and, for device reads, torch tensors or
raw device pointers) into the C ABI of ``libhemelb_hip.so``; every step of
the lattice update runs in the library's HIP kernels.  See
``include/hemelb_hip.h`` for the meaning, layout and error behaviour of each
call.
"""
from __future__ import annotations

import ctypes as ct

import numpy as np

from . import _lib
from ._lib import (HL_ALTERNATE, HL_BOTH_EACH_STEP, HL_COUPLE_VELOCITY, HL_DEBUG_CHECKS, HL_DRIVE_GRAPH, HL_DRIVE_LAUNCH,  # noqa: F401
                   HL_E_DEVICE, HL_E_DIVERGED, HL_E_INVAL, HL_E_NOMEM, HL_E_RANGE, HL_E_STATE,
                   HL_F16_OFFSET, HL_F16_SCALED, HL_F16_STOCHASTIC, HL_F32_OFFSET, HL_F64, HL_INLET_VEL, HL_OK,
                   HL_OUTLET_P, HL_ORDER_BOUNDARY_MORTON, HL_ORDER_BRICK, HL_ORDER_BRICK_32, HL_ORDER_BULK_MORTON,
                   HL_ORDER_INTERLEAVE, HL_SCHED_FUSED, HL_SCHED_PAIRS, HL_SCHED_XCD_BRICKS, HL_SCHED_XCD_REMAP,
                   HL_SCHED_XCD_RUNS, HL_SCHEME_AA, HL_W_MACH, HL_W_TAU, HL_WALL_BOUZIDI, HL_WALL_SBB, hl_info)

PRECISIONS = {"f64": HL_F64, "f32": HL_F32_OFFSET, "f16": HL_F16_OFFSET, "f16w": HL_F16_SCALED, "f16sr": HL_F16_STOCHASTIC}


class HLError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} [{code}]")
        self.code = code


def lib():
    return _lib.load()


def status_string(code):
    return lib().hl_status_string(int(code)).decode()


def hl_validate_sites(nbr, n_iolet):
    """Host-only check of a site list (no device needed); returns the code."""
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    n = nbr.shape[1] if nbr.ndim == 2 else nbr.size // 19
    return lib().hl_validate_sites(n, nbr.ctypes.data_as(ct.POINTER(ct.c_int32)), int(n_iolet))


def hl_copy_bandwidth(dst, src, nbytes, reps=20, stream=None):
    """Measured copy ceiling in GB/s: ``nbytes`` copied from ``src`` to ``dst``
    (torch tensors or raw device pointers, caller-owned) ``reps`` times on
    ``stream`` (a torch stream, a raw handle or None)."""
    d = dst.data_ptr() if hasattr(dst, "data_ptr") else int(dst)
    s = src.data_ptr() if hasattr(src, "data_ptr") else int(src)
    st = getattr(stream, "cuda_stream", stream)
    out = ct.c_double(0.0)
    rc = lib().hl_copy_bandwidth(ct.c_void_p(d), ct.c_void_p(s), int(nbytes), int(reps),
                                 ct.c_void_p(st or 0), ct.byref(out))
    if rc != HL_OK:
        raise HLError(rc, f"hl_copy_bandwidth failed: {status_string(rc)}")
    return out.value


def _pd(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def hl_coupling_map(outlet_centres, inlet_centres):
    """Sec. 3 distance map (host only): (owner int32 [n_in], dist float64
    [n_in]) for centres given as (n, 3) arrays."""
    oc = np.ascontiguousarray(np.asarray(outlet_centres, dtype=np.float64).reshape(-1, 3).T)
    ic = np.ascontiguousarray(np.asarray(inlet_centres, dtype=np.float64).reshape(-1, 3).T)
    n_out, n_in = oc.shape[1], ic.shape[1]
    owner = np.zeros(n_in, np.int32)
    dist = np.zeros(n_in)
    rc = lib().hl_coupling_map(n_out, _pd(oc), n_in, _pd(ic), owner.ctypes.data_as(ct.POINTER(ct.c_int32)),
                               _pd(dist))
    if rc != HL_OK:
        raise HLError(rc, f"hl_coupling_map failed: {status_string(rc)}")
    return owner, dist


def hl_velocity_factors(dp, L, A, A0):
    """Eq. (2) (host only): v_i / v_0 for the veins of one arterial outlet."""
    dp, L, A = (np.ascontiguousarray(v, dtype=np.float64).ravel() for v in (dp, L, A))
    v = np.zeros(dp.size)
    rc = lib().hl_velocity_factors(dp.size, _pd(dp), _pd(L), _pd(A), float(A0), _pd(v))
    if rc != HL_OK:
        raise HLError(rc, f"hl_velocity_factors failed: {status_string(rc)}")
    return v


class Context:
    """One library context: several domains stepped together on one GPU."""

    def __init__(self, device=0, precision="f64", order=0):
        self._l = lib()
        self._h = ct.c_void_p()
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        rc = self._l.hl_create(ct.byref(self._h), int(device), prec, int(order))
        if rc != HL_OK:
            raise HLError(rc, f"hl_create failed: {status_string(rc)}")
        self.precision = prec
        self.n = []
        self.n_iolet = []

    # -- plumbing ---------------------------------------------------------
    def _chk(self, rc, what):
        if rc < 0:
            msg = self._l.hl_last_error(self._h).decode()
            raise HLError(rc, f"{what}: {msg or status_string(rc)}")
        return rc

    def close(self):
        if self._h:
            self._l.hl_destroy(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        """``stream``: a torch.cuda.Stream, an integer hipStream_t or None."""
        ptr = getattr(stream, "cuda_stream", stream)
        return self._chk(self._l.hl_set_stream(self._h, ct.c_void_p(ptr or 0)), "hl_set_stream")

    # -- geometry ---------------------------------------------------------
    def add_domain(self):
        d = ct.c_int32()
        self._chk(self._l.hl_add_domain(self._h, ct.byref(d)), "hl_add_domain")
        self.n.append(0)
        self.n_iolet.append(0)
        return d.value

    def load_sites(self, dom, coords, nbr, n_iolet, q_site=None, q_dir=None, q=None):
        coords = np.ascontiguousarray(coords, dtype=np.int32)
        nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        n = coords.shape[1]
        if q is None or len(q) == 0:
            nq, qs, qd, qq = 0, None, None, None
        else:
            qs = np.ascontiguousarray(q_site, dtype=np.int64)
            qd = np.ascontiguousarray(q_dir, dtype=np.int8)
            qq = np.ascontiguousarray(q, dtype=np.float32)
            nq = qs.size
        rc = self._l.hl_load_sites(
            self._h, dom, n, coords.ctypes.data_as(ct.POINTER(ct.c_int32)),
            nbr.ctypes.data_as(ct.POINTER(ct.c_int32)), int(n_iolet), nq,
            None if qs is None else qs.ctypes.data_as(ct.POINTER(ct.c_int64)),
            None if qd is None else qd.ctypes.data_as(ct.POINTER(ct.c_int8)),
            None if qq is None else qq.ctypes.data_as(ct.POINTER(ct.c_float)))
        self._chk(rc, "hl_load_sites")
        self.n[dom] = n
        self.n_iolet[dom] = int(n_iolet)

    def load_geometry(self, dom, geo):
        """Load an object with ``coords``, ``nbr``, ``iolets`` (kind, centre,
        normal, radius) and optional ``q_site``, ``q_dir``, ``q``."""
        self.load_sites(dom, geo.coords, geo.nbr, len(geo.iolets), geo.q_site, geo.q_dir, geo.q)
        for k, io in enumerate(geo.iolets):
            kind = HL_INLET_VEL if io.kind == "inlet" else HL_OUTLET_P
            self.set_iolet(dom, k, kind, io.centre, io.normal, io.radius)

    def set_wall_normals(self, dom, sites, normals):
        sites = np.ascontiguousarray(sites, dtype=np.int64)
        normals = np.ascontiguousarray(normals, dtype=np.float64)
        return self._chk(self._l.hl_set_wall_normals(self._h, dom, sites.size,
                                                     sites.ctypes.data_as(ct.POINTER(ct.c_int64)),
                                                     _pd(normals)), "hl_set_wall_normals")

    # -- physics ----------------------------------------------------------
    def set_wall_mode(self, dom, mode):
        return self._chk(self._l.hl_set_wall_mode(self._h, dom, int(mode)), "hl_set_wall_mode")

    def set_tau(self, dom, tau):
        return self._chk(self._l.hl_set_tau(self._h, dom, float(tau)), "hl_set_tau")

    def set_iolet(self, dom, k, kind, centre, normal, radius):
        c = np.ascontiguousarray(centre, dtype=np.float64)
        nr = np.ascontiguousarray(normal, dtype=np.float64)
        return self._chk(self._l.hl_set_iolet(self._h, dom, k, int(kind), _pd(c), _pd(nr), float(radius)),
                         "hl_set_iolet")

    def _series(self, fn, name, dom, k, a0, a, b, period):
        nh = len(a)
        aa = np.ascontiguousarray(a if nh else [0.0], dtype=np.float64)
        bb = np.ascontiguousarray(b if nh else [0.0], dtype=np.float64)
        return self._chk(fn(self._h, dom, k, float(a0), nh, _pd(aa), _pd(bb), float(period)), name)

    def set_inlet_velocity(self, dom, k, a0, a=(), b=(), period=1.0):
        return self._series(self._l.hl_set_inlet_velocity, "hl_set_inlet_velocity", dom, k, a0, a, b, period)

    def set_outlet_density(self, dom, k, rho, a=(), b=(), period=1.0):
        return self._series(self._l.hl_set_outlet_density, "hl_set_outlet_density", dom, k, rho, a, b, period)

    def set_body_force(self, dom, F0, omega=0.0):
        F = np.ascontiguousarray(F0, dtype=np.float64)
        return self._chk(self._l.hl_set_body_force(self._h, dom, _pd(F), float(omega)), "hl_set_body_force")

    def couple(self, dom_a, outlet, dom_b, inlet, s_vel, dp_ratio):
        return self._chk(self._l.hl_couple(self._h, dom_a, outlet, dom_b, inlet, float(s_vel), float(dp_ratio)),
                         "hl_couple")

    def set_coupling_mode(self, mode):
        return self._chk(self._l.hl_set_coupling_mode(self._h, int(mode)), "hl_set_coupling_mode")

    # -- stepping ---------------------------------------------------------
    def commit(self):
        return self._chk(self._l.hl_commit(self._h), "hl_commit")

    def step(self, n):
        return self._chk(self._l.hl_step(self._h, int(n)), "hl_step")

    def sync(self):
        return self._chk(self._l.hl_sync(self._h), "hl_sync")

    @property
    def t(self):
        v = ct.c_int64()
        self._chk(self._l.hl_get_time(self._h, ct.byref(v)), "hl_get_time")
        return v.value

    def set_drive(self, drive, steps_per_graph=16):
        return self._chk(self._l.hl_set_drive(self._h, int(drive), int(steps_per_graph)), "hl_set_drive")

    # -- reads ------------------------------------------------------------
    def density(self, dom=0):
        out = np.empty(self.n[dom])
        self._chk(self._l.hl_read_density(self._h, dom, _pd(out)), "hl_read_density")
        return out

    def velocity(self, dom=0):
        out = np.empty((3, self.n[dom]))
        self._chk(self._l.hl_read_velocity(self._h, dom, _pd(out)), "hl_read_velocity")
        return out

    def wss(self, dom=0):
        out = np.empty(self.n[dom])
        self._chk(self._l.hl_read_wss(self._h, dom, _pd(out)), "hl_read_wss")
        return out

    def populations(self, dom=0):
        out = np.empty((19, self.n[dom]))
        self._chk(self._l.hl_read_populations(self._h, dom, _pd(out)), "hl_read_populations")
        return out

    def set_populations(self, dom, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        if f.shape != (19, self.n[dom]):
            raise ValueError("populations must have shape (19, n)")
        return self._chk(self._l.hl_set_populations(self._h, dom, _pd(f)), "hl_set_populations")

    def iolet_stats(self, dom=0):
        k = max(self.n_iolet[dom], 1)
        mu, mp = np.zeros(k), np.zeros(k)
        self._chk(self._l.hl_read_iolet_stats(self._h, dom, _pd(mu), _pd(mp)), "hl_read_iolet_stats")
        return mu[: self.n_iolet[dom]], mp[: self.n_iolet[dom]]

    def iolet_bc(self, dom=0, which=0):
        out = np.zeros(max(self.n_iolet[dom], 1))
        self._chk(self._l.hl_read_iolet_bc(self._h, dom, int(which), _pd(out)), "hl_read_iolet_bc")
        return out[: self.n_iolet[dom]]

    def _device(self, fn, name, dom, dst):
        ptr = dst.data_ptr() if hasattr(dst, "data_ptr") else int(dst)
        return self._chk(fn(self._h, dom, ct.c_void_p(ptr)), name)

    def density_device(self, dom, dst):
        return self._device(self._l.hl_read_density_device, "hl_read_density_device", dom, dst)

    def velocity_device(self, dom, dst):
        return self._device(self._l.hl_read_velocity_device, "hl_read_velocity_device", dom, dst)

    def wss_device(self, dom, dst):
        return self._device(self._l.hl_read_wss_device, "hl_read_wss_device", dom, dst)

    def observables_device_noalloc(self, dom, rho=None, u=None, wss=None):
        """Density, velocity and wall shear stress into caller device buffers
        (torch tensors or raw pointers; None skips one) without any device
        allocation (``hl_read_observables_device_noalloc``)."""
        ptr = [ct.c_void_p(0 if b is None else (b.data_ptr() if hasattr(b, "data_ptr") else int(b)))
               for b in (rho, u, wss)]
        return self._chk(self._l.hl_read_observables_device_noalloc(self._h, dom, *ptr),
                         "hl_read_observables_device_noalloc")

    # -- checkpoints, schedule -------------------------------------------
    def get_state(self):
        n = ct.c_size_t(0)
        self._chk(self._l.hl_get_state(self._h, None, ct.byref(n)), "hl_get_state")
        buf = ct.create_string_buffer(n.value)
        self._chk(self._l.hl_get_state(self._h, buf, ct.byref(n)), "hl_get_state")
        return buf.raw

    def set_state(self, blob):
        buf = ct.create_string_buffer(blob, len(blob))
        return self._chk(self._l.hl_set_state(self._h, buf, len(blob)), "hl_set_state")

    def autotune(self, budget_ms=500):
        return self._chk(self._l.hl_autotune(self._h, int(budget_ms)), "hl_autotune")

    def autotune_report(self):
        """(candidates, best ms/step, runner-up ms/step, spread of the best's repeats)."""
        n, b, r, sp = ct.c_int32(), ct.c_double(), ct.c_double(), ct.c_double()
        self._chk(self._l.hl_autotune_report(self._h, ct.byref(n), ct.byref(b), ct.byref(r), ct.byref(sp)),
                  "hl_autotune_report")
        return n.value, b.value, r.value, sp.value

    def schedule(self):
        b, f = ct.c_int32(), ct.c_int32()
        self._chk(self._l.hl_get_schedule(self._h, ct.byref(b), ct.byref(f)), "hl_get_schedule")
        return b.value, f.value

    def set_schedule(self, block, flags=0):
        return self._chk(self._l.hl_set_schedule(self._h, int(block), int(flags)), "hl_set_schedule")

    def time_kernels(self, nsteps):
        """Mean per-step duration (ms) of the bulk-site and boundary-site kernels."""
        b, n = ct.c_double(), ct.c_double()
        self._chk(self._l.hl_time_kernels(self._h, int(nsteps), ct.byref(b), ct.byref(n)), "hl_time_kernels")
        return b.value, n.value

    def info(self):
        inf = hl_info()
        self._chk(self._l.hl_get_info(self._h, ct.byref(inf)), "hl_get_info")
        return {name: getattr(inf, name) for name, _ in inf._fields_}
