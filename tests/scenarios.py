"""Build one scenario (geometry + physics settings) both in the CPU oracle and
in the GPU library, and compare their outputs with the error metrics used
throughout the tests:

  e_u       = max |u - u_ref| / max(max |u_ref|, 1e-4)
  e_rho     = max |rho - rho_ref| / max(max |rho_ref - rho0|, 1e-2)
  e_f       = max |f - f_ref| / max(max |f_ref - w rho0|, 1e-3)
  e_wss     = max |wss - wss_ref| / max(max |wss_ref|, 1e-6)
  e_iolet_u = max |mean_u - mean_u_ref| / max(max |mean_u_ref|, 1e-4)
  e_iolet_p = max |mean_p - mean_p_ref| / max(max |mean_p_ref|, 0.01 / 3)

Each error is measured against the size of its signal: the deviation from
the rest state for the density and the populations, the values themselves
for the velocity, the wall shear stress and the iolet means.  The floors (in
lattice units: 1e-4 for a velocity, 1 % of rho0 for the density, 1e-3 for a
population offset, 1e-6 for a stress) keep each ratio meaningful where the
signal is at round-off level, e.g. a domain that is still at rest or the
density of a force-driven periodic pipe.  The iolet gauge pressure is a
density deviation, p = (mean rho - rho0)/3, and shares the density's floor
(0.01/3): with full populations stored in FP64, rho itself is resolved only to
about 1e-16, so smaller pressures cannot carry 12 significant digits.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
U_FLOOR, RHO_FLOOR, F_FLOOR, WSS_FLOOR, P_FLOOR = 1e-4, 1e-2, 1e-3, 1e-6, 1e-2 / 3


@dataclass
class Dom:
    geo: object
    tau: float = 0.8
    bouzidi: bool = False
    F0: tuple = (0.0, 0.0, 0.0)
    omega: float = 0.0
    inlets: dict = field(default_factory=dict)    # k -> (a0, a, b, period)
    outlets: dict = field(default_factory=dict)   # k -> (rho, a, b, period)


@dataclass
class Scenario:
    doms: list
    pairs: list = field(default_factory=list)     # (da, ka, db, kb, s, delta)
    mode: int = 0


def from_workload(wl):
    """Scenario from a synth.workloads.Workload."""
    doms = [Dom(d.geo, d.tau, d.bouzidi, tuple(d.F0), d.omega, dict(d.inlets), dict(d.outlets)) for d in wl.domains]
    return Scenario(doms, list(wl.pairs), wl.mode)


def build_oracle(sc, oracle):
    s = oracle.System(len(sc.doms))
    for d, dm in enumerate(sc.doms):
        s.set_geometry(d, dm.geo)
        s.set_params(d, dm.tau, oracle.BOUZIDI if dm.bouzidi else oracle.SBB)
        if any(dm.F0):
            s.set_force(d, dm.F0, dm.omega)
        for k, io in enumerate(dm.geo.iolets):
            if io.kind == "inlet" and k in dm.inlets:
                a0, a, b, T = dm.inlets[k]
                s.set_iolet(d, k, oracle.INLET, io.centre, io.normal, io.radius, a0, a, b, T)
            if io.kind == "outlet" and k in dm.outlets:
                r0, a, b, T = dm.outlets[k]
                s.set_iolet(d, k, oracle.OUTLET, io.centre, io.normal, io.radius, r0, a, b, T)
    for p in sc.pairs:
        s.couple(*p)
    s.set_coupling_mode(sc.mode)
    s.init()
    return s


def build_gpu(sc, hl, precision="f64", order=0):
    ctx = hl.Context(0, precision, order=order)
    for d, dm in enumerate(sc.doms):
        ctx.add_domain()
        ctx.load_geometry(d, dm.geo)
        ctx.set_tau(d, dm.tau)
        ctx.set_wall_mode(d, hl.HL_WALL_BOUZIDI if dm.bouzidi else hl.HL_WALL_SBB)
        if any(dm.F0):
            ctx.set_body_force(d, dm.F0, dm.omega)
        for k, (a0, a, b, T) in dm.inlets.items():
            ctx.set_inlet_velocity(d, k, a0, a, b, T)
        for k, (r0, a, b, T) in dm.outlets.items():
            ctx.set_outlet_density(d, k, r0, a, b, T)
    for p in sc.pairs:
        ctx.couple(*p)
    ctx.set_coupling_mode(sc.mode)
    return ctx


def rel(a, b, scale, floor=0.0):
    scale = max(float(np.max(np.abs(scale))) if np.size(scale) else 0.0, floor)
    if scale == 0.0:
        return float(np.max(np.abs(a - b)))
    return float(np.max(np.abs(a - b)) / scale)


def errors(ctx, osys, dom=0, with_f=True, with_wss=True, dom_o=None):
    do = dom if dom_o is None else dom_o
    rho_r, u_r = osys.moments(do)
    out = {
        "e_u": rel(ctx.velocity(dom), u_r, u_r, U_FLOOR),
        "e_rho": rel(ctx.density(dom), rho_r, rho_r - 1.0, RHO_FLOOR),
    }
    if with_f:
        f_r = osys.f(do)
        out["e_f"] = rel(ctx.populations(dom), f_r, f_r - W[:, None], F_FLOOR)
    if with_wss:
        w_r = osys.wss(do)
        out["e_wss"] = rel(ctx.wss(dom), w_r, w_r, WSS_FLOOR)
    if osys.n_iolet[do]:
        mu_r, mp_r, _ = osys.iolet_stats(do)
        mu, mp = ctx.iolet_stats(dom)
        out["e_iolet_u"] = rel(mu, mu_r, mu_r, U_FLOOR)
        out["e_iolet_p"] = rel(mp, mp_r, mp_r, P_FLOOR)
    return out
