"""The other workload configurations on the GPU: the full-size Womersley pipe
against the analytic solution, and reduced-size twins of the coupled
arterial-venous pair and of the uneven ensemble against the FP64 oracle."""
import os

import numpy as np
import pytest

import synth
from scenarios import build_gpu, build_oracle, errors, from_workload

pytestmark = pytest.mark.gpu
THREADS = min(8, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def hl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_04144_amd as hl
    hl.lib()
    return hl


def womersley_error(ctx, wl, phases=8):
    meta = wl.meta
    geo = wl.domains[0].geo
    ax, ay = meta["axis"]
    r = np.sqrt((geo.coords[0] - ax) ** 2 + (geo.coords[1] - ay) ** 2)
    per = meta["period"]
    amp = np.max(np.abs(synth.workloads.womersley_profile(np.zeros(1), np.arange(64) * per / 64, meta)))
    errs = []
    for k in range(phases):
        u = ctx.velocity(0)[2]
        ana = synth.workloads.womersley_profile(r, ctx.t, meta)
        errs.append(float(np.sqrt(np.mean((u - ana) ** 2)) / amp))
        ctx.step(int(round(per / phases)))
    return max(errs)


@pytest.mark.parametrize("alpha", [10.0, 4.0])
def test_womersley_full_size(hl, alpha):
    """Pipe of radius 32 and length 1024 (3.3 M sites), tau 0.8, five periods:
    FP64 follows Womersley's profile within the staircase error; FP32 and FP16
    offset storage report their errors against the FP64 run."""
    wl = synth.workloads.womersley(alpha=alpha)
    sc = from_workload(wl)
    per = wl.meta["period"]
    n0 = int(round(4 * per))
    res = {}
    for prec in ("f64", "f32", "f16"):
        ctx = build_gpu(sc, hl, prec)
        ctx.step(n0)
        err = womersley_error(ctx, wl)
        res[prec] = (err, ctx.velocity(0), ctx.density(0))
        ctx.close()
        print(f"womersley alpha={alpha} {prec}: max relative L2 vs analytic over the 5th period {err:.4f}",
              flush=True)
    assert res["f64"][0] < 0.03
    u64 = res["f64"][1]
    for prec, bound in (("f32", 1e-4), ("f16", 2e-2)):
        e_u = np.abs(res[prec][1] - u64).max() / np.abs(u64).max()
        print(f"womersley alpha={alpha} {prec} vs f64: e_u={e_u:.2e}", flush=True)
        assert e_u < bound
        assert res[prec][0] < 0.03


@pytest.mark.parametrize("order", [2, 16 | 8])
def test_coupled_pair_twin(hl, oracle_mod, order):
    """Reduced twin of the coupled pair (depth 3, root radius 10, veins x1.5,
    8 pairs 1:1, pulsatile inlet), 800 steps so that flow has crossed into the
    venous tree: FP64 matches the oracle to 1e-12 in both domains, FP32 offset
    storage within the stated bound.  Two-lattice and in-place layouts."""
    wl = synth.workloads.coupled_pair(depth=3, r0=10.0, lam=6.0, period=300.0)
    sc = from_workload(wl)
    o = build_oracle(sc, oracle_mod)
    o.step(800, THREADS)
    g = build_gpu(sc, hl, "f64", order=order)
    g.step(800)
    for d in (0, 1):
        err = errors(g, o, d)
        print("coupled twin fp64", d, err, flush=True)
        assert max(err.values()) <= 1e-12, err
        np.testing.assert_allclose(g.iolet_bc(d, which=1), o.last_bc(d), rtol=1e-12, atol=1e-15)
    g32 = build_gpu(sc, hl, "f32", order=order)
    g32.step(800)
    for d in (0, 1):
        err = errors(g32, o, d, with_f=False, with_wss=False)
        print("coupled twin fp32", d, err, flush=True)
        assert err["e_u"] < 1e-3


def test_ensemble_twin(hl, oracle_mod):
    """Reduced twin of the ensemble: six trees of uneven size, each with its
    own tau and 3-harmonic inlet waveform, advanced in one context."""
    wl = synth.workloads.ensemble(count=6, lo=1.5e4, hi=8e4, depth=3, lam=6.0)
    sc = from_workload(wl)
    o = build_oracle(sc, oracle_mod)
    o.step(150, THREADS)
    g = build_gpu(sc, hl, "f64")
    g.set_schedule(128, 0)
    g.step(150)
    for d in range(len(sc.doms)):
        err = errors(g, o, d)
        assert max(err.values()) <= 1e-12, (d, err)
