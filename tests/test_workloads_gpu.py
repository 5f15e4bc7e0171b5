"""The workload configurations on the GPU: the branching artery at full size
in the layouts and schedule the benchmark times, the full-size Womersley pipe
against the analytic solution, and reduced-size twins of the coupled
arterial-venous pair and of the uneven ensemble against the FP64 oracle."""
import os

import numpy as np
import pytest

import synth
from scenarios import Dom, Scenario, build_gpu, build_oracle, errors, from_workload

pytestmark = pytest.mark.gpu
THREADS = min(8, os.cpu_count() or 1)
TOL64 = 1e-12


@pytest.fixture(scope="module")
def hl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_04144_amd as hl
    hl.lib()
    return hl


def test_branching_artery_full_size(hl, oracle_mod):
    """The benchmark workload at full size (Murray tree of depth 8, root radius
    40, 768^3 box, 6,064,894 sites, Bouzidi walls, tau 0.55, steady inlet) in
    the configurations the benchmark times: 32^3 bricks with the fused XCD-runs
    schedule, two lattices in FP64 and FP32 offset storage and in place in
    FP16 offset storage, each against the FP64 oracle after five steps (an odd
    count, so the in-place run ends on an odd sweep).  Every output is
    compared, not a sample: the oracle takes about a second per step here."""
    geo = synth.branching_artery(box=768)
    assert geo.n == 6064894
    sc = Scenario([Dom(geo, tau=0.55, bouzidi=True, inlets={0: (0.01, (), (), 1.0)})])
    o = build_oracle(sc, oracle_mod)
    o.step(5, min(16, os.cpu_count() or 1))
    sched = hl.HL_SCHED_FUSED | hl.HL_SCHED_XCD_REMAP | hl.HL_SCHED_XCD_RUNS
    bricks = hl.HL_ORDER_BRICK | hl.HL_ORDER_BRICK_32
    for prec, order, bound in (("f64", bricks, TOL64), ("f32", bricks, 1e-3),
                               ("f16", bricks | hl.HL_SCHEME_AA, 2e-2)):
        print(f"branching artery full size: {prec} layout {order}", flush=True)
        g = build_gpu(sc, hl, prec, order=order)
        g.commit()
        g.set_schedule(256, sched)
        g.step(5)
        full = prec == "f64"
        err = errors(g, o, 0, with_f=full, with_wss=full)
        g.close()
        print(f"branching artery full size {prec}: {err}", flush=True)
        if full:
            assert max(err.values()) <= bound, err
        else:
            assert err["e_u"] < bound and err["e_iolet_u"] < bound, err


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
    for prec in ("f64", "f32", "f16", "f16w", "f16sr"):
        ctx = build_gpu(sc, hl, prec)
        ctx.step(n0)
        err = womersley_error(ctx, wl)
        res[prec] = (err, ctx.velocity(0), ctx.density(0))
        ctx.close()
        print(f"womersley alpha={alpha} {prec}: max relative L2 vs analytic over the 5th period {err:.4f}",
              flush=True)
    assert res["f64"][0] < 0.03
    u64 = res["f64"][1]
    for prec, bound in (("f32", 1e-4), ("f16", 2e-2), ("f16w", 2e-2), ("f16sr", 2e-2)):
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


def _areas(geo):
    codes = geo.nbr[1:]
    return np.array([int(np.count_nonzero((codes == -2 - k).any(axis=0))) for k in range(len(geo.iolets))])


@pytest.mark.parametrize("order", [2, 16 | 8])
def test_coupled_13_to_1(hl, oracle_mod, order):
    """13 venous inlets per arterial outlet (the ratio of the leg vasculature,
    Sec. 3): a depth-2 arterial tree (4 outlets) coupled through the greedy
    map and Eq. (2) to 52 venous tubes.  The veins are placed, for the map,
    in a cluster around each outlet, so the greedy map gives every outlet 13.
    FP64 matches the oracle in both domains; at steady state each artery's
    outflow reappears in its veins."""
    from paper_2010_04144_amd import coupling
    art = synth.tree_geometry(2, 8.0, 20100414 + 13, lam=6.0)
    ven = synth.tubes(52, radius=3.0, length=16)
    rng = np.random.default_rng(20100414 + 14)
    aa, av = _areas(art), _areas(ven)
    outlets = list(range(1, 5))
    inlets = list(range(52))
    oc = np.array([art.iolets[k].centre for k in outlets])
    sep = min(np.linalg.norm(oc[i] - oc[j]) for i in range(4) for j in range(i + 1, 4))
    dirs = rng.normal(size=(52, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    pos = [oc[j % 4] + dirs[j] * sep * (0.05 + 0.3 * j / 52) for j in inlets]
    pairs = coupling.build_pairs(0, outlets, oc, aa[1:5], 1, inlets, pos, av[:52], rng.uniform(0.3, 0.7, 52))
    counts = [sum(1 for p in pairs if p[1] == i) for i in outlets]
    assert counts == [13, 13, 13, 13], counts
    sc = Scenario([Dom(art, tau=0.8, bouzidi=True, inlets={0: (0.02, (), (), 1.0)}),
                   Dom(ven, tau=0.8)], pairs=pairs, mode=0)
    o = build_oracle(sc, oracle_mod)
    o.step(300, THREADS)
    g = build_gpu(sc, hl, "f64", order=order)
    g.step(300)
    for d in (0, 1):
        err = errors(g, o, d)
        print("13:1 fp64 domain", d, err, flush=True)
        assert max(err.values()) <= 1e-12, (d, err)
    g.step(2700)
    mu_a, _ = g.iolet_stats(0)
    mu_v, _ = g.iolet_stats(1)
    for i in outlets:
        veins = [p[3] for p in pairs if p[1] == i]
        flux_a = aa[i] * mu_a[i]
        flux_v = sum(av[j] * mu_v[j] for j in veins)
        print("artery", i, "veins", len(veins), "flux", flux_a, flux_v, flush=True)
        assert abs(flux_v - flux_a) / abs(flux_a) < 0.03
