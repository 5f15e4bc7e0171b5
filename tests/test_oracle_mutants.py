"""Mutation check of the oracle pins.

Each mutant plants one plausible slip (a swapped branch operand, a dropped
factor, a wrong sign or index) in a copy of the oracle's C source, builds it
on the CPU in a temporary folder, and runs the pins named beside it against
that copy in a child process (ORACLE_LIB_OVERRIDE): every named pin must
fail.  The unmodified source, built the same way, passes them all.  This is
what shows that the pins fix the oracle rather than restate it.
"""
import os
import re
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbgk_oracle.c")
PINS = "tests/test_oracle_pins.py"

# (name, text in the oracle source, replacement, pins that must fail)
MUTANTS = [
    ("bouzidi far branch: own populations swapped",
     "v = fsi / (2.0 * q) + (1.0 - 1.0 / (2.0 * q)) * d->fs[(size_t)ib * n + x];",
     "v = d->fs[(size_t)ib * n + x] / (2.0 * q) + (1.0 - 1.0 / (2.0 * q)) * fsi;",
     ["test_bouzidi_at_half_is_bounce_back", "test_bouzidi_far_wall_second_order"]),
    ("bouzidi near branch: weights swapped",
     "if (back >= 0) v = 2.0 * q * fsi + (1.0 - 2.0 * q) * d->fs[(size_t)i * n + back];",
     "if (back >= 0) v = (1.0 - 2.0 * q) * fsi + 2.0 * q * d->fs[(size_t)i * n + back];",
     ["test_bouzidi_second_order_vs_bounce_back_first_order"]),
    ("bouzidi near branch: wrong fallback without a second node",
     "if (back >= 0) v = 2.0 * q * fsi + (1.0 - 2.0 * q) * d->fs[(size_t)i * n + back];",
     "if (back >= 0) v = 2.0 * q * fsi + (1.0 - 2.0 * q) * d->fs[(size_t)i * n + back];"
     " else v = d->fs[(size_t)ib * n + x];",
     ["test_bouzidi_without_second_node_is_bounce_back"]),
    ("series: 2 pi dropped",
     "double ph = 2.0 * M_PI * (double)m * t / s->period;",
     "double ph = (double)m * t / s->period;",
     ["test_waveform_series_period_mean_and_harmonics"]),
    ("series: harmonic number dropped",
     "double ph = 2.0 * M_PI * (double)m * t / s->period;",
     "double ph = 2.0 * M_PI * t / s->period;",
     ["test_waveform_series_period_mean_and_harmonics"]),
    ("series: cosine and sine coefficients swapped",
     "v = v + s->a[m - 1] * cos(ph) + s->b[m - 1] * sin(ph);",
     "v = v + s->a[m - 1] * sin(ph) + s->b[m - 1] * cos(ph);",
     ["test_waveform_series_period_mean_and_harmonics"]),
    ("equilibrium: second-order coefficient",
     "feq[i] = W[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);",
     "feq[i] = W[i] * rho * (1.0 + 3.0 * cu + 4.0 * cu * cu - 1.5 * uu);",
     ["test_feq_moments", "test_sparse_addressing_matches_dense_bruteforce"]),
    ("Guo source: sign of u",
     "s = s + (3.0 * (C[i][a] - u[a]) + 9.0 * cu * C[i][a]) * F[a];",
     "s = s + (3.0 * (C[i][a] + u[a]) + 9.0 * cu * C[i][a]) * F[a];",
     ["test_collision_conserves_and_relaxes", "test_sparse_addressing_matches_dense_bruteforce"]),
    ("moments: half-force shift dropped",
     "for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * F[a]) / r;",
     "for (int a = 0; a < 3; ++a) u[a] = j[a] / r;",
     ["test_sparse_addressing_matches_dense_bruteforce", "test_plane_poiseuille_exact_at_magic_tau"]),
    ("streaming: pushed into the opposite direction",
     "d->fn[(size_t)i * n + y] = fsi;",
     "d->fn[(size_t)ib * n + y] = fsi;",
     ["test_sparse_addressing_matches_dense_bruteforce"]),
    ("inlet: sign of the Ladd term",
     "d->fn[(size_t)ib * n + x] = fsi - 6.0 * W[i] * RHO0 * cu;",
     "d->fn[(size_t)ib * n + x] = fsi + 6.0 * W[i] * RHO0 * cu;",
     ["test_open_domain_mass_budget", "test_hagen_poiseuille_cylinder",
      "test_plug_flow_is_a_fixed_point_of_the_open_boundaries"]),
    ("inlet: profile divided by R instead of R^2",
     "double v = 1.0 - r2 / (io->R * io->R);",
     "double v = 1.0 - r2 / io->R;",
     ["test_open_domain_mass_budget"]),
    ("outlet: equilibrium of the wrong direction",
     "d->fn[(size_t)ib * n + x] = feq[ib];",
     "d->fn[(size_t)ib * n + x] = feq[i];",
     ["test_open_domain_mass_budget", "test_plug_flow_is_a_fixed_point_of_the_open_boundaries"]),
    ("iolet mean pressure: the density summed instead of its deviation",
     "sr[k] = sr[k] + (d->rho[x] - RHO0);",
     "sr[k] = sr[k] + d->rho[x];",
     ["test_iolet_means_are_site_averages"]),
    ("iolet mean density: wrong count",
     "io->mean_drho = cnt[k] ? sr[k] / (double)cnt[k] : 0.0;",
     "io->mean_drho = cnt[k] ? sr[k] / (double)(cnt[k] + 1) : 0.0;",
     ["test_iolet_means_are_site_averages"]),
    ("wall shear stress: viscous prefactor",
     "double pref = -(1.0 - 1.0 / (2.0 * d->tau));",
     "double pref = -(1.0 - 1.0 / d->tau);",
     ["test_wall_shear_stress_plane_poiseuille"]),
    ("Eq. (2): distance ratio inverted",
     "double ratio = (dp[i] * L[0] * A[i]) / (dp[0] * L[i] * A[0]);",
     "double ratio = (dp[i] * L[i] * A[i]) / (dp[0] * L[0] * A[0]);",
     ["test_velocity_factors_conserve_mass", "test_velocity_factors_paper_example"]),
    ("coupling reverse rule: Eq. (1) solved with the wrong sign",
     "sum = sum + pv / (1.0 - o->delta);",
     "sum = sum + pv / (1.0 + o->delta);",
     ["test_coupled_1to3_reaches_eq2_ratios", "test_reverse_rule_sets_the_pressure_drop"]),
    ("coupling reverse rule: venous pressures summed, not averaged",
     "out->held = RHO0 + 3.0 * (sum / (double)cnt);",
     "out->held = RHO0 + 3.0 * sum;",
     ["test_coupled_1to3_reaches_eq2_ratios"]),
    ("coupling reverse rule: pressure not converted to density",
     "out->held = RHO0 + 3.0 * (sum / (double)cnt);",
     "out->held = RHO0 + (sum / (double)cnt);",
     ["test_coupled_1to3_reaches_eq2_ratios", "test_reverse_rule_sets_the_pressure_drop"]),
    ("coupling forward rule: velocity factor dropped",
     "in->held = in->phibar > 0.0 ? pr->s * s->d[pr->da].io[pr->ka].mean_u / in->phibar : 0.0;",
     "in->held = in->phibar > 0.0 ? s->d[pr->da].io[pr->ka].mean_u / in->phibar : 0.0;",
     ["test_coupled_1to3_reaches_eq2_ratios"]),
    ("coupling forward rule: mean velocity used as the profile peak",
     "in->held = in->phibar > 0.0 ? pr->s * s->d[pr->da].io[pr->ka].mean_u / in->phibar : 0.0;",
     "in->held = in->phibar > 0.0 ? pr->s * s->d[pr->da].io[pr->ka].mean_u : 0.0;",
     ["test_coupled_1to3_reaches_eq2_ratios"]),
    ("coupling: both directions exchanged on the same step parity",
     "int rev = (s->mode & COUPLE_BOTH) || (s->t % 2 == 1);",
     "int rev = (s->mode & COUPLE_BOTH) || (s->t % 2 == 0);",
     ["test_exchange_directions_per_step"]),
    ("body force: sine for cosine",
     "double c = cos(d->omega * (double)t);",
     "double c = sin(d->omega * (double)t);",
     ["test_time_dependent_force_momentum_budget", "test_womersley_pipe"]),
    ("body force: taken one step late",
     "double c = cos(d->omega * (double)t);",
     "double c = cos(d->omega * (double)(t + 1));",
     ["test_time_dependent_force_momentum_budget"]),
    ("collision: relaxation rate tau for 1/tau",
     "fstar[i] = f[i] - (f[i] - feq[i]) / tau + pref * W[i] * s;",
     "fstar[i] = f[i] - (f[i] - feq[i]) * tau + pref * W[i] * s;",
     ["test_collision_conserves_and_relaxes"]),
    ("Guo source: prefactor 1 - 1/tau",
     "double pref = 1.0 - 1.0 / (2.0 * tau);",
     "double pref = 1.0 - 1.0 / tau;",
     ["test_collision_conserves_and_relaxes", "test_time_dependent_force_momentum_budget"]),
    ("inlet: Ladd factor halved",
     "d->fn[(size_t)ib * n + x] = fsi - 6.0 * W[i] * RHO0 * cu;",
     "d->fn[(size_t)ib * n + x] = fsi - 3.0 * W[i] * RHO0 * cu;",
     ["test_open_domain_mass_budget", "test_hagen_poiseuille_cylinder"]),
    ("inlet profile: distance along the normal kept",
     "double r2 = dd - dn * dn;",
     "double r2 = dd;",
     ["test_open_domain_mass_budget"]),
    ("outlet: equilibrium at rest instead of at the site's velocity",
     "for (int a = 0; a < 3; ++a) u[a] = d->u[(size_t)a * n + x];\n                    or_feq(io->bc, u, feq);",
     "for (int a = 0; a < 3; ++a) u[a] = 0.0;\n                    or_feq(io->bc, u, feq);",
     ["test_open_domain_mass_budget", "test_hagen_poiseuille_cylinder",
      "test_plug_flow_is_a_fixed_point_of_the_open_boundaries"]),
    ("series: evaluated one step ahead",
     "io->bc = io->coupled ? io->held : series_at(&io->wave, (double)s->t);",
     "io->bc = io->coupled ? io->held : series_at(&io->wave, (double)(s->t + 1));",
     ["test_waveform_series_period_mean_and_harmonics"]),
    ("wall shear stress: normal traction kept",
     "double sx = tr[0] - tn * nv[0], sy = tr[1] - tn * nv[1], sz = tr[2] - tn * nv[2];",
     "double sx = tr[0] + 0.0 * tn, sy = tr[1], sz = tr[2];",
     ["test_wall_shear_stress_is_the_tangential_traction"]),
    ("Eq. (2): area factor dropped",
     "v[i] = (A0 / A[i]) * ratio / sum;",
     "v[i] = ratio / sum;",
     ["test_velocity_factors_conserve_mass"]),
    ("iolet means: a site counted once per link to the iolet, not once",
     "if (!seen) ks[nk++] = k;\n        }\n        for (int m = 0; m < nk; ++m) {\n            int k = ks[m];",
     "ks[nk++] = k; (void)seen;\n        }\n        for (int m = 0; m < nk; ++m) {\n            int k = ks[m];",
     ["test_iolet_means_are_site_averages"]),
    ("iolet means: velocity taken along the opposite normal",
     "for (int a = 0; a < 3; ++a) un = un + d->u[(size_t)a * d->n + x] * d->io[k].nrm[a];",
     "for (int a = 0; a < 3; ++a) un = un - d->u[(size_t)a * d->n + x] * d->io[k].nrm[a];",
     ["test_iolet_means_are_site_averages", "test_coupled_1to3_reaches_eq2_ratios"]),
    ("moments: rest population left out of the density",
     "        r = r + f[i];\n",
     "        r = r + (i ? f[i] : 0.0);\n",
     ["test_collision_conserves_and_relaxes", "test_mass_conserved_in_closed_domains"]),
    ("streaming: rest population not collided",
     "d->fn[x] = d->fs[x]; /* rest population stays */",
     "d->fn[x] = d->f[x]; /* rest population stays */",
     ["test_mass_conserved_in_closed_domains", "test_sparse_addressing_matches_dense_bruteforce"]),
    ("bouzidi far branch: weight 1 - 1/q",
     "v = fsi / (2.0 * q) + (1.0 - 1.0 / (2.0 * q)) * d->fs[(size_t)ib * n + x];",
     "v = fsi / (2.0 * q) + (1.0 - 1.0 / q) * d->fs[(size_t)ib * n + x];",
     ["test_bouzidi_at_half_is_bounce_back", "test_bouzidi_far_wall_second_order"]),
    ("bouzidi near branch: second node's population of the opposite direction",
     "if (back >= 0) v = 2.0 * q * fsi + (1.0 - 2.0 * q) * d->fs[(size_t)i * n + back];",
     "if (back >= 0) v = 2.0 * q * fsi + (1.0 - 2.0 * q) * d->fs[(size_t)ib * n + back];",
     ["test_bouzidi_second_order_vs_bounce_back_first_order"]),
    ("inlet profile: not clamped at zero beyond the radius",
     "return v > 0.0 ? v : 0.0;",
     "return v;",
     ["test_open_domain_mass_budget"]),
    ("inlet: Ladd term at the site's density instead of rho0",
     "d->fn[(size_t)ib * n + x] = fsi - 6.0 * W[i] * RHO0 * cu;",
     "d->fn[(size_t)ib * n + x] = fsi - 6.0 * W[i] * d->rho[x] * cu;",
     ["test_open_domain_mass_budget"]),
    ("coupling forward rule: profile factor summed over the inlet, not averaged",
     "io->phibar = cnt[j] ? sp[j] / (double)cnt[j] : 0.0;",
     "io->phibar = cnt[j] ? sp[j] : 0.0;",
     ["test_coupled_1to3_reaches_eq2_ratios"]),
    ("velocity reverse: vein mean multiplied by s instead of divided",
     "sum = sum + s->d[o->db].io[o->kb].mean_u / o->s;",
     "sum = sum + s->d[o->db].io[o->kb].mean_u * o->s;",
     ["test_velocity_reverse_rule_from_outside"]),
    ("velocity reverse: mean imposed as the peak",
     "out->held = out->phibar > 0.0 ? (sum / (double)cnt) / out->phibar : 0.0;",
     "out->held = out->phibar > 0.0 ? (sum / (double)cnt) : 0.0;",
     ["test_velocity_reverse_rule_from_outside"]),
    ("velocity reverse: outlet driven along its inward normal",
     "for (int a = 0; a < 3; ++a) cu = cu + C[i][a] * (io->bc * phi * io->nrm[a]);",
     "for (int a = 0; a < 3; ++a) cu = cu + C[i][a] * (io->bc * phi * io->nrm[a])"
     " * (io->kind == KIND_OUTLET ? -1.0 : 1.0);",
     ["test_velocity_reverse_rule_from_outside"]),
]


def _build(src_text, folder, tag):
    from oracle import build as ob
    src = os.path.join(folder, f"{tag}.c")
    with open(src, "w") as fh:
        fh.write(src_text)
    return ob.build(src=src, out=os.path.join(folder, f"{tag}.so"))


def _run_pins(lib, names):
    """Run the named pins against the oracle build `lib`; return the set of
    those that failed."""
    env = dict(os.environ, ORACLE_LIB_OVERRIDE=lib, OMP_NUM_THREADS="1")
    sel = " or ".join(names)
    p = subprocess.run([sys.executable, "-m", "pytest", PINS, "-q", "-rfE", "-p", "no:cacheprovider",
                        "-m", "not gpu", "-k", sel], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    failed = set(re.findall(r"^(?:FAILED|ERROR) \S+::(\w+)", p.stdout, flags=re.M))
    ran = re.search(r"(\d+) (passed|failed)", p.stdout)
    assert ran, p.stdout[-2000:] + p.stderr[-2000:]
    return failed, p


def test_every_mutant_is_caught():
    with open(SRC) as fh:
        text = fh.read()
    for name, old, new, _ in MUTANTS:
        assert text.count(old) == 1, f"mutation site not found once: {name}"
    names = sorted({t for *_, pins in MUTANTS for t in pins})
    with tempfile.TemporaryDirectory() as tmp:
        jobs = [("control", text, names)]
        for k, (name, old, new, pins) in enumerate(MUTANTS):
            jobs.append((name, text.replace(old, new), pins))

        def one(job):
            tag = f"m{jobs.index(job)}"
            lib = _build(job[1], tmp, tag)
            failed, p = _run_pins(lib, job[2])
            return job[0], job[2], failed, p

        with ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
            results = list(ex.map(one, jobs))
    problems = []
    for name, pins, failed, p in results:
        if name == "control":
            if failed:
                problems.append(f"unmodified oracle fails {sorted(failed)}")
            continue
        missed = [t for t in pins if t not in failed]
        if missed:
            problems.append(f"{name}: {missed} still pass")
    assert not problems, "\n".join(problems)
