/*
 * Plain FP64 CPU oracle for the sparse D3Q19 LBGK path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library.  It shares no
 * code, header, table or constant with the GPU library.
 *
 * What it computes (McCullough et al., "Towards Blood Flow in the Virtual
 * Human: Efficient Self-Coupling of HemeLB", Sec. 2 first paragraph: D3Q19
 * lattice, single-relaxation-time collision, velocity and pressure
 * boundaries, rigid walls; Sec. 2.3 and Sec. 3: self-coupling by averaged
 * boundary values, Eq. (1)-(2), forward/reverse alternation).  The paper does
 * not print the lattice Boltzmann formulas themselves, so each step below
 * follows the textbook form named beside it:
 *
 *   1. moments of f(n):  rho = sum_i f_i,  u = (sum_i c_i f_i + F(n)/2) / rho
 *   2. iolet means over the sites bordering each inlet/outlet (sites in the
 *      caller's order): mean u.n and mean (rho - rho0), pressure c_s^2 times
 *      the latter (the deviations are summed, not the densities, so that the
 *      leading rho0 of every term does not swamp a small mean)
 *   3. boundary values for step n: waveform series at t = n, or the coupled
 *      values (forward: venous inlet peak = s mean_u(arterial outlet) / phibar,
 *      phibar = mean inlet profile factor over the inlet's sites, so that the
 *      site mean of the imposed velocity is s times the arterial mean;
 *      reverse: arterial outlet pressure = mean over its veins of
 *      p_vein / (1 - dP/P0), which is Eq. (1) solved for P0; in the
 *      velocity-reverse mode the reverse half instead sets the arterial
 *      outlet's target mean velocity to the mean over its veins of
 *      mean_u(vein) / s, imposed as a peak of that value / phibar)
 *   4. LBGK collision with Guo's forcing term (Guo, Zheng & Shi 2002, which
 *      Sec. 3 names for the explicit force):
 *        f*_i = f_i - (f_i - feq_i)/tau
 *               + (1 - 1/(2 tau)) w_i [3 (c_i - u) + 9 (c_i.u) c_i] . F
 *        feq_i = w_i rho [1 + 3 c_i.u + 4.5 (c_i.u)^2 - 1.5 u.u]
 *      (second-order equilibrium of Qian, d'Humieres & Lallemand 1992)
 *   5. push streaming: f_i(x + c_i, n+1) = f*_i(x) when x + c_i is fluid;
 *      otherwise the link (x, i) sets f_ib(x, n+1) (ib = opposite of i):
 *        wall, halfway bounce-back:   f*_i(x)
 *        wall, Bouzidi (linear, BFL 2001) with wall at x + q c_i:
 *          q <  1/2:  2q f*_i(x) + (1 - 2q) f*_i(x - c_i)
 *          q >= 1/2:  f*_i(x)/(2q) + (1 - 1/(2q)) f*_ib(x)
 *          (halfway bounce-back when x - c_i is not fluid)
 *        velocity inlet k (Ladd):  f*_i(x) - 6 w_i rho0 (c_i . u_w),
 *          u_w = U_k(n) max(0, 1 - r^2/R_k^2) n_k, r = distance of x from
 *          the iolet axis
 *        pressure outlet k:        feq_ib(rho_out_k(n), u(x, n))
 *        coupled arterial outlet in the velocity-reverse mode: the Ladd
 *          rule above with the outlet's outward normal
 *   6. swap the two arrays.
 *
 * The reverse half of the coupling in step 3 is a reading of Sec. 3 that no
 * printed number fixes; the tests pin what follows from it (flux
 * conservation, settling to the Eq. (2) ratios, and the steady pressure drop
 * of two coupled tubes scaling with 1/(1 - dP/P0) as Eq. (1) requires).
 * The velocity-reverse mode (VEL), another reading that runs away as read,
 * is pinned in the early part of a run: the outlet value it sets, recomputed
 * from the per-site moments and the geometry, and the mass budget of its
 * velocity-driven outlet.
 *
 * Sums run over directions in index order and over sites in caller order.
 * Build with -ffp-contract=off so every product and sum is rounded as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19
#define RHO0 1.0
#define MAXH 8

/* D3Q19 velocities of the site-list interface: rest, faces, edges, with
 * opposite directions adjacent (1,2), (3,4), ..., (17,18). */
static const int C[Q][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double W[Q];

static void init_weights(void) {
    W[0] = 1.0 / 3.0;
    for (int i = 1; i <= 6; ++i) W[i] = 1.0 / 18.0;
    for (int i = 7; i < Q; ++i) W[i] = 1.0 / 36.0;
}

static int opposite(int i) {
    if (i == 0) return 0;
    return (i % 2 == 1) ? i + 1 : i - 1;
}

typedef struct {
    double a0;
    int nh;
    double a[MAXH], b[MAXH];
    double period;
} series_t;

/* Boundary value of an uncoupled iolet at step t: a0 plus a truncated Fourier
 * series of period T (the pulsatile inflow of the runs of Sec. 3; the
 * coefficients are inputs).  Step 3 of the header. */
static double series_at(const series_t *s, double t) {
    double v = s->a0;
    for (int m = 1; m <= s->nh; ++m) {
        double ph = 2.0 * M_PI * (double)m * t / s->period;
        v = v + s->a[m - 1] * cos(ph) + s->b[m - 1] * sin(ph);
    }
    return v;
}

enum { KIND_INLET = 0, KIND_OUTLET = 1 };
enum { WALL_SBB = 0, WALL_BOUZIDI = 1 };
/* coupling mode bits: both directions every step; velocity-reverse */
enum { COUPLE_ALTERNATE = 0, COUPLE_BOTH = 1, COUPLE_VEL = 2 };

typedef struct {
    int kind;
    double c[3], nrm[3], R;
    series_t wave;     /* inlet peak velocity U(t) or outlet density rho(t) */
    int coupled;       /* 1 when a coupling pair drives this iolet */
    double held;       /* held coupled value (U for inlets, rho for outlets,
                          U for outlets in the velocity-reverse mode) */
    int ladd;          /* 1 when its links take the Ladd velocity rule */
    double bc;         /* value used by the current stream step */
    double phibar;     /* mean profile factor over the bordering sites */
    /* means of the current f */
    int64_t area;
    double mean_u, mean_drho;  /* iolet means of u.n and of rho - rho0 */
} iolet_t;

typedef struct {
    int64_t n;
    int32_t *coords;   /* [3][n] */
    int32_t *nbr;      /* [19][n] */
    double *q;         /* [19][n] */
    double *wn;        /* [3][n] wall normals given by the caller, or NULL */
    double *f, *fn, *fs;
    double *rho, *u;   /* [n], [3][n] moments of f at the current step */
    int n_iolet;
    iolet_t *io;
    double tau;
    int wall_mode;
    double F0[3], omega;
} domain_t;

typedef struct {
    int da, ka, db, kb;
    double s, delta;
} pair_t;

typedef struct {
    int ndom;
    domain_t *d;
    int npair;
    pair_t *pairs;
    int mode;
    int64_t t;
    int ready;
} or_sys;

/* ------------------------------------------------------------------ */
/* single-site building blocks                                          */
/* ------------------------------------------------------------------ */

void or_lattice(int *c, double *w) {
    init_weights();
    for (int i = 0; i < Q; ++i) {
        for (int a = 0; a < 3; ++a) c[3 * i + a] = C[i][a];
        w[i] = W[i];
    }
}

/* Second-order D3Q19 equilibrium (Qian, d'Humieres & Lallemand 1992) for the
 * lattice of Sec. 2, first paragraph; c_s^2 = 1/3. */
void or_feq(double rho, const double *u, double *feq) {
    init_weights();
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        double cu = C[i][0] * u[0] + C[i][1] * u[1] + C[i][2] * u[2];
        feq[i] = W[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* Moments of one site's populations: rho and u = (j + F/2)/rho, the
 * half-force shift of Guo, Zheng & Shi (2002). */
void or_moments_site(const double *f, const double *F, double *rho, double *u) {
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        r = r + f[i];
        for (int a = 0; a < 3; ++a) j[a] = j[a] + C[i][a] * f[i];
    }
    *rho = r;
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * F[a]) / r;
}

/* LBGK collision (the single relaxation time of Sec. 2) with Guo forcing
 * (named in Sec. 3) for one site.  Step 4 of the header. */
void or_collide_site(const double *f, const double *F, double tau, double *fstar) {
    init_weights();
    double rho, u[3], feq[Q];
    or_moments_site(f, F, &rho, u);
    or_feq(rho, u, feq);
    double pref = 1.0 - 1.0 / (2.0 * tau);
    for (int i = 0; i < Q; ++i) {
        double cu = C[i][0] * u[0] + C[i][1] * u[1] + C[i][2] * u[2];
        double s = 0.0;
        for (int a = 0; a < 3; ++a) s = s + (3.0 * (C[i][a] - u[a]) + 9.0 * cu * C[i][a]) * F[a];
        fstar[i] = f[i] - (f[i] - feq[i]) / tau + pref * W[i] * s;
    }
}

/* Inlet profile factor max(0, 1 - r^2/R^2), r = distance from the axis: the
 * parabolic velocity profile of a velocity iolet (Sec. 2, velocity
 * boundaries; R the iolet radius). */
static double profile(const iolet_t *io, const int32_t *coords, int64_t n, int64_t x) {
    double d[3], dn = 0.0, dd = 0.0;
    for (int a = 0; a < 3; ++a) {
        d[a] = (double)coords[a * n + x] - io->c[a];
        dn = dn + d[a] * io->nrm[a];
        dd = dd + d[a] * d[a];
    }
    double r2 = dd - dn * dn;
    double v = 1.0 - r2 / (io->R * io->R);
    return v > 0.0 ? v : 0.0;
}

/* ------------------------------------------------------------------ */
/* system                                                               */
/* ------------------------------------------------------------------ */

or_sys *or_create(int ndom) {
    init_weights();
    or_sys *s = (or_sys *)calloc(1, sizeof(or_sys));
    s->ndom = ndom;
    s->d = (domain_t *)calloc((size_t)ndom, sizeof(domain_t));
    for (int k = 0; k < ndom; ++k) s->d[k].tau = 1.0;
    return s;
}

static void free_domain(domain_t *d) {
    free(d->coords); free(d->nbr); free(d->q); free(d->wn);
    free(d->f); free(d->fn); free(d->fs); free(d->rho); free(d->u); free(d->io);
    memset(d, 0, sizeof(*d));
}

void or_destroy(or_sys *s) {
    if (!s) return;
    for (int k = 0; k < s->ndom; ++k) free_domain(&s->d[k]);
    free(s->d); free(s->pairs); free(s);
}

int or_set_sites(or_sys *s, int dom, int64_t n, const int32_t *coords, const int32_t *nbr, int n_iolet) {
    if (dom < 0 || dom >= s->ndom || n < 0) return -1;
    domain_t *d = &s->d[dom];
    double tau = d->tau;
    free_domain(d);
    d->tau = tau;
    d->n = n;
    size_t nn = (size_t)(n > 0 ? n : 1);
    d->coords = (int32_t *)malloc(3 * nn * sizeof(int32_t));
    d->nbr = (int32_t *)malloc(Q * nn * sizeof(int32_t));
    memcpy(d->coords, coords, 3 * (size_t)n * sizeof(int32_t));
    memcpy(d->nbr, nbr, Q * (size_t)n * sizeof(int32_t));
    d->q = (double *)malloc(Q * nn * sizeof(double));
    for (size_t k = 0; k < Q * (size_t)n; ++k) d->q[k] = 0.5;
    d->f = (double *)calloc(Q * nn, sizeof(double));
    d->fn = (double *)calloc(Q * nn, sizeof(double));
    d->fs = (double *)calloc(Q * nn, sizeof(double));
    d->rho = (double *)calloc(nn, sizeof(double));
    d->u = (double *)calloc(3 * nn, sizeof(double));
    d->n_iolet = n_iolet;
    d->io = (iolet_t *)calloc((size_t)(n_iolet > 0 ? n_iolet : 1), sizeof(iolet_t));
    for (int k = 0; k < n_iolet; ++k) {
        d->io[k].R = 1.0;
        d->io[k].wave.period = 1.0;
        d->io[k].nrm[2] = 1.0;
    }
    return 0;
}

int or_set_q(or_sys *s, int dom, int64_t nq, const int64_t *site, const int8_t *dir, const float *q) {
    domain_t *d = &s->d[dom];
    for (int64_t k = 0; k < nq; ++k) {
        if (site[k] < 0 || site[k] >= d->n || dir[k] < 1 || dir[k] >= Q) return -1;
        d->q[(size_t)dir[k] * d->n + site[k]] = (double)q[k];
    }
    return 0;
}

int or_set_wall_normals(or_sys *s, int dom, const double *wn) {
    domain_t *d = &s->d[dom];
    free(d->wn);
    d->wn = NULL;
    if (wn) {
        d->wn = (double *)malloc(3 * (size_t)d->n * sizeof(double));
        memcpy(d->wn, wn, 3 * (size_t)d->n * sizeof(double));
    }
    return 0;
}

int or_set_params(or_sys *s, int dom, double tau, int wall_mode) {
    s->d[dom].tau = tau;
    s->d[dom].wall_mode = wall_mode;
    return 0;
}

int or_set_force(or_sys *s, int dom, const double *F0, double omega) {
    for (int a = 0; a < 3; ++a) s->d[dom].F0[a] = F0[a];
    s->d[dom].omega = omega;
    return 0;
}

int or_set_iolet(or_sys *s, int dom, int k, int kind, const double *c, const double *nrm, double R,
                 double a0, int nh, const double *a, const double *b, double period) {
    domain_t *d = &s->d[dom];
    if (k < 0 || k >= d->n_iolet || nh < 0 || nh > MAXH) return -1;
    iolet_t *io = &d->io[k];
    io->kind = kind;
    double nn = sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
    for (int q = 0; q < 3; ++q) {
        io->c[q] = c[q];
        io->nrm[q] = nrm[q] / nn;
    }
    io->R = R;
    io->wave.a0 = a0;
    io->wave.nh = nh;
    for (int m = 0; m < nh; ++m) {
        io->wave.a[m] = a[m];
        io->wave.b[m] = b[m];
    }
    io->wave.period = period;
    return 0;
}

int or_couple(or_sys *s, int da, int ka, int db, int kb, double sv, double delta) {
    s->pairs = (pair_t *)realloc(s->pairs, (size_t)(s->npair + 1) * sizeof(pair_t));
    pair_t *p = &s->pairs[s->npair++];
    p->da = da; p->ka = ka; p->db = db; p->kb = kb; p->s = sv; p->delta = delta;
    s->d[da].io[ka].coupled = 1;
    s->d[db].io[kb].coupled = 1;
    return 0;
}

/* Coupling mode bits (COUPLE_BOTH, COUPLE_VEL); set before or_init. */
void or_set_coupling_mode(or_sys *s, int mode) { s->mode = mode; }

/* Body force of step t, F0 cos(omega t): the explicit Guo force of Sec. 3,
 * here a uniform drive (omega = 0 for a steady one). */
static void body_force(const domain_t *d, int64_t t, double *F) {
    double c = cos(d->omega * (double)t);
    for (int a = 0; a < 3; ++a) F[a] = d->F0[a] * c;
}

/* Step 1: moments of the current f at every site. */
static void moments(domain_t *d, int64_t t, int nthreads) {
    double F[3];
    body_force(d, t, F);
    (void)nthreads;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t x = 0; x < d->n; ++x) {
        double fl[Q], r, u[3];
        for (int i = 0; i < Q; ++i) fl[i] = d->f[(size_t)i * d->n + x];
        or_moments_site(fl, F, &r, u);
        d->rho[x] = r;
        for (int a = 0; a < 3; ++a) d->u[(size_t)a * d->n + x] = u[a];
    }
}

/* Step 2: means over the sites that border each iolet (Sec. 2.3: only
 * averaged values cross a coupled boundary).  One pass over the sites in
 * caller order; a site adds to every iolet it borders. */
static void iolet_means(domain_t *d) {
    double *su = (double *)calloc((size_t)(d->n_iolet + 1), sizeof(double));
    double *sr = (double *)calloc((size_t)(d->n_iolet + 1), sizeof(double));
    int64_t *cnt = (int64_t *)calloc((size_t)(d->n_iolet + 1), sizeof(int64_t));
    for (int64_t x = 0; x < d->n; ++x) {
        int ks[Q], nk = 0;
        for (int i = 1; i < Q; ++i) {
            int32_t v = d->nbr[(size_t)i * d->n + x];
            if (v > -2) continue;
            int k = -2 - v, seen = 0;
            for (int m = 0; m < nk; ++m)
                if (ks[m] == k) seen = 1;
            if (!seen) ks[nk++] = k;
        }
        for (int m = 0; m < nk; ++m) {
            int k = ks[m];
            double un = 0.0;
            for (int a = 0; a < 3; ++a) un = un + d->u[(size_t)a * d->n + x] * d->io[k].nrm[a];
            su[k] = su[k] + un;
            sr[k] = sr[k] + (d->rho[x] - RHO0);
            cnt[k] = cnt[k] + 1;
        }
    }
    for (int k = 0; k < d->n_iolet; ++k) {
        iolet_t *io = &d->io[k];
        io->area = cnt[k];
        io->mean_u = cnt[k] ? su[k] / (double)cnt[k] : 0.0;
        io->mean_drho = cnt[k] ? sr[k] / (double)cnt[k] : 0.0;
    }
    free(su); free(sr); free(cnt);
}

/* Step 3: boundary values for the stream that follows step t (Sec. 3: the
 * coupled exchange with Eq. (1)-(2), alternating direction; series values
 * for the other iolets). */
static void boundary_values(or_sys *s) {
    int fwd = (s->mode & COUPLE_BOTH) || (s->t % 2 == 0);
    int rev = (s->mode & COUPLE_BOTH) || (s->t % 2 == 1);
    if (fwd) {
        for (int p = 0; p < s->npair; ++p) {
            pair_t *pr = &s->pairs[p];
            iolet_t *in = &s->d[pr->db].io[pr->kb];
            in->held = in->phibar > 0.0 ? pr->s * s->d[pr->da].io[pr->ka].mean_u / in->phibar : 0.0;
        }
    }
    if (rev) {
        for (int p = 0; p < s->npair; ++p) {
            pair_t *pr = &s->pairs[p];
            iolet_t *out = &s->d[pr->da].io[pr->ka];
            /* each arterial outlet once, at its first pair */
            int first = 1;
            for (int q = 0; q < p; ++q)
                if (s->pairs[q].da == pr->da && s->pairs[q].ka == pr->ka) first = 0;
            if (!first) continue;
            double sum = 0.0;
            int cnt = 0;
            for (int q = 0; q < s->npair; ++q) {
                pair_t *o = &s->pairs[q];
                if (o->da != pr->da || o->ka != pr->ka) continue;
                if (s->mode & COUPLE_VEL) {
                    /* the vein carries s times the artery's mean velocity */
                    sum = sum + s->d[o->db].io[o->kb].mean_u / o->s;
                } else {
                    double pv = s->d[o->db].io[o->kb].mean_drho / 3.0;
                    sum = sum + pv / (1.0 - o->delta);
                }
                cnt = cnt + 1;
            }
            if (s->mode & COUPLE_VEL)
                out->held = out->phibar > 0.0 ? (sum / (double)cnt) / out->phibar : 0.0;
            else
                out->held = RHO0 + 3.0 * (sum / (double)cnt);
        }
    }
    for (int k = 0; k < s->ndom; ++k) {
        domain_t *d = &s->d[k];
        for (int j = 0; j < d->n_iolet; ++j) {
            iolet_t *io = &d->io[j];
            io->bc = io->coupled ? io->held : series_at(&io->wave, (double)s->t);
        }
    }
}

/* Steps 4-5 for one domain: collide into fs, push-stream into fn (the D3Q19
 * stream of Sec. 2 with rigid walls, halfway or Bouzidi-Firdaouss-Lallemand
 * 2001, Ladd velocity and equilibrium pressure links). */
static void collide_stream(domain_t *d, int64_t t, int nthreads) {
    double F[3];
    body_force(d, t, F);
    const int64_t n = d->n;
    (void)nthreads;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t x = 0; x < n; ++x) {
        double fl[Q], fo[Q];
        for (int i = 0; i < Q; ++i) fl[i] = d->f[(size_t)i * n + x];
        or_collide_site(fl, F, d->tau, fo);
        for (int i = 0; i < Q; ++i) d->fs[(size_t)i * n + x] = fo[i];
    }
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t x = 0; x < n; ++x) {
        d->fn[x] = d->fs[x]; /* rest population stays */
        for (int i = 1; i < Q; ++i) {
            int32_t y = d->nbr[(size_t)i * n + x];
            int ib = opposite(i);
            double fsi = d->fs[(size_t)i * n + x];
            if (y >= 0) {
                d->fn[(size_t)i * n + y] = fsi;
            } else if (y == -1) {
                double v = fsi;
                if (d->wall_mode == WALL_BOUZIDI) {
                    double q = d->q[(size_t)i * n + x];
                    int32_t back = d->nbr[(size_t)ib * n + x]; /* x - c_i */
                    if (q < 0.5) {
                        if (back >= 0) v = 2.0 * q * fsi + (1.0 - 2.0 * q) * d->fs[(size_t)i * n + back];
                    } else {
                        v = fsi / (2.0 * q) + (1.0 - 1.0 / (2.0 * q)) * d->fs[(size_t)ib * n + x];
                    }
                }
                d->fn[(size_t)ib * n + x] = v;
            } else {
                int k = -2 - y;
                const iolet_t *io = &d->io[k];
                if (io->ladd) {
                    double phi = profile(io, d->coords, n, x);
                    double cu = 0.0;
                    for (int a = 0; a < 3; ++a) cu = cu + C[i][a] * (io->bc * phi * io->nrm[a]);
                    d->fn[(size_t)ib * n + x] = fsi - 6.0 * W[i] * RHO0 * cu;
                } else {
                    double u[3], feq[Q];
                    for (int a = 0; a < 3; ++a) u[a] = d->u[(size_t)a * n + x];
                    or_feq(io->bc, u, feq);
                    d->fn[(size_t)ib * n + x] = feq[ib];
                }
            }
        }
    }
}

int or_init(or_sys *s) {
    init_weights();
    s->t = 0;
    for (int k = 0; k < s->ndom; ++k) {
        domain_t *d = &s->d[k];
        for (int i = 0; i < Q; ++i)
            for (int64_t x = 0; x < d->n; ++x) d->f[(size_t)i * d->n + x] = W[i] * RHO0;
        /* mean inlet profile factor over each iolet's bordering sites,
         * one pass over the sites in caller order */
        double *sp = (double *)calloc((size_t)(d->n_iolet + 1), sizeof(double));
        int64_t *cnt = (int64_t *)calloc((size_t)(d->n_iolet + 1), sizeof(int64_t));
        for (int64_t x = 0; x < d->n; ++x) {
            int ks[Q], nk = 0;
            for (int i = 1; i < Q; ++i) {
                int32_t v = d->nbr[(size_t)i * d->n + x];
                if (v > -2) continue;
                int k = -2 - v, seen = 0;
                for (int m = 0; m < nk; ++m)
                    if (ks[m] == k) seen = 1;
                if (!seen) ks[nk++] = k;
            }
            for (int m = 0; m < nk; ++m) {
                sp[ks[m]] = sp[ks[m]] + profile(&d->io[ks[m]], d->coords, d->n, x);
                cnt[ks[m]] = cnt[ks[m]] + 1;
            }
        }
        for (int j = 0; j < d->n_iolet; ++j) {
            iolet_t *io = &d->io[j];
            io->ladd = io->kind == KIND_INLET || (io->coupled && (s->mode & COUPLE_VEL));
            /* a velocity-driven outlet starts from rest */
            io->held = (io->ladd && io->kind == KIND_OUTLET) ? 0.0 : series_at(&io->wave, 0.0);
            io->phibar = cnt[j] ? sp[j] / (double)cnt[j] : 0.0;
        }
        free(sp);
        free(cnt);
    }
    s->ready = 1;
    return 0;
}

int or_set_f(or_sys *s, int dom, const double *f) {
    domain_t *d = &s->d[dom];
    memcpy(d->f, f, Q * (size_t)d->n * sizeof(double));
    return 0;
}

/* State injection for comparisons from a state another run reached: the step
 * counter (it selects the waveform phase and the forward/reverse half of the
 * exchange) and the held coupled value of iolet k (the one a step that does
 * not recompute it keeps).  Neither changes any arithmetic of the step. */
int or_set_time(or_sys *s, int64_t t) {
    if (t < 0) return -1;
    s->t = t;
    return 0;
}

int or_set_held(or_sys *s, int dom, int k, double v) {
    if (dom < 0 || dom >= s->ndom || k < 0 || k >= s->d[dom].n_iolet) return -1;
    s->d[dom].io[k].held = v;
    return 0;
}

/* nsteps lattice updates, each taking steps 1-6 of the header in order for
 * every domain (Sec. 2.2 counts these as the update steps). */
int or_step(or_sys *s, int64_t nsteps, int nthreads) {
    if (!s->ready) return -3;
    if (nthreads < 1) nthreads = 1;
    for (int64_t it = 0; it < nsteps; ++it) {
        for (int k = 0; k < s->ndom; ++k) {
            moments(&s->d[k], s->t, nthreads);
            iolet_means(&s->d[k]);
        }
        boundary_values(s);
        for (int k = 0; k < s->ndom; ++k) {
            domain_t *d = &s->d[k];
            collide_stream(d, s->t, nthreads);
            double *tmp = d->f;
            d->f = d->fn;
            d->fn = tmp;
        }
        s->t = s->t + 1;
    }
    return 0;
}

int64_t or_time(const or_sys *s) { return s->t; }

int or_read_f(or_sys *s, int dom, double *f) {
    domain_t *d = &s->d[dom];
    memcpy(f, d->f, Q * (size_t)d->n * sizeof(double));
    return 0;
}

/* Post-collision populations of the last step (valid after or_step). */
int or_read_fpost(or_sys *s, int dom, double *f) {
    domain_t *d = &s->d[dom];
    memcpy(f, d->fs, Q * (size_t)d->n * sizeof(double));
    return 0;
}

int or_read_moments(or_sys *s, int dom, double *rho, double *u) {
    domain_t *d = &s->d[dom];
    moments(d, s->t, 1);
    memcpy(rho, d->rho, (size_t)d->n * sizeof(double));
    memcpy(u, d->u, 3 * (size_t)d->n * sizeof(double));
    return 0;
}

/* Means at the current step and the boundary values that the next stream
 * will use (both recomputed from the current state). */
int or_read_iolet_stats(or_sys *s, int dom, double *mean_u, double *mean_p, int64_t *area) {
    for (int k = 0; k < s->ndom; ++k) {
        moments(&s->d[k], s->t, 1);
        iolet_means(&s->d[k]);
    }
    domain_t *d = &s->d[dom];
    for (int k = 0; k < d->n_iolet; ++k) {
        mean_u[k] = d->io[k].mean_u;
        mean_p[k] = d->io[k].mean_drho / 3.0;
        area[k] = d->io[k].area;
    }
    return 0;
}

/* Wall shear stress (the quantity Sec. 1 names as what 3D flow resolves along
 * artery walls) at every site with at least one wall link (0 elsewhere):
 * sigma = -(1 - 1/(2 tau)) sum_i (f_i - feq_i) c_i c_i, traction t = sigma n,
 * wss = |t - (t.n) n|; n is the caller's normal or the normalised
 * -sum of the wall-link directions. */
int or_read_wss(or_sys *s, int dom, double *wss) {
    domain_t *d = &s->d[dom];
    moments(d, s->t, 1);
    const int64_t n = d->n;
    for (int64_t x = 0; x < n; ++x) {
        double nv[3] = {0.0, 0.0, 0.0};
        int walls = 0;
        for (int i = 1; i < Q; ++i) {
            if (d->nbr[(size_t)i * n + x] == -1) {
                walls = 1;
                for (int a = 0; a < 3; ++a) nv[a] = nv[a] - C[i][a];
            }
        }
        wss[x] = 0.0;
        if (!walls) continue;
        if (d->wn)
            for (int a = 0; a < 3; ++a) nv[a] = d->wn[(size_t)a * n + x];
        double nl = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
        if (nl == 0.0) continue;
        for (int a = 0; a < 3; ++a) nv[a] = nv[a] / nl;
        double u[3], feq[Q];
        for (int a = 0; a < 3; ++a) u[a] = d->u[(size_t)a * n + x];
        or_feq(d->rho[x], u, feq);
        double P[3][3] = {{0}};
        for (int i = 0; i < Q; ++i) {
            double ne = d->f[(size_t)i * n + x] - feq[i];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) P[a][b] = P[a][b] + ne * C[i][a] * C[i][b];
        }
        double pref = -(1.0 - 1.0 / (2.0 * d->tau));
        double tr[3];
        for (int a = 0; a < 3; ++a) {
            tr[a] = 0.0;
            for (int b = 0; b < 3; ++b) tr[a] = tr[a] + pref * P[a][b] * nv[b];
        }
        double tn = tr[0] * nv[0] + tr[1] * nv[1] + tr[2] * nv[2];
        double sx = tr[0] - tn * nv[0], sy = tr[1] - tn * nv[1], sz = tr[2] - tn * nv[2];
        wss[x] = sqrt(sx * sx + sy * sy + sz * sz);
    }
    return 0;
}

/* Boundary values (inlet peak velocity or outlet density, per iolet) that
 * the last completed step, t-1 -> t, used. */
int or_read_bc(or_sys *s, int dom, double *bc) {
    domain_t *d = &s->d[dom];
    for (int k = 0; k < d->n_iolet; ++k) bc[k] = d->io[k].bc;
    return 0;
}

/* Eq. (2): velocity factor of each of the N veins coupled to one arterial
 * outlet, from pressure-drop factors dP_i/P0, distances L_i, areas A_i and
 * the arterial outlet area A0.  The expression is written as printed, with
 * the first vein as the reference of the ratios. */
void or_velocity_factors(int nv, const double *dp, const double *L, const double *A, double A0, double *v) {
    double sum = 0.0;
    for (int j = 0; j < nv; ++j) sum = sum + (dp[j] * L[0] * A[j]) / (dp[0] * L[j] * A[0]);
    for (int i = 0; i < nv; ++i) {
        double ratio = (dp[i] * L[0] * A[i]) / (dp[0] * L[i] * A[0]);
        v[i] = (A0 / A[i]) * ratio / sum;
    }
}
