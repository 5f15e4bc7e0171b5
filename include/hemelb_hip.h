/*
 * hemelb_hip.h -- C ABI of the MI355X (gfx950) sparse D3Q19 LBGK library.
 *
 * The library advances one or more vascular domains (arterial tree, venous
 * tree, ensemble members) with the lattice Boltzmann method the paper uses
 * (McCullough et al., "Towards Blood Flow in the Virtual Human: Efficient
 * Self-Coupling of HemeLB", Sec. 2 first paragraph: D3Q19 lattice,
 * single-relaxation-time collision, velocity and pressure boundaries, rigid
 * walls, Newtonian fluid) over a sparse, indirectly addressed list of fluid
 * sites (Sec. 1: the code targets sparse vascular geometries), and couples
 * domains through averaged boundary values (Sec. 2.3 and Sec. 3, Eq. (1)-(2)).
 *
 * Conventions for every call
 *  - Return value: HL_OK (0) on success, a negative HL_E_* code on error, a
 *    positive HL_W_* code for a warning (the call still took effect).
 *    hl_last_error(ctx) describes the last failure on that context.
 *  - Ownership: every input array belongs to the caller and is copied before
 *    the call returns.  Output buffers are allocated by the caller.  Device
 *    memory belongs to the context and is released by hl_destroy.
 *  - Threads: one context per host thread; calls on one context must not
 *    overlap.
 *  - Streams: all device work is queued on the context's stream (see
 *    hl_set_stream).  hl_step returns before the work finishes; every read
 *    waits for it.
 *  - Sites: a domain's sites are numbered 0..n-1 by the caller ("caller
 *    order"); every read returns values in that order.  The library keeps its
 *    own internal order (bulk sites first, then boundary sites grouped by
 *    iolet) and never exposes it.
 *  - Directions: index 0 is rest; 1..6 are +x,-x,+y,-y,+z,-z; 7..18 are the
 *    edges (+x+y,-x-y), (+x-y,-x+y), (+x+z,-x-z), (+x-z,-x+z), (+y+z,-y-z),
 *    (+y-z,-y+z).  Opposite directions are adjacent: opp(i) = i+1 for odd i.
 *  - Units are lattice units; the reference density rho0 is 1.
 */
#ifndef HEMELB_HIP_H
#define HEMELB_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes (every call that takes a context returns HL_E_INVAL when
 * the context is NULL) */
#define HL_OK 0
#define HL_E_INVAL (-1)    /* malformed argument or inconsistent input */
#define HL_E_RANGE (-2)    /* index or code out of range */
#define HL_E_STATE (-3)    /* call not allowed in the current state */
#define HL_E_NOMEM (-4)    /* device or host allocation failed */
#define HL_E_DEVICE (-5)   /* no usable gfx950 device, or a HIP call failed */
#define HL_E_DIVERGED (-6) /* a non-finite density appeared during stepping */
#define HL_W_MACH 1        /* inlet speed gives Ma = sqrt(3) U >= 0.1 */
#define HL_W_TAU 2         /* tau > 1 (outside the preferred range (1/2, 1]) */

/* storage precision of the populations, fixed at hl_create */
#define HL_F64 0        /* FP64 storage and arithmetic */
#define HL_F32_OFFSET 1 /* FP32 storage of f_i - w_i rho0, FP32 arithmetic */
#define HL_F16_OFFSET 2 /* FP16 storage of f_i - w_i rho0, FP32 arithmetic */
/* FP16 storage of (f_i - w_i rho0) / w_i, FP32 arithmetic: the offset of
 * every direction is held at the same relative precision (the plain offset
 * form spends FP16's 11-bit mantissa on values 3x to 12x smaller for the
 * face and edge directions than for the rest population) */
#define HL_F16_SCALED 3
/* FP16 storage of f_i - w_i rho0 rounded stochastically on every store (round
 * up with probability equal to the fraction of the FP16 step below the value;
 * the random bits are a hash of the lattice element and the step, so runs are
 * reproducible), FP32 arithmetic */
#define HL_F16_STOCHASTIC 4

/* wall treatment */
#define HL_WALL_SBB 0     /* halfway bounce-back */
#define HL_WALL_BOUZIDI 1 /* linear interpolated bounce-back (Bouzidi, Firdaouss & Lallemand 2001) */

/* iolet kinds */
#define HL_INLET_VEL 0
#define HL_OUTLET_P 1

/* coupling modes */
#define HL_ALTERNATE 0      /* forward on even steps, reverse on odd steps (Sec. 3) */
#define HL_BOTH_EACH_STEP 1 /* both directions every step */
/* bit, with either of the above: the reverse exchange drives each coupled
 * arterial outlet as a velocity (Ladd) boundary, parabolic over its cut plane,
 * whose site mean is the mean over its veins of mean_u(vein) / s_vel, instead
 * of setting its pressure.  The second reading of the reverse direction of
 * Sec. 3; it has no pressure feedback and grows without bound in the 1:3
 * layout within about 100 steps, so it is offered for study, not as the
 * default. */
#define HL_COUPLE_VELOCITY 2

/* step drivers */
#define HL_DRIVE_LAUNCH 0 /* plain kernel launches per step */
#define HL_DRIVE_GRAPH 1  /* replay of a captured HIP graph of several steps (default) */

/* hl_create flags: internal site order inside each class of sites (bulk
 * sites; boundary sites of one domain or one iolet).  The caller order is
 * kept by default; Morton order (bit-interleaved x, y, z) keeps spatial
 * neighbours close in memory. */
#define HL_ORDER_BULK_MORTON 1u
#define HL_ORDER_BOUNDARY_MORTON 2u
/* keep wall sites in place among the bulk sites (only iolet sites are
 * grouped); a work-group whose sites all lack boundary links takes the bulk
 * kernel, any other one the boundary kernel */
#define HL_ORDER_INTERLEAVE 4u
/* brick-local layout: sites are grouped by 16^3 bricks of the voxel grid;
 * inside a brick the bulk sites whose neighbours all share the brick (their
 * pull indices are read as int16 deltas, see hl_info.n_near), the other bulk
 * sites, the wall sites whose fluid neighbours share the brick (int16 deltas
 * too), the other wall sites, each group in lexicographic order; iolet sites
 * stay grouped per iolet.  Every group starts on a whole 64-site tile of the
 * population storage. */
#define HL_ORDER_BRICK 8u
/* in-place AA-pattern streaming: one population lattice instead of two
 * (half the population memory); even steps touch only each site's own
 * populations, odd steps gather and scatter through the pull table */
#define HL_SCHEME_AA 16u
/* with HL_ORDER_BRICK: bricks of 32^3 voxels instead of 16^3 (fewer brick faces,
 * larger groups; HL_E_INVAL without HL_ORDER_BRICK) */
#define HL_ORDER_BRICK_32 32u
/* debug: before the first upload, check the planned layout exhaustively on
 * the host against the caller's site lists (every pull index in range and on
 * a real site, equal to the caller's neighbour through the site order, int16
 * deltas decoding to the same site, every site in exactly one work-group);
 * hl_commit then fails with HL_E_RANGE or HL_E_INVAL and a message instead of
 * uploading a faulty table.  Costs host time of the order of the planning. */
#define HL_DEBUG_CHECKS 64u

/* schedule flags */
#define HL_SCHED_XCD_REMAP 1u /* hand each XCD a contiguous range of site blocks */
#define HL_SCHED_FUSED 2u     /* one launch over all work-groups in storage order, each taking the
                                 bulk or the boundary path */
#define HL_SCHED_XCD_RUNS 8u  /* with HL_SCHED_XCD_REMAP: runs of 64 consecutive site blocks go to the
                                 XCDs in turn instead of one contiguous range each */
#define HL_SCHED_PAIRS 4u     /* two adjacent sites per lane on bulk sites (vector loads and stores where
                                 the two sources are adjacent): the split schedule's bulk kernel, or,
                                 with HL_SCHED_FUSED, the bulk work-groups of the fused launch (each then
                                 takes up to twice the work-group size in sites); ignored with
                                 HL_SCHEME_AA, HL_F16_SCALED and HL_F16_STOCHASTIC */
#define HL_SCHED_XCD_BRICKS 16u /* with HL_SCHED_FUSED alone, in a brick layout: the work-groups are cut
                                 into runs of at least 64 that end only at brick boundaries, and each
                                 run goes to the XCD holding the fewest so far, so a brick's lines are
                                 fetched and written through one XCD's L2 while the XCDs sweep the
                                 site list side by side */

typedef struct hl_ctx hl_ctx;

/* Library description of a committed context. */
typedef struct {
    int64_t n_sites;        /* all domains */
    int64_t n_bulk;         /* sites with no boundary link */
    int64_t n_boundary;     /* sites with at least one wall or iolet link */
    int64_t n_iolet_sites;  /* sites bordering an iolet */
    int32_t n_domains;
    int32_t n_iolets;       /* all domains */
    int32_t n_blocks_bulk;  /* work-groups of one step over bulk sites */
    int32_t n_blocks_bnd;   /* work-groups of one step over boundary sites */
    int32_t precision;
    int32_t block_size;
    int32_t sched_flags;
    int32_t drive;
    int64_t device_bytes;   /* device memory held by the context */
    double bytes_per_site;  /* algorithmic HBM bytes per bulk site update (int32 pull indices) */
    int64_t n_near;         /* sites addressed through int16 pull deltas (18 x 2 B instead of 18 x 4 B) */
} hl_info;

/* ---- context ----------------------------------------------------------- */

/* Create a context on HIP device `device` storing populations in `precision`
 * (HL_F64, HL_F32_OFFSET, HL_F16_OFFSET, HL_F16_SCALED, HL_F16_STOCHASTIC); `flags` is 0 or a combination of
 * HL_ORDER_*, HL_SCHEME_AA and HL_DEBUG_CHECKS bits.  Errors: HL_E_INVAL (bad
 * precision or flags), HL_E_DEVICE (no such device, or not gfx950).  *out is
 * NULL on error.  Infrastructure: no passage of the paper defines it. */
int hl_create(hl_ctx **out, int device, int precision, uint64_t flags);

/* Release the context and its device memory after the work queued on its
 * stream has finished.  NULL is allowed; calling it twice on the same pointer
 * is not.  Infrastructure: no passage of the paper defines it. */
void hl_destroy(hl_ctx *ctx);

/* Message for the last failing call on ctx (valid until the next call).
 * Infrastructure (no defining passage), as is hl_status_string. */
const char *hl_last_error(const hl_ctx *ctx);

/* Static text for a status code. */
const char *hl_status_string(int code);

/* Queue all device work of ctx on `hip_stream` (a hipStream_t; NULL selects
 * the null stream).  The stream must outlive the context's use of it.  Work
 * already queued on the previous stream is waited for before the switch, so
 * nothing on the new stream overlaps it.  HL_E_DEVICE when that wait fails.
 * Infrastructure: no passage of the paper defines it. */
int hl_set_stream(hl_ctx *ctx, void *hip_stream);

/* Add an empty domain and return its id (0, 1, ... in call order).  A domain
 * is one instance of the method with its own geometry, relaxation time and
 * iolets: an arterial or a venous tree of the self-coupled pair (Sec. 2.3:
 * several instances in one simulation exchanging only boundary averages), or
 * an ensemble member.  Every domain of a context advances in the same
 * launches.  HL_E_INVAL for NULL arguments; HL_E_STATE after the first step. */
int hl_add_domain(hl_ctx *ctx, int32_t *dom_id);

/* ---- geometry ------------------------------------------------------------ */

/* Check a site list without a device (Sec. 1: the code works on sparse lists
 * of fluid sites of vascular geometries; Sec. 2.2: blocks of sites with their
 * neighbour links).  nbr is int32 [19][n] (direction-major), caller-owned and
 * only read:
 * nbr[i*n + x] is the caller index of the fluid site at x + c_i, -1 when that
 * voxel is wall, -2-k when it lies beyond the cut plane of iolet k.  Element
 * offsets are 64-bit, so 19 n may exceed 2^31 (Sec. 2.1: element counts beyond
 * 32-bit ranges).
 * Errors: HL_E_RANGE (n < 0 or n > 2^31-1, an index >= n, a code below
 * -1-n_iolet, nbr[0][x] != x); HL_E_INVAL (a fluid link without its reverse
 * link, nbr[i][x] = y but nbr[opp(i)][y] != x; a site bordering two iolets). */
int hl_validate_sites(int64_t n, const int32_t *nbr, int64_t n_iolet);

/* Load the sparse site list of domain `dom` (Sec. 1: sparse vascular
 * geometry; Sec. 2.2: blocks of sites).  coords: int32 [3][n] voxel
 * coordinates (used for inlet profiles); nbr: as in hl_validate_sites;
 * n_iolet: number of iolets the codes refer to.  Wall links may carry the
 * wall distance fraction q in (0, 1] (the wall lies at x + q c_i): n_q entries
 * (q_site[j], q_dir[j], q[j]) of links whose nbr code is -1; links without an
 * entry use q = 1/2.  Iolets must then be described with hl_set_iolet.
 * Errors: those of hl_validate_sites; HL_E_RANGE for a q entry that is not a
 * wall link or q outside (0, 1]; HL_E_STATE after the first step. */
int hl_load_sites(hl_ctx *ctx, int32_t dom, int64_t n, const int32_t *coords, const int32_t *nbr,
                  int32_t n_iolet, int64_t n_q, const int64_t *q_site, const int8_t *q_dir,
                  const float *q);

/* Optional unit normals (double [3][n_w], either orientation; copied) of wall
 * sites site[0..n_w) (caller indices), used by the wall shear stress (Sec. 1
 * names wall shear stress as the quantity 3D models add); sites without one
 * use the normalised negative sum of their wall-link directions.  HL_E_INVAL
 * for NULL arrays with n_w > 0; HL_E_RANGE for a site index outside the
 * domain; HL_E_STATE after the first step. */
int hl_set_wall_normals(hl_ctx *ctx, int32_t dom, int64_t n_w, const int64_t *site, const double *nrm);

/* ---- physics --------------------------------------------------------------- */

/* Wall treatment of the domain: HL_WALL_SBB or HL_WALL_BOUZIDI (Sec. 2:
 * rigid walls; the interpolated form is the linear one of Bouzidi et al.
 * 2001, falling back to halfway bounce-back where the second node is not
 * fluid).  Allowed at any time. */
int hl_set_wall_mode(hl_ctx *ctx, int32_t dom, int mode);

/* Relaxation time (Sec. 3.3: nu = (tau - 1/2)/3 in lattice units).  HL_E_INVAL
 * for tau <= 1/2 or non-finite; HL_W_TAU for tau > 1.  Allowed at any time. */
int hl_set_tau(hl_ctx *ctx, int32_t dom, double tau);

/* Describe iolet k of the domain: kind HL_INLET_VEL or HL_OUTLET_P, a point
 * on its cut plane, its normal (into the fluid for an inlet, out of it for an
 * outlet; normalised here) and its radius.  Defaults: inlet at rest, outlet
 * at rho0.  HL_E_RANGE for k outside the domain's iolets; HL_E_INVAL for a
 * zero normal or radius <= 0; HL_E_STATE after the first step. */
int hl_set_iolet(hl_ctx *ctx, int32_t dom, int32_t k, int kind, const double centre[3],
                 const double normal[3], double radius);

/* Inlet peak velocity U(t) = a0 + sum_{m=1..nh} a[m-1] cos(2 pi m t/T) +
 * b[m-1] sin(2 pi m t/T) at step t (nh <= 8; nh = 0 means steady), imposed
 * with a parabolic profile U(t) max(0, 1 - r^2/R^2) along the normal by
 * momentum-corrected bounce-back (Ladd 1994) (Sec. 2: velocity boundaries;
 * Sec. 3.3: velocity at the inlets).  HL_W_MACH when sqrt(3) max|U| >= 0.1
 * (Sec. 3.3 stability bound).  HL_E_INVAL for an outlet, nh outside 0..8, or
 * period <= 0 with nh > 0.  Allowed at any time. */
int hl_set_inlet_velocity(hl_ctx *ctx, int32_t dom, int32_t k, double a0, int nh, const double *a,
                          const double *b, double period);

/* Outlet density rho(t), same series form, imposed as the equilibrium at
 * rho(t) and the site's own velocity (Sec. 2: pressure boundaries; Sec. 3.3:
 * pressure at the outlets).  Errors as hl_set_inlet_velocity. */
int hl_set_outlet_density(hl_ctx *ctx, int32_t dom, int32_t k, double rho0, int nh, const double *a,
                          const double *b, double period);

/* Uniform body force F(t) = F0 cos(omega t) on the domain, applied with Guo's
 * forcing scheme (Guo, Zheng & Shi 2002, named in Sec. 3).  Allowed at any
 * time. */
int hl_set_body_force(hl_ctx *ctx, int32_t dom, const double F0[3], double omega);

/* Couple outlet `outlet` of domain dom_a (arterial) to inlet `inlet` of
 * domain dom_b (venous) (Sec. 2.3; Sec. 3, Eq. (1)-(2)).  s_vel = v_i/v_0 of
 * Eq. (2); dp_ratio = dP_i/P_0 in (0, 1).  Forward: the venous inlet's peak
 * velocity is set so that its site-mean imposed velocity equals s_vel times
 * the arterial outlet's mean velocity.  Reverse: the arterial outlet density
 * is rho0 + 3 p with p the mean over its veins of p_vein / (1 - dp_ratio)
 * (Eq. (1) solved for P_0).  One outlet may have several inlets (1:N); an
 * inlet may be coupled once.  Errors: HL_E_RANGE (ids), HL_E_INVAL (kinds,
 * dp_ratio outside (0,1), inlet already coupled), HL_E_STATE after the first
 * step. */
int hl_couple(hl_ctx *ctx, int32_t dom_a, int32_t outlet, int32_t dom_b, int32_t inlet, double s_vel,
              double dp_ratio);

/* HL_ALTERNATE (default; Sec. 3: the direction alternates at each swap) or
 * HL_BOTH_EACH_STEP, either optionally with HL_COUPLE_VELOCITY.  HL_E_INVAL
 * for other bits; HL_E_STATE after the first step. */
int hl_set_coupling_mode(hl_ctx *ctx, int mode);

/* ---- stepping ---------------------------------------------------------------- */

/* Build the device layout and the initial state (equilibrium at rho0, rest,
 * t = 0).  Implied by the first hl_step or read.  Errors: HL_E_STATE when no
 * domain holds a site; HL_E_NOMEM; HL_E_DEVICE. */
int hl_commit(hl_ctx *ctx);

/* Advance every domain by nsteps lattice updates (Sec. 2.2 times update
 * steps with initialisation and output excluded).  Asynchronous on the
 * context stream.  HL_E_INVAL for nsteps < 0; HL_E_DIVERGED when an earlier
 * step produced a non-finite density (sticky until hl_set_state or
 * hl_set_populations); HL_E_DEVICE when a launch fails, after which part of
 * the batch may already be queued and the step counter no longer matches the
 * lattice: the only calls that remain meaningful are hl_last_error and
 * hl_destroy. */
int hl_step(hl_ctx *ctx, int64_t nsteps);

/* Wait for the context stream; HL_E_DIVERGED as above.  Infrastructure (no
 * defining passage), as are hl_get_time and hl_set_drive. */
int hl_sync(hl_ctx *ctx);

/* Current step counter t. */
int hl_get_time(hl_ctx *ctx, int64_t *t);

/* Choose how hl_step drives the device: HL_DRIVE_LAUNCH or HL_DRIVE_GRAPH
 * (steps_per_graph >= 1; ignored for launches). */
int hl_set_drive(hl_ctx *ctx, int drive, int32_t steps_per_graph);

/* ---- reads (moments of the post-stream populations f(t)) ------------------- */

/* Density rho(t) per site, double [n]. */
int hl_read_density(hl_ctx *ctx, int32_t dom, double *out);
/* Velocity u(t) = (sum_i c_i f_i + F(t)/2) / rho, double [3][n]. */
int hl_read_velocity(hl_ctx *ctx, int32_t dom, double *out);
/* Wall shear stress, double [n], 0 at sites without a wall link:
 * |t - (t.n) n| with traction t = sigma n and the viscous stress
 * sigma = -(1 - 1/(2 tau)) sum_i (f_i - feq_i) c_i c_i at the site
 * (Sec. 1 names wall shear stress as an output of 3D models). */
int hl_read_wss(hl_ctx *ctx, int32_t dom, double *out);
/* Populations f_i(t), double [19][n] (full values, not offsets). */
int hl_read_populations(hl_ctx *ctx, int32_t dom, double *out);
/* Replace the domain's populations f_i(t), double [19][n]; the other domains
 * keep theirs.  The next step collides from these values. */
int hl_set_populations(hl_ctx *ctx, int32_t dom, const double *f);
/* Per-iolet means over the sites bordering each iolet at step t (Sec. 2.3:
 * only averages cross a coupled boundary): mean of u.n and the gauge
 * pressure (mean rho - rho0)/3.  Arrays of the domain's iolet count. */
int hl_read_iolet_stats(hl_ctx *ctx, int32_t dom, double *mean_u, double *mean_p);
/* Boundary value per iolet (inlet peak velocity or outlet density): which = 0
 * for the next step t -> t+1, which = 1 for the step t-1 -> t (t > 0). */
int hl_read_iolet_bc(hl_ctx *ctx, int32_t dom, int which, double *out);

/* Device variants: write into caller device memory (double, same layouts) on
 * the context stream, without a host copy. */
int hl_read_density_device(hl_ctx *ctx, int32_t dom, void *dptr);
int hl_read_velocity_device(hl_ctx *ctx, int32_t dom, void *dptr);
int hl_read_wss_device(hl_ctx *ctx, int32_t dom, void *dptr);

/* Allocation-free variant of the three device reads above, for callers that
 * cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  Writes the domain's density (double [n]),
 * velocity (double [3][n]) and wall shear stress (double [n]) at step t, in
 * caller order, into the caller's device buffers rho, u and wss (any of them
 * may be NULL to skip it), on the context stream, with the same values as
 * hl_read_density_device, hl_read_velocity_device and hl_read_wss_device.
 * It calls no hipMalloc, hipFree or allocating routine: the observables are
 * staged through a fixed device scratch array of the library (64 MiB on every
 * device the library runs on, held until the process ends), in passes of
 * 1,677,696 internal sites, so contexts of any size are served.  Every call on
 * one device shares that scratch: calls that overlap on one device (other
 * streams, other threads, other contexts) race and must be serialised by the
 * caller.  The context must be committed (hl_commit, or a step or read before)
 * because committing allocates.  Errors: HL_E_RANGE (domain), HL_E_STATE (not
 * committed), HL_E_DEVICE (a launch failed). */
int hl_read_observables_device_noalloc(hl_ctx *ctx, int32_t dom, void *rho, void *u, void *wss);

/* ---- checkpoints ------------------------------------------------------------ */

/* Copy the complete dynamic state (both population lattices, outlet velocity
 * history, step counter, coupling values, divergence flag) into buf.  With
 * buf == NULL only *bytes is set.  HL_E_INVAL when *bytes is too small.
 * Infrastructure (checkpoints; no defining passage), as is hl_set_state. */
int hl_get_state(hl_ctx *ctx, void *buf, size_t *bytes);
/* Restore a state taken from a context with the same geometry and
 * precision.  HL_E_INVAL on a size, layout or version mismatch. */
int hl_set_state(hl_ctx *ctx, const void *buf, size_t bytes);

/* ---- schedule ---------------------------------------------------------------- */

/* Time candidate schedules for about budget_ms and keep the fastest: work-group
 * size {64, 128, 256} x {split, fused} x {plain, contiguous XCD ranges, XCD
 * runs}, the brick-aligned XCD runs in brick layouts, and the two-sites-per-
 * lane bulk path (split and fused) where it applies.  Every candidate is timed once; the three
 * fastest are then timed five more times each and the one with the lowest
 * median is kept.  The schedule, drive and dynamic state are restored on every
 * exit, including errors, so results do not change.  Infrastructure (the
 * paper's CPU load balancing of Sec. 2.2.1 is prior art, not this): no
 * defining passage; likewise hl_get_schedule, hl_set_schedule, hl_get_info,
 * hl_time_kernels and hl_copy_bandwidth. */
int hl_autotune(hl_ctx *ctx, int budget_ms);
/* Outcome of the last hl_autotune on ctx: the number of candidates, the
 * median step time of the kept schedule and of the runner-up (ms), and the
 * spread (max - min) / median of the kept schedule's repeated timings.
 * HL_E_STATE before any hl_autotune. */
int hl_autotune_report(hl_ctx *ctx, int32_t *n_candidates, double *best_ms, double *runner_up_ms, double *spread);
int hl_get_schedule(hl_ctx *ctx, int32_t *block_size, int32_t *flags);
/* block_size in {64, 128, 256}; flags of HL_SCHED_*. */
int hl_set_schedule(hl_ctx *ctx, int32_t block_size, int32_t flags);

/* Description of the committed context. */
int hl_get_info(hl_ctx *ctx, hl_info *out);

/* Measurement: advance nsteps (1..100000) steps with plain launches and HIP
 * events recorded on the context stream around each kernel; return the mean
 * duration in milliseconds of the bulk-site kernel and of the boundary-site
 * kernel of one step (with HL_SCHED_FUSED: 0 and the fused kernel).  The
 * one-work-group finalize kernel (queued every step only when domains are
 * coupled) and the step-counter update after the steps are not included.  The
 * steps are real steps (t advances). */
int hl_time_kernels(hl_ctx *ctx, int64_t nsteps, double *ms_bulk, double *ms_bnd);

/* ---- coupling construction (host only, no context or device) ------------- */

/* The distance-based map of Sec. 3: arterial outlets in index order each take
 * the nearest venous inlet not yet taken (ties: lowest inlet index), so every
 * outlet gets one when there are at least as many inlets; every inlet left
 * then joins its nearest outlet (ties: lowest outlet index).  out_c: double
 * [3][n_out] and in_c: double [3][n_in] iolet centres (caller-owned, read
 * only).  Writes owner[j] (outlet of inlet j) and dist[j] (the centre distance,
 * L_i of Eq. (1)-(2)) for j < n_in.  HL_E_INVAL for NULL arrays, n_out < 1 or
 * n_in < 0. */
int hl_coupling_map(int32_t n_out, const double *out_c, int32_t n_in, const double *in_c, int32_t *owner,
                    double *dist);

/* Eq. (2) of Sec. 3: the velocity factor v_i / v_0 of each of the nv veins of
 * one arterial outlet, from their pressure-drop factors dp[i] = dP_i / P_0,
 * distances L[i] and areas A[i] and the outlet area A0 (arrays of nv doubles,
 * caller-owned).  The factors satisfy sum_i A_i v_i = A_0 v_0 (the veins carry
 * the outlet's flow).  Writes v[0..nv).  HL_E_INVAL for nv < 1, NULL arrays or
 * a non-positive or non-finite input. */
int hl_velocity_factors(int32_t nv, const double *dp, const double *L, const double *A, double A0, double *v);

/* Measured copy ceiling (no context): copy `bytes` bytes from src to dst, two
 * device buffers of the current device that the caller owns (16-byte aligned,
 * not overlapping, bytes a positive multiple of 16), with one 16-byte element
 * per lane and non-temporal loads and stores; one untimed launch, then reps
 * (1..1000) launches timed with HIP events on `stream` (NULL: the default
 * stream).  *gbps = bytes read plus bytes written per second, in GB/s.  It is
 * the practical HBM bound the step kernels' bandwidth is compared with, next
 * to the published peak.  dst is overwritten with src.  HL_E_INVAL on a bad
 * argument, HL_E_RANGE when the copy needs more than 2^31 - 1 work-groups,
 * HL_E_DEVICE when a HIP call fails. */
int hl_copy_bandwidth(void *dst, const void *src, int64_t bytes, int32_t reps, void *stream, double *gbps);

#ifdef __cplusplus
}
#endif
#endif
