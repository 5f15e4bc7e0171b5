// Internal layout shared by the host driver (hl_api.cpp) and the gfx950
// kernels (hl_kernels.hip).  Nothing here is part of the public C ABI.
//
// Device layout of a committed context (all domains concatenated):
//   sites      internal order: bulk sites of every domain, then wall-only
//              boundary sites per domain, then the sites bordering each
//              iolet, grouped by global iolet id.
//   lat[2]     populations, structure of arrays [19][N]; FP64 holds f_i,
//              FP32/FP16 hold the offset g_i = f_i - w_i rho0.  lat[t&1]
//              holds the post-collision state f*(t); lat[(t+1)&1] holds
//              f*(t-1), or the raw f(t) right after a (re)initialisation.
//   src        int32 [18][N] pull table: src[j-1][s] is the internal index of
//              the site at x_s - c_j, or -1 (wall link) / -2-g (iolet g).
//   bq         float, the wall fractions q of the wall links (src = -1) of
//              each boundary site b in direction order j = 1..18, starting at
//              bq_off[b] (uint32 [Nb + 1]); q of the link (s, opp(j)).
//   bphi       double [Nb] inlet profile factor max(0, 1 - r^2/R^2).
//   bnrm       double [3][Nb] unit wall normal (0 for sites without walls).
//   uprev[2]   [3][Nio] velocity of each iolet site at step t (parity t&1).
#pragma once
#include <stdint.h>

namespace hl {

constexpr int Q = 19;
// Populations are stored tile-major: tiles of TILE sites, each holding its
// 19 direction rows contiguously (element (i, s) at
// ((s / TILE) * Q + i) * TILE + s % TILE); the lattice spans Npad sites.
constexpr int TILE_SHIFT = 6;
constexpr int TILE = 1 << TILE_SHIFT;
constexpr int MAXH = 8;
constexpr double RHO0 = 1.0;

// Entry classes: bulk site (every link fluid) with int32 pull indices, wall
// or iolet boundary site, bulk site whose upstream sites all lie within 32767
// places (int16 pull deltas, K_NEAR), or wall site whose fluid upstream sites
// do (int16 deltas, INT16_MIN for a wall link, K_NEARWALL).
enum : int32_t { K_BULK = 0, K_WALL = 1, K_IOLET = 2, K_NEAR = 3, K_NEARWALL = 4 };
constexpr int CLASS_BITS = 3;
// (constexpr: usable in host code built without HIP and in device code)
constexpr int tag_class(int32_t tag) { return tag & ((1 << CLASS_BITS) - 1); }
constexpr int tag_iolet(int32_t tag) { return tag >> CLASS_BITS; }
enum : int32_t { KIND_INLET = 0, KIND_OUTLET = 1 };
enum : int32_t { WALL_SBB = 0, WALL_BOUZIDI = 1 };
// coupling mode bits: both directions every step; velocity-driven reverse
enum : int32_t { COUPLE_ALTERNATE = 0, COUPLE_BOTH = 1, COUPLE_VEL = 2 };
enum : int32_t { PREC_F64 = 0, PREC_F32 = 1, PREC_F16 = 2, PREC_F16W = 3, PREC_F16SR = 4 };

// One work-group's share of sites: a contiguous internal range inside one
// domain and one class.  tag = class | (global iolet id << CLASS_BITS).
struct Entry {
    int32_t start;
    int32_t count;
    int32_t seg;
    int32_t tag;
};

// Per-domain constants read uniformly by a work-group.
struct SegDev {
    double inv_tau;    // 1/tau
    double guo_pref;   // 1 - 1/(2 tau)
    double F0[3];      // body force amplitude
    double omega;      // body force angular frequency
    int32_t wall_mode;
    int32_t has_force;
};

struct IoletDev {
    double nrm[3];     // unit normal (into the fluid for inlets, out for outlets)
    double area;       // number of bordering sites
    double phibar;     // mean profile factor over those sites (velocity-driven iolets)
    double a0, a[MAXH], b[MAXH], period;
    int32_t nh, kind, coupled, seg;  // kind: the link rule (KIND_INLET: Ladd velocity, KIND_OUTLET: pressure)
    int32_t e_lo, e_hi;       // schedule entries covering the iolet's sites
    int32_t pair_lo, pair_n;  // coupling pairs whose arterial outlet is this iolet
};

struct PairDev {
    int32_t out_g, in_g;
    double s, delta;
};

struct Ctrl {
    int64_t t;          // step of the stored state
    int32_t direct;     // 1: lat[(t+1)&1] holds raw f(t)
    int32_t nan_flag;   // sticky non-finite density flag
};

struct KArgs {
    int64_t N, NB, IO0, Nb, Nio;
    int64_t Npad;            // N rounded up to whole tiles (lattice extent)
    void *lat0, *lat1;
    const int32_t *src;
    const int16_t *d16;      // [18][N] upstream site minus s for K_NEAR / K_NEARWALL sites
    const float *bq;
    const uint32_t *bq_off;
    const double *bphi;
    void *up0, *up1;
    const double *bnrm;
    const Entry *entries;
    int32_t e_off;           // first entry of this launch
    const SegDev *seg;
    const IoletDev *io;
    const PairDev *pairs;
    int32_t n_io, n_pairs;
    int32_t couple_mode, xcd_remap;  // xcd_remap: 0 none, 1 contiguous eighths, C > 1 runs of C entries
    const Entry *entries2;   // bulk entries of 2 x block sites (two sites per lane)
    int32_t aa;              // 1: one in-place lattice (lat0), AA-pattern sweeps
    int32_t dt;              // steps since the stored counter: a launch works on step ctrl->t + dt
    int32_t n_pairs_blocks;  // > 0: the bulk launch runs the two-sites-per-lane kernel
    int32_t pair_fused;      // 1: fused launch whose bulk entries hold up to 2 x block sites, two per lane
    int32_t io_e0, io_e1;    // entry span covering every iolet's entries (empty: io_e0 == io_e1)
    const int32_t *emap;     // brick-aligned XCD order of the fused launch: work-group b takes entry
    int32_t n_emap;          // emap[b] (nothing when < 0); n_emap work-groups (null: storage order)
    Ctrl *ctrl;
    double *partials;  // [2][n_entries]
    double *stats;     // [2][n_io]: mean u.n, mean rho - rho0
    double *bc;        // [2][n_io] boundary values by step parity
    double *held;      // [n_io] held coupled values
    double *obs;       // [5][obs_stride] rho, ux, uy, uz, wss of the sites in [obs_lo, obs_hi)
    int64_t obs_lo, obs_hi, obs_stride;
    double *fout;      // [19][N] full f(t) or null
    const double *fin; // [19][N] full f(t) to load
};

// Kernel launchers (hl_kernels.hip).  Each returns a hipError_t value.
// part: 0 = every launch of a step, 1 = the bulk-site kernel, 2 = the
// boundary-site (or fused) kernel, 3 = the finalize kernel.
// fused: one launch over all n_bnd entries (storage order), each work-group
// choosing the bulk or the boundary path from its entry class.
int launch_step(int prec, const KArgs &a, int n_bulk, int n_bnd, int block, void *stream, int part = 0,
                bool fused = false);
int launch_init(int prec, const KArgs &a, int n_entries, int block, void *stream);
// After a batch of n steps launched with dt = 0 .. n-1: advance the stored step
// counter by n (one work-item).
int launch_advance(const KArgs &a, int64_t n, void *stream);
// Iolet means and boundary values of the current step from the partial sums
// of the last step (two lattices; contexts whose steps skip the finalize).
int launch_stats(const KArgs &a, void *stream);
int launch_observe(int prec, const KArgs &a, int n_entries, int block, void *stream);
int launch_load_raw(int prec, const KArgs &a, void *stream);
int launch_fill_rest(int prec, const KArgs &a, void *stream);
// out[k] = src[c2g[k] - lo] for the caller sites k < n whose internal index
// lies in [lo, hi) (the others are left as they are).
int launch_gather_obs(const double *src, const int64_t *c2g, int64_t n, double *out, int64_t lo, int64_t hi,
                      void *stream);
// Fixed device scratch of the allocation-free observables read: a file-scope
// device array of NOALLOC_SCRATCH_DOUBLES doubles in each device's copy of the
// library.  noalloc_scratch_setup() looks up its device address once per
// device (call it with that device current; returns a hipError_t value);
// noalloc_scratch() returns the address found for a device, or null.
constexpr int64_t NOALLOC_SCRATCH_DOUBLES = (int64_t)8 << 20;  // 64 MiB
int noalloc_scratch_setup(int device);
double *noalloc_scratch(int device);
// In-place (AA-pattern) scheme: one sweep t -> t+1 (odd = t & 1), and the
// moments-only pass that computes the iolet means and boundary values of t.
int launch_aa_step(int prec, const KArgs &a, int n_bulk, int n_bnd, int block, void *stream, int part, bool fused,
                   int odd);
int launch_aa_moments(int prec, const KArgs &a, int n_entries, int block, void *stream, int odd);
int launch_aa_load_odd(int prec, const KArgs &a, int n_entries, int block, void *stream);

}  // namespace hl
