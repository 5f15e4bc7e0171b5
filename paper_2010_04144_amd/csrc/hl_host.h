// Host-side model of a context: the caller's domains, iolets and coupling
// pairs, and the device layout planned from them (site order, pull tables,
// link data, work-group schedule).  Plain C++ with no HIP dependency, so the
// planning code (hl_layout.cpp) also builds and runs on a machine without a
// GPU, under the address and undefined-behaviour sanitizers.  Nothing here is
// part of the public C ABI.
#pragma once
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "hl_internal.h"

namespace hl {

// Fourier series a0 + sum_m a_m cos(2 pi m t / T) + b_m sin(2 pi m t / T).
struct Series {
    double a0 = 0.0;
    int nh = 0;
    double a[MAXH] = {0}, b[MAXH] = {0};
    double period = 1.0;
    double at(double t) const {
        double v = a0;
        for (int m = 1; m <= nh; ++m) {
            const double ph = 2.0 * M_PI * (double)m * t / period;
            v = v + a[m - 1] * std::cos(ph) + b[m - 1] * std::sin(ph);
        }
        return v;
    }
    double bound() const {
        double v = std::fabs(a0);
        for (int m = 0; m < nh; ++m) v += std::fabs(a[m]) + std::fabs(b[m]);
        return v;
    }
};

struct IoletH {
    int kind = KIND_INLET;
    double c[3] = {0, 0, 0}, nrm[3] = {0, 0, 1}, R = 1.0;
    Series wave;
    bool coupled = false;
};

// One vascular tree (or ensemble member) as the caller described it.
struct Domain {
    int64_t n = 0;
    std::vector<int32_t> coords, nbr;  // [3][n], [19][n]; released after the upload
    std::vector<int64_t> q_site;
    std::vector<int8_t> q_dir;
    std::vector<float> q;
    std::vector<int64_t> wn_site;
    std::vector<double> wn;
    int32_t n_iolet = 0;
    std::vector<IoletH> io;
    double tau = 1.0;
    int wall_mode = WALL_SBB;
    double F0[3] = {0, 0, 0}, omega = 0.0;
    // planned
    std::vector<int64_t> c2g;  // caller index -> internal index
    int32_t io_base = 0;       // global id of the domain's first iolet
};

struct PairH {
    int da, ka, db, kb;
    double s, delta;
};

// A contiguous internal range of one class in one domain.
struct Range {
    int64_t start, count;
    int32_t seg, tag;
    bool mixed = false;   // interleaved bulk and wall sites, split per work-group
    int64_t brick = -1;   // brick of the range in the brick layouts (-1: none, e.g. iolet groups)
};

// Everything the device needs, planned on the host.
struct Layout {
    int64_t N = 0, NB = 0, IO0 = 0, Nb = 0, Nio = 0, Npad = 0;
    int64_t n_sites = 0, n_bulk_sites = 0, n_io_sites = 0, n_near_sites = 0;
    std::vector<Range> ranges;
    std::vector<uint8_t> site_wall;  // interleaved layout: 1 where a site has a boundary link
    std::vector<int32_t> src;        // [18][N] pull table
    std::vector<int16_t> d16;        // [18][N] int16 pull deltas (empty when no site uses them)
    std::vector<float> bq;           // wall fractions of the wall links, boundary site by site, in direction order
    std::vector<uint32_t> bq_off;    // [Nb + 1] first entry of each boundary site in bq
    std::vector<double> bphi, bnrm;  // [Nb], [3][Nb]
    std::vector<IoletDev> hio;
    std::vector<PairDev> hpairs;
    std::vector<SegDev> hseg;
    // schedule
    std::vector<Entry> entries, entries2;
    std::vector<int32_t> entry_range;  // range of each entry
    int n_bulk_blocks = 0, n_bnd_blocks = 0;
    // brick-aligned XCD order (HL_SCHED_XCD_BRICKS): work-group b of the fused
    // launch takes entry emap[b], or nothing when emap[b] < 0
    std::vector<int32_t> emap;
    int bulk_chunk = 0;  // sites per bulk entry (2 x block in the fused two-sites-per-lane schedule)
};

// Checks of a caller's site list (no device needed): codes in range, every
// fluid link paired with its reverse, one iolet per site.  0 or HL_E_*.
int validate_sites(int64_t n, const int32_t *nbr, int64_t n_iolet, std::string &err);

SegDev seg_of(const Domain &d);

// Site order, pull tables, link data and iolet/pair tables of the domains.
// Sets each domain's c2g and io_base.  Returns 0, or an HL_E_* code with a
// message in err.
// couple_mode: HL_COUPLE_VELOCITY makes every coupled outlet a velocity
// (Ladd) boundary with the parabolic profile of its cut plane.
int plan_layout(std::vector<Domain> &doms, const std::vector<PairH> &pairs, uint64_t order_flags, int couple_mode,
                Layout &L, std::string &err);
// True when iolet io takes the Ladd velocity rule.
inline bool velocity_driven(const IoletH &io, int couple_mode) {
    return io.kind == KIND_INLET || (io.coupled && (couple_mode & COUPLE_VEL));
}

// Work-group entries for `block` sites per work-group under the HL_SCHED_*
// flags (and the brick-aligned XCD map when asked for), plus each iolet's
// entry span.  pair_bulk: with HL_SCHED_FUSED | HL_SCHED_PAIRS, bulk entries
// hold up to 2 x block sites (the kernel takes two adjacent sites per lane).
void plan_schedule(Layout &L, int block, int sched_flags, bool pair_bulk = false);

// Exhaustive host check of a planned layout against the caller's site lists
// (while they are still held): every internal index in range and on a real
// site, the pull table equal to the caller's neighbour table through the site
// permutation, the int16 deltas decoding to the same indices, every site in
// exactly one entry of at most `block` sites, the XCD map a permutation of the
// entries.  Returns 0 or HL_E_RANGE / HL_E_INVAL with a message in err.
int check_layout(const std::vector<Domain> &doms, const Layout &L, int block, std::string &err);

// Sec. 3 coupling construction.  Greedy map: outlets in index order each take
// the nearest free inlet (ties: lowest index), then every inlet left joins its
// nearest outlet.  centres are [3][n].  owner[j] and dist[j] per inlet.
void coupling_map(int32_t n_out, const double *out_c, int32_t n_in, const double *in_c, int32_t *owner,
                  double *dist);
// Eq. (2): v_i / v_0 for the nv veins of one outlet.
void velocity_factors(int32_t nv, const double *dp, const double *L, const double *A, double A0, double *v);

}  // namespace hl
