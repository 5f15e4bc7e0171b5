// Host planning of the device layout: internal site order, pull tables,
// link data, iolet and coupling tables, the work-group schedule, the host
// check of all of it, and the Sec. 3 coupling construction.  No HIP calls:
// the device allocation and upload live in hl_api.cpp.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>

#include "hemelb_hip.h"
#include "hl_host.h"

namespace hl {

namespace {

constexpr int CXh[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CYh[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZh[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
inline int opp_h(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// Spread the low 21 bits of v to every third bit.
inline uint64_t spread3(uint64_t v) {
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}

int failf(std::string &err, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    return code;
}

}  // namespace

int validate_sites(int64_t n, const int32_t *nbr, int64_t n_iolet, std::string &err) {
    if (n < 0 || n > INT32_MAX) return failf(err, HL_E_RANGE, "site count %lld out of range", (long long)n);
    if (n_iolet < 0 || n_iolet > (1 << 20)) return failf(err, HL_E_RANGE, "iolet count out of range");
    if (n > 0 && !nbr) return failf(err, HL_E_INVAL, "nbr is NULL");
    for (int64_t x = 0; x < n; ++x)
        if (nbr[x] != x) return failf(err, HL_E_RANGE, "nbr[0][%lld] must equal the site index", (long long)x);
    for (int i = 1; i < Q; ++i) {
        const int32_t *row = nbr + (size_t)i * n;
        const int32_t *back = nbr + (size_t)opp_h(i) * n;
        for (int64_t x = 0; x < n; ++x) {
            const int32_t v = row[x];
            if (v >= 0) {
                if (v >= n) return failf(err, HL_E_RANGE, "nbr[%d][%lld] = %d >= n", i, (long long)x, v);
                if (back[v] != x)
                    return failf(err, HL_E_INVAL, "link (%lld, %d) has no reverse link", (long long)x, i);
            } else if (v < -1 - n_iolet) {
                return failf(err, HL_E_RANGE, "nbr[%d][%lld] = %d is not a known code", i, (long long)x, v);
            }
        }
    }
    for (int64_t x = 0; x < n; ++x) {
        int32_t k = 0;
        for (int i = 1; i < Q; ++i) {
            const int32_t v = nbr[(size_t)i * n + x];
            if (v <= -2) {
                if (k != 0 && k != v)
                    return failf(err, HL_E_INVAL, "site %lld borders two iolets", (long long)x);
                k = v;
            }
        }
    }
    return HL_OK;
}

SegDev seg_of(const Domain &d) {
    SegDev s{};
    s.inv_tau = 1.0 / d.tau;
    s.guo_pref = 1.0 - 1.0 / (2.0 * d.tau);
    for (int k = 0; k < 3; ++k) s.F0[k] = d.F0[k];
    s.omega = d.omega;
    s.wall_mode = d.wall_mode;
    s.has_force = (d.F0[0] != 0.0 || d.F0[1] != 0.0 || d.F0[2] != 0.0) ? 1 : 0;
    return s;
}

int plan_layout(std::vector<Domain> &doms, const std::vector<PairH> &pairs, uint64_t order_flags, int couple_mode,
                Layout &L, std::string &err) {
    L = Layout{};
    int64_t total = 0;
    for (auto &d : doms) total += d.n;
    if (total == 0) return failf(err, HL_E_STATE, "no domain holds a site");
    if (total > INT32_MAX) return failf(err, HL_E_RANGE, "more than 2^31-1 sites in one context");
    const int D = (int)doms.size();

    // classes: -1 bulk, -2 wall only, k >= 0 iolet k
    std::vector<std::vector<int32_t>> cls(D);
    int32_t io_count = 0;
    for (int d = 0; d < D; ++d) {
        Domain &dm = doms[d];
        dm.io_base = io_count;
        io_count += dm.n_iolet;
        cls[d].assign(dm.n, -1);
        for (int64_t x = 0; x < dm.n; ++x) {
            int32_t k = -1;
            bool wall = false;
            for (int i = 1; i < Q; ++i) {
                const int32_t v = dm.nbr[(size_t)i * dm.n + x];
                if (v == -1) wall = true;
                if (v <= -2) k = -2 - v;
            }
            cls[d][x] = k >= 0 ? k : (wall ? -2 : -1);
        }
    }
    L.n_sites = total;
    for (int d = 0; d < D; ++d)
        for (auto v : cls[d]) {
            if (v == -1) ++L.n_bulk_sites;
            if (v >= 0) ++L.n_io_sites;
        }
    // internal order: bulk, wall, iolet groups; inside a group caller order or
    // Morton order of the coordinates.  Every group starts on a whole tile: a
    // work-group's wavefronts then own whole tiles, and no tile row is written
    // by two work-groups.
    int64_t pos = 0;
    auto align_tile = [&]() { pos = (pos + TILE - 1) & ~(int64_t)(TILE - 1); };
    auto place = [&](int d, int32_t key, bool morton) {
        Domain &dm = doms[d];
        align_tile();
        std::vector<int64_t> idx;
        for (int64_t x = 0; x < dm.n; ++x)
            if (cls[d][x] == key) idx.push_back(x);
        if (morton) {
            std::vector<std::pair<uint64_t, int64_t>> kv(idx.size());
            for (size_t m = 0; m < idx.size(); ++m) {
                const int64_t x = idx[m];
                const uint64_t mx = (uint64_t)(dm.coords[x] + (1 << 20));
                const uint64_t my = (uint64_t)(dm.coords[(size_t)dm.n + x] + (1 << 20));
                const uint64_t mz = (uint64_t)(dm.coords[(size_t)2 * dm.n + x] + (1 << 20));
                kv[m] = {spread3(mx) | (spread3(my) << 1) | (spread3(mz) << 2), x};
            }
            std::sort(kv.begin(), kv.end());
            for (size_t m = 0; m < idx.size(); ++m) idx[m] = kv[m].second;
        }
        for (int64_t x : idx) dm.c2g[x] = pos++;
        return (int64_t)idx.size();
    };
    const bool mb = (order_flags & HL_ORDER_BULK_MORTON) != 0;
    const bool mw = (order_flags & HL_ORDER_BOUNDARY_MORTON) != 0;
    const bool inter = (order_flags & HL_ORDER_INTERLEAVE) != 0;
    const bool brick = (order_flags & HL_ORDER_BRICK) != 0;
    if (brick) {
        // per domain: bricks (16^3, or 32^3 with HL_ORDER_BRICK_32) in
        // lexicographic brick order; inside a brick the near bulk sites, the
        // other bulk sites, then the wall sites, each in lexicographic order.
        // Bulk sites whose 18 upstream sites all lie in their own brick (and
        // are not iolet sites) form a group of their own (class 0, tagged
        // K_NEAR when their pull deltas fit in int16, checked once the order
        // is final); other bulk sites class 1; wall sites whose fluid upstream
        // sites satisfy the same condition class 2 (K_NEARWALL), other wall
        // sites class 3.
        const int bb = (order_flags & HL_ORDER_BRICK_32) ? 5 : 4;  // log2 of the brick edge
        const uint64_t bm = (1u << bb) - 1;
        int64_t brick_base = 0;  // bricks of earlier domains
        for (int d = 0; d < D; ++d) {
            Domain &dm = doms[d];
            dm.c2g.assign(dm.n, -1);
            std::vector<std::pair<uint64_t, int64_t>> kv;
            int64_t mn[3] = {INT64_MAX, INT64_MAX, INT64_MAX};
            for (int64_t x = 0; x < dm.n; ++x)
                for (int a = 0; a < 3; ++a) mn[a] = std::min<int64_t>(mn[a], dm.coords[(size_t)a * dm.n + x]);
            auto brick_of = [&](int64_t x) {
                const uint64_t px = (uint64_t)(dm.coords[x] - mn[0]);
                const uint64_t py = (uint64_t)(dm.coords[(size_t)dm.n + x] - mn[1]);
                const uint64_t pz = (uint64_t)(dm.coords[(size_t)2 * dm.n + x] - mn[2]);
                return ((pz >> bb) << 34) | ((py >> bb) << 17) | (px >> bb);
            };
            for (int64_t x = 0; x < dm.n; ++x) {
                const int32_t k = cls[d][x];
                if (k >= 0) continue;
                const uint64_t px = (uint64_t)(dm.coords[x] - mn[0]);
                const uint64_t py = (uint64_t)(dm.coords[(size_t)dm.n + x] - mn[1]);
                const uint64_t pz = (uint64_t)(dm.coords[(size_t)2 * dm.n + x] - mn[2]);
                const uint64_t bkey = brick_of(x);
                const uint64_t lkey = ((pz & bm) << (2 * bb)) | ((py & bm) << bb) | (px & bm);
                // near: every fluid upstream site in this brick and not an
                // iolet site (iolet groups sit after all bricks, far away)
                bool near = true;
                for (int j = 1; j < Q && near; ++j) {
                    const int32_t y = dm.nbr[(size_t)j * dm.n + x];
                    if (y >= 0 && (brick_of(y) != bkey || cls[d][y] >= 0)) near = false;
                }
                const uint64_t cl = (k == -1) ? (near ? 0 : 1) : (near ? 2 : 3);
                kv.push_back({(bkey << (3 * bb + 2)) | (cl << (3 * bb)) | lkey, x});
            }
            std::sort(kv.begin(), kv.end());
            size_t m = 0;
            int64_t nbricks = 0;
            uint64_t last_brick = ~0ULL;
            while (m < kv.size()) {
                const uint64_t grp = kv[m].first >> (3 * bb);  // brick and class
                const uint64_t bk = grp >> 2;
                if (bk != last_brick) {
                    last_brick = bk;
                    ++nbricks;
                }
                align_tile();
                const int64_t st = pos;
                while (m < kv.size() && (kv[m].first >> (3 * bb)) == grp) {
                    dm.c2g[kv[m].second] = pos++;
                    ++m;
                }
                static const int32_t tag_of[4] = {K_NEAR, K_BULK, K_NEARWALL, K_WALL};
                Range r{st, pos - st, d, tag_of[grp & 3]};
                r.brick = brick_base + nbricks - 1;
                L.ranges.push_back(r);
            }
            brick_base += nbricks;
        }
        L.NB = 0;
    } else if (inter) {
        // bulk and wall sites together, in one range per domain
        for (int d = 0; d < D; ++d) {
            for (auto &v : cls[d])
                if (v == -2) v = -3;  // wall, placed with the bulk sites below
            doms[d].c2g.assign(doms[d].n, -1);
        }
        for (int d = 0; d < D; ++d) {
            auto &cd = cls[d];
            std::vector<int32_t> saved = cd;
            for (auto &v : cd)
                if (v == -3) v = -1;
            align_tile();
            const int64_t st = pos;
            place(d, -1, mb);
            cd = saved;
            if (pos > st) {
                Range r{st, pos - st, d, K_BULK};
                r.mixed = true;
                L.ranges.push_back(r);
            }
        }
        L.NB = 0;
        L.site_wall.assign(pos, 0);
        for (int d = 0; d < D; ++d)
            for (int64_t x = 0; x < doms[d].n; ++x)
                if (cls[d][x] == -3) L.site_wall[doms[d].c2g[x]] = 1;
        for (int d = 0; d < D; ++d)
            for (auto &v : cls[d])
                if (v == -3) v = -2;
    } else {
        for (int d = 0; d < D; ++d) {
            doms[d].c2g.assign(doms[d].n, -1);
            align_tile();
            const int64_t st = pos;
            if (place(d, -1, mb) > 0) L.ranges.push_back({st, pos - st, d, K_BULK});
        }
        align_tile();
        L.NB = pos;
        for (int d = 0; d < D; ++d) {
            align_tile();
            const int64_t st = pos;
            if (place(d, -2, mw) > 0) L.ranges.push_back({st, pos - st, d, K_WALL});
        }
    }
    align_tile();
    L.IO0 = pos;
    std::vector<int64_t> io_lo(io_count, 0), io_n(io_count, 0);
    for (int d = 0; d < D; ++d) {
        Domain &dm = doms[d];
        for (int k = 0; k < dm.n_iolet; ++k) {
            align_tile();
            const int64_t st = pos;
            place(d, k, mw);
            io_lo[dm.io_base + k] = st;
            io_n[dm.io_base + k] = pos - st;
            if (pos > st) L.ranges.push_back({st, pos - st, d, K_IOLET | ((dm.io_base + k) << CLASS_BITS)});
        }
    }
    align_tile();
    L.N = pos;  // padded: every range starts, and N ends, on a whole tile
    L.Npad = (L.N + TILE - 1) / TILE * TILE;
    L.Nb = L.N - L.NB;
    L.Nio = L.N - L.IO0;
    const int64_t N = L.N, NB = L.NB, Nb = L.Nb;

    // pull table, wall fractions, inlet profile, wall normals
    L.src.assign((size_t)18 * N, 0);
    std::vector<float> qfull((size_t)18 * std::max<int64_t>(Nb, 1), 0.5f);  // [18][Nb], compacted below
    L.bphi.assign(std::max<int64_t>(Nb, 1), 0.0);
    L.bnrm.assign((size_t)3 * std::max<int64_t>(Nb, 1), 0.0);
    L.hio.assign(io_count, IoletDev{});
    for (int d = 0; d < D; ++d) {
        Domain &dm = doms[d];
        for (int64_t x = 0; x < dm.n; ++x) {
            const int64_t g = dm.c2g[x];
            for (int j = 1; j < Q; ++j) {
                const int32_t up = dm.nbr[(size_t)opp_h(j) * dm.n + x];
                int32_t v;
                if (up >= 0)
                    v = (int32_t)dm.c2g[up];
                else if (up == -1)
                    v = -1;
                else
                    v = -2 - (dm.io_base + (-2 - up));
                L.src[(size_t)(j - 1) * N + g] = v;
            }
        }
        for (size_t e = 0; e < dm.q.size(); ++e) {
            const int64_t g = dm.c2g[dm.q_site[e]];
            const int j = opp_h(dm.q_dir[e]);
            qfull[(size_t)(j - 1) * Nb + (g - NB)] = dm.q[e];
        }
        std::vector<double> userw;
        std::vector<char> has_user;
        if (!dm.wn_site.empty()) {
            userw.assign((size_t)3 * dm.n, 0.0);
            has_user.assign(dm.n, 0);
            const size_t nw = dm.wn_site.size();
            for (size_t e = 0; e < nw; ++e) {
                const int64_t x = dm.wn_site[e];
                has_user[x] = 1;
                for (int a = 0; a < 3; ++a) userw[(size_t)a * dm.n + x] = dm.wn[a * nw + e];
            }
        }
        for (int64_t x = 0; x < dm.n; ++x) {
            const int64_t g = dm.c2g[x];
            if (g < NB) continue;
            const int64_t b = g - NB;
            double nv[3] = {0, 0, 0};
            bool wall = false;
            for (int i = 1; i < Q; ++i)
                if (dm.nbr[(size_t)i * dm.n + x] == -1) {
                    wall = true;
                    nv[0] -= CXh[i];
                    nv[1] -= CYh[i];
                    nv[2] -= CZh[i];
                }
            if (wall) {
                if (!has_user.empty() && has_user[x])
                    for (int a = 0; a < 3; ++a) nv[a] = userw[(size_t)a * dm.n + x];
                const double nl = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
                if (nl > 0.0)
                    for (int a = 0; a < 3; ++a) L.bnrm[(size_t)a * Nb + b] = nv[a] / nl;
            }
            const int32_t k = cls[d][x];
            if (k >= 0 && velocity_driven(dm.io[k], couple_mode)) {
                const IoletH &io = dm.io[k];
                double dv[3], dn = 0.0, dd = 0.0;
                for (int a = 0; a < 3; ++a) {
                    dv[a] = (double)dm.coords[(size_t)a * dm.n + x] - io.c[a];
                    dn = dn + dv[a] * io.nrm[a];
                    dd = dd + dv[a] * dv[a];
                }
                const double r2 = dd - dn * dn;
                const double v = 1.0 - r2 / (io.R * io.R);
                L.bphi[b] = v > 0.0 ? v : 0.0;
            }
        }
        for (int k = 0; k < dm.n_iolet; ++k) {
            const int g = dm.io_base + k;
            IoletDev &io = L.hio[g];
            const IoletH &ih = dm.io[k];
            for (int a = 0; a < 3; ++a) io.nrm[a] = ih.nrm[a];
            io.area = (double)io_n[g];
            double sp = 0.0;
            for (int64_t s = io_lo[g]; s < io_lo[g] + io_n[g]; ++s) sp = sp + L.bphi[s - NB];
            io.phibar = io_n[g] ? sp / (double)io_n[g] : 0.0;
            io.a0 = ih.wave.a0;
            io.nh = ih.wave.nh;
            io.period = ih.wave.period;
            for (int m = 0; m < MAXH; ++m) {
                io.a[m] = ih.wave.a[m];
                io.b[m] = ih.wave.b[m];
            }
            io.kind = velocity_driven(ih, couple_mode) ? KIND_INLET : KIND_OUTLET;
            io.coupled = ih.coupled ? 1 : 0;
            io.seg = d;
        }
    }
    // wall fractions of the wall links only, boundary site by site
    {
        size_t nw = 0;
        for (int64_t b = 0; b < Nb; ++b)
            for (int j = 1; j < Q; ++j) nw += L.src[(size_t)(j - 1) * N + NB + b] == -1;
        if (nw > (size_t)UINT32_MAX) return failf(err, HL_E_RANGE, "%zu wall links exceed the 32-bit offsets", nw);
        L.bq.clear();
        L.bq.reserve(std::max<size_t>(nw, 1));
        L.bq_off.assign((size_t)Nb + 1, 0);
        for (int64_t b = 0; b < Nb; ++b) {
            L.bq_off[b] = (uint32_t)L.bq.size();
            for (int j = 1; j < Q; ++j)
                if (L.src[(size_t)(j - 1) * N + NB + b] == -1) L.bq.push_back(qfull[(size_t)(j - 1) * Nb + b]);
        }
        L.bq_off[Nb] = (uint32_t)L.bq.size();
        if (L.bq.empty()) L.bq.push_back(0.5f);  // one element, never read
    }
    // coupling pairs grouped by arterial outlet, call order kept
    {
        std::vector<size_t> order(pairs.size());
        for (size_t p = 0; p < order.size(); ++p) order[p] = p;
        auto outg = [&](size_t p) { return doms[pairs[p].da].io_base + pairs[p].ka; };
        std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return outg(x) < outg(y); });
        for (size_t p : order) {
            const PairH &ph = pairs[p];
            PairDev pd;
            pd.out_g = doms[ph.da].io_base + ph.ka;
            pd.in_g = doms[ph.db].io_base + ph.kb;
            pd.s = ph.s;
            pd.delta = ph.delta;
            IoletDev &o = L.hio[pd.out_g];
            if (o.pair_n == 0) o.pair_lo = (int32_t)L.hpairs.size();
            o.pair_n++;
            L.hpairs.push_back(pd);
        }
    }
    // int16 pull deltas of the K_NEAR and K_NEARWALL groups (INT16_MIN for a
    // wall link); a group with a delta beyond the int16 range falls back to
    // the int32 table (K_BULK or K_WALL).  The table is kept only when some
    // group uses it.
    bool any_near = false;
    for (const Range &g : L.ranges) any_near = any_near || g.tag == K_NEAR || g.tag == K_NEARWALL;
    if (any_near) L.d16.assign(L.src.size(), 0);
    for (Range &g : L.ranges) {
        if (g.tag != K_NEAR && g.tag != K_NEARWALL) continue;
        bool fits = true;
        for (int j = 1; j < Q && fits; ++j)
            for (int64_t s = g.start; s < g.start + g.count; ++s) {
                const int32_t v = L.src[(size_t)(j - 1) * N + s];
                const int64_t dl = (int64_t)v - s;
                if (v < -1 || (v >= 0 && (dl < -32767 || dl > 32767))) {
                    fits = false;
                    break;
                }
                L.d16[(size_t)(j - 1) * N + s] = (v == -1) ? (int16_t)INT16_MIN : (int16_t)dl;
            }
        if (fits)
            L.n_near_sites += g.count;
        else
            g.tag = (g.tag == K_NEAR) ? K_BULK : K_WALL;
    }
    if (L.n_near_sites == 0) std::vector<int16_t>().swap(L.d16);
    for (auto &d : doms) L.hseg.push_back(seg_of(d));
    return HL_OK;
}

namespace {

// Brick-aligned XCD order of the fused launch.  Work-group b runs on XCD
// b mod 8 (the dispatcher deals work-groups to the XCDs in turn), and each
// XCD has its own L2.  The entries, in storage order, are cut into runs of at
// least `run` entries that end only where a brick ends (iolet groups, which
// have no brick, are cut every `run` entries); each run goes to the XCD with
// the fewest entries so far (ties: lowest XCD), so the XCDs sweep the site
// list side by side while a brick's lines are fetched and written by one L2.
// XCD x's k-th entry then sits at position 8 k + x of the map; positions past
// the end of an XCD's share hold -1.
void plan_xcd_bricks(Layout &L, int run) {
    const int n = (int)L.entries.size();
    std::vector<std::vector<int32_t>> seq(8);
    std::vector<int64_t> load(8, 0);
    int e = 0;
    auto brick = [&](int k) { return L.ranges[L.entry_range[k]].brick; };
    while (e < n) {
        // whole bricks until the run holds at least `run` entries
        int end = e + 1;
        for (; end < n; ++end)
            if (end - e >= run && (brick(end) < 0 || brick(end) != brick(end - 1))) break;
        int x = 0;
        for (int k = 1; k < 8; ++k)
            if (load[k] < load[x]) x = k;
        for (int k = e; k < end; ++k) seq[x].push_back(k);
        load[x] += end - e;
        e = end;
    }
    size_t len = 0;
    for (auto &s : seq) len = std::max(len, s.size());
    L.emap.assign(8 * len, -1);
    for (int x = 0; x < 8; ++x)
        for (size_t k = 0; k < seq[x].size(); ++k) L.emap[8 * k + x] = seq[x][k];
}

}  // namespace

// Split the class ranges into work-group entries of at most `block` sites:
// entries for the bulk kernel first, then those for the boundary kernel.  In
// the interleaved layout a chunk of a mixed range goes to the bulk kernel
// when none of its sites has a boundary link.  The fused schedule keeps every
// entry in storage order for a single launch (n_bulk_blocks = 0).
void plan_schedule(Layout &L, int block, int sched_flags, bool pair_bulk) {
    std::vector<Entry> bulk, bnd;
    std::vector<int32_t> rbulk, rbnd;
    for (auto &io : L.hio) io.e_lo = io.e_hi = 0;
    const bool fused_pairs = pair_bulk && (sched_flags & HL_SCHED_FUSED) && (sched_flags & HL_SCHED_PAIRS);
    L.bulk_chunk = fused_pairs ? 2 * block : block;
    for (size_t r = 0; r < L.ranges.size(); ++r) {
        const Range &g = L.ranges[r];
        const int chunk = (!g.mixed && (g.tag == K_BULK || g.tag == K_NEAR)) ? L.bulk_chunk : block;
        for (int64_t off = 0; off < g.count; off += chunk) {
            Entry e;
            e.start = (int32_t)(g.start + off);
            e.count = (int32_t)std::min<int64_t>(chunk, g.count - off);
            e.seg = g.seg;
            e.tag = g.tag;
            if (g.mixed) {
                bool wall = false;
                for (int32_t k = 0; k < e.count && !wall; ++k) wall = L.site_wall[(size_t)e.start + k] != 0;
                e.tag = wall ? K_WALL : K_BULK;
            }
            const int ek = tag_class(e.tag);
            if ((ek == K_BULK || ek == K_NEAR) && !(sched_flags & HL_SCHED_FUSED)) {
                bulk.push_back(e);
                rbulk.push_back((int32_t)r);
            } else {
                bnd.push_back(e);
                rbnd.push_back((int32_t)r);
            }
        }
    }
    L.entries = bulk;
    L.entries.insert(L.entries.end(), bnd.begin(), bnd.end());
    L.entry_range = rbulk;
    L.entry_range.insert(L.entry_range.end(), rbnd.begin(), rbnd.end());
    L.entries2.clear();
    for (const Entry &e : bulk) {
        // merge consecutive bulk entries of one range class into chunks of
        // 2 x block sites (two sites per lane)
        if (!L.entries2.empty()) {
            Entry &l = L.entries2.back();
            if (l.seg == e.seg && l.tag == e.tag && l.start + l.count == e.start && l.count + e.count <= 2 * block) {
                l.count += e.count;
                continue;
            }
        }
        L.entries2.push_back(e);
    }
    L.n_bulk_blocks = (int)bulk.size();
    L.n_bnd_blocks = (int)bnd.size();
    for (int e = 0; e < (int)L.entries.size(); ++e) {
        const Entry &en = L.entries[e];
        if (tag_class(en.tag) != K_IOLET) continue;
        auto &io = L.hio[tag_iolet(en.tag)];
        if (io.e_hi == 0) io.e_lo = e;
        io.e_hi = e + 1;
    }
    L.emap.clear();
    if ((sched_flags & HL_SCHED_XCD_BRICKS) && (sched_flags & HL_SCHED_FUSED)) plan_xcd_bricks(L, 64);
}

int check_layout(const std::vector<Domain> &doms, const Layout &L, int block, std::string &err) {
    const int64_t N = L.N;
    if (L.src.size() != (size_t)18 * N) return failf(err, HL_E_INVAL, "pull table holds %zu entries", L.src.size());
    // the site permutation: caller sites onto distinct internal sites below N
    std::vector<int8_t> owner((size_t)N, 0);
    for (size_t d = 0; d < doms.size(); ++d) {
        const Domain &dm = doms[d];
        if ((int64_t)dm.c2g.size() != dm.n) return failf(err, HL_E_INVAL, "domain %zu has no site map", d);
        for (int64_t x = 0; x < dm.n; ++x) {
            const int64_t g = dm.c2g[x];
            if (g < 0 || g >= N) return failf(err, HL_E_RANGE, "site %lld of domain %zu maps to %lld", (long long)x, d, (long long)g);
            if (owner[g]) return failf(err, HL_E_INVAL, "internal site %lld holds two caller sites", (long long)g);
            owner[g] = 1;
        }
    }
    // the pull table against the caller's neighbour table
    for (size_t d = 0; d < doms.size(); ++d) {
        const Domain &dm = doms[d];
        if (dm.nbr.size() != (size_t)Q * dm.n) return failf(err, HL_E_STATE, "site list of domain %zu released", d);
        for (int64_t x = 0; x < dm.n; ++x) {
            const int64_t g = dm.c2g[x];
            for (int j = 1; j < Q; ++j) {
                const int32_t up = dm.nbr[(size_t)opp_h(j) * dm.n + x];
                const int32_t v = L.src[(size_t)(j - 1) * N + g];
                const int32_t want = up >= 0 ? (int32_t)dm.c2g[up] : (up == -1 ? -1 : -2 - (dm.io_base + (-2 - up)));
                if (v != want)
                    return failf(err, HL_E_INVAL, "pull index (%d, %lld) is %d, not %d", j, (long long)g, v, want);
                if (v >= 0 && (v >= N || !owner[v]))
                    return failf(err, HL_E_RANGE, "pull index (%d, %lld) = %d is no site", j, (long long)g, v);
                if (v <= -2 && -2 - v >= (int32_t)L.hio.size())
                    return failf(err, HL_E_RANGE, "pull index (%d, %lld) names iolet %d", j, (long long)g, -2 - v);
            }
        }
    }
    // wall fractions: one per wall link of each boundary site, the caller's q
    // (or 1/2 where none was given) at the link's rank among the site's walls
    if (L.bq_off.size() != (size_t)L.Nb + 1 || L.bq.empty() || L.bq_off[0] != 0)
        return failf(err, HL_E_INVAL, "wall-fraction offsets hold %zu entries for %lld boundary sites", L.bq_off.size(),
                     (long long)L.Nb);
    for (int64_t b = 0; b < L.Nb; ++b) {
        int64_t nwall = 0;
        for (int j = 1; j < Q; ++j) nwall += L.src[(size_t)(j - 1) * N + L.NB + b] == -1;
        if ((int64_t)L.bq_off[b + 1] - (int64_t)L.bq_off[b] != nwall)
            return failf(err, HL_E_INVAL, "boundary site %lld has %lld wall links but %lld fractions", (long long)b,
                         (long long)nwall, (long long)L.bq_off[b + 1] - (long long)L.bq_off[b]);
    }
    if ((size_t)L.bq_off[L.Nb] > L.bq.size()) return failf(err, HL_E_RANGE, "wall-fraction list too short");
    for (int j = 1; j < Q; ++j)  // the kernels read a site's fractions only at or above NB
        for (int64_t s = 0; s < L.NB; ++s)
            if (L.src[(size_t)(j - 1) * N + s] == -1)
                return failf(err, HL_E_INVAL, "site %lld below the boundary region has a wall link", (long long)s);
    for (size_t d = 0; d < doms.size(); ++d) {
        const Domain &dm = doms[d];
        std::vector<float> given((size_t)18 * dm.n, -1.0f);
        for (size_t e = 0; e < dm.q.size(); ++e) given[(size_t)(opp_h(dm.q_dir[e]) - 1) * dm.n + dm.q_site[e]] = dm.q[e];
        for (int64_t x = 0; x < dm.n; ++x) {
            const int64_t g = dm.c2g[x];
            if (g < L.NB) continue;
            uint32_t k = L.bq_off[g - L.NB];
            for (int j = 1; j < Q; ++j) {
                if (L.src[(size_t)(j - 1) * N + g] != -1) continue;
                const float want = given[(size_t)(j - 1) * dm.n + x] >= 0.0f ? given[(size_t)(j - 1) * dm.n + x] : 0.5f;
                if (L.bq[k] != want)
                    return failf(err, HL_E_INVAL, "wall fraction (%d, %lld) of domain %zu is %g, not %g", j,
                                 (long long)x, d, (double)L.bq[k], (double)want);
                ++k;
            }
        }
    }
    // padding slots hold no link
    for (int j = 1; j < Q; ++j)
        for (int64_t s = 0; s < N; ++s)
            if (!owner[s] && L.src[(size_t)(j - 1) * N + s] != 0)
                return failf(err, HL_E_INVAL, "padding site %lld has a pull index", (long long)s);
    // entries: every real site in exactly one entry, classes consistent
    std::vector<int8_t> seen((size_t)N, 0);
    for (size_t e = 0; e < L.entries.size(); ++e) {
        const Entry &en = L.entries[e];
        const int k = tag_class(en.tag);
        const int most = (k == K_BULK || k == K_NEAR) ? std::max(block, L.bulk_chunk) : block;
        if (en.count < 1 || en.count > most || en.start < 0 || (int64_t)en.start + en.count > N)
            return failf(err, HL_E_RANGE, "entry %zu covers [%d, %d)", e, en.start, en.start + en.count);
        if (most > block && (en.start & 1))
            return failf(err, HL_E_INVAL, "two-sites-per-lane entry %zu starts on an odd site", e);
        for (int32_t s = en.start; s < en.start + en.count; ++s) {
            if (seen[s]) return failf(err, HL_E_INVAL, "site %d is in two entries", s);
            seen[s] = 1;
            bool bnd = false;
            for (int j = 1; j < Q; ++j) bnd = bnd || L.src[(size_t)(j - 1) * N + s] < 0;
            if (owner[s] && (k == K_BULK || k == K_NEAR) && bnd)
                return failf(err, HL_E_INVAL, "boundary site %d in a bulk entry", s);
            if ((k == K_NEAR || k == K_NEARWALL) && owner[s]) {
                if (L.d16.size() != L.src.size()) return failf(err, HL_E_INVAL, "int16 entry without its table");
                for (int j = 1; j < Q; ++j) {
                    const int16_t dl = L.d16[(size_t)(j - 1) * N + s];
                    const int32_t v = L.src[(size_t)(j - 1) * N + s];
                    const int32_t dec = dl == INT16_MIN ? -1 : s + dl;
                    if (dec != v) return failf(err, HL_E_INVAL, "int16 delta (%d, %d) decodes to %d, not %d", j, s, dec, v);
                }
            }
            if (k == K_IOLET && owner[s]) {
                bool hit = false;
                for (int j = 1; j < Q; ++j) hit = hit || L.src[(size_t)(j - 1) * N + s] == -2 - tag_iolet(en.tag);
                if (!hit) return failf(err, HL_E_INVAL, "site %d does not border the iolet of its entry", s);
            }
        }
    }
    for (int64_t s = 0; s < N; ++s)
        if (owner[s] && !seen[s]) return failf(err, HL_E_INVAL, "site %lld is in no entry", (long long)s);
    // the XCD map: every entry exactly once
    if (!L.emap.empty()) {
        std::vector<int8_t> hit(L.entries.size(), 0);
        for (int32_t e : L.emap) {
            if (e < -1 || e >= (int32_t)L.entries.size()) return failf(err, HL_E_RANGE, "XCD map names entry %d", e);
            if (e < 0) continue;
            if (hit[e]) return failf(err, HL_E_INVAL, "XCD map names entry %d twice", e);
            hit[e] = 1;
        }
        for (size_t e = 0; e < hit.size(); ++e)
            if (!hit[e]) return failf(err, HL_E_INVAL, "XCD map misses entry %zu", e);
    }
    return HL_OK;
}

void coupling_map(int32_t n_out, const double *out_c, int32_t n_in, const double *in_c, int32_t *owner,
                  double *dist) {
    auto d2 = [&](int32_t i, int32_t j) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double v = out_c[(size_t)a * n_out + i] - in_c[(size_t)a * n_in + j];
            s += v * v;
        }
        return std::sqrt(s);
    };
    std::vector<char> taken(n_in, 0);
    for (int32_t j = 0; j < n_in; ++j) owner[j] = -1;
    int32_t left = n_in;
    for (int32_t i = 0; i < n_out && left > 0; ++i) {
        int32_t best = -1;
        double bd = 0.0;
        for (int32_t j = 0; j < n_in; ++j) {
            if (taken[j]) continue;
            const double v = d2(i, j);
            if (best < 0 || v < bd) {
                best = j;
                bd = v;
            }
        }
        taken[best] = 1;
        owner[best] = i;
        --left;
    }
    for (int32_t j = 0; j < n_in; ++j) {
        if (owner[j] >= 0) continue;
        int32_t best = 0;
        double bd = d2(0, j);
        for (int32_t i = 1; i < n_out; ++i) {
            const double v = d2(i, j);
            if (v < bd) {
                best = i;
                bd = v;
            }
        }
        owner[j] = best;
    }
    for (int32_t j = 0; j < n_in; ++j) dist[j] = d2(owner[j], j);
}

void velocity_factors(int32_t nv, const double *dp, const double *L, const double *A, double A0, double *v) {
    // Eq. (1) with a resistance per unit length proportional to 1/A_i gives
    // a flow share q_i proportional to dp_i A_i / L_i; the shares add up to
    // the outlet's flow (A0 v0), so v_i / v0 = (A0 / A_i) r_i / sum_k r_k with
    // r_i = dp_i A_i / L_i, here written as ratios to the first vein
    std::vector<double> r(nv);
    double sum = 0.0;
    for (int32_t i = 0; i < nv; ++i) {
        r[i] = (dp[i] / dp[0]) * (A[i] / A[0]) * (L[0] / L[i]);
        sum += r[i];
    }
    for (int32_t i = 0; i < nv; ++i) v[i] = (A0 / A[i]) * (r[i] / sum);
}

}  // namespace hl
