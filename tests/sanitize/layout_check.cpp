// Host-only driver of the library's layout planner (hl_layout.cpp), built
// with the address and undefined-behaviour sanitizers by
// tests/test_sanitizers.py.  It reads the site lists the test wrote, plans
// the layout in every site order and schedule the library offers, and runs
// the planner's exhaustive check on each; any out-of-bounds access or
// undefined operation in the planning code aborts the run.
//
// Input file (little-endian): int32 n_domains, then per domain int64 n,
// int32 n_iolet, int32 coords[3][n], int32 nbr[19][n], int64 n_q,
// int64 q_site[n_q], int8 q_dir[n_q], float q[n_q], and per iolet int32 kind,
// double centre[3], double normal[3], double radius.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "hemelb_hip.h"
#include "hl_host.h"

template <typename T>
static void rd(FILE *f, T *p, size_t n) {
    if (n && fread(p, sizeof(T), n, f) != n) {
        fprintf(stderr, "short read\n");
        exit(2);
    }
}

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t nd = 0;
    rd(f, &nd, 1);
    std::vector<hl::Domain> doms(nd);
    for (auto &d : doms) {
        rd(f, &d.n, 1);
        rd(f, &d.n_iolet, 1);
        d.coords.resize((size_t)3 * d.n);
        d.nbr.resize((size_t)19 * d.n);
        rd(f, d.coords.data(), d.coords.size());
        rd(f, d.nbr.data(), d.nbr.size());
        int64_t nq = 0;
        rd(f, &nq, 1);
        d.q_site.resize(nq);
        d.q_dir.resize(nq);
        d.q.resize(nq);
        rd(f, d.q_site.data(), nq);
        rd(f, d.q_dir.data(), nq);
        rd(f, d.q.data(), nq);
        d.io.resize(d.n_iolet);
        for (auto &io : d.io) {
            int32_t kind = 0;
            rd(f, &kind, 1);
            io.kind = kind;
            rd(f, io.c, 3);
            rd(f, io.nrm, 3);
            rd(f, &io.R, 1);
        }
        std::string err;
        if (hl::validate_sites(d.n, d.nbr.data(), d.n_iolet, err) != HL_OK) {
            fprintf(stderr, "validate: %s\n", err.c_str());
            return 1;
        }
    }
    fclose(f);
    // couple every outlet of domain 0 to the inlets of domain 1 when there are two
    std::vector<hl::PairH> pairs;
    if (nd == 2) {
        int kb = 0;
        for (int ka = 0; ka < doms[0].n_iolet && kb < doms[1].n_iolet; ++ka) {
            if (doms[0].io[ka].kind != hl::KIND_OUTLET) continue;
            while (kb < doms[1].n_iolet && doms[1].io[kb].kind != hl::KIND_INLET) ++kb;
            if (kb == doms[1].n_iolet) break;
            pairs.push_back({0, ka, 1, kb, 1.0, 0.5});
            doms[0].io[ka].coupled = doms[1].io[kb].coupled = true;
            ++kb;
        }
    }
    const uint64_t orders[] = {0,
                               HL_ORDER_BULK_MORTON,
                               HL_ORDER_BOUNDARY_MORTON,
                               HL_ORDER_BULK_MORTON | HL_ORDER_BOUNDARY_MORTON,
                               HL_ORDER_INTERLEAVE,
                               HL_ORDER_INTERLEAVE | HL_ORDER_BULK_MORTON,
                               HL_ORDER_BRICK,
                               HL_ORDER_BRICK | HL_ORDER_BRICK_32,
                               HL_ORDER_BRICK | HL_SCHEME_AA};
    const int scheds[] = {0,
                          HL_SCHED_FUSED,
                          HL_SCHED_XCD_REMAP,
                          HL_SCHED_XCD_REMAP | HL_SCHED_XCD_RUNS | HL_SCHED_FUSED,
                          HL_SCHED_PAIRS,
                          HL_SCHED_FUSED | HL_SCHED_XCD_BRICKS,
                          HL_SCHED_FUSED | HL_SCHED_PAIRS | HL_SCHED_XCD_REMAP | HL_SCHED_XCD_RUNS,
                          HL_SCHED_FUSED | HL_SCHED_PAIRS | HL_SCHED_XCD_BRICKS};
    int plans = 0;
    for (uint64_t o : orders) {
        hl::Layout L;
        std::string err;
        std::vector<hl::Domain> dd = doms;
        if (hl::plan_layout(dd, pairs, o, (o & HL_ORDER_BRICK) ? HL_COUPLE_VELOCITY : 0, L, err) != HL_OK) {
            fprintf(stderr, "plan_layout(order %llu): %s\n", (unsigned long long)o, err.c_str());
            return 1;
        }
        for (int s : scheds)
            for (int block : {64, 128, 256}) {
                hl::plan_schedule(L, block, s, true);
                if ((s & HL_SCHED_XCD_BRICKS) && (o & HL_ORDER_BRICK) && L.emap.empty()) {
                    fprintf(stderr, "no XCD map for order %llu\n", (unsigned long long)o);
                    return 1;
                }
                if (hl::check_layout(dd, L, block, err) != HL_OK) {
                    fprintf(stderr, "check_layout(order %llu, sched %d, block %d): %s\n", (unsigned long long)o, s,
                            block, err.c_str());
                    return 1;
                }
                ++plans;
            }
    }
    // the coupling construction on the iolet centres of the two domains
    if (nd == 2) {
        std::vector<double> oc, ic;
        for (int a = 0; a < 3; ++a)
            for (auto &io : doms[0].io) oc.push_back(io.c[a]);
        for (int a = 0; a < 3; ++a)
            for (auto &io : doms[1].io) ic.push_back(io.c[a]);
        std::vector<int32_t> owner(doms[1].n_iolet);
        std::vector<double> dist(doms[1].n_iolet);
        hl::coupling_map(doms[0].n_iolet, oc.data(), doms[1].n_iolet, ic.data(), owner.data(), dist.data());
        std::vector<double> dp(doms[1].n_iolet, 0.4), L(dist), A(doms[1].n_iolet, 2.0), v(doms[1].n_iolet);
        for (auto &x : L) x += 1.0;
        hl::velocity_factors(doms[1].n_iolet, dp.data(), L.data(), A.data(), 3.0, v.data());
    }
    printf("layout_check: %d domains, %d plans checked\n", nd, plans);
    return 0;
}
