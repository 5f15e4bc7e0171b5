// Host side of the C ABI declared in include/hemelb_hip.h: argument checks,
// the internal site order and pull table, the work-group schedule, device
// memory, the step driver (plain launches or a replayed HIP graph), reads,
// checkpoints and the schedule autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "hemelb_hip.h"
#include "hl_host.h"

using hl::Q;
using hl::Domain;
using hl::IoletH;
using hl::PairH;
using hl::Series;

struct hl_ctx {
    int device = 0, precision = 0;
    uint64_t order_flags = 0;
    bool aa = false;          // in-place AA-pattern scheme
    int64_t stats_t = -1;     // step whose iolet means / boundary values are on the device
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    std::string err;
    std::vector<Domain> doms;
    std::vector<PairH> pairs;
    int couple_mode = hl::COUPLE_ALTERNATE;
    bool committed = false;
    int block = 256;
    int sched_flags = 0;
    int drive = HL_DRIVE_GRAPH;
    int steps_per_graph = 16;
    int64_t t_host = 0;
    hl::Layout L;  // planned layout and schedule
    bool debug_checks = false;
    // last hl_autotune: candidates, median ms/step of the kept and the
    // runner-up schedule, spread of the kept one's repeats
    int32_t tune_n = 0;
    double tune_best = 0.0, tune_second = 0.0, tune_spread = 0.0;
    // device memory
    void *lat[2] = {nullptr, nullptr};
    int32_t *d_src = nullptr;
    int16_t *d_d16 = nullptr;
    int32_t *d_emap = nullptr;
    std::vector<int64_t *> d_c2g;  // per domain: caller index -> internal index (device reads)
    float *d_bq = nullptr;
    uint32_t *d_bq_off = nullptr;
    double *d_bphi = nullptr, *d_bnrm = nullptr;
    void *d_up[2] = {nullptr, nullptr};
    hl::Entry *d_entries = nullptr, *d_entries2 = nullptr;
    hl::SegDev *d_seg = nullptr;
    hl::IoletDev *d_io = nullptr;
    hl::PairDev *d_pairs = nullptr;
    hl::Ctrl *d_ctrl = nullptr;
    double *d_partials = nullptr, *d_stats = nullptr, *d_bc = nullptr, *d_held = nullptr;
    double *d_obs = nullptr, *d_fbuf = nullptr;
    int64_t dev_bytes = 0;
    int64_t obs_t = -1;
    hipGraphExec_t gexec = nullptr;
    int graph_steps = 0;
    int *h_nan = nullptr;  // pinned copy of the divergence flag
};

namespace {

int fail(hl_ctx *c, int code, const char *fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIPC(ctx, call)                                                                         \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail((ctx), e_ == hipErrorOutOfMemory ? HL_E_NOMEM : HL_E_DEVICE, "%s: %s", #call, \
                        hipGetErrorString(e_));                                                 \
    } while (0)

size_t store_bytes(int prec) { return prec == hl::PREC_F64 ? 8 : (prec == hl::PREC_F32 ? 4 : 2); }
size_t arith_bytes(int prec) { return prec == hl::PREC_F64 ? 8 : 4; }

int check_dom(hl_ctx *c, int32_t dom) {
    if (!c) return HL_E_INVAL;
    if (dom < 0 || dom >= (int32_t)c->doms.size()) return fail(c, HL_E_RANGE, "domain %d does not exist", dom);
    return HL_OK;
}

template <typename T>
int dalloc(hl_ctx *c, T **p, size_t count) {
    size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc((void **)p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(c, HL_E_NOMEM, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    c->dev_bytes += (int64_t)bytes;
    return HL_OK;
}

void dfree(void *p) {
    if (p) (void)hipFree(p);
}

void free_device(hl_ctx *c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    c->graph_steps = 0;
    void *ps[] = {c->lat[0], c->lat[1], c->d_src, c->d_d16, c->d_bq, c->d_bq_off, c->d_bphi, c->d_bnrm, c->d_up[0], c->d_up[1],
                  c->d_entries, c->d_entries2, c->d_seg, c->d_io, c->d_pairs, c->d_ctrl, c->d_partials, c->d_stats,
                  c->d_bc, c->d_held, c->d_obs, c->d_fbuf};
    for (void *p : ps) dfree(p);
    for (auto &p : c->d_c2g) dfree(p);
    c->d_c2g.clear();
    dfree(c->d_emap);
    c->d_emap = nullptr;
    c->lat[0] = c->lat[1] = nullptr;
    c->d_src = nullptr;
    c->d_d16 = nullptr;
    c->d_bq = nullptr;
    c->d_bq_off = nullptr;
    c->d_bphi = c->d_bnrm = nullptr;
    c->d_up[0] = c->d_up[1] = nullptr;
    c->d_entries = nullptr;
    c->d_entries2 = nullptr;
    c->d_seg = nullptr;
    c->d_io = nullptr;
    c->d_pairs = nullptr;
    c->d_ctrl = nullptr;
    c->d_partials = c->d_stats = c->d_bc = c->d_held = c->d_obs = c->d_fbuf = nullptr;
    c->dev_bytes = 0;
}

// Storage forms and schemes with the two-sites-per-lane bulk path.
bool pairs_supported(const hl_ctx *c) {
    return !c->aa && c->precision != hl::PREC_F16W && c->precision != hl::PREC_F16SR;
}

hl::KArgs make_args(hl_ctx *c) {
    hl::KArgs a{};
    a.N = c->L.N;
    a.NB = c->L.NB;
    a.IO0 = c->L.IO0;
    a.Nb = c->L.Nb;
    a.Nio = c->L.Nio;
    a.Npad = c->L.Npad;
    a.lat0 = c->lat[0];
    a.lat1 = c->lat[1];
    a.src = c->d_src;
    a.d16 = c->d_d16;
    a.bq = c->d_bq;
    a.bq_off = c->d_bq_off;
    a.bphi = c->d_bphi;
    a.up0 = c->d_up[0];
    a.up1 = c->d_up[1];
    a.bnrm = c->d_bnrm;
    a.entries = c->d_entries;
    a.entries2 = c->d_entries2;
    a.n_pairs_blocks = ((c->sched_flags & HL_SCHED_PAIRS) && !(c->sched_flags & HL_SCHED_FUSED) && pairs_supported(c))
                           ? (int32_t)c->L.entries2.size() : 0;
    a.pair_fused = (c->L.bulk_chunk > c->block) ? 1 : 0;
    a.seg = c->d_seg;
    a.io = c->d_io;
    a.pairs = c->d_pairs;
    a.n_io = (int32_t)c->L.hio.size();
    a.n_pairs = (int32_t)c->L.hpairs.size();
    a.io_e0 = a.io_e1 = 0;
    for (const auto &io : c->L.hio) {
        if (io.e_hi <= io.e_lo) continue;
        if (a.io_e0 == a.io_e1) {
            a.io_e0 = io.e_lo;
            a.io_e1 = io.e_hi;
        } else {
            a.io_e0 = std::min(a.io_e0, io.e_lo);
            a.io_e1 = std::max(a.io_e1, io.e_hi);
        }
    }
    a.couple_mode = c->couple_mode;
    a.xcd_remap = !(c->sched_flags & HL_SCHED_XCD_REMAP) ? 0 : ((c->sched_flags & HL_SCHED_XCD_RUNS) ? 64 : 1);
    a.emap = c->L.emap.empty() ? nullptr : c->d_emap;
    a.n_emap = (int32_t)c->L.emap.size();
    a.ctrl = c->d_ctrl;
    a.aa = c->aa ? 1 : 0;
    a.dt = 0;
    a.partials = c->d_partials;
    a.stats = c->d_stats;
    a.bc = c->d_bc;
    a.held = c->d_held;
    a.obs = c->d_obs;
    a.obs_lo = 0;
    a.obs_hi = c->L.N;
    a.obs_stride = c->L.N;
    a.fout = nullptr;
    a.fin = nullptr;
    return a;
}

int upload_schedule(hl_ctx *c) {
    dfree(c->d_entries);
    dfree(c->d_entries2);
    dfree(c->d_partials);
    c->d_entries = nullptr;
    c->d_entries2 = nullptr;
    c->d_partials = nullptr;
    int rc;
    if ((rc = dalloc(c, &c->d_entries, c->L.entries.size())) != HL_OK) return rc;
    if ((rc = dalloc(c, &c->d_entries2, c->L.entries2.size())) != HL_OK) return rc;
    if (!c->L.entries2.empty())
        HIPC(c, hipMemcpy(c->d_entries2, c->L.entries2.data(), c->L.entries2.size() * sizeof(hl::Entry),
                          hipMemcpyHostToDevice));
    if ((rc = dalloc(c, &c->d_partials, 2 * c->L.entries.size())) != HL_OK) return rc;
    dfree(c->d_emap);
    c->d_emap = nullptr;
    if (!c->L.emap.empty()) {
        if ((rc = dalloc(c, &c->d_emap, c->L.emap.size())) != HL_OK) return rc;
        HIPC(c, hipMemcpy(c->d_emap, c->L.emap.data(), c->L.emap.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    HIPC(c, hipMemcpy(c->d_entries, c->L.entries.data(), c->L.entries.size() * sizeof(hl::Entry),
                      hipMemcpyHostToDevice));
    if (!c->L.hio.empty())
        HIPC(c, hipMemcpy(c->d_io, c->L.hio.data(), c->L.hio.size() * sizeof(hl::IoletDev), hipMemcpyHostToDevice));
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    c->graph_steps = 0;
    return HL_OK;
}

// n steps as plain launches; t0 is the step counter before the first one (the
// in-place scheme alternates its even and odd kernels).
// (Launch k of the batch works on step t0 + k through its dt; the stored
// counter advances once after the batch.  The per-step finalize kernel runs
// only when the context couples domains.)
int launch_steps_plain(hl_ctx *c, int64_t n, hipStream_t st, int64_t t0) {
    if (n <= 0) return HL_OK;
    hl::KArgs a = make_args(c);
    const bool fused = (c->sched_flags & HL_SCHED_FUSED) != 0;
    for (int64_t k = 0; k < n; ++k) {
        a.dt = (int32_t)k;
        int e = c->aa ? hl::launch_aa_step(c->precision, a, c->L.n_bulk_blocks, c->L.n_bnd_blocks, c->block, st, 0, fused,
                                           (int)((t0 + k) & 1))
                      : hl::launch_step(c->precision, a, c->L.n_bulk_blocks, c->L.n_bnd_blocks, c->block, st, 0, fused);
        if (e != 0) return fail(c, HL_E_DEVICE, "step launch failed: %s", hipGetErrorString((hipError_t)e));
    }
    a.dt = 0;
    int e = hl::launch_advance(a, n, st);
    if (e != 0) return fail(c, HL_E_DEVICE, "advance launch failed: %s", hipGetErrorString((hipError_t)e));
    return HL_OK;
}

// Steps of a batch longer than this go in several launches sequences (dt is int32).
constexpr int64_t MAX_BATCH = (int64_t)1 << 30;

int ensure_graph(hl_ctx *c) {
    if (c->gexec && c->graph_steps == c->steps_per_graph) return HL_OK;
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    if (!c->cap_stream) HIPC(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIPC(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = launch_steps_plain(c, c->steps_per_graph, c->cap_stream, 0);  // replayed from even steps only
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (rc != HL_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(c, HL_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(c, HL_E_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    c->graph_steps = c->steps_per_graph;
    return HL_OK;
}

int run_steps(hl_ctx *c, int64_t n) {
    if (n <= 0) return HL_OK;  // keeps the means of the current step valid
    int64_t rest = n, t = c->t_host;
    if (c->aa && (c->steps_per_graph & 1)) c->steps_per_graph *= 2;  // graphs keep the sweep parity
    if (c->drive == HL_DRIVE_GRAPH && n >= c->steps_per_graph + (t & 1)) {
        if (c->aa && (t & 1)) {
            int rc = launch_steps_plain(c, 1, c->stream, t);
            if (rc != HL_OK) return rc;
            ++t;
            --rest;
        }
        int rc = ensure_graph(c);
        if (rc != HL_OK) return rc;
        while (rest >= c->graph_steps) {
            HIPC(c, hipGraphLaunch(c->gexec, c->stream));
            rest -= c->graph_steps;
            t += c->graph_steps;
        }
    }
    while (rest > 0) {
        const int64_t m = std::min(rest, MAX_BATCH);
        int rc = launch_steps_plain(c, m, c->stream, t);
        if (rc != HL_OK) return rc;
        rest -= m;
        t += m;
    }
    c->t_host += n;
    c->obs_t = -1;
    // coupled contexts finalize every step; the others compute their iolet
    // means on demand
    c->stats_t = c->L.hpairs.empty() ? -1 : (c->aa ? c->t_host - 1 : c->t_host);
    HIPC(c, hipMemcpyAsync(c->h_nan, &c->d_ctrl->nan_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    return HL_OK;
}

int upload_params(hl_ctx *c) {
    if (!c->committed) return HL_OK;
    for (size_t d = 0; d < c->doms.size(); ++d) c->L.hseg[d] = hl::seg_of(c->doms[d]);
    HIPC(c, hipStreamSynchronize(c->stream));
    HIPC(c, hipMemcpy(c->d_seg, c->L.hseg.data(), c->L.hseg.size() * sizeof(hl::SegDev), hipMemcpyHostToDevice));
    return HL_OK;
}

// Re-evaluate the boundary value of an uncoupled iolet for the coming step
// after its waveform changed.
int refresh_series(hl_ctx *c, int32_t dom, int32_t k) {
    if (!c->committed) return HL_OK;
    Domain &d = c->doms[dom];
    const int g = d.io_base + k;
    hl::IoletDev &io = c->L.hio[g];
    const Series &s = d.io[k].wave;
    io.a0 = s.a0;
    io.nh = s.nh;
    io.period = s.period;
    for (int m = 0; m < hl::MAXH; ++m) {
        io.a[m] = s.a[m];
        io.b[m] = s.b[m];
    }
    HIPC(c, hipStreamSynchronize(c->stream));
    HIPC(c, hipMemcpy(c->d_io + g, &io, sizeof io, hipMemcpyHostToDevice));
    if (!io.coupled) {
        const double v = s.at((double)c->t_host);
        HIPC(c, hipMemcpy(c->d_bc + (c->t_host & 1) * c->L.hio.size() + g, &v, sizeof v, hipMemcpyHostToDevice));
    }
    return HL_OK;
}

int read_nan(hl_ctx *c) {
    HIPC(c, hipStreamSynchronize(c->stream));
    int v = 0;
    HIPC(c, hipMemcpy(&v, &c->d_ctrl->nan_flag, sizeof v, hipMemcpyDeviceToHost));
    *c->h_nan = v;
    if (v) return fail(c, HL_E_DIVERGED, "a non-finite density appeared");
    return HL_OK;
}

int observe(hl_ctx *c, bool with_f) {
    int rc;
    if (!c->d_obs && (rc = dalloc(c, &c->d_obs, 5 * (size_t)c->L.N)) != HL_OK) return rc;
    if (with_f && !c->d_fbuf && (rc = dalloc(c, &c->d_fbuf, (size_t)Q * c->L.N)) != HL_OK) return rc;
    if (!with_f && c->obs_t == c->t_host) return HL_OK;
    hl::KArgs a = make_args(c);
    a.fout = with_f ? c->d_fbuf : nullptr;
    int e = hl::launch_observe(c->precision, a, (int)c->L.entries.size(), c->block, c->stream);
    if (e != 0) return fail(c, HL_E_DEVICE, "observe launch failed: %s", hipGetErrorString((hipError_t)e));
    c->obs_t = c->t_host;
    return HL_OK;
}

// Collide the raw f(t) in lat[(t+1)&1] into f*(t) and recompute the means
// and boundary values of step t.
int reinit(hl_ctx *c) {
    hl::KArgs a = make_args(c);
    int e;
    if (c->aa) {
        // the lattice holds f(t) in natural slots: mark it and take its moments
        HIPC(c, hipStreamSynchronize(c->stream));
        const int one = 1;
        HIPC(c, hipMemcpy(&c->d_ctrl->direct, &one, sizeof one, hipMemcpyHostToDevice));
        e = hl::launch_aa_moments(c->precision, a, (int)c->L.entries.size(), c->block, c->stream, (int)(c->t_host & 1));
    } else {
        e = hl::launch_init(c->precision, a, (int)c->L.entries.size(), c->block, c->stream);
    }
    if (e != 0) return fail(c, HL_E_DEVICE, "init launch failed: %s", hipGetErrorString((hipError_t)e));
    c->obs_t = -1;
    c->stats_t = c->t_host;
    return HL_OK;
}

// Iolet means and boundary values of the current step, when the last steps
// did not leave them: the in-place scheme reduces f(t) during the sweep
// t -> t+1, so it runs the moments pass (idempotent: the next sweep
// recomputes the same values); two lattices reduce f(t) in the step that
// produces it, so the partial sums of the last step only need the finalize.
int ensure_stats(hl_ctx *c) {
    if (c->stats_t == c->t_host) return HL_OK;
    hl::KArgs a = make_args(c);
    int e = c->aa ? hl::launch_aa_moments(c->precision, a, (int)c->L.entries.size(), c->block, c->stream,
                                          (int)(c->t_host & 1))
                  : hl::launch_stats(a, c->stream);
    if (e != 0) return fail(c, HL_E_DEVICE, "moments launch failed: %s", hipGetErrorString((hipError_t)e));
    c->stats_t = c->t_host;
    return HL_OK;
}

int commit(hl_ctx *c) {
    if (c->committed) return HL_OK;
    HIPC(c, hipSetDevice(c->device));
    int rc = hl::plan_layout(c->doms, c->pairs, c->order_flags, c->couple_mode, c->L, c->err);
    if (rc != HL_OK) return rc;
    hl::plan_schedule(c->L, c->block, c->sched_flags, pairs_supported(c));
    if (c->debug_checks && (rc = hl::check_layout(c->doms, c->L, c->block, c->err)) != HL_OK) return rc;
    const int D = (int)c->doms.size();
    const int64_t Nio = c->L.Nio;

    // device memory
    const size_t S = store_bytes(c->precision), A = arith_bytes(c->precision);
    for (int p = 0; p < 2; ++p) {
        if (p == 0 || !c->aa) {
            HIPC(c, hipMalloc(&c->lat[p], (size_t)Q * c->L.Npad * S));
            c->dev_bytes += (int64_t)((size_t)Q * c->L.Npad * S);
        }
        HIPC(c, hipMalloc(&c->d_up[p], std::max<size_t>((size_t)3 * Nio * A, 8)));
        c->dev_bytes += (int64_t)std::max<size_t>((size_t)3 * Nio * A, 8);
    }
    const hl::Layout &L = c->L;
    if ((rc = dalloc(c, &c->d_src, L.src.size())) != HL_OK) return rc;
    if (!L.d16.empty() && (rc = dalloc(c, &c->d_d16, L.d16.size())) != HL_OK) return rc;
    if ((rc = dalloc(c, &c->d_bq, L.bq.size())) != HL_OK) return rc;
    if ((rc = dalloc(c, &c->d_bq_off, L.bq_off.size())) != HL_OK) return rc;
    if ((rc = dalloc(c, &c->d_bphi, L.bphi.size())) != HL_OK) return rc;
    if ((rc = dalloc(c, &c->d_bnrm, L.bnrm.size())) != HL_OK) return rc;
    if ((rc = dalloc(c, &c->d_seg, c->L.hseg.size())) != HL_OK) return rc;
    if ((rc = dalloc(c, &c->d_io, c->L.hio.size())) != HL_OK) return rc;
    if ((rc = dalloc(c, &c->d_pairs, c->L.hpairs.size())) != HL_OK) return rc;
    if ((rc = dalloc(c, &c->d_ctrl, 1)) != HL_OK) return rc;
    const size_t nio1 = std::max<size_t>(c->L.hio.size(), 1);
    if ((rc = dalloc(c, &c->d_stats, 2 * nio1)) != HL_OK) return rc;
    if ((rc = dalloc(c, &c->d_bc, 2 * nio1)) != HL_OK) return rc;
    if ((rc = dalloc(c, &c->d_held, nio1)) != HL_OK) return rc;
    HIPC(c, hipMemcpy(c->d_src, L.src.data(), L.src.size() * 4, hipMemcpyHostToDevice));
    if (!L.d16.empty()) HIPC(c, hipMemcpy(c->d_d16, L.d16.data(), L.d16.size() * 2, hipMemcpyHostToDevice));
    HIPC(c, hipMemcpy(c->d_bq, L.bq.data(), L.bq.size() * 4, hipMemcpyHostToDevice));
    HIPC(c, hipMemcpy(c->d_bq_off, L.bq_off.data(), L.bq_off.size() * 4, hipMemcpyHostToDevice));
    HIPC(c, hipMemcpy(c->d_bphi, L.bphi.data(), L.bphi.size() * 8, hipMemcpyHostToDevice));
    HIPC(c, hipMemcpy(c->d_bnrm, L.bnrm.data(), L.bnrm.size() * 8, hipMemcpyHostToDevice));
    HIPC(c, hipMemcpy(c->d_seg, c->L.hseg.data(), c->L.hseg.size() * sizeof(hl::SegDev), hipMemcpyHostToDevice));
    if (!c->L.hpairs.empty())
        HIPC(c, hipMemcpy(c->d_pairs, c->L.hpairs.data(), c->L.hpairs.size() * sizeof(hl::PairDev),
                          hipMemcpyHostToDevice));
    if ((rc = upload_schedule(c)) != HL_OK) return rc;
    // caller index -> internal index per domain, for the device reads
    c->d_c2g.assign(c->doms.size(), nullptr);
    for (int d = 0; d < D; ++d) {
        if ((rc = dalloc(c, &c->d_c2g[d], c->doms[d].n)) != HL_OK) return rc;
        if (c->doms[d].n)
            HIPC(c, hipMemcpy(c->d_c2g[d], c->doms[d].c2g.data(), c->doms[d].n * sizeof(int64_t),
                              hipMemcpyHostToDevice));
    }
    std::vector<double> held(nio1, 0.0), zeros(2 * nio1, 0.0);
    for (int d = 0; d < D; ++d)
        for (int k = 0; k < c->doms[d].n_iolet; ++k) {
            // a velocity-driven coupled outlet starts from rest
            const hl::IoletH &io = c->doms[d].io[k];
            const bool vel_outlet = io.kind == hl::KIND_OUTLET && hl::velocity_driven(io, c->couple_mode);
            held[c->doms[d].io_base + k] = vel_outlet ? 0.0 : io.wave.at(0.0);
        }
    HIPC(c, hipMemcpy(c->d_held, held.data(), held.size() * 8, hipMemcpyHostToDevice));
    HIPC(c, hipMemcpy(c->d_bc, zeros.data(), zeros.size() * 8, hipMemcpyHostToDevice));
    HIPC(c, hipMemcpy(c->d_stats, zeros.data(), zeros.size() * 8, hipMemcpyHostToDevice));
    hl::Ctrl ctrl{};
    HIPC(c, hipMemcpy(c->d_ctrl, &ctrl, sizeof ctrl, hipMemcpyHostToDevice));
    // geometry arrays and uploaded tables are no longer needed on the host
    for (auto &d : c->doms) {
        std::vector<int32_t>().swap(d.nbr);
        std::vector<int32_t>().swap(d.coords);
    }
    std::vector<int32_t>().swap(c->L.src);
    std::vector<int16_t>().swap(c->L.d16);
    std::vector<float>().swap(c->L.bq);
    std::vector<uint32_t>().swap(c->L.bq_off);
    std::vector<double>().swap(c->L.bphi);
    std::vector<double>().swap(c->L.bnrm);
    c->committed = true;
    c->t_host = 0;
    // initial state: rest equilibrium at rho0, collided into f*(0)
    hl::KArgs a = make_args(c);
    int e = hl::launch_fill_rest(c->precision, a, c->stream);
    if (e != 0) return fail(c, HL_E_DEVICE, "fill launch failed: %s", hipGetErrorString((hipError_t)e));
    if ((rc = reinit(c)) != HL_OK) return rc;
    HIPC(c, hipStreamSynchronize(c->stream));
    return HL_OK;
}

int validate(hl_ctx *c, int64_t n, const int32_t *nbr, int64_t n_iolet) {
    std::string err;
    const int rc = hl::validate_sites(n, nbr, n_iolet, err);
    return rc == HL_OK ? HL_OK : fail(c, rc, "%s", err.c_str());
}

int parse_series(hl_ctx *c, Series &s, double a0, int nh, const double *a, const double *b, double period) {
    if (nh < 0 || nh > hl::MAXH) return fail(c, HL_E_INVAL, "nh = %d outside 0..%d", nh, hl::MAXH);
    if (nh > 0 && (!(period > 0.0) || !a || !b)) return fail(c, HL_E_INVAL, "period must be > 0 with harmonics");
    if (!std::isfinite(a0)) return fail(c, HL_E_INVAL, "non-finite series");
    s = Series{};
    s.a0 = a0;
    s.nh = nh;
    s.period = nh > 0 ? period : 1.0;
    for (int m = 0; m < nh; ++m) {
        if (!std::isfinite(a[m]) || !std::isfinite(b[m])) return fail(c, HL_E_INVAL, "non-finite series");
        s.a[m] = a[m];
        s.b[m] = b[m];
    }
    return HL_OK;
}

struct StateHeader {
    char magic[8];
    int32_t version, precision;
    int64_t N, Nio, n_io, bytes;
};

size_t state_bytes(hl_ctx *c) {
    const size_t S = store_bytes(c->precision), A = arith_bytes(c->precision);
    const size_t nio = c->L.hio.size();
    const size_t nlat = c->aa ? 1 : 2;
    return sizeof(StateHeader) + sizeof(hl::Ctrl) + nlat * (size_t)Q * c->L.Npad * S + 2 * (size_t)3 * c->L.Nio * A +
           (2 + 2 + 1) * nio * sizeof(double);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *hl_status_string(int code) {
    switch (code) {
        case HL_OK: return "ok";
        case HL_E_INVAL: return "invalid argument";
        case HL_E_RANGE: return "index or code out of range";
        case HL_E_STATE: return "call not allowed in the current state";
        case HL_E_NOMEM: return "allocation failed";
        case HL_E_DEVICE: return "device error";
        case HL_E_DIVERGED: return "simulation diverged";
        case HL_W_MACH: return "warning: Mach number >= 0.1";
        case HL_W_TAU: return "warning: tau > 1";
        default: return "unknown status";
    }
}

const char *hl_last_error(const hl_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int hl_create(hl_ctx **out, int device, int precision, uint64_t flags) {
    if (!out) return HL_E_INVAL;
    *out = nullptr;
    if (precision < HL_F64 || precision > HL_F16_STOCHASTIC) return HL_E_INVAL;
    if (flags & ~(uint64_t)(HL_ORDER_BULK_MORTON | HL_ORDER_BOUNDARY_MORTON | HL_ORDER_INTERLEAVE | HL_ORDER_BRICK |
                            HL_SCHEME_AA | HL_ORDER_BRICK_32 | HL_DEBUG_CHECKS))
        return HL_E_INVAL;
    if ((flags & HL_ORDER_BRICK_32) && !(flags & HL_ORDER_BRICK)) return HL_E_INVAL;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return HL_E_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return HL_E_DEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return HL_E_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return HL_E_DEVICE;
    // once per device: the address of the fixed scratch of the
    // allocation-free observables read
    if (hl::noalloc_scratch_setup(device) != (int)hipSuccess) return HL_E_DEVICE;
    hl_ctx *c = new hl_ctx();
    c->device = device;
    c->precision = precision;
    c->order_flags = flags;
    c->aa = (flags & HL_SCHEME_AA) != 0;
    c->debug_checks = (flags & HL_DEBUG_CHECKS) != 0;
    if (hipHostMalloc((void **)&c->h_nan, sizeof(int), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return HL_E_NOMEM;
    }
    *c->h_nan = 0;
    *out = c;
    return HL_OK;
}

void hl_destroy(hl_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->committed) (void)hipStreamSynchronize(ctx->stream);
    free_device(ctx);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->h_nan) (void)hipHostFree(ctx->h_nan);
    delete ctx;
}

int hl_set_stream(hl_ctx *ctx, void *hip_stream) {
    if (!ctx) return HL_E_INVAL;
    hipStream_t next = (hipStream_t)hip_stream;
    if (next == ctx->stream) return HL_OK;
    // work queued on the old stream finishes before anything is queued on the
    // new one (later reads, steps and hl_destroy wait on the new stream only)
    if (ctx->committed) {
        HIPC(ctx, hipSetDevice(ctx->device));
        HIPC(ctx, hipStreamSynchronize(ctx->stream));
    }
    ctx->stream = next;
    return HL_OK;
}

int hl_add_domain(hl_ctx *ctx, int32_t *dom_id) {
    if (!ctx || !dom_id) return HL_E_INVAL;
    if (ctx->committed) return fail(ctx, HL_E_STATE, "domains cannot be added after the first step");
    ctx->doms.emplace_back();
    *dom_id = (int32_t)ctx->doms.size() - 1;
    return HL_OK;
}

int hl_validate_sites(int64_t n, const int32_t *nbr, int64_t n_iolet) { return validate(nullptr, n, nbr, n_iolet); }

int hl_load_sites(hl_ctx *ctx, int32_t dom, int64_t n, const int32_t *coords, const int32_t *nbr, int32_t n_iolet,
                  int64_t n_q, const int64_t *q_site, const int8_t *q_dir, const float *q) {
    int rc = check_dom(ctx, dom);
    if (rc) return rc;
    if (ctx->committed) return fail(ctx, HL_E_STATE, "sites cannot be loaded after the first step");
    if ((rc = validate(ctx, n, nbr, n_iolet)) != HL_OK) return rc;
    if (n > 0 && !coords) return fail(ctx, HL_E_INVAL, "coords is NULL");
    if (n_q < 0 || (n_q > 0 && (!q_site || !q_dir || !q))) return fail(ctx, HL_E_INVAL, "bad wall-fraction arrays");
    for (int64_t e = 0; e < n_q; ++e) {
        if (q_site[e] < 0 || q_site[e] >= n || q_dir[e] < 1 || q_dir[e] >= Q)
            return fail(ctx, HL_E_RANGE, "wall fraction %lld names no link", (long long)e);
        if (nbr[(size_t)q_dir[e] * n + q_site[e]] != -1)
            return fail(ctx, HL_E_RANGE, "wall fraction %lld is not on a wall link", (long long)e);
        if (!(q[e] > 0.0f && q[e] <= 1.0f)) return fail(ctx, HL_E_RANGE, "wall fraction %lld outside (0,1]", (long long)e);
    }
    Domain &d = ctx->doms[dom];
    d.n = n;
    d.coords.assign(coords, coords + 3 * (size_t)n);
    d.nbr.assign(nbr, nbr + (size_t)Q * n);
    d.q_site.assign(q_site, q_site + n_q);
    d.q_dir.assign(q_dir, q_dir + n_q);
    d.q.assign(q, q + n_q);
    d.n_iolet = n_iolet;
    d.io.assign(n_iolet, IoletH{});
    for (auto &io : d.io) io.wave.a0 = 0.0;
    d.wn_site.clear();
    d.wn.clear();
    return HL_OK;
}

int hl_set_wall_normals(hl_ctx *ctx, int32_t dom, int64_t n_w, const int64_t *site, const double *nrm) {
    int rc = check_dom(ctx, dom);
    if (rc) return rc;
    if (ctx->committed) return fail(ctx, HL_E_STATE, "normals cannot change after the first step");
    Domain &d = ctx->doms[dom];
    if (n_w < 0 || (n_w > 0 && (!site || !nrm))) return fail(ctx, HL_E_INVAL, "bad normal arrays");
    for (int64_t e = 0; e < n_w; ++e)
        if (site[e] < 0 || site[e] >= d.n) return fail(ctx, HL_E_RANGE, "normal %lld names no site", (long long)e);
    d.wn_site.assign(site, site + n_w);
    d.wn.assign(nrm, nrm + 3 * (size_t)n_w);
    return HL_OK;
}

int hl_set_wall_mode(hl_ctx *ctx, int32_t dom, int mode) {
    int rc = check_dom(ctx, dom);
    if (rc) return rc;
    if (mode != HL_WALL_SBB && mode != HL_WALL_BOUZIDI) return fail(ctx, HL_E_INVAL, "unknown wall mode %d", mode);
    ctx->doms[dom].wall_mode = mode;
    return upload_params(ctx);
}

int hl_set_tau(hl_ctx *ctx, int32_t dom, double tau) {
    int rc = check_dom(ctx, dom);
    if (rc) return rc;
    if (!std::isfinite(tau) || tau <= 0.5) return fail(ctx, HL_E_INVAL, "tau = %g must exceed 1/2", tau);
    ctx->doms[dom].tau = tau;
    rc = upload_params(ctx);
    if (rc) return rc;
    return tau > 1.0 ? HL_W_TAU : HL_OK;
}

int hl_set_iolet(hl_ctx *ctx, int32_t dom, int32_t k, int kind, const double centre[3], const double normal[3],
                 double radius) {
    int rc = check_dom(ctx, dom);
    if (rc) return rc;
    if (ctx->committed) return fail(ctx, HL_E_STATE, "iolets cannot change after the first step");
    Domain &d = ctx->doms[dom];
    if (k < 0 || k >= d.n_iolet) return fail(ctx, HL_E_RANGE, "iolet %d does not exist", k);
    if (kind != HL_INLET_VEL && kind != HL_OUTLET_P) return fail(ctx, HL_E_INVAL, "unknown iolet kind");
    if (!centre || !normal) return fail(ctx, HL_E_INVAL, "NULL centre or normal");
    const double nl = std::sqrt(normal[0] * normal[0] + normal[1] * normal[1] + normal[2] * normal[2]);
    if (!(nl > 0.0) || !(radius > 0.0)) return fail(ctx, HL_E_INVAL, "zero normal or radius");
    IoletH &io = d.io[k];
    if (io.coupled && io.kind != kind) return fail(ctx, HL_E_INVAL, "iolet %d is coupled", k);
    io.kind = kind;
    for (int a = 0; a < 3; ++a) {
        io.c[a] = centre[a];
        io.nrm[a] = normal[a] / nl;
    }
    io.R = radius;
    io.wave = Series{};
    io.wave.a0 = (kind == HL_OUTLET_P) ? hl::RHO0 : 0.0;
    return HL_OK;
}

static int set_series(hl_ctx *ctx, int32_t dom, int32_t k, int kind, double a0, int nh, const double *a,
                      const double *b, double period) {
    int rc = check_dom(ctx, dom);
    if (rc) return rc;
    Domain &d = ctx->doms[dom];
    if (k < 0 || k >= d.n_iolet) return fail(ctx, HL_E_RANGE, "iolet %d does not exist", k);
    if (d.io[k].kind != kind) return fail(ctx, HL_E_INVAL, "iolet %d has the other kind", k);
    Series s;
    if ((rc = parse_series(ctx, s, a0, nh, a, b, period)) != HL_OK) return rc;
    d.io[k].wave = s;
    if ((rc = refresh_series(ctx, dom, k)) != HL_OK) return rc;
    if (kind == HL_INLET_VEL && std::sqrt(3.0) * s.bound() >= 0.1) return HL_W_MACH;
    return HL_OK;
}

int hl_set_inlet_velocity(hl_ctx *ctx, int32_t dom, int32_t k, double a0, int nh, const double *a, const double *b,
                          double period) {
    return set_series(ctx, dom, k, HL_INLET_VEL, a0, nh, a, b, period);
}

int hl_set_outlet_density(hl_ctx *ctx, int32_t dom, int32_t k, double rho0, int nh, const double *a,
                          const double *b, double period) {
    if (ctx && !(rho0 > 0.0)) return fail(ctx, HL_E_INVAL, "outlet density must be positive");
    return set_series(ctx, dom, k, HL_OUTLET_P, rho0, nh, a, b, period);
}

int hl_set_body_force(hl_ctx *ctx, int32_t dom, const double F0[3], double omega) {
    int rc = check_dom(ctx, dom);
    if (rc) return rc;
    if (!F0 || !std::isfinite(F0[0]) || !std::isfinite(F0[1]) || !std::isfinite(F0[2]) || !std::isfinite(omega))
        return fail(ctx, HL_E_INVAL, "bad body force");
    for (int a = 0; a < 3; ++a) ctx->doms[dom].F0[a] = F0[a];
    ctx->doms[dom].omega = omega;
    return upload_params(ctx);
}

int hl_couple(hl_ctx *ctx, int32_t dom_a, int32_t outlet, int32_t dom_b, int32_t inlet, double s_vel,
              double dp_ratio) {
    int rc;
    if ((rc = check_dom(ctx, dom_a)) || (rc = check_dom(ctx, dom_b))) return rc;
    if (ctx->committed) return fail(ctx, HL_E_STATE, "coupling cannot change after the first step");
    Domain &a = ctx->doms[dom_a], &b = ctx->doms[dom_b];
    if (outlet < 0 || outlet >= a.n_iolet || inlet < 0 || inlet >= b.n_iolet)
        return fail(ctx, HL_E_RANGE, "iolet index out of range");
    if (a.io[outlet].kind != HL_OUTLET_P || b.io[inlet].kind != HL_INLET_VEL)
        return fail(ctx, HL_E_INVAL, "coupling runs from an outlet to an inlet");
    if (b.io[inlet].coupled) return fail(ctx, HL_E_INVAL, "inlet already coupled");
    if (!(dp_ratio > 0.0 && dp_ratio < 1.0) || !std::isfinite(s_vel))
        return fail(ctx, HL_E_INVAL, "dp_ratio must lie in (0,1)");
    ctx->pairs.push_back({dom_a, outlet, dom_b, inlet, s_vel, dp_ratio});
    a.io[outlet].coupled = true;
    b.io[inlet].coupled = true;
    return HL_OK;
}

int hl_set_coupling_mode(hl_ctx *ctx, int mode) {
    if (!ctx) return HL_E_INVAL;
    if (ctx->committed) return fail(ctx, HL_E_STATE, "coupling mode cannot change after the first step");
    if (mode & ~(HL_BOTH_EACH_STEP | HL_COUPLE_VELOCITY)) return fail(ctx, HL_E_INVAL, "unknown coupling mode");
    ctx->couple_mode = mode;
    return HL_OK;
}

int hl_commit(hl_ctx *ctx) {
    if (!ctx) return HL_E_INVAL;
    return commit(ctx);
}

int hl_step(hl_ctx *ctx, int64_t nsteps) {
    if (!ctx) return HL_E_INVAL;
    if (nsteps < 0) return fail(ctx, HL_E_INVAL, "nsteps < 0");
    int rc = commit(ctx);
    if (rc) return rc;
    if (*ctx->h_nan) return fail(ctx, HL_E_DIVERGED, "a non-finite density appeared");
    HIPC(ctx, hipSetDevice(ctx->device));
    return run_steps(ctx, nsteps);
}

int hl_sync(hl_ctx *ctx) {
    if (!ctx) return HL_E_INVAL;
    if (!ctx->committed) return HL_OK;
    return read_nan(ctx);
}

int hl_get_time(hl_ctx *ctx, int64_t *t) {
    if (!ctx || !t) return HL_E_INVAL;
    *t = ctx->t_host;
    return HL_OK;
}

int hl_set_drive(hl_ctx *ctx, int drive, int32_t steps_per_graph) {
    if (!ctx) return HL_E_INVAL;
    if (drive != HL_DRIVE_LAUNCH && drive != HL_DRIVE_GRAPH) return fail(ctx, HL_E_INVAL, "unknown drive");
    if (drive == HL_DRIVE_GRAPH && steps_per_graph < 1) return fail(ctx, HL_E_INVAL, "steps_per_graph < 1");
    ctx->drive = drive;
    if (drive == HL_DRIVE_GRAPH) ctx->steps_per_graph = steps_per_graph;
    return HL_OK;
}

static int read_component(hl_ctx *ctx, int32_t dom, int comp, int ncomp, double *out) {
    int rc = check_dom(ctx, dom);
    if (rc) return rc;
    if (!out) return fail(ctx, HL_E_INVAL, "NULL output");
    if ((rc = commit(ctx)) != HL_OK) return rc;
    HIPC(ctx, hipSetDevice(ctx->device));
    if ((rc = observe(ctx, false)) != HL_OK) return rc;
    const int64_t N = ctx->L.N;
    std::vector<double> buf((size_t)ncomp * N);
    HIPC(ctx, hipMemcpyAsync(buf.data(), ctx->d_obs + (size_t)comp * N, buf.size() * 8, hipMemcpyDeviceToHost,
                             ctx->stream));
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    const Domain &d = ctx->doms[dom];
    for (int m = 0; m < ncomp; ++m)
        for (int64_t x = 0; x < d.n; ++x) out[(size_t)m * d.n + x] = buf[(size_t)m * N + d.c2g[x]];
    return read_nan(ctx);
}

int hl_read_density(hl_ctx *ctx, int32_t dom, double *out) { return read_component(ctx, dom, 0, 1, out); }
int hl_read_velocity(hl_ctx *ctx, int32_t dom, double *out) { return read_component(ctx, dom, 1, 3, out); }
int hl_read_wss(hl_ctx *ctx, int32_t dom, double *out) { return read_component(ctx, dom, 4, 1, out); }

int hl_read_populations(hl_ctx *ctx, int32_t dom, double *out) {
    int rc = check_dom(ctx, dom);
    if (rc) return rc;
    if (!out) return fail(ctx, HL_E_INVAL, "NULL output");
    if ((rc = commit(ctx)) != HL_OK) return rc;
    HIPC(ctx, hipSetDevice(ctx->device));
    if ((rc = observe(ctx, true)) != HL_OK) return rc;
    const int64_t N = ctx->L.N;
    std::vector<double> buf((size_t)Q * N);
    HIPC(ctx, hipMemcpyAsync(buf.data(), ctx->d_fbuf, buf.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    const Domain &d = ctx->doms[dom];
    for (int i = 0; i < Q; ++i)
        for (int64_t x = 0; x < d.n; ++x) out[(size_t)i * d.n + x] = buf[(size_t)i * N + d.c2g[x]];
    return read_nan(ctx);
}

int hl_set_populations(hl_ctx *ctx, int32_t dom, const double *f) {
    int rc = check_dom(ctx, dom);
    if (rc) return rc;
    if (!f) return fail(ctx, HL_E_INVAL, "NULL populations");
    if ((rc = commit(ctx)) != HL_OK) return rc;
    HIPC(ctx, hipSetDevice(ctx->device));
    if ((rc = observe(ctx, true)) != HL_OK) return rc;
    const int64_t N = ctx->L.N;
    std::vector<double> buf((size_t)Q * N);
    HIPC(ctx, hipMemcpyAsync(buf.data(), ctx->d_fbuf, buf.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    const Domain &d = ctx->doms[dom];
    for (int i = 0; i < Q; ++i)
        for (int64_t x = 0; x < d.n; ++x) buf[(size_t)i * N + d.c2g[x]] = f[(size_t)i * d.n + x];
    HIPC(ctx, hipMemcpy(ctx->d_fbuf, buf.data(), buf.size() * 8, hipMemcpyHostToDevice));
    int zero = 0;
    HIPC(ctx, hipMemcpy(&ctx->d_ctrl->nan_flag, &zero, sizeof zero, hipMemcpyHostToDevice));
    *ctx->h_nan = 0;
    hl::KArgs a = make_args(ctx);
    a.fin = ctx->d_fbuf;
    int e = (ctx->aa && (ctx->t_host & 1))
                ? hl::launch_aa_load_odd(ctx->precision, a, (int)ctx->L.entries.size(), ctx->block, ctx->stream)
                : hl::launch_load_raw(ctx->precision, a, ctx->stream);
    if (e != 0) return fail(ctx, HL_E_DEVICE, "load launch failed: %s", hipGetErrorString((hipError_t)e));
    if ((rc = reinit(ctx)) != HL_OK) return rc;
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    return HL_OK;
}

int hl_read_iolet_stats(hl_ctx *ctx, int32_t dom, double *mean_u, double *mean_p) {
    int rc = check_dom(ctx, dom);
    if (rc) return rc;
    if ((rc = commit(ctx)) != HL_OK) return rc;
    const Domain &d = ctx->doms[dom];
    if (d.n_iolet == 0) return HL_OK;
    if (!mean_u || !mean_p) return fail(ctx, HL_E_INVAL, "NULL output");
    HIPC(ctx, hipSetDevice(ctx->device));
    if ((rc = ensure_stats(ctx)) != HL_OK) return rc;
    const size_t nio = ctx->L.hio.size();
    std::vector<double> st(2 * nio);
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    HIPC(ctx, hipMemcpy(st.data(), ctx->d_stats, st.size() * 8, hipMemcpyDeviceToHost));
    for (int k = 0; k < d.n_iolet; ++k) {
        mean_u[k] = st[d.io_base + k];
        mean_p[k] = st[nio + d.io_base + k] / 3.0;  // the device holds the mean of rho - rho0
    }
    return read_nan(ctx);
}

int hl_read_iolet_bc(hl_ctx *ctx, int32_t dom, int which, double *out) {
    int rc = check_dom(ctx, dom);
    if (rc) return rc;
    if (which != 0 && which != 1) return fail(ctx, HL_E_INVAL, "which must be 0 or 1");
    if ((rc = commit(ctx)) != HL_OK) return rc;
    if (which == 1 && ctx->t_host == 0) return fail(ctx, HL_E_STATE, "no step has been taken");
    const Domain &d = ctx->doms[dom];
    if (d.n_iolet == 0) return HL_OK;
    if (!out) return fail(ctx, HL_E_INVAL, "NULL output");
    HIPC(ctx, hipSetDevice(ctx->device));
    if ((rc = ensure_stats(ctx)) != HL_OK) return rc;
    const size_t nio = ctx->L.hio.size();
    std::vector<double> bc(2 * nio);
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    HIPC(ctx, hipMemcpy(bc.data(), ctx->d_bc, bc.size() * 8, hipMemcpyDeviceToHost));
    const int64_t par = (ctx->t_host - which) & 1;
    for (int k = 0; k < d.n_iolet; ++k) out[k] = bc[par * nio + d.io_base + k];
    return read_nan(ctx);
}

static int read_device(hl_ctx *ctx, int32_t dom, int comp, int ncomp, void *dptr) {
    int rc = check_dom(ctx, dom);
    if (rc) return rc;
    if (!dptr) return fail(ctx, HL_E_INVAL, "NULL device pointer");
    if ((rc = commit(ctx)) != HL_OK) return rc;
    HIPC(ctx, hipSetDevice(ctx->device));
    if ((rc = observe(ctx, false)) != HL_OK) return rc;
    Domain &d = ctx->doms[dom];
    for (int m = 0; m < ncomp; ++m) {
        int e = hl::launch_gather_obs(ctx->d_obs + (size_t)(comp + m) * ctx->L.N, ctx->d_c2g[dom], d.n,
                                      (double *)dptr + (size_t)m * d.n, 0, ctx->L.N, ctx->stream);
        if (e != 0) return fail(ctx, HL_E_DEVICE, "gather launch failed");
    }
    return HL_OK;
}

int hl_read_observables_device_noalloc(hl_ctx *ctx, int32_t dom, void *rho, void *u, void *wss) {
    int rc = check_dom(ctx, dom);
    if (rc) return rc;
    if (!ctx->committed) return fail(ctx, HL_E_STATE, "the context must be committed first (this call allocates nothing)");
    if (!rho && !u && !wss) return HL_OK;
    HIPC(ctx, hipSetDevice(ctx->device));
    double *scr = hl::noalloc_scratch(ctx->device);
    if (!scr) return fail(ctx, HL_E_DEVICE, "no scratch address for device %d", ctx->device);
    // passes over windows of W internal sites: the observables of a window
    // are staged in the scratch ([5][W] doubles) and scattered to the caller
    // order; the next pass reuses the scratch (same stream)
    const int64_t W = hl::NOALLOC_SCRATCH_DOUBLES / 5 / hl::TILE * hl::TILE;
    const Domain &d = ctx->doms[dom];
    void *outs[3] = {rho, u, wss};
    const int comps[3] = {0, 1, 4}, ncomp[3] = {1, 3, 1};
    for (int64_t g0 = 0; g0 < ctx->L.N; g0 += W) {
        hl::KArgs a = make_args(ctx);
        a.obs = scr;
        a.obs_lo = g0;
        a.obs_hi = std::min(g0 + W, ctx->L.N);
        a.obs_stride = W;
        a.fout = nullptr;
        int e = hl::launch_observe(ctx->precision, a, (int)ctx->L.entries.size(), ctx->block, ctx->stream);
        if (e != 0) return fail(ctx, HL_E_DEVICE, "observe launch failed: %s", hipGetErrorString((hipError_t)e));
        for (int q = 0; q < 3; ++q) {
            if (!outs[q]) continue;
            for (int m = 0; m < ncomp[q]; ++m) {
                e = hl::launch_gather_obs(scr + (size_t)(comps[q] + m) * W, ctx->d_c2g[dom], d.n,
                                          (double *)outs[q] + (size_t)m * d.n, a.obs_lo, a.obs_hi, ctx->stream);
                if (e != 0) return fail(ctx, HL_E_DEVICE, "gather launch failed");
            }
        }
    }
    return HL_OK;
}

int hl_read_density_device(hl_ctx *ctx, int32_t dom, void *dptr) { return read_device(ctx, dom, 0, 1, dptr); }
int hl_read_velocity_device(hl_ctx *ctx, int32_t dom, void *dptr) { return read_device(ctx, dom, 1, 3, dptr); }
int hl_read_wss_device(hl_ctx *ctx, int32_t dom, void *dptr) { return read_device(ctx, dom, 4, 1, dptr); }

int hl_get_state(hl_ctx *ctx, void *buf, size_t *bytes) {
    if (!ctx || !bytes) return HL_E_INVAL;
    int rc = commit(ctx);
    if (rc) return rc;
    const size_t need = state_bytes(ctx);
    if (!buf) {
        *bytes = need;
        return HL_OK;
    }
    if (*bytes < need) return fail(ctx, HL_E_INVAL, "state buffer holds %zu of %zu bytes", *bytes, need);
    *bytes = need;
    HIPC(ctx, hipSetDevice(ctx->device));
    if ((rc = ensure_stats(ctx)) != HL_OK) return rc;  // the saved means and values are those of step t
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    char *p = (char *)buf;
    StateHeader h{};
    std::memcpy(h.magic, "HLSTATE", 8);
    h.version = 1;
    h.precision = ctx->precision | (ctx->aa ? 0x100 : 0);
    h.N = ctx->L.N;
    h.Nio = ctx->L.Nio;
    h.n_io = (int64_t)ctx->L.hio.size();
    h.bytes = (int64_t)need;
    std::memcpy(p, &h, sizeof h);
    p += sizeof h;
    const size_t S = store_bytes(ctx->precision), A = arith_bytes(ctx->precision), nio = ctx->L.hio.size();
    HIPC(ctx, hipMemcpy(p, ctx->d_ctrl, sizeof(hl::Ctrl), hipMemcpyDeviceToHost));
    p += sizeof(hl::Ctrl);
    for (int k = 0; k < (ctx->aa ? 1 : 2); ++k) {
        HIPC(ctx, hipMemcpy(p, ctx->lat[k], (size_t)Q * ctx->L.Npad * S, hipMemcpyDeviceToHost));
        p += (size_t)Q * ctx->L.Npad * S;
    }
    for (int k = 0; k < 2; ++k) {
        if (ctx->L.Nio) HIPC(ctx, hipMemcpy(p, ctx->d_up[k], (size_t)3 * ctx->L.Nio * A, hipMemcpyDeviceToHost));
        p += (size_t)3 * ctx->L.Nio * A;
    }
    if (nio) {
        HIPC(ctx, hipMemcpy(p, ctx->d_stats, 2 * nio * 8, hipMemcpyDeviceToHost));
        HIPC(ctx, hipMemcpy(p + 2 * nio * 8, ctx->d_bc, 2 * nio * 8, hipMemcpyDeviceToHost));
        HIPC(ctx, hipMemcpy(p + 4 * nio * 8, ctx->d_held, nio * 8, hipMemcpyDeviceToHost));
    }
    return HL_OK;
}

int hl_set_state(hl_ctx *ctx, const void *buf, size_t bytes) {
    if (!ctx || !buf) return HL_E_INVAL;
    int rc = commit(ctx);
    if (rc) return rc;
    const size_t need = state_bytes(ctx);
    StateHeader h;
    if (bytes < sizeof h) return fail(ctx, HL_E_INVAL, "state too short");
    std::memcpy(&h, buf, sizeof h);
    if (std::memcmp(h.magic, "HLSTATE", 8) != 0 || h.version != 1)
        return fail(ctx, HL_E_INVAL, "not a state buffer of this library version");
    if (bytes != need || h.bytes != (int64_t)need || h.precision != (ctx->precision | (ctx->aa ? 0x100 : 0)) ||
        h.N != ctx->L.N ||
        h.Nio != ctx->L.Nio || h.n_io != (int64_t)ctx->L.hio.size())
        return fail(ctx, HL_E_INVAL, "state layout does not match this context");
    HIPC(ctx, hipSetDevice(ctx->device));
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    const char *p = (const char *)buf + sizeof h;
    const size_t S = store_bytes(ctx->precision), A = arith_bytes(ctx->precision), nio = ctx->L.hio.size();
    hl::Ctrl ctrl;
    std::memcpy(&ctrl, p, sizeof ctrl);
    HIPC(ctx, hipMemcpy(ctx->d_ctrl, &ctrl, sizeof ctrl, hipMemcpyHostToDevice));
    p += sizeof(hl::Ctrl);
    for (int k = 0; k < (ctx->aa ? 1 : 2); ++k) {
        HIPC(ctx, hipMemcpy(ctx->lat[k], p, (size_t)Q * ctx->L.Npad * S, hipMemcpyHostToDevice));
        p += (size_t)Q * ctx->L.Npad * S;
    }
    for (int k = 0; k < 2; ++k) {
        if (ctx->L.Nio) HIPC(ctx, hipMemcpy(ctx->d_up[k], p, (size_t)3 * ctx->L.Nio * A, hipMemcpyHostToDevice));
        p += (size_t)3 * ctx->L.Nio * A;
    }
    if (nio) {
        HIPC(ctx, hipMemcpy(ctx->d_stats, p, 2 * nio * 8, hipMemcpyHostToDevice));
        HIPC(ctx, hipMemcpy(ctx->d_bc, p + 2 * nio * 8, 2 * nio * 8, hipMemcpyHostToDevice));
        HIPC(ctx, hipMemcpy(ctx->d_held, p + 4 * nio * 8, nio * 8, hipMemcpyHostToDevice));
    }
    ctx->t_host = ctrl.t;
    *ctx->h_nan = ctrl.nan_flag;
    ctx->obs_t = -1;
    ctx->stats_t = ctx->t_host;
    return HL_OK;
}

int hl_get_schedule(hl_ctx *ctx, int32_t *block_size, int32_t *flags) {
    if (!ctx || !block_size || !flags) return HL_E_INVAL;
    *block_size = ctx->block;
    *flags = ctx->sched_flags;
    return HL_OK;
}

int hl_set_schedule(hl_ctx *ctx, int32_t block_size, int32_t flags) {
    if (!ctx) return HL_E_INVAL;
    if (block_size != 64 && block_size != 128 && block_size != 256)
        return fail(ctx, HL_E_INVAL, "block size %d not in {64, 128, 256}", block_size);
    if (flags & ~(int32_t)(HL_SCHED_XCD_REMAP | HL_SCHED_FUSED | HL_SCHED_PAIRS | HL_SCHED_XCD_RUNS |
                           HL_SCHED_XCD_BRICKS))
        return fail(ctx, HL_E_INVAL, "unknown schedule flags");
    if ((flags & HL_SCHED_XCD_RUNS) && !(flags & HL_SCHED_XCD_REMAP))
        return fail(ctx, HL_E_INVAL, "HL_SCHED_XCD_RUNS needs HL_SCHED_XCD_REMAP");
    if ((flags & HL_SCHED_XCD_BRICKS) &&
        (!(flags & HL_SCHED_FUSED) || (flags & (HL_SCHED_XCD_REMAP | HL_SCHED_XCD_RUNS)) ||
         !(ctx->order_flags & HL_ORDER_BRICK)))
        return fail(ctx, HL_E_INVAL, "HL_SCHED_XCD_BRICKS needs HL_SCHED_FUSED alone and a brick layout");
    const bool rebuild = block_size != ctx->block ||
                         ((flags ^ ctx->sched_flags) & (HL_SCHED_FUSED | HL_SCHED_XCD_BRICKS | HL_SCHED_PAIRS));
    ctx->block = block_size;
    ctx->sched_flags = flags;
    if (!ctx->committed) return HL_OK;
    HIPC(ctx, hipSetDevice(ctx->device));
    int rc;
    if (rebuild && (rc = ensure_stats(ctx)) != HL_OK) return rc;  // from the partials about to be replaced
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    if (rebuild) {
        hl::plan_schedule(ctx->L, ctx->block, ctx->sched_flags, pairs_supported(ctx));
        return upload_schedule(ctx);
    }
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    ctx->gexec = nullptr;
    ctx->graph_steps = 0;
    return HL_OK;
}

int hl_autotune(hl_ctx *ctx, int budget_ms) {
    if (!ctx) return HL_E_INVAL;
    if (budget_ms < 1) return fail(ctx, HL_E_INVAL, "budget must be positive");
    int rc = commit(ctx);
    if (rc) return rc;
    HIPC(ctx, hipSetDevice(ctx->device));
    size_t bytes = 0;
    if ((rc = hl_get_state(ctx, nullptr, &bytes)) != HL_OK) return rc;
    std::vector<char> saved(bytes);
    if ((rc = hl_get_state(ctx, saved.data(), &bytes)) != HL_OK) return rc;
    // On every exit the caller's drive comes back, the events go away and,
    // unless a schedule was chosen, the caller's schedule and dynamic state
    // are restored (a failing trial leaves nothing behind).
    struct Guard {
        hl_ctx *c;
        int drive, block, flags;
        const std::vector<char> *state;
        bool done = false;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Guard() {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            c->drive = drive;
            if (!done) {
                const std::string err = c->err;  // keep the message of the failure
                (void)hl_set_schedule(c, block, flags);
                (void)hl_set_state(c, state->data(), state->size());
                c->err = err;
            }
        }
    } guard{ctx, ctx->drive, ctx->block, ctx->sched_flags, &saved};
    ctx->drive = HL_DRIVE_LAUNCH;
    struct Cand { int block, flags; double ms; };
    std::vector<Cand> cands;
    const bool pairs_ok = pairs_supported(ctx);
    const bool bricks = (ctx->order_flags & HL_ORDER_BRICK) != 0;
    const int R1 = (int)HL_SCHED_XCD_REMAP, RR = (int)(HL_SCHED_XCD_REMAP | HL_SCHED_XCD_RUNS);
    const int F = (int)HL_SCHED_FUSED, P = (int)HL_SCHED_PAIRS, B = (int)HL_SCHED_XCD_BRICKS;
    for (int b : {64, 128, 256}) {
        for (int f : {0, R1, RR, F, F | R1, F | RR, P, P | R1, P | RR, F | P | RR})
            if (pairs_ok || !(f & HL_SCHED_PAIRS)) cands.push_back({b, f, 0.0});
        if (bricks) cands.push_back({b, F | B, 0.0});
        if (bricks && pairs_ok) cands.push_back({b, F | P | B, 0.0});
    }
    HIPC(ctx, hipEventCreate(&guard.e0));
    HIPC(ctx, hipEventCreate(&guard.e1));
    hipEvent_t e0 = guard.e0, e1 = guard.e1;
    auto time_steps = [&](int64_t n, double *ms_per_step) -> int {
        int r;
        if ((r = run_steps(ctx, 1)) != HL_OK) return r;
        HIPC(ctx, hipEventRecord(e0, ctx->stream));
        if ((r = run_steps(ctx, n)) != HL_OK) return r;
        HIPC(ctx, hipEventRecord(e1, ctx->stream));
        HIPC(ctx, hipEventSynchronize(e1));
        float ms = 0.0f;
        HIPC(ctx, hipEventElapsedTime(&ms, e0, e1));
        *ms_per_step = (double)ms / (double)n;
        return HL_OK;
    };
    // steps per trial from two timed steps of the current schedule: 60 % of
    // the budget for one trial of every candidate, 40 % for five more trials
    // of the three fastest
    constexpr int REPEAT = 5, TOP = 3;
    int64_t reps = 2;
    {
        double per = 0.0;
        if ((rc = time_steps(2, &per)) != HL_OK) return rc;
        per = std::max(1e-3, per);
        const double trials = (double)cands.size() / 0.6;
        reps = std::max<int64_t>(2, (int64_t)((double)budget_ms / (per * trials)));
        reps = std::min<int64_t>(reps, 200);
    }
    for (auto &cd : cands) {
        if ((rc = hl_set_schedule(ctx, cd.block, cd.flags)) != HL_OK) return rc;
        if ((rc = time_steps(reps, &cd.ms)) != HL_OK) return rc;
    }
    std::vector<Cand> top = cands;
    std::sort(top.begin(), top.end(), [](const Cand &x, const Cand &y) { return x.ms < y.ms; });
    top.resize(std::min<size_t>(top.size(), TOP));
    std::vector<std::vector<double>> runs(top.size());
    for (int r = 0; r < REPEAT; ++r)
        for (size_t k = 0; k < top.size(); ++k) {  // interleaved, so a slow spell hits all three
            if ((rc = hl_set_schedule(ctx, top[k].block, top[k].flags)) != HL_OK) return rc;
            double ms = 0.0;
            if ((rc = time_steps(reps, &ms)) != HL_OK) return rc;
            runs[k].push_back(ms);
        }
    std::vector<double> med(top.size());
    for (size_t k = 0; k < top.size(); ++k) {
        std::vector<double> v = runs[k];
        std::sort(v.begin(), v.end());
        med[k] = v[v.size() / 2];
    }
    size_t best = 0;
    for (size_t k = 1; k < top.size(); ++k)
        if (med[k] < med[best]) best = k;
    if ((rc = hl_set_schedule(ctx, top[best].block, top[best].flags)) != HL_OK) return rc;
    if ((rc = hl_set_state(ctx, saved.data(), saved.size())) != HL_OK) return rc;
    guard.done = true;
    const auto mm = std::minmax_element(runs[best].begin(), runs[best].end());
    ctx->tune_n = (int32_t)cands.size();
    ctx->tune_best = med[best];
    ctx->tune_second = med[best];
    bool second = false;
    for (size_t k = 0; k < top.size(); ++k)
        if (k != best && (!second || med[k] < ctx->tune_second)) {
            ctx->tune_second = med[k];
            second = true;
        }
    ctx->tune_spread = med[best] > 0.0 ? (*mm.second - *mm.first) / med[best] : 0.0;
    return HL_OK;
}

int hl_autotune_report(hl_ctx *ctx, int32_t *n_candidates, double *best_ms, double *runner_up_ms, double *spread) {
    if (!ctx || !n_candidates || !best_ms || !runner_up_ms || !spread) return HL_E_INVAL;
    if (ctx->tune_n == 0) return fail(ctx, HL_E_STATE, "no autotuning has run on this context");
    *n_candidates = ctx->tune_n;
    *best_ms = ctx->tune_best;
    *runner_up_ms = ctx->tune_second;
    *spread = ctx->tune_spread;
    return HL_OK;
}

int hl_coupling_map(int32_t n_out, const double *out_c, int32_t n_in, const double *in_c, int32_t *owner,
                    double *dist) {
    if (n_out < 1 || n_in < 0 || !out_c || (n_in > 0 && (!in_c || !owner || !dist))) return HL_E_INVAL;
    hl::coupling_map(n_out, out_c, n_in, in_c, owner, dist);
    return HL_OK;
}

int hl_velocity_factors(int32_t nv, const double *dp, const double *L, const double *A, double A0, double *v) {
    if (nv < 1 || !dp || !L || !A || !v || !(A0 > 0.0) || !std::isfinite(A0)) return HL_E_INVAL;
    for (int32_t i = 0; i < nv; ++i)
        if (!(dp[i] > 0.0) || !(L[i] > 0.0) || !(A[i] > 0.0) || !std::isfinite(dp[i]) || !std::isfinite(L[i]) ||
            !std::isfinite(A[i]))
            return HL_E_INVAL;
    hl::velocity_factors(nv, dp, L, A, A0, v);
    return HL_OK;
}

int hl_time_kernels(hl_ctx *ctx, int64_t nsteps, double *ms_bulk, double *ms_bnd) {
    if (!ctx || !ms_bulk || !ms_bnd) return HL_E_INVAL;
    if (nsteps < 1 || nsteps > 100000) return fail(ctx, HL_E_INVAL, "nsteps must lie in 1..100000");
    int rc = commit(ctx);
    if (rc) return rc;
    if (*ctx->h_nan) return fail(ctx, HL_E_DIVERGED, "a non-finite density appeared");
    HIPC(ctx, hipSetDevice(ctx->device));
    std::vector<hipEvent_t> ev((size_t)3 * nsteps, nullptr);
    for (auto &e : ev) HIPC(ctx, hipEventCreate(&e));
    hl::KArgs a = make_args(ctx);
    const bool fu = (ctx->sched_flags & HL_SCHED_FUSED) != 0;
    int err = 0;
    auto part = [&](int64_t k, int which) {
        a.dt = (int32_t)k;
        const int odd = (int)((ctx->t_host + k) & 1);
        return ctx->aa ? hl::launch_aa_step(ctx->precision, a, ctx->L.n_bulk_blocks, ctx->L.n_bnd_blocks, ctx->block,
                                            ctx->stream, which, fu, odd)
                       : hl::launch_step(ctx->precision, a, ctx->L.n_bulk_blocks, ctx->L.n_bnd_blocks, ctx->block,
                                         ctx->stream, which, fu);
    };
    for (int64_t k = 0; k < nsteps && !err; ++k) {
        HIPC(ctx, hipEventRecord(ev[3 * k], ctx->stream));
        err = part(k, 1);
        HIPC(ctx, hipEventRecord(ev[3 * k + 1], ctx->stream));
        if (!err) err = part(k, 2);
        HIPC(ctx, hipEventRecord(ev[3 * k + 2], ctx->stream));
        if (!err) err = part(k, 3);
    }
    a.dt = 0;
    if (!err) err = hl::launch_advance(a, nsteps, ctx->stream);
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    double sb = 0.0, sn = 0.0;
    for (int64_t k = 0; k < nsteps; ++k) {
        float m1 = 0.0f, m2 = 0.0f;
        HIPC(ctx, hipEventElapsedTime(&m1, ev[3 * k], ev[3 * k + 1]));
        HIPC(ctx, hipEventElapsedTime(&m2, ev[3 * k + 1], ev[3 * k + 2]));
        sb += m1;
        sn += m2;
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (err) return fail(ctx, HL_E_DEVICE, "step launch failed: %s", hipGetErrorString((hipError_t)err));
    ctx->t_host += nsteps;
    ctx->obs_t = -1;
    ctx->stats_t = ctx->L.hpairs.empty() ? -1 : (ctx->aa ? ctx->t_host - 1 : ctx->t_host);
    *ms_bulk = sb / (double)nsteps;
    *ms_bnd = sn / (double)nsteps;
    return HL_OK;
}

int hl_get_info(hl_ctx *ctx, hl_info *out) {
    if (!ctx || !out) return HL_E_INVAL;
    int rc = commit(ctx);
    if (rc) return rc;
    std::memset(out, 0, sizeof *out);
    out->n_sites = ctx->L.n_sites;
    out->n_bulk = ctx->L.n_bulk_sites;
    out->n_near = ctx->L.n_near_sites;
    out->n_boundary = ctx->L.n_sites - ctx->L.n_bulk_sites;
    out->n_iolet_sites = ctx->L.n_io_sites;
    out->n_domains = (int32_t)ctx->doms.size();
    out->n_iolets = (int32_t)ctx->L.hio.size();
    out->n_blocks_bulk = ctx->L.n_bulk_blocks;
    out->n_blocks_bnd = ctx->L.n_bnd_blocks;
    out->precision = ctx->precision;
    out->block_size = ctx->block;
    out->sched_flags = ctx->sched_flags;
    out->drive = ctx->drive;
    out->device_bytes = ctx->dev_bytes;
    // two-lattice: 19 reads + 19 writes + 18 int32 indices per step; in-place:
    // the same on odd steps, no indices on even steps
    out->bytes_per_site = 2.0 * Q * (double)store_bytes(ctx->precision) + (ctx->aa ? 9.0 : 18.0) * 4.0;
    return HL_OK;
}

}  // extern "C"
