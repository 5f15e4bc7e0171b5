// gfx950 kernels of the sparse D3Q19 LBGK step.
//
// One lane owns one fluid site.  A step t -> t+1 is the fused pull form of
// the stream-and-collide update (Sec. 2 of the paper: D3Q19, single
// relaxation time, rigid walls, velocity and pressure boundaries):
//   1. gather f_j(x, t+1) = f*_j(x - c_j, t) through the pull table (int32
//      indices, or int16 deltas for sites whose neighbours share their brick),
//   2. replace the populations whose upstream voxel is not fluid by the
//      boundary rule of that link (halfway or Bouzidi wall, Ladd velocity
//      inlet, equilibrium pressure outlet),
//   3. take the moments, relax toward the second-order equilibrium with
//      Guo's forcing term, and store f*(t+1) to the other lattice.
// The in-place (AA-pattern) sweeps further below perform the same update on
// a single lattice.
// Work-groups whose sites border an iolet also reduce (in FP64, in a fixed
// order) the mean velocity along the iolet normal and the mean density; a
// one-work-group kernel queued after them turns those means into the
// boundary values of the next step, including the arterial-venous coupling
// of Sec. 2.3 and Sec. 3 (forward on even steps, reverse on odd steps,
// Eq. (1)-(2)).  Stream order alone separates the kernels of a step: no
// device-wide fences or atomics are needed.
//
// The lattice is bandwidth-bound (about 1 flop per byte), so there is no
// matrix-core work here: the design goal is coalesced SoA traffic.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <mutex>
#include <type_traits>

#include "hl_internal.h"

namespace hl {

// Velocity set of the site-list interface (rest, faces, edges; opposite
// directions adjacent).
static constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

template <typename R>
__device__ __forceinline__ constexpr R wgt(int i) {
    return i == 0 ? R(1.0) / R(3.0) : (i <= 6 ? R(1.0) / R(18.0) : R(1.0) / R(36.0));
}

// a / b in the arithmetic type: IEEE division in FP64 (the operation of the
// FP64 reference form); in FP32 a times the hardware reciprocal of b (1 ulp;
// the divisors here, a density near rho0 and 2q in [1, 2], are far from the
// denormal range), which the compiler shares between quotients with the
// same divisor.
__device__ __forceinline__ double over(double a, double b) { return a / b; }
__device__ __forceinline__ float over(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// Storage type -> arithmetic type.  FP64 stores f, FP32/FP16 store offsets.
template <typename T> struct Arith { using R = float; static constexpr bool OFF = true; };
template <> struct Arith<double> { using R = double; static constexpr bool OFF = false; };

// Population storage.  ld/st take the lattice row (direction slot) so that
// the weight-normalised FP16 form can scale by w_row (w_i = w_opp(i), so the
// row alone fixes the weight in both the natural and the swapped layout).
struct h16w {
    __half v;
};
// FP16 offset storage rounded stochastically on every store.
struct h16sr {
    __half v;
};

// Random bits for stochastic rounding, a function of (lattice element, step)
// only, so a run is reproducible bit for bit: C. Wellons' "lowbias32"
// integer hash (hash-prospector, 2018) chained over the step, the high and
// the low half of the element index.
__device__ __forceinline__ uint32_t lowbias32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
template <typename T>
__device__ __forceinline__ uint32_t rkey(size_t idx, int64_t t) {
    if constexpr (std::is_same<T, h16sr>::value)
        return lowbias32((uint32_t)idx ^ lowbias32((uint32_t)(idx >> 32) ^ lowbias32((uint32_t)t)));
    else
        return 0u;
}

// Stochastic rounding to FP16: the value truncated toward zero (lo) or the
// next FP16 value away from zero (hi), hi with probability (v - lo)/(hi - lo),
// so the stored value is unbiased.  v - lo is exact in FP32 and hi - lo is a
// power of two; u is uniform on [0, 1) with 24 bits from r.
__device__ __forceinline__ __half half_sr(float v, uint32_t r) {
    const __half lo = __float2half_rz(v);
    const float flo = __half2float(lo);
    const float rem = fabsf(v - flo);
    const __half hi = __ushort_as_half((unsigned short)(__half_as_ushort(lo) + 1));
    const float ulp = fabsf(__half2float(hi) - flo);
    const float u = (float)(r >> 8) * 0x1p-24f;
    return (rem > 0.0f && u * ulp < rem) ? hi : lo;
}
__device__ __forceinline__ double ldc(const double *p, int) { return *p; }
__device__ __forceinline__ float ldc(const float *p, int) { return *p; }
__device__ __forceinline__ float ldc(const __half *p, int) { return __half2float(*p); }
__device__ __forceinline__ float ldc(const h16w *p, int row) { return __half2float(p->v) * wgt<float>(row); }
__device__ __forceinline__ float ldc(const h16sr *p, int) { return __half2float(p->v); }
// NT: non-temporal store (the two-lattice step writes a lattice it does not
// read, in every storage form); the in-place sweeps store to lines they have
// just read and keep them cached (NT = false).
template <bool NT = true>
__device__ __forceinline__ void stc(double *p, double v, int, uint32_t = 0) {
    if (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}
template <bool NT = true>
__device__ __forceinline__ void stc(float *p, float v, int, uint32_t = 0) {
    if (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}
// FP16 forms: the 16-bit pattern is stored as an unsigned short so that the
// two-lattice step can store it non-temporally as well.
template <bool NT>
__device__ __forceinline__ void st16(void *p, __half h) {
    const unsigned short bits = __half_as_ushort(h);
    if (NT)
        __builtin_nontemporal_store(bits, (unsigned short *)p);
    else
        *(unsigned short *)p = bits;
}
template <bool NT = true>
__device__ __forceinline__ void stc(__half *p, float v, int, uint32_t = 0) { st16<NT>(p, __float2half_rn(v)); }
template <bool NT = true>
__device__ __forceinline__ void stc(h16w *p, float v, int row, uint32_t = 0) {
    st16<NT>(p, __float2half_rn(v * (row == 0 ? 3.0f : (row <= 6 ? 18.0f : 36.0f))));
}
template <bool NT = true>
__device__ __forceinline__ void stc(h16sr *p, float v, int, uint32_t key = 0) { st16<NT>(p, half_sr(v, key)); }

// Lattice element of direction i at site s.  Sites are grouped in tiles of
// TILE consecutive sites; a tile holds its 19 direction rows one after the
// other (tile-major SoA), so a wavefront's accesses to one direction stay a
// contiguous run while all populations of a tile share a few DRAM pages.
__device__ __forceinline__ size_t lidx(int i, int64_t s) {
    return ((((size_t)s >> TILE_SHIFT) * Q + (size_t)i) << TILE_SHIFT) | ((size_t)s & (TILE - 1));
}

// Wall fractions of site s (b = s - NB), one per direction j: q of the wall
// link fed into j when sr[j] == -1 and the walls are Bouzidi walls, read from
// the site's run of the compact list (its wall links in direction order),
// else 1/2.  bz is uniform over the work-group.  The observation and moments
// passes take this path for bulk sites too, where b may be negative: the
// offset is read only for a site with a wall link, which the layout places at
// or above NB.
__device__ __forceinline__ void wall_fractions(const KArgs &a, int64_t b, bool bz, const int32_t (&sr)[Q],
                                               float (&qv)[Q]) {
    bool wall = false;
#pragma unroll
    for (int j = 1; j < Q; ++j) wall = wall || sr[j] == -1;
    const float *qp = a.bq + ((bz && wall) ? a.bq_off[b] : 0u);
    int k = 0;
#pragma unroll
    for (int j = 1; j < Q; ++j) {
        const bool w = bz && sr[j] == -1;
        qv[j] = w ? qp[k] : 0.5f;
        k += w ? 1 : 0;
    }
}

// Entry classes whose sites take the bulk path (every link fluid).
__device__ __forceinline__ bool bulk_class(int klass) { return klass == K_BULK || klass == K_NEAR; }

// Pull indices of a bulk site: from the int16 delta table for a K_NEAR work-
// group (half the index traffic), else from the int32 table.  The class is
// uniform over the work-group, so the branch does not diverge.  Index lines
// are read once per step, so they are loaded non-temporally and leave the L2
// to the lattice lines that neighbouring gathers reuse.
__device__ __forceinline__ void pull_indices(const KArgs &a, int klass, int64_t s, int32_t (&sr)[Q]) {
    const int64_t N = a.N;
    if (klass == K_NEAR) {
#pragma unroll
        for (int j = 1; j < Q; ++j) sr[j] = (int32_t)s + (int32_t)__builtin_nontemporal_load(a.d16 + (size_t)(j - 1) * N + s);
    } else {
#pragma unroll
        for (int j = 1; j < Q; ++j) sr[j] = __builtin_nontemporal_load(a.src + (size_t)(j - 1) * N + s);
    }
}

// Pull indices of a boundary site (-1 for a wall link, -2-g for iolet g): from
// the int16 delta table for a K_NEARWALL work-group (INT16_MIN marks a wall
// link), else from the int32 table.
__device__ __forceinline__ void boundary_indices(const KArgs &a, int klass, int64_t s, int32_t (&sr)[Q]) {
    const int64_t N = a.N;
    if (klass == K_NEARWALL) {
#pragma unroll
        for (int j = 1; j < Q; ++j) {
            const int d = __builtin_nontemporal_load(a.d16 + (size_t)(j - 1) * N + s);
            sr[j] = (d == -32768) ? -1 : (int32_t)s + d;
        }
    } else {
#pragma unroll
        for (int j = 1; j < Q; ++j) sr[j] = __builtin_nontemporal_load(a.src + (size_t)(j - 1) * N + s);
    }
}

template <typename T>
__device__ __forceinline__ const T *lat_ptr(const KArgs &a, int64_t parity) {
    return (const T *)((parity & 1) ? a.lat1 : a.lat0);
}

// XCD-aware order: work-group b runs on XCD b % 8.  xcd_remap 1: each XCD
// takes one contiguous eighth of the entries; xcd_remap = C > 1: runs of C
// consecutive entries go to the XCDs in turn (entries past the last whole
// round keep their place), so neighbouring sites share an L2 while the XCDs
// sweep the site list together.
__device__ __forceinline__ int block_index(int xcd_remap) {
    const int b = blockIdx.x;
    if (!xcd_remap) return b;
    const int G = gridDim.x;
    const int x = b & 7, k = b >> 3;
    if (xcd_remap == 1) {
        const int per = G >> 3, rem = G & 7;
        return x * per + (x < rem ? x : rem) + k;
    }
    const int C = xcd_remap;
    const int G8 = G / (8 * C) * (8 * C);
    if (b >= G8) return b;
    return ((k / C) * 8 + x) * C + (k % C);
}

// Entry of this work-group: from the brick-aligned XCD map when the host
// built one (negative: no work), else through block_index.
__device__ __forceinline__ int entry_index(const KArgs &a) {
    if (a.emap) return a.emap[blockIdx.x];
    return a.e_off + block_index(a.xcd_remap);
}

// Step of a launch: the stored counter plus the launch's offset in its batch
// (the counter is advanced once per batch).
__device__ __forceinline__ int64_t step_time(const KArgs &a) { return a.ctrl->t + a.dt; }

// ---------------------------------------------------------------------------
// Step 1-2: the populations f_j(x, p+1) of site s, streamed from f*(p).
// BND selects the boundary path (pull codes may be negative).
// ---------------------------------------------------------------------------
template <typename T, bool BND>
__device__ __forceinline__ void gather(const KArgs &a, const Entry &e, const SegDev &sg, int64_t p,
                                       int64_t s, typename Arith<T>::R (&x)[Q]) {
    using R = typename Arith<T>::R;
    constexpr bool OFF = Arith<T>::OFF;
    const T *__restrict__ lin = lat_ptr<T>(a, p);
    int32_t sr[Q];
    if (BND)
        boundary_indices(a, tag_class(e.tag), s, sr);
    else
        pull_indices(a, tag_class(e.tag), s, sr);
    x[0] = ldc(lin + lidx(0, s), 0);
#pragma unroll
    for (int j = 1; j < Q; ++j) {
        if (BND)
            x[j] = (sr[j] >= 0) ? ldc(lin + lidx(j, sr[j]), j) : R(0);
        else
            x[j] = ldc(lin + lidx(j, sr[j]), j);
    }
    if (!BND) return;

    const int64_t b = s - a.NB;
    const int klass = tag_class(e.tag);
    int kind = KIND_INLET;
    R U = 0, nx = 0, ny = 0, nz = 0, phi = 0;
    R rho_out = 0, drho_out = 0, ux = 0, uy = 0, uz = 0;
    if (klass == K_IOLET) {
        const int g = tag_iolet(e.tag);
        const IoletDev &io = a.io[g];
        kind = io.kind;
        const double v = a.bc[(p & 1) * a.n_io + g];
        if (kind == KIND_INLET) {
            U = (R)v;
            nx = (R)io.nrm[0];
            ny = (R)io.nrm[1];
            nz = (R)io.nrm[2];
            phi = (R)a.bphi[b];
        } else {
            rho_out = (R)v;
            drho_out = (R)(v - RHO0);
            const R *up = (const R *)((p & 1) ? a.up1 : a.up0);
            const int64_t vi = s - a.IO0;
            ux = up[vi];
            uy = up[a.Nio + vi];
            uz = up[2 * a.Nio + vi];
        }
    }
    // Phase 1: issue every load the boundary rules need before using any of
    // them, so the memory latencies overlap instead of queueing behind the
    // per-direction branches.
    const bool bz = sg.wall_mode == WALL_BOUZIDI;
    const bool outlet = klass == K_IOLET && kind == KIND_OUTLET;
    R own[Q];  // f*_i(s) where a rule reads it
    float qv[Q];  // wall fraction of the wall link fed into direction j (stored as float)
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int ib = opp(i);
        // f*_i(s) feeds direction ib (bounce-back, Bouzidi, inlet) and, for a
        // Bouzidi wall link, direction i itself (q >= 1/2)
        const bool need = (sr[ib] == -1) || (sr[ib] <= -2 && !outlet) || (bz && sr[i] == -1);
        own[i] = need ? ldc(lin + lidx(i, s), i) : R(0);
    }
    wall_fractions(a, b, bz, sr, qv);
    // Phase 2: the boundary rules, from registers only.
#pragma unroll
    for (int j = 1; j < Q; ++j) {
        if (sr[j] >= 0) continue;
        const int jb = opp(j);
        if (sr[j] == -1) {
            // wall link (s, jb): the wall lies at x_s + q c_jb
            if (bz) {
                const R q = (R)qv[j];
                if (q < R(0.5)) {
                    // second node x_s - c_jb = x_s + c_j, pulled as x[jb]
                    x[j] = (sr[jb] >= 0) ? R(2) * q * own[jb] + (R(1) - R(2) * q) * x[jb] : own[jb];
                } else {
                    x[j] = over(own[jb], R(2) * q) + (R(1) - over(R(1), R(2) * q)) * own[j];
                }
            } else {
                x[j] = own[jb];
            }
        } else if (kind == KIND_INLET) {
            // Ladd: f_j = f*_jb - 6 w rho0 (c_jb . u_w), u_w = U phi n
            const R cn = R(CX[jb]) * nx + R(CY[jb]) * ny + R(CZ[jb]) * nz;
            x[j] = own[jb] - R(6) * wgt<R>(j) * R(RHO0) * (cn * (U * phi));
        } else {
            // pressure outlet: equilibrium at rho_out and the site's velocity
            const R cu = R(CX[j]) * ux + R(CY[j]) * uy + R(CZ[j]) * uz;
            const R uu = ux * ux + uy * uy + uz * uz;
            const R poly = R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu;
            if (OFF)
                x[j] = wgt<R>(j) * (drho_out + rho_out * poly);
            else
                x[j] = wgt<R>(j) * rho_out * (R(1) + poly);
        }
    }
}

// Deterministic FP64 sum over the work-group; the result is valid in lane 0
// of wave 0.
__device__ __forceinline__ double block_sum(double v, double *lds) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) r += lds[w];
    }
    __syncthreads();
    return r;
}

__device__ double series_at(const IoletDev &io, int64_t t) {
    double v = io.a0;
    for (int m = 1; m <= io.nh; ++m) {
        const double ph = 2.0 * M_PI * (double)m * (double)t / io.period;
        v = v + io.a[m - 1] * cos(ph) + io.b[m - 1] * sin(ph);
    }
    return v;
}

// Boundary values of the iolets without coupling for the stream tn -> tn+1,
// written by the first work-group of a step's boundary (or fused) launch.
// The launch itself reads the other parity, so the write races with nothing.
__device__ __forceinline__ void publish_series(const KArgs &a, int64_t tn) {
    if (blockIdx.x != 0) return;
    for (int k = threadIdx.x; k < a.n_io; k += blockDim.x) {
        const IoletDev &io = a.io[k];
        if (!io.coupled) a.bc[(tn & 1) * a.n_io + k] = series_at(io, tn);
    }
}

// One work-group after the site kernels of a step (stream order, no
// fences): iolet means of f(tn) from the per-work-group partial sums,
// coupling, boundary values for the stream tn -> tn+1.  t is the launch's
// step (stored counter + dt); the stored counter itself is advanced by
// k_advance once per batch.  Contexts without coupling run it only on demand
// (their steps publish the boundary series themselves).
// mode: FIN_STEP (two-lattice step: f(t+1) was reduced; tn = t+1),
// FIN_RAW (two-lattice reinitialisation: f(t) reduced; tn = t; direct := 1),
// FIN_AA_SWEEP (in-place sweep: f(t) reduced; tn = t),
// FIN_AA_MOMENTS (moments-only pass: f(t) reduced; tn = t),
// FIN_STATS (two lattices, on demand: the last step reduced f(t); tn = t).
enum { FIN_STEP = 0, FIN_RAW = 1, FIN_AA_SWEEP = 2, FIN_AA_MOMENTS = 3, FIN_STATS = 4 };

// Partial sums staged per pass of the iolet sums (16 B each).
constexpr int FIN_CHUNK = 2048;

__global__ void __launch_bounds__(256) k_finalize(KArgs a, int mode) {
    __shared__ double2 stage[FIN_CHUNK];
    const int64_t t = step_time(a);
    const int64_t tn = (mode == FIN_STEP) ? t + 1 : t;
    double *mu = a.stats;
    double *mr = a.stats + a.n_io;
    // Iolet sums over the per-work-group partials.  The partials of the span
    // of iolet entries pass through LDS in coalesced chunks; each thread adds
    // its iolets' entries from left to right (between chunks the running
    // sums wait in mu/mr), so the order is that of a plain sequential sum.
    // An iolet's mean, and its next boundary value when it is not coupled,
    // are final as soon as its sums are; coupled values follow the exchange.
    const int nchunk = (a.io_e1 - a.io_e0 + FIN_CHUNK - 1) / FIN_CHUNK;
    for (int c = 0; c < max(nchunk, 1); ++c) {
        const int c0 = a.io_e0 + c * FIN_CHUNK, c1 = min(c0 + FIN_CHUNK, a.io_e1);
        if (c > 0) __syncthreads();
        for (int e = c0 + (int)threadIdx.x; e < c1; e += blockDim.x)
            stage[e - c0] = make_double2(a.partials[2 * e], a.partials[2 * e + 1]);
        __syncthreads();
        const bool last = c + 1 >= nchunk;
        for (int k = threadIdx.x; k < a.n_io; k += blockDim.x) {
            const IoletDev &io = a.io[k];
            const int lo = max(io.e_lo, c0), hi = min(io.e_hi, c1);
            double su = (c > 0) ? mu[k] : 0.0, sr = (c > 0) ? mr[k] : 0.0;
            for (int e = lo; e < hi; ++e) {
                su = su + stage[e - c0].x;
                sr = sr + stage[e - c0].y;
            }
            if (!last) {
                mu[k] = su;
                mr[k] = sr;
                continue;
            }
            mu[k] = io.area > 0.0 ? su / io.area : 0.0;
            mr[k] = io.area > 0.0 ? sr / io.area : 0.0;  // mean of rho - rho0
            if (!isfinite(su) || !isfinite(sr)) a.ctrl->nan_flag = 1;
            if (!io.coupled) a.bc[(tn & 1) * a.n_io + k] = series_at(io, tn);
        }
    }
    if (a.n_pairs > 0) {
        __syncthreads();
        const bool fwd = (a.couple_mode & COUPLE_BOTH) || (tn % 2 == 0);
        const bool rev = (a.couple_mode & COUPLE_BOTH) || (tn % 2 == 1);
        if (fwd) {
            for (int p = threadIdx.x; p < a.n_pairs; p += blockDim.x) {
                const PairDev pr = a.pairs[p];
                const double pb = a.io[pr.in_g].phibar;
                a.held[pr.in_g] = pb > 0.0 ? pr.s * mu[pr.out_g] / pb : 0.0;
            }
        }
        if (rev) {
            for (int k = threadIdx.x; k < a.n_io; k += blockDim.x) {
                const IoletDev &io = a.io[k];
                if (io.pair_n == 0) continue;
                double sum = 0.0;
                if (a.couple_mode & COUPLE_VEL) {
                    // velocity-driven outlet: the mean over its veins of
                    // mean_u(vein) / s, imposed as a peak of that over phibar
                    for (int p = io.pair_lo; p < io.pair_lo + io.pair_n; ++p) {
                        const PairDev pr = a.pairs[p];
                        sum = sum + mu[pr.in_g] / pr.s;
                    }
                    a.held[k] = io.phibar > 0.0 ? (sum / (double)io.pair_n) / io.phibar : 0.0;
                } else {
                    for (int p = io.pair_lo; p < io.pair_lo + io.pair_n; ++p) {
                        const PairDev pr = a.pairs[p];
                        const double pv = mr[pr.in_g] / 3.0;
                        sum = sum + pv / (1.0 - pr.delta);
                    }
                    a.held[k] = RHO0 + 3.0 * (sum / (double)io.pair_n);
                }
            }
        }
        __syncthreads();
        for (int k = threadIdx.x; k < a.n_io; k += blockDim.x)
            if (a.io[k].coupled) a.bc[(tn & 1) * a.n_io + k] = a.held[k];
    }
    if (mode == FIN_RAW && threadIdx.x == 0) a.ctrl->direct = 1;
}

// The stored step counter after a batch of n steps; a reloaded lattice is no
// longer the raw state.
__global__ void k_advance(KArgs a, int64_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        a.ctrl->t += n;
        a.ctrl->direct = 0;
    }
}

// Moments and LBGK collision with Guo forcing for one site: x holds f(t)
// (or its offset) on entry and f*(t) on exit; returns true when the density
// is not finite.
template <typename R, bool OFF>
__device__ __forceinline__ bool collide_site(R (&x)[Q], const SegDev &sg, R Fx, R Fy, R Fz) {
    R m0 = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        m0 += x[i];
        if (CX[i]) jx += R(CX[i]) * x[i];
        if (CY[i]) jy += R(CY[i]) * x[i];
        if (CZ[i]) jz += R(CZ[i]) * x[i];
    }
    R rho, drho = 0;
    if (OFF) {
        drho = m0;
        rho = R(RHO0) + drho;
    } else {
        rho = m0;
    }
    const R ux = over(jx + R(0.5) * Fx, rho);
    const R uy = over(jy + R(0.5) * Fy, rho);
    const R uz = over(jz + R(0.5) * Fz, rho);
    const R it = (R)sg.inv_tau;
    const R uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const R cu = R(CX[i]) * ux + R(CY[i]) * uy + R(CZ[i]) * uz;
        const R poly = R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu;
        const R eq = OFF ? wgt<R>(i) * (drho + rho * poly) : wgt<R>(i) * rho * (R(1) + poly);
        R o = x[i] - (x[i] - eq) * it;
        if (sg.has_force) {
            const R sF = (R(3) * (R(CX[i]) - ux) + R(9) * cu * R(CX[i])) * Fx +
                         (R(3) * (R(CY[i]) - uy) + R(9) * cu * R(CY[i])) * Fy +
                         (R(3) * (R(CZ[i]) - uz) + R(9) * cu * R(CZ[i])) * Fz;
            o += (R)sg.guo_pref * wgt<R>(i) * sF;
        }
        x[i] = o;
    }
    return !isfinite(rho);
}

// M_FUSEDP: the fused launch whose bulk entries take two adjacent sites per lane
enum { M_BULK = 0, M_BND = 1, M_RAW = 2, M_FUSED = 3, M_FUSEDP = 4 };

// Storage forms with a two-sites-per-lane bulk path (the weight-normalised and
// stochastic FP16 forms store through their own conversions).
template <typename T>
constexpr bool pair_ok() {
    return std::is_same<T, double>::value || std::is_same<T, float>::value || std::is_same<T, __half>::value;
}
template <typename T>
__device__ __forceinline__ void pair_sites(const KArgs &a, const Entry &e);

// ---------------------------------------------------------------------------
// The step kernel.  M_BULK / M_BND: pull step t -> t+1 over bulk or boundary
// entries.  M_RAW: collide the raw f(t) held in lat[(t+1)&1] into lat[t&1]
// (initialisation and population loads), without advancing t.
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__device__ __forceinline__ void step_body(const KArgs &a) {
    using R = typename Arith<T>::R;
    constexpr bool OFF = Arith<T>::OFF;
    __shared__ double lds[8];
    const int64_t t = step_time(a);
    const int64_t tn = (MODE == M_RAW) ? t : t + 1;
    if constexpr (MODE == M_BND || MODE == M_FUSED || MODE == M_FUSEDP) publish_series(a, tn);
    const int eidx = entry_index(a);
    if (eidx < 0) return;  // uniform over the work-group
    const Entry e = a.entries[eidx];
    const int klass = tag_class(e.tag);
    if constexpr (MODE == M_FUSEDP) {
        // bulk entries of up to two work-groups' sites, two adjacent sites per lane
        if (bulk_class(klass)) {
            pair_sites<T>(a, e);
            return;
        }
    }
    const SegDev &sg = a.seg[e.seg];
    // one site per lane; the initialisation pass over a bulk entry of the
    // two-sites-per-lane schedule (up to 2 x blockDim sites) takes two rounds
    const int rounds = (MODE == M_RAW) ? (e.count + (int)blockDim.x - 1) / (int)blockDim.x : 1;
    for (int round = 0; round < rounds; ++round) {
    const int tid = (int)threadIdx.x + round * (int)blockDim.x;
    const bool act = tid < e.count;
    const int64_t s = (int64_t)e.start + tid;

    R x[Q];
    if (act) {
        if (MODE == M_RAW) {
            const T *__restrict__ raw = lat_ptr<T>(a, t + 1);
#pragma unroll
            for (int i = 0; i < Q; ++i) x[i] = ldc(raw + lidx(i, s), i);
        } else if (MODE == M_FUSED || MODE == M_FUSEDP) {
            if (bulk_class(klass))
                gather<T, false>(a, e, sg, t, s, x);
            else
                gather<T, true>(a, e, sg, t, s, x);
        } else {
            gather<T, MODE == M_BND>(a, e, sg, t, s, x);
        }
    }

    // moments of f(tn)
    R Fx = 0, Fy = 0, Fz = 0;
    if (sg.has_force) {
        const double c = cos(sg.omega * (double)tn);
        Fx = (R)(sg.F0[0] * c);
        Fy = (R)(sg.F0[1] * c);
        Fz = (R)(sg.F0[2] * c);
    }
    R rho = 0, drho = 0, ux = 0, uy = 0, uz = 0;
    bool bad = false;
    if (act) {
        R m0 = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            m0 += x[i];
            if (CX[i]) jx += R(CX[i]) * x[i];
            if (CY[i]) jy += R(CY[i]) * x[i];
            if (CZ[i]) jz += R(CZ[i]) * x[i];
        }
        if (OFF) {
            drho = m0;
            rho = R(RHO0) + drho;
        } else {
            rho = m0;
        }
        ux = over(jx + R(0.5) * Fx, rho);
        uy = over(jy + R(0.5) * Fy, rho);
        uz = over(jz + R(0.5) * Fz, rho);
        bad = !isfinite(rho);

        if (klass == K_IOLET) {
            R *up = (R *)((tn & 1) ? a.up1 : a.up0);
            const int64_t vi = s - a.IO0;
            up[vi] = ux;
            up[a.Nio + vi] = uy;
            up[2 * a.Nio + vi] = uz;
        }

        // LBGK collision with Guo forcing
        const R it = (R)sg.inv_tau;
        const R uu = ux * ux + uy * uy + uz * uz;
        T *__restrict__ lout = (T *)((tn & 1) ? a.lat1 : a.lat0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const R cu = R(CX[i]) * ux + R(CY[i]) * uy + R(CZ[i]) * uz;
            const R poly = R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu;
            const R eq = OFF ? wgt<R>(i) * (drho + rho * poly) : wgt<R>(i) * rho * (R(1) + poly);
            R o = x[i] - (x[i] - eq) * it;
            if (sg.has_force) {
                const R sF = (R(3) * (R(CX[i]) - ux) + R(9) * cu * R(CX[i])) * Fx +
                             (R(3) * (R(CY[i]) - uy) + R(9) * cu * R(CY[i])) * Fy +
                             (R(3) * (R(CZ[i]) - uz) + R(9) * cu * R(CZ[i])) * Fz;
                o += (R)sg.guo_pref * wgt<R>(i) * sF;
            }
            stc(lout + lidx(i, s), o, i, rkey<T>(lidx(i, s), tn));
        }
    }
    if (__ballot(bad) != 0 && (threadIdx.x & 63) == 0) a.ctrl->nan_flag = 1;

    if (klass == K_IOLET) {
        const IoletDev &io = a.io[tag_iolet(e.tag)];
        double un = 0.0, rh = 0.0;  // u.n and rho - rho0 (summed as deviations: no cancellation)
        if (act) {
            un = (double)ux * io.nrm[0] + (double)uy * io.nrm[1] + (double)uz * io.nrm[2];
            rh = OFF ? (double)drho : (double)rho - RHO0;
        }
        const double su = block_sum(un, lds);
        const double sr = block_sum(rh, lds);
        if (threadIdx.x == 0) {
            a.partials[2 * eidx] = su;
            a.partials[2 * eidx + 1] = sr;
        }
    }
    }  // rounds
}

template <typename T, int MODE>
__global__ void __launch_bounds__(256) k_step(KArgs a) {
    step_body<T, MODE>(a);
}

// ---------------------------------------------------------------------------
// Bulk sites, two adjacent sites per lane.  Range starts and N are whole
// tiles (even), so the pull indices, the rest population and the stores of a
// lane move as aligned 2-element vectors; a gather moves as one vector (4-byte
// alignment, so the compiler splits it where the target needs that) when the
// two sources are adjacent in one tile, else as two loads.  Same arithmetic
// as the one-site kernel.
// ---------------------------------------------------------------------------
template <typename T> struct Vec2;
template <> struct Vec2<double> { typedef double elem; typedef double type __attribute__((ext_vector_type(2))); };
template <> struct Vec2<float> { typedef float elem; typedef float type __attribute__((ext_vector_type(2))); };
template <> struct Vec2<__half> { typedef _Float16 elem; typedef _Float16 type __attribute__((ext_vector_type(2))); };
typedef int32_t int2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double cvt(double v) { return v; }
__device__ __forceinline__ float cvt(float v) { return v; }
__device__ __forceinline__ float cvt(_Float16 v) { return (float)v; }

template <typename T>
__device__ __forceinline__ void pair_sites(const KArgs &a, const Entry &e) {
    using R = typename Arith<T>::R;
    using V2 = typename Vec2<T>::type;
    using E = typename Vec2<T>::elem;
    constexpr bool OFF = Arith<T>::OFF;
    const int64_t t = step_time(a);
    const int64_t tn = t + 1;
    const SegDev &sg = a.seg[e.seg];
    const int base = 2 * (int)threadIdx.x;
    if (base >= e.count) return;
    const bool two = base + 1 < e.count;
    const int64_t s = (int64_t)e.start + base;
    const int64_t N = a.N;
    const T *__restrict__ lin = lat_ptr<T>(a, t);
    T *__restrict__ lout = (T *)((tn & 1) ? a.lat1 : a.lat0);

    R x0[Q], x1[Q];
    if (two) {
        const V2 v = *(const V2 *)(lin + lidx(0, s));  // s even: s, s+1 share a tile
        x0[0] = cvt(v.x);
        x1[0] = cvt(v.y);
    } else {
        x0[0] = ldc(lin + lidx(0, s), 0);
        x1[0] = R(0);
    }
    const bool near = tag_class(e.tag) == K_NEAR;
#pragma unroll
    for (int j = 1; j < Q; ++j) {
        const int32_t *sp = a.src + (size_t)(j - 1) * N + s;
        const int16_t *dp = near ? a.d16 + (size_t)(j - 1) * N + s : nullptr;
        if (two) {
            int2v sv;
            if (near) {
                // the two int16 deltas of sites s, s+1 as one aligned dword (s and N even)
                const uint32_t pk = *(const uint32_t *)dp;
                sv.x = (int32_t)s + (int32_t)(int16_t)(uint16_t)(pk & 0xffffu);
                sv.y = (int32_t)s + 1 + (int32_t)(int16_t)(uint16_t)(pk >> 16);
            } else {
                sv = *(const int2v *)sp;
            }
            if (sv.y == sv.x + 1 && (sv.x & (TILE - 1)) != TILE - 1) {
                // adjacent sources in one tile: one vector load
                V2 v;
                __builtin_memcpy(&v, lin + lidx(j, sv.x), sizeof(V2));
                x0[j] = cvt(v.x);
                x1[j] = cvt(v.y);
            } else {
                x0[j] = ldc(lin + lidx(j, sv.x), j);
                x1[j] = ldc(lin + lidx(j, sv.y), j);
            }
        } else {
            x0[j] = ldc(lin + lidx(j, near ? (int32_t)s + (int32_t)dp[0] : sp[0]), j);
            x1[j] = R(0);
        }
    }
    R Fx = 0, Fy = 0, Fz = 0;
    if (sg.has_force) {
        const double c = cos(sg.omega * (double)tn);
        Fx = (R)(sg.F0[0] * c);
        Fy = (R)(sg.F0[1] * c);
        Fz = (R)(sg.F0[2] * c);
    }
    const bool bad0 = collide_site<R, OFF>(x0, sg, Fx, Fy, Fz);
    const bool bad1 = two ? collide_site<R, OFF>(x1, sg, Fx, Fy, Fz) : false;
    if (__ballot(bad0 || bad1) != 0 && (threadIdx.x & 63) == 0) a.ctrl->nan_flag = 1;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        T *p = lout + lidx(i, s);
        if (two) {
            V2 v;
            v.x = (E)x0[i];
            v.y = (E)x1[i];
            __builtin_nontemporal_store(v, (V2 *)p);
        } else {
            stc(p, x0[i], i);
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_bulk2(KArgs a) {
    pair_sites<T>(a, a.entries2[block_index(a.xcd_remap)]);
}

// The same kernel with the register budget of six waves per SIMD: used for the
// FP32/FP16 boundary and fused variants, whose boundary path would otherwise
// drop occupancy to five waves (FP64 would spill, so it keeps k_step).
template <typename T, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) k_step_occ(KArgs a) {
    step_body<T, MODE>(a);
}

template <typename T, int MODE>
static void launch_mode(int grid, int block, hipStream_t st, const KArgs &a) {
    if constexpr (MODE == M_FUSED && pair_ok<T>()) {
        if (a.pair_fused) {
            // the two-sites-per-lane bulk path in its own kernel, so that the
            // plain fused kernel keeps its register budget
            if constexpr (std::is_same<T, __half>::value)
                hipLaunchKernelGGL((k_step_occ<T, M_FUSEDP>), dim3(grid), dim3(block), 0, st, a);
            else
                hipLaunchKernelGGL((k_step<T, M_FUSEDP>), dim3(grid), dim3(block), 0, st, a);
            return;
        }
    }
    if constexpr (MODE == M_BULK && !std::is_same<T, h16w>::value && !std::is_same<T, h16sr>::value) {
        if (a.n_pairs_blocks > 0) {
            hipLaunchKernelGGL((k_bulk2<T>), dim3(a.n_pairs_blocks), dim3(block), 0, st, a);
            return;
        }
    }
    if constexpr (std::is_same<T, double>::value || MODE == M_BULK || MODE == M_RAW)
        hipLaunchKernelGGL((k_step<T, MODE>), dim3(grid), dim3(block), 0, st, a);
    else
        hipLaunchKernelGGL((k_step_occ<T, MODE>), dim3(grid), dim3(block), 0, st, a);
}

// ===========================================================================
// In-place (AA-pattern) streaming: one lattice A[19][N].
//   even t: A holds f(t) in natural slots (A[i][x] = f_i(x)), except boundary
//           slots left for a fixup by the previous odd sweep.  The even sweep
//           reads its own slots, collides, and stores f*_i(x) into A[opp(i)][x]
//           (swapped); halfway and Bouzidi q >= 1/2 wall values, which need
//           only this site's f*, are stored there ready for the next read.
//   odd t:  A holds f*(t-1) in swapped slots.  The odd sweep gathers
//           f_j(x) = A[opp(j)][x - c_j], collides, and scatters f*_k(x) to
//           A[k][x + c_k] (natural slots of the next step); a link whose
//           destination is not fluid writes its boundary value (or the raw
//           f*_k(x) when the rule needs data of another site or the boundary
//           values of step t) into A[opp(k)][x].
// Every slot is read and written by one thread only within a sweep, so a
// sweep needs no second lattice.  The Bouzidi q < 1/2 interpolation, the
// Ladd inlet term and the pressure-outlet equilibrium of the stream
// t-1 -> t are applied when reading (they use step t-1's boundary values).
// ===========================================================================
template <typename T, bool BND, int ODD>
__device__ __forceinline__ void aa_read(const KArgs &a, const Entry &e, const SegDev &sg, int64_t t, int64_t s,
                                        int direct, typename Arith<T>::R (&x)[Q], int32_t (&sr)[Q],
                                        float (&qv)[Q]) {
    using R = typename Arith<T>::R;
    constexpr bool OFF = Arith<T>::OFF;
    const T *__restrict__ A = (const T *)a.lat0;
    // the pull table: needed by odd sweeps (gather/scatter) and by boundary sites
    if (BND)
        boundary_indices(a, tag_class(e.tag), s, sr);
    else if (ODD)
        pull_indices(a, tag_class(e.tag), s, sr);
    if (!ODD) {
#pragma unroll
        for (int i = 0; i < Q; ++i) x[i] = ldc(A + lidx(i, s), i);
    } else {
        // (after a reload at an odd step the lattice holds f(t) in the same
        // arrangement, so the same gather reads it back)
        x[0] = ldc(A + lidx(0, s), 0);
#pragma unroll
        for (int j = 1; j < Q; ++j) {
            const int jb = opp(j);
            if (BND) {
                // one load from the selected slot (rows j and jb share a weight)
                const T *p = (sr[j] >= 0) ? A + lidx(jb, sr[j]) : A + lidx(j, s);
                x[j] = ldc(p, j);
            } else {
                x[j] = ldc(A + lidx(jb, sr[j]), jb);
            }
        }
    }
    if (!BND) return;
    const bool bz = sg.wall_mode == WALL_BOUZIDI;
    const int64_t b = s - a.NB;
    wall_fractions(a, b, bz, sr, qv);
    if (direct) return;
    // boundary rules of the stream t-1 -> t; x[j] holds f*_jb(s, t-1) (or a
    // final value) for every direction whose upstream voxel is not fluid.
    // Candidate values are computed for every lane and selected, so the
    // divergent link mix of boundary sites costs no branches.
    const int64_t p = t - 1;
    const int klass = tag_class(e.tag);
    if (bz) {
        // halfway and q >= 1/2 values were stored final; q < 1/2 needs the
        // second node x_s + c_j, whose population arrived as x[jb] (never
        // rewritten here: the rule applies only when jb is a fluid link)
#pragma unroll
        for (int j = 1; j < Q; ++j) {
            const int jb = opp(j);
            const R q = (R)qv[j];
            const R vw = R(2) * q * x[j] + (R(1) - R(2) * q) * x[jb];
            x[j] = (sr[j] == -1 && q < R(0.5) && sr[jb] >= 0) ? vw : x[j];
        }
    }
    if (klass == K_IOLET) {
        const int g = tag_iolet(e.tag);
        const IoletDev &io = a.io[g];
        const double v = a.bc[(p & 1) * a.n_io + g];
        if (io.kind == KIND_INLET) {
            // Ladd: f_j = f*_jb - 6 w rho0 (c_jb . u_w), u_w = U phi n
            const R Uphi = (R)v * (R)a.bphi[b];
            const R nx = (R)io.nrm[0], ny = (R)io.nrm[1], nz = (R)io.nrm[2];
#pragma unroll
            for (int j = 1; j < Q; ++j) {
                const int jb = opp(j);
                const R cn = R(CX[jb]) * nx + R(CY[jb]) * ny + R(CZ[jb]) * nz;
                const R vi = x[j] - R(6) * wgt<R>(j) * R(RHO0) * (cn * Uphi);
                x[j] = (sr[j] <= -2) ? vi : x[j];
            }
        } else {
            // pressure outlet: equilibrium at rho_out and the site's velocity
            // of step t-1
            const R rho_out = (R)v, drho_out = (R)(v - RHO0);
            const R *up = (const R *)((p & 1) ? a.up1 : a.up0);
            const int64_t vi = s - a.IO0;
            const R ux = up[vi], uy = up[a.Nio + vi], uz = up[2 * a.Nio + vi];
            const R uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
            for (int j = 1; j < Q; ++j) {
                const R cu = R(CX[j]) * ux + R(CY[j]) * uy + R(CZ[j]) * uz;
                const R poly = R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu;
                const R vo = OFF ? wgt<R>(j) * (drho_out + rho_out * poly) : wgt<R>(j) * rho_out * (R(1) + poly);
                x[j] = (sr[j] <= -2) ? vo : x[j];
            }
        }
    }
}

// Moments of f(t) in x: iolet velocity history, partial sums of the iolet
// work-groups, divergence flag.  Returns rho and u through the references.
template <typename T>
__device__ __forceinline__ void aa_moments(const KArgs &a, const Entry &e, int eidx, int64_t t, int64_t s, bool act,
                                           const typename Arith<T>::R (&x)[Q], typename Arith<T>::R Fx,
                                           typename Arith<T>::R Fy, typename Arith<T>::R Fz, double *lds) {
    using R = typename Arith<T>::R;
    constexpr bool OFF = Arith<T>::OFF;
    const int klass = tag_class(e.tag);
    R rho = 1, drho = 0, ux = 0, uy = 0, uz = 0;
    bool bad = false;
    if (act) {
        R m0 = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            m0 += x[i];
            if (CX[i]) jx += R(CX[i]) * x[i];
            if (CY[i]) jy += R(CY[i]) * x[i];
            if (CZ[i]) jz += R(CZ[i]) * x[i];
        }
        rho = OFF ? R(RHO0) + m0 : m0;
        drho = OFF ? m0 : m0 - R(RHO0);
        ux = over(jx + R(0.5) * Fx, rho);
        uy = over(jy + R(0.5) * Fy, rho);
        uz = over(jz + R(0.5) * Fz, rho);
        bad = !isfinite(rho);
        if (klass == K_IOLET) {
            R *up = (R *)((t & 1) ? a.up1 : a.up0);
            const int64_t vi = s - a.IO0;
            up[vi] = ux;
            up[a.Nio + vi] = uy;
            up[2 * a.Nio + vi] = uz;
        }
    }
    if (__ballot(bad) != 0 && (threadIdx.x & 63) == 0) a.ctrl->nan_flag = 1;
    if (klass == K_IOLET) {
        const IoletDev &io = a.io[tag_iolet(e.tag)];
        double un = 0.0, rh = 0.0;  // u.n and rho - rho0 (summed as deviations: no cancellation)
        if (act) {
            un = (double)ux * io.nrm[0] + (double)uy * io.nrm[1] + (double)uz * io.nrm[2];
            rh = OFF ? (double)drho : (double)rho - RHO0;
        }
        const double su = block_sum(un, lds);
        const double sr = block_sum(rh, lds);
        if (threadIdx.x == 0) {
            a.partials[2 * eidx] = su;
            a.partials[2 * eidx + 1] = sr;
        }
    }
}

template <typename R>
__device__ __forceinline__ void body_force(const SegDev &sg, int64_t t, R &Fx, R &Fy, R &Fz) {
    Fx = Fy = Fz = 0;
    if (sg.has_force) {
        const double c = cos(sg.omega * (double)t);
        Fx = (R)(sg.F0[0] * c);
        Fy = (R)(sg.F0[1] * c);
        Fz = (R)(sg.F0[2] * c);
    }
}

// One in-place sweep t -> t+1 (MODE: M_BULK, M_BND or M_FUSED).
template <typename T, int MODE, int ODD>
__device__ __forceinline__ void aa_sweep_body(const KArgs &a) {
    using R = typename Arith<T>::R;
    constexpr bool OFF = Arith<T>::OFF;
    __shared__ double lds[8];
    const int64_t t = step_time(a);
    // the raw (reloaded) state is seen only by the first sweep of a batch
    const int direct = a.dt == 0 ? a.ctrl->direct : 0;
    // the sweep reads the values of step t-1 and publishes those of step t
    if constexpr (MODE != M_BULK) publish_series(a, t);
    const int eidx = entry_index(a);
    if (eidx < 0) return;  // uniform over the work-group
    const Entry e = a.entries[eidx];
    const int klass = tag_class(e.tag);
    const SegDev &sg = a.seg[e.seg];
    const bool act = (int)threadIdx.x < e.count;
    const int64_t s = (int64_t)e.start + threadIdx.x;
    T *__restrict__ A = (T *)a.lat0;
    R x[Q];
    float qv[Q];
    int32_t sr[Q];
    // FP16 storage: the wall fractions of a boundary site wait out the
    // collision in LDS, not in registers (the boundary path's register count
    // sets the occupancy of the fused sweep: 5 instead of 4 waves per SIMD);
    // each lane reads back only its own column.  FP32 and FP64 measured
    // faster with them in registers.
    constexpr bool QLDS = sizeof(T) == 2;
    __shared__ float lq[QLDS ? (Q - 1) * 256 : 1];
    const bool bnd = (MODE == M_BND) || (MODE == M_FUSED && !bulk_class(klass));
    const bool bz = bnd && sg.wall_mode == WALL_BOUZIDI;
    if (act) {
        if (MODE == M_BULK || (MODE == M_FUSED && !bnd)) {
            aa_read<T, false, ODD>(a, e, sg, t, s, direct, x, sr, qv);
        } else {
            aa_read<T, true, ODD>(a, e, sg, t, s, direct, x, sr, qv);
            if (QLDS && bz) {
#pragma unroll
                for (int j = 1; j < Q; ++j) lq[(j - 1) * 256 + threadIdx.x] = qv[j];
            }
        }
    }
    R Fx, Fy, Fz;
    body_force(sg, t, Fx, Fy, Fz);
    aa_moments<T>(a, e, eidx, t, s, act, x, Fx, Fy, Fz, lds);
    if (!act) return;
    R(&f)[Q] = x;
    collide_site<R, OFF>(f, sg, Fx, Fy, Fz);
    if (!ODD) {
        // swapped stores; slot m receives f*_opp(m), or the final wall value
        // of the pulled direction m when x_s - c_m is a Bouzidi wall (q >= 1/2)
        stc<false>(A + lidx(0, s), f[0], 0, rkey<T>(lidx(0, s), t));
        if (bz) {
#pragma unroll
            for (int m = 1; m < Q; ++m) {
                const int mb = opp(m);
                const R q = (R)(QLDS ? lq[(m - 1) * 256 + threadIdx.x] : qv[m]);
                const R vb = over(f[mb], R(2) * q) + (R(1) - over(R(1), R(2) * q)) * f[m];
                stc<false>(A + lidx(m, s), (sr[m] == -1 && q >= R(0.5)) ? vb : f[mb], m, rkey<T>(lidx(m, s), t));
            }
        } else {
#pragma unroll
            for (int m = 1; m < Q; ++m) stc<false>(A + lidx(m, s), f[opp(m)], m, rkey<T>(lidx(m, s), t));
        }
    } else {
        stc<false>(A + lidx(0, s), f[0], 0, rkey<T>(lidx(0, s), t));
        if (bnd) {
            // a link whose destination x_s + c_k is not fluid keeps f*_k (or
            // its final Bouzidi q >= 1/2 wall value) in the site's own slot
            // opp(k): one store to the selected slot (rows k and opp(k) share
            // a weight)
#pragma unroll
            for (int k = 1; k < Q; ++k) {
                const int kb = opp(k);
                const int32_t dst = sr[kb];  // the site at x_s + c_k
                R v = f[k];
                if (bz) {
                    const R q = (R)(QLDS ? lq[(kb - 1) * 256 + threadIdx.x] : qv[kb]);
                    const R vb = over(f[k], R(2) * q) + (R(1) - over(R(1), R(2) * q)) * f[kb];
                    v = (dst == -1 && q >= R(0.5)) ? vb : v;
                }
                const size_t di = (dst >= 0) ? lidx(k, dst) : lidx(kb, s);
                stc<false>(A + di, v, k, rkey<T>(di, t));
            }
        } else {
            // bulk site: every neighbour is fluid
#pragma unroll
            for (int k = 1; k < Q; ++k) stc<false>(A + lidx(k, sr[opp(k)]), f[k], k, rkey<T>(lidx(k, sr[opp(k)]), t));
        }
    }
}

template <typename T, int MODE, int ODD>
__global__ void __launch_bounds__(256) k_aa(KArgs a) {
    aa_sweep_body<T, MODE, ODD>(a);
}

// FP32/FP16 boundary and fused sweeps with the register budget of four waves
// per SIMD (their odd form would otherwise run three).
template <typename T, int MODE, int ODD>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) k_aa_occ(KArgs a) {
    aa_sweep_body<T, MODE, ODD>(a);
}

template <typename T, int MODE, int ODD>
static void launch_aa_mode(int grid, int block, hipStream_t st, const KArgs &a) {
    if constexpr (std::is_same<T, double>::value || MODE == M_BULK)
        hipLaunchKernelGGL((k_aa<T, MODE, ODD>), dim3(grid), dim3(block), 0, st, a);
    else
        hipLaunchKernelGGL((k_aa_occ<T, MODE, ODD>), dim3(grid), dim3(block), 0, st, a);
}

// Moments-only pass over f(t) (iolet means and history at step t).
template <typename T, int ODD>
__global__ void __launch_bounds__(256) k_aa_moments(KArgs a) {
    using R = typename Arith<T>::R;
    __shared__ double lds[8];
    const int64_t t = a.ctrl->t;
    const int direct = a.ctrl->direct;
    const int eidx = blockIdx.x;
    const Entry e = a.entries[eidx];
    const SegDev &sg = a.seg[e.seg];
    const bool act = (int)threadIdx.x < e.count;
    const int64_t s = (int64_t)e.start + threadIdx.x;
    R x[Q];
    float qv[Q];
    int32_t sr[Q];
    if (act) aa_read<T, true, ODD>(a, e, sg, t, s, direct, x, sr, qv);
    R Fx, Fy, Fz;
    body_force(sg, t, Fx, Fy, Fz);
    aa_moments<T>(a, e, eidx, t, s, act, x, Fx, Fy, Fz, lds);
}

// ---------------------------------------------------------------------------
// Observables of f(t): density, velocity, wall shear stress (FP64), and
// optionally the full populations.  f(t) is re-streamed from f*(t-1) with
// the boundary values of step t-1, or read directly after a reload.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_observe(KArgs a) {
    using R = typename Arith<T>::R;
    constexpr bool OFF = Arith<T>::OFF;
    const int64_t t = a.ctrl->t;
    const int direct = a.ctrl->direct;
    const Entry e = a.entries[blockIdx.x];
    const SegDev &sg = a.seg[e.seg];
    // one site per lane, in rounds when the entry holds more sites than lanes
    // (bulk entries of the two-sites-per-lane schedule)
    for (int k = threadIdx.x; k < e.count; k += blockDim.x) {
    const int64_t s = (int64_t)e.start + k;
    if (s < a.obs_lo || s >= a.obs_hi) continue;  // outside this pass's window
    const int64_t N = a.N;
    R x[Q];
    if (a.aa) {
        float qv[Q];
        int32_t sr[Q];
        if (t & 1)
            aa_read<T, true, 1>(a, e, sg, t, s, direct, x, sr, qv);
        else
            aa_read<T, true, 0>(a, e, sg, t, s, direct, x, sr, qv);
    } else if (direct) {
        const T *__restrict__ raw = lat_ptr<T>(a, t + 1);
#pragma unroll
        for (int i = 0; i < Q; ++i) x[i] = ldc(raw + lidx(i, s), i);
    } else {
        gather<T, true>(a, e, sg, t - 1, s, x);
    }
    double f[Q];
    double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        f[i] = (double)x[i] + (OFF ? wgt<double>(i) * RHO0 : 0.0);
        rho += f[i];
        jx += CX[i] * f[i];
        jy += CY[i] * f[i];
        jz += CZ[i] * f[i];
    }
    double F[3] = {0.0, 0.0, 0.0};
    if (sg.has_force) {
        const double c = cos(sg.omega * (double)t);
        for (int d = 0; d < 3; ++d) F[d] = sg.F0[d] * c;
    }
    const double ux = (jx + 0.5 * F[0]) / rho;
    const double uy = (jy + 0.5 * F[1]) / rho;
    const double uz = (jz + 0.5 * F[2]) / rho;
    double wss = 0.0;
    const int64_t b = s - a.NB;
    if (b >= 0) {
        const double n0 = a.bnrm[b], n1 = a.bnrm[a.Nb + b], n2 = a.bnrm[2 * a.Nb + b];
        if (n0 != 0.0 || n1 != 0.0 || n2 != 0.0) {
            const double uu = ux * ux + uy * uy + uz * uz;
            double P[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const double cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
                const double fe = wgt<double>(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
                const double ne = f[i] - fe;
                const double c3[3] = {(double)CX[i], (double)CY[i], (double)CZ[i]};
                for (int p = 0; p < 3; ++p)
                    for (int q = 0; q < 3; ++q) P[p][q] += ne * c3[p] * c3[q];
            }
            const double pref = -sg.guo_pref;
            const double nv[3] = {n0, n1, n2};
            double tr[3];
            for (int p = 0; p < 3; ++p) tr[p] = pref * (P[p][0] * nv[0] + P[p][1] * nv[1] + P[p][2] * nv[2]);
            const double tn = tr[0] * nv[0] + tr[1] * nv[1] + tr[2] * nv[2];
            const double sx = tr[0] - tn * nv[0], sy = tr[1] - tn * nv[1], sz = tr[2] - tn * nv[2];
            wss = sqrt(sx * sx + sy * sy + sz * sz);
        }
    }
    const int64_t w = s - a.obs_lo, W = a.obs_stride;
    a.obs[w] = rho;
    a.obs[W + w] = ux;
    a.obs[2 * W + w] = uy;
    a.obs[3 * W + w] = uz;
    a.obs[4 * W + w] = wss;
    if (a.fout) {
#pragma unroll
        for (int i = 0; i < Q; ++i) a.fout[(size_t)i * N + s] = f[i];
    }
    }  // sites
}

// Full f(t) (double) -> raw storage in lat[(t+1)&1].
template <typename T>
__global__ void k_load_raw(KArgs a) {
    using R = typename Arith<T>::R;
    constexpr bool OFF = Arith<T>::OFF;
    const int64_t t = a.ctrl->t;
    T *raw = (T *)((!a.aa && ((t + 1) & 1)) ? a.lat1 : a.lat0);
    const int64_t total = (int64_t)Q * a.N;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(k / a.N);
        const int64_t s = k - (int64_t)i * a.N;
        const double v = a.fin[k] - (OFF ? wgt<double>(i) * RHO0 : 0.0);
        stc(raw + lidx(i, s), (R)v, i, rkey<T>(lidx(i, s), t));
    }
}

// Rest state f_i = w_i rho0 as raw storage in lat[(t+1)&1].
template <typename T>
__global__ void k_fill_rest(KArgs a) {
    using R = typename Arith<T>::R;
    constexpr bool OFF = Arith<T>::OFF;
    const int64_t t = a.ctrl->t;
    T *raw = (T *)((!a.aa && ((t + 1) & 1)) ? a.lat1 : a.lat0);
    // every element of the tiled lattice, padding sites included
    const int64_t total = (int64_t)Q * a.Npad;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)((k >> TILE_SHIFT) % Q);
        stc(raw + k, OFF ? R(0) : (R)(wgt<double>(i) * RHO0), i, rkey<T>((size_t)k, t));
    }
}

// obs component (internal order) -> caller order, in device memory.
__global__ void k_gather_obs(const double *__restrict__ src, const int64_t *__restrict__ c2g, int64_t n,
                             double *__restrict__ out, int64_t lo, int64_t hi) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = c2g[k];
        if (g >= lo && g < hi) out[k] = src[g - lo];
    }
}

// Staging of the allocation-free observables read (see hl_internal.h).  In
// host code `scratch` names a host-side stand-in, never the device array:
// kernels receive the address hipGetSymbolAddress returns for the device.
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

int noalloc_scratch_setup(int device) {
    if (device < 0 || device >= MAX_DEVICES) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return (int)hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    g_scratch_ptr[device] = (double *)ptr;
    return (int)hipSuccess;
}

double *noalloc_scratch(int device) {
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

// Full f(t) (double, internal order) -> the in-place lattice at an odd step,
// in the arrangement the odd sweep gathers from: f_j(x) at
// A[opp(j)][x - c_j] when that site is fluid, else at A[j][x].
template <typename T>
__global__ void __launch_bounds__(256) k_aa_load_odd(KArgs a) {
    using R = typename Arith<T>::R;
    constexpr bool OFF = Arith<T>::OFF;
    const Entry e = a.entries[blockIdx.x];
    if ((int)threadIdx.x >= e.count) return;
    const int64_t s = (int64_t)e.start + threadIdx.x;
    const int64_t N = a.N;
    T *A = (T *)a.lat0;
    const int64_t t = a.ctrl->t;
    stc(A + lidx(0, s), (R)(a.fin[s] - (OFF ? wgt<double>(0) * RHO0 : 0.0)), 0, rkey<T>(lidx(0, s), t));
#pragma unroll
    for (int j = 1; j < Q; ++j) {
        const R v = (R)(a.fin[(size_t)j * N + s] - (OFF ? wgt<double>(j) * RHO0 : 0.0));
        const int32_t up = a.src[(size_t)(j - 1) * N + s];
        if (up >= 0)
            stc(A + lidx(opp(j), up), v, opp(j), rkey<T>(lidx(opp(j), up), t));
        else
            stc(A + lidx(j, s), v, j, rkey<T>(lidx(j, s), t));
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// part: 0 = every launch of the step, 1 = the bulk-site kernel, 2 = the
// boundary-site (or fused) kernel, 3 = the finalize kernel (launched only
// when domains are coupled).
template <typename T>
static int step_t(const KArgs &a0, int n_bulk, int n_bnd, int block, hipStream_t st, int part, bool fused) {
    KArgs a = a0;
    if (fused) {
        a.e_off = 0;
        if ((part == 0 || part == 2) && n_bnd > 0) launch_mode<T, M_FUSED>(a.emap ? a.n_emap : n_bnd, block, st, a);
    } else {
        if (n_bulk > 0 && (part == 0 || part == 1)) {
            a.e_off = 0;
            launch_mode<T, M_BULK>(n_bulk, block, st, a);
        }
        if (n_bnd > 0 && (part == 0 || part == 2)) {
            a.e_off = n_bulk;
            launch_mode<T, M_BND>(n_bnd, block, st, a);
        }
    }
    if ((part == 0 || part == 3) && a.n_pairs > 0)
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, a, (int)FIN_STEP);
    return (int)hipGetLastError();
}

template <typename T>
static int init_t(const KArgs &a0, int n_entries, int block, hipStream_t st) {
    KArgs a = a0;
    a.e_off = 0;
    a.xcd_remap = 0;
    a.emap = nullptr;  // one work-group per entry, in entry order
    hipLaunchKernelGGL((k_step<T, M_RAW>), dim3(n_entries), dim3(block), 0, st, a);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, a, (int)FIN_RAW);
    return (int)hipGetLastError();
}

int launch_advance(const KArgs &a, int64_t n, void *stream) {
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, (hipStream_t)stream, a, n);
    return (int)hipGetLastError();
}

int launch_stats(const KArgs &a0, void *stream) {
    KArgs a = a0;
    a.dt = 0;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, (hipStream_t)stream, a, (int)FIN_STATS);
    return (int)hipGetLastError();
}

static int grid_for(int64_t total) {
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

// Storage-type dispatch: calls f with a value of the storage type of `prec`.
template <typename F>
static int by_prec(int prec, F &&f) {
    switch (prec) {
    case PREC_F64: return f(double());
    case PREC_F32: return f(float());
    case PREC_F16: return f(__half());
    case PREC_F16W: return f(h16w());
    default: return f(h16sr());
    }
}

int launch_step(int prec, const KArgs &a, int n_bulk, int n_bnd, int block, void *stream, int part, bool fused) {
    hipStream_t st = (hipStream_t)stream;
    return by_prec(prec, [&](auto z) { return step_t<decltype(z)>(a, n_bulk, n_bnd, block, st, part, fused); });
}

int launch_init(int prec, const KArgs &a, int n_entries, int block, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    return by_prec(prec, [&](auto z) { return init_t<decltype(z)>(a, n_entries, block, st); });
}

int launch_observe(int prec, const KArgs &a, int n_entries, int block, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    return by_prec(prec, [&](auto z) {
        hipLaunchKernelGGL(k_observe<decltype(z)>, dim3(n_entries), dim3(block), 0, st, a);
        return (int)hipGetLastError();
    });
}

int launch_load_raw(int prec, const KArgs &a, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    const int g = grid_for((int64_t)Q * a.N);
    return by_prec(prec, [&](auto z) {
        hipLaunchKernelGGL(k_load_raw<decltype(z)>, dim3(g), dim3(256), 0, st, a);
        return (int)hipGetLastError();
    });
}

template <typename T, int ODD>
static int aa_step_t(const KArgs &a0, int n_bulk, int n_bnd, int block, hipStream_t st, int part, bool fused) {
    KArgs a = a0;
    if (fused) {
        a.e_off = 0;
        if ((part == 0 || part == 2) && n_bnd > 0)
            launch_aa_mode<T, M_FUSED, ODD>(a.emap ? a.n_emap : n_bnd, block, st, a);
    } else {
        if (n_bulk > 0 && (part == 0 || part == 1)) {
            a.e_off = 0;
            launch_aa_mode<T, M_BULK, ODD>(n_bulk, block, st, a);
        }
        if (n_bnd > 0 && (part == 0 || part == 2)) {
            a.e_off = n_bulk;
            launch_aa_mode<T, M_BND, ODD>(n_bnd, block, st, a);
        }
    }
    if ((part == 0 || part == 3) && a.n_pairs > 0)
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, a, (int)FIN_AA_SWEEP);
    return (int)hipGetLastError();
}

int launch_aa_step(int prec, const KArgs &a, int n_bulk, int n_bnd, int block, void *stream, int part, bool fused,
                   int odd) {
    hipStream_t st = (hipStream_t)stream;
    return by_prec(prec, [&](auto z) {
        using T = decltype(z);
        return odd ? aa_step_t<T, 1>(a, n_bulk, n_bnd, block, st, part, fused)
                   : aa_step_t<T, 0>(a, n_bulk, n_bnd, block, st, part, fused);
    });
}

template <typename T>
static void aa_moments_t(const KArgs &a, int n_entries, int block, hipStream_t st, int odd) {
    if (odd)
        hipLaunchKernelGGL((k_aa_moments<T, 1>), dim3(n_entries), dim3(block), 0, st, a);
    else
        hipLaunchKernelGGL((k_aa_moments<T, 0>), dim3(n_entries), dim3(block), 0, st, a);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, a, (int)FIN_AA_MOMENTS);
}

int launch_aa_moments(int prec, const KArgs &a, int n_entries, int block, void *stream, int odd) {
    hipStream_t st = (hipStream_t)stream;
    return by_prec(prec, [&](auto z) {
        aa_moments_t<decltype(z)>(a, n_entries, block, st, odd);
        return (int)hipGetLastError();
    });
}

int launch_aa_load_odd(int prec, const KArgs &a, int n_entries, int block, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    return by_prec(prec, [&](auto z) {
        hipLaunchKernelGGL(k_aa_load_odd<decltype(z)>, dim3(n_entries), dim3(block), 0, st, a);
        return (int)hipGetLastError();
    });
}

int launch_gather_obs(const double *src, const int64_t *c2g, int64_t n, double *out, int64_t lo, int64_t hi,
                      void *stream) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_gather_obs, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, src, c2g, n, out, lo, hi);
    return (int)hipGetLastError();
}

int launch_fill_rest(int prec, const KArgs &a, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    const int g = grid_for((int64_t)Q * a.Npad);
    return by_prec(prec, [&](auto z) {
        hipLaunchKernelGGL(k_fill_rest<decltype(z)>, dim3(g), dim3(256), 0, st, a);
        return (int)hipGetLastError();
    });
}

}  // namespace hl
