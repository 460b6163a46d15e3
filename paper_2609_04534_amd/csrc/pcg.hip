// Preconditioned conjugate gradients for the coupled SIPG operator of a mesh
// plan: A x = b in FP64 with the cell-wise fast-diagonalization block-Jacobi
// preconditioner of Sec. 5.2 (z = D^{-1} r, the cell blocks of
// eq. (cell_block) with the interior stencil on every cell), applied in FP64
// or FP32, or by one multigrid V-cycle (the paper's solver, Sec. 5: the same
// block inverse inside Chebyshev smoothing on every level; mg.hip), set with
// tp_pcg_set_multigrid.
//
// One iteration is five launches, none of which needs the host:
//   1. q = A p with the per-workgroup partial sums of (p, q)
//   2. one workgroup: alpha = (r, z) / (p, q)
//   3. x += alpha p, r -= alpha q, z = D^{-1} r, partial sums of (r, z), (r, r)
//   4. one workgroup: beta = (r, z)_new / (r, z), convergence test on (r, r)
//   5. p = z + beta p
// The state (scalars, iteration count, done flag) lives in device memory;
// once the flag is set every later kernel returns at its first instruction,
// so the host enqueues iterations in chunks and reads the state once per
// chunk.  Reductions sum per-workgroup partials in a fixed order (no
// atomics), so a solve is deterministic.
#include <algorithm>
#include <cmath>
#include <new>

#include "sipg.h"

namespace tpfdm {

namespace {

__device__ __forceinline__ bool finite(double v) { return v == v && v <= 1.7976931348623157e308 && v >= -1.7976931348623157e308; }

// 1.  q = A p, partial (p, q) per workgroup (HERM: the two-layer face
// terms of the Hermite-type basis).
template <int N, int LB, bool HERM = false>
__global__ __launch_bounds__(64, 2) void k_pcg_aq(const double* __restrict__ p, double* __restrict__ q, MeshArgs G,
                                                Pair<N, double> R, FaceRef<N, double> F,
                                                const PcgState* __restrict__ st, double* __restrict__ part) {
    if (st->done) return;
    constexpr int N3 = N * N * N;
    __shared__ double sa[N * N][64], sbt[N * N][64];
    const int64_t c = static_cast<int64_t>(lane_tile(blockIdx.x, gridDim.x, plane_tiles<N, double, HERM>(G))) * 64 + threadIdx.x;
    const int lb = LB >= 0 ? LB : G.logB;
    double dot = 0.0;
    if (c < G.ncells) {
        double acc[N3];
        sipg_cell<N, double, double, LB, HERM>(p, G, R, F, c, acc, sa, sbt);
        const int64_t base = G.offset + block_base(c, lb, N3);
#pragma unroll
        for (int e = 0; e < N3; ++e) {
            const int64_t o = base + (static_cast<int64_t>(e) << lb);
            q[o] = acc[e];
            dot = fma(acc[e], p[o], dot);
        }
    }
    dot = wave_sum(dot);
    if (threadIdx.x == 0) part[blockIdx.x] = dot;
}

// Fixed-order sum of count partials by one 256-thread workgroup.
__device__ __forceinline__ double block_sum(const double* __restrict__ part, int64_t count, double* red) {
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (static_cast<int>(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// 0.  After the start kernel: (r, z), (r, r), (b, b) -> state.  norm 0:
// converged when (r, r) <= rtol^2 (b, b); norm 1: when (r, z) <= rtol^2
// (r_0, z_0), the preconditioned residual norm reduced by rtol.
__global__ __launch_bounds__(256) void k_pcg_reduce_start(const double* __restrict__ part, int64_t count,
                                                          PcgState* __restrict__ st, double rtol, int maxit,
                                                          int norm) {
    __shared__ double red[256];
    const double rz = block_sum(part, count, red);
    const double rr = block_sum(part + count, count, red);
    const double bb = block_sum(part + 2 * count, count, red);
    if (threadIdx.x == 0) {
        PcgState s;
        s.rz = rz;
        s.pq = 0.0;
        s.rr = rr;
        s.bb = bb;
        s.alpha = 0.0;
        s.beta = 0.0;
        s.tol2 = rtol * rtol * (norm ? rz : bb);
        s.iter = 0;
        s.maxit = maxit;
        s.norm = norm;
        s.done = !(finite(rz) && finite(rr) && finite(bb)) ? 2 : ((norm ? rz : rr) <= s.tol2 ? 1 : (maxit <= 0 ? 3 : 0));
        *st = s;
    }
}

// 2.  alpha = (r, z) / (p, q).
__global__ __launch_bounds__(256) void k_pcg_reduce_alpha(const double* __restrict__ part, int64_t count,
                                                          PcgState* __restrict__ st) {
    if (st->done) return;
    __shared__ double red[256];
    const double pq = block_sum(part, count, red);
    if (threadIdx.x == 0) {
        st->pq = pq;
        if (!(pq > 0.0) || !finite(pq)) {
            st->done = 2;
        } else {
            st->alpha = st->rz / pq;
        }
    }
}

// 4.  beta, the iteration count and the convergence test.
__global__ __launch_bounds__(256) void k_pcg_reduce_beta(const double* __restrict__ part, int64_t count,
                                                         PcgState* __restrict__ st) {
    if (st->done) return;
    __shared__ double red[256];
    const double rz = block_sum(part, count, red);
    const double rr = block_sum(part + count, count, red);
    if (threadIdx.x == 0) {
        const double rz_old = st->rz;
        st->beta = rz / rz_old;
        st->rz = rz;
        st->rr = rr;
        const int it = st->iter + 1;
        st->iter = it;
        if (!finite(rz) || !finite(rr)) st->done = 2;
        else if ((st->norm ? rz : rr) <= st->tol2) st->done = 1;
        else if (it >= st->maxit) st->done = 3;
    }
}

// z = D^{-1} r for the lane's cell in precision TI: v holds the cell's
// residual (already rounded to TI), z is written in FP64; returns the
// partial (r, z) of the cell with r re-read in FP64.
template <int N, typename TI, int LB>
__device__ __forceinline__ double precondition(TI (&v)[N * N * N], const double* __restrict__ r,
                                               double* __restrict__ z, int64_t base, int lb, const Eig<N, TI>& E,
                                               TI sx, TI sy, TI sz) {
    constexpr int N3 = N * N * N;
    lane_fdm_inplace<N, TI>(v, E, sx, sy, sz);
    double rz = 0.0;
#pragma unroll
    for (int e = 0; e < N3; ++e) {
        const int64_t o = base + (static_cast<int64_t>(e) << lb);
        const double zv = static_cast<double>(v[e]);
        z[o] = zv;
        rz = fma(r[o], zv, rz);
    }
    return rz;
}

// Start: x = x0 and r = b - q with q = A x0, or x = 0 and r = b; z = D^{-1} r; p = z;
// partials (r, z), (r, r), (b, b).
template <int N, typename TI, int LB>
__global__ __launch_bounds__(64, 2) void k_pcg_start(const double* __restrict__ b, const double* __restrict__ q,
                                                   const double* __restrict__ x0, double* __restrict__ x,
                                                   double* __restrict__ r, double* __restrict__ z,
                                                   double* __restrict__ p, MeshArgs G, Eig<N, TI> E,
                                                   double* __restrict__ part, int64_t count) {
    constexpr int N3 = N * N * N;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 64 + threadIdx.x;
    const int lb = LB >= 0 ? LB : G.logB;
    double rz = 0.0, rr = 0.0, bb = 0.0;
    if (c < G.ncells) {
        const int64_t base = G.offset + block_base(c, lb, N3);
        TI v[N3];
#pragma unroll
        for (int e = 0; e < N3; ++e) {
            const int64_t o = base + (static_cast<int64_t>(e) << lb);
            const double bv = b[o];
            const double rv = q ? bv - q[o] : bv;   // (q: A x0, or null for x0 = 0)
            x[o] = q ? x0[o] : 0.0;   // the solver's iterate starts from the guess
            r[o] = rv;
            v[e] = static_cast<TI>(rv);
            rr = fma(rv, rv, rr);
            bb = fma(bv, bv, bb);
        }
        rz = precondition<N, TI, LB>(v, r, z, base, lb, E, static_cast<TI>(G.sx), static_cast<TI>(G.sy),
                                     static_cast<TI>(G.sz));
#pragma unroll
        for (int e = 0; e < N3; ++e) {
            const int64_t o = base + (static_cast<int64_t>(e) << lb);
            p[o] = z[o];
        }
    }
    rz = wave_sum(rz);
    rr = wave_sum(rr);
    bb = wave_sum(bb);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = rz;
        part[count + blockIdx.x] = rr;
        part[2 * count + blockIdx.x] = bb;
    }
}

// 3.  x += alpha p, r -= alpha q, z = D^{-1} r; partials (r, z), (r, r).
template <int N, typename TI, int LB>
__global__ __launch_bounds__(64, 2) void k_pcg_update(double* __restrict__ x, double* __restrict__ r,
                                                    double* __restrict__ z, const double* __restrict__ p,
                                                    const double* __restrict__ q, MeshArgs G, Eig<N, TI> E,
                                                    const PcgState* __restrict__ st, double* __restrict__ part,
                                                    int64_t count) {
    if (st->done) return;
    constexpr int N3 = N * N * N;
    const double alpha = st->alpha;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 64 + threadIdx.x;
    const int lb = LB >= 0 ? LB : G.logB;
    double rz = 0.0, rr = 0.0;
    if (c < G.ncells) {
        const int64_t base = G.offset + block_base(c, lb, N3);
        TI v[N3];
#pragma unroll
        for (int e = 0; e < N3; ++e) {
            const int64_t o = base + (static_cast<int64_t>(e) << lb);
            x[o] = fma(alpha, p[o], x[o]);
            const double rv = fma(-alpha, q[o], r[o]);
            r[o] = rv;
            v[e] = static_cast<TI>(rv);
            rr = fma(rv, rv, rr);
        }
        rz = precondition<N, TI, LB>(v, r, z, base, lb, E, static_cast<TI>(G.sx), static_cast<TI>(G.sy),
                                     static_cast<TI>(G.sz));
    }
    rz = wave_sum(rz);
    rr = wave_sum(rr);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = rz;
        part[count + blockIdx.x] = rr;
    }
}

// 5.  p = z + beta p over the whole vector (padding lanes included: they are
// never read as cell data).
// z in FP64, or in FP32 when it is the result of an FP32-storage V-cycle.
template <typename TZ>
__global__ __launch_bounds__(256) void k_pcg_dir(const TZ* __restrict__ z, double* __restrict__ p, int64_t n,
                                                 const PcgState* __restrict__ st) {
    if (st->done) return;
    const double beta = st->beta;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * 256)
        p[i] = fma(beta, p[i], static_cast<double>(z[i]));
}

// ---------------------------------------------------------------- multigrid preconditioning
// The V-cycle is a sequence of launches over all levels, so with it the
// start and the update only form residuals; z and (r, z) come from the
// multigrid kernels.

// Start: x = x0 and r = b - q, or x = 0 and r = b; partials (r, r), (b, b).
template <int N, int LB>
__global__ __launch_bounds__(64) void k_pcg_start_res(const double* __restrict__ b, const double* __restrict__ q,
                                                      const double* __restrict__ x0, double* __restrict__ x,
                                                      double* __restrict__ r, MeshArgs G,
                                                      double* __restrict__ part, int64_t count) {
    constexpr int N3 = N * N * N;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 64 + threadIdx.x;
    const int lb = LB >= 0 ? LB : G.logB;
    double rr = 0.0, bb = 0.0;
    if (c < G.ncells) {
        const int64_t base = G.offset + block_base(c, lb, N3);
#pragma unroll 8
        for (int e = 0; e < N3; ++e) {
            const int64_t o = base + (static_cast<int64_t>(e) << lb);
            const double bv = b[o];
            const double rv = q ? bv - q[o] : bv;   // (q: A x0, or null for x0 = 0)
            x[o] = q ? x0[o] : 0.0;
            r[o] = rv;
            rr = fma(rv, rv, rr);
            bb = fma(bv, bv, bb);
        }
    }
    rr = wave_sum(rr);
    bb = wave_sum(bb);
    if (threadIdx.x == 0) {
        part[count + blockIdx.x] = rr;
        part[2 * count + blockIdx.x] = bb;
    }
}

// x += alpha p, r -= alpha q; partial (r, r).
template <int N, int LB>
__global__ __launch_bounds__(64) void k_pcg_axpy(double* __restrict__ x, double* __restrict__ r,
                                                 const double* __restrict__ p, const double* __restrict__ q,
                                                 MeshArgs G, const PcgState* __restrict__ st,
                                                 double* __restrict__ part, int64_t count) {
    if (st->done) return;
    constexpr int N3 = N * N * N;
    const double alpha = st->alpha;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 64 + threadIdx.x;
    const int lb = LB >= 0 ? LB : G.logB;
    double rr = 0.0;
    if (c < G.ncells) {
        const int64_t base = G.offset + block_base(c, lb, N3);
#pragma unroll
        for (int e = 0; e < N3; ++e) {
            const int64_t o = base + (static_cast<int64_t>(e) << lb);
            x[o] = fma(alpha, p[o], x[o]);
            const double rv = fma(-alpha, q[o], r[o]);
            r[o] = rv;
            rr = fma(rv, rv, rr);
        }
    }
    rr = wave_sum(rr);
    if (threadIdx.x == 0) part[count + blockIdx.x] = rr;
}

// ---------------------------------------------------------------- n >= 5
// One cell per wave: lane (a, b) owns the z-pencil (a, b, 0..n-1) for the
// vector updates; the preconditioner runs the even-odd FDM inverse of the
// cell in an LDS slab; q = A p is the wave body of the coupled operator.

// 1.  q = A p, partial (p, q) per workgroup (one cell); HERM: the
// Hermite-type basis (sign-flipped tables, see wave_sipg_cell).
template <int N, bool VP, bool HERM>
__global__ __launch_bounds__(64, 2) void k_pcg_aq_wave(const double* __restrict__ p, double* __restrict__ q,
                                                     MeshArgs G, const double* __restrict__ tab,
                                                     FaceRef<N, double> F, const PcgState* __restrict__ st,
                                                     double* __restrict__ part) {
    if (st->done) return;
    constexpr int TAB = 2 * (EOShape<N>::SE + EOShape<N>::SO);
    __shared__ WaveLds<N, double> L;
    // the FP64 tables are read at wave-uniform global addresses (scalar
    // loads), not from registers or LDS
    static_assert(TAB > 0, "table");
    const int64_t c = xcd_tile(blockIdx.x, gridDim.x);
    double y[N];
    wave_sipg_cell<N, double, VP, HERM>(p, G, tab, F, c, L, y);
    const Pencil<N> pc(1);
    double dot = 0.0;
    if (pc.act) {
        const int64_t base = G.offset + block_base(c, G.logB, N * N * N);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int64_t o = base + (static_cast<int64_t>((i * N + pc.pa) * N + pc.pb) << G.logB);
            q[o] = y[i];
            dot = fma(y[i], p[o], dot);
        }
    }
    dot = wave_sum(dot);
    if (threadIdx.x == 0) part[blockIdx.x] = dot;
}

// Inverse tables of the wave kernels: SE | SO in registers, lam in LDS.
template <int N, typename TI>
__device__ __forceinline__ void load_inverse_tables(const TI* __restrict__ tab, TI* stab,
                                                    TI (&T)[EOShape<N>::SE + EOShape<N>::SO]) {
    constexpr int TABM = EOShape<N>::SE + EOShape<N>::SO;
    for (int e = threadIdx.x; e < TABM + N; e += 64) stab[e] = tab[e];
    wave_sync();
#pragma unroll
    for (int i = 0; i < TABM; ++i) T[i] = stab[i];
}

// z = D^{-1} r of the wave's cell in precision TI (rv: the lane's z-pencil of
// r in FP64), written in FP64 at zp (one vector store per 16 bytes when VP:
// the pencil is contiguous); returns the lane's partial (r, z).  HERM: the
// inverse tables are those of the sign-flipped Hermite-type coefficients, so
// r enters and z leaves the slab multiplied by its sign.
template <int N, typename TI, bool VP = false, bool HERM = false>
__device__ __forceinline__ double wave_precondition(const double (&rv)[N], double* __restrict__ zp, int lb,
                                                    const Pencil<N>& pc, TI* slab, const TI* T, const TI* lam,
                                                    TI sx, TI sy, TI sz) {
    using SL = Slab<N>;
    auto sg = [&](int k) {
        return HERM ? hermite_sign(N, pc.pa) * hermite_sign(N, pc.pb) * hermite_sign(N, k) : 1.0;
    };
    if (pc.act) {
#pragma unroll
        for (int k = 0; k < N; ++k) slab[SL::at(pc.pa, pc.pb, k)] = static_cast<TI>(sg(k) * rv[k]);
    }
    wave_sync();
    eo_inverse_lds<N, TI>(pc, slab, T, T + EOShape<N>::SE, lam, sx, sy, sz);
    double rz = 0.0;
    if (pc.act) {
        double zv[N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            zv[k] = sg(k) * static_cast<double>(slab[SL::at(pc.pa, pc.pb, k)]);
            rz = fma(rv[k], zv[k], rz);
        }
        pencil_store<N, VP>(zp, zv, lb);
    }
    return rz;
}

// Start (see k_pcg_start), one cell per workgroup.
template <int N, typename TI, bool HERM>
__global__ __launch_bounds__(64, 2) void k_pcg_start_wave(const double* __restrict__ b, const double* __restrict__ q,
                                                        const double* __restrict__ x0, double* __restrict__ x,
                                                        double* __restrict__ r, double* __restrict__ z,
                                                        double* __restrict__ p, MeshArgs G,
                                                        const TI* __restrict__ tab, double* __restrict__ part,
                                                        int64_t count) {
    constexpr int TABM = EOShape<N>::SE + EOShape<N>::SO;
    __shared__ TI slab[Slab<N>::size];
    __shared__ TI stab[TABM + N];
    TI T[TABM];
    load_inverse_tables<N, TI>(tab, stab, T);
    const int64_t c = blockIdx.x;
    const Pencil<N> pc(1);
    const int lb = G.logB;
    const int64_t pb = G.offset + block_base(c, lb, N * N * N) +
                       (static_cast<int64_t>((pc.pa * N + pc.pb) * N) << lb);
    double rv[N], rr = 0.0, bb = 0.0;
    if (pc.act) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const int64_t o = pb + (static_cast<int64_t>(k) << lb);
            const double bv = b[o];
            rv[k] = q ? bv - q[o] : bv;
            x[o] = q ? x0[o] : 0.0;
            r[o] = rv[k];
            rr = fma(rv[k], rv[k], rr);
            bb = fma(bv, bv, bb);
        }
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) rv[k] = 0.0;
    }
    double rz = wave_precondition<N, TI, false, HERM>(rv, z + pb, lb, pc, slab, T, stab + TABM,
                                                      static_cast<TI>(G.sx),
                                         static_cast<TI>(G.sy), static_cast<TI>(G.sz));
    if (pc.act) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const int64_t o = pb + (static_cast<int64_t>(k) << lb);
            p[o] = z[o];
        }
    }
    rz = wave_sum(rz);
    rr = wave_sum(rr);
    bb = wave_sum(bb);
    if (threadIdx.x == 0) {
        part[c] = rz;
        part[count + c] = rr;
        part[2 * count + c] = bb;
    }
}

// 3.  (see k_pcg_update), one cell per workgroup; VP: the lane's pencils are
// contiguous (layout B = 1), moved with vector loads and stores.
template <int N, typename TI, bool VP, bool HERM>
__global__ __launch_bounds__(64, 2) void k_pcg_update_wave(double* __restrict__ x, double* __restrict__ r,
                                                         double* __restrict__ z, const double* __restrict__ p,
                                                         const double* __restrict__ q, MeshArgs G,
                                                         const TI* __restrict__ tab, const PcgState* __restrict__ st,
                                                         double* __restrict__ part, int64_t count) {
    if (st->done) return;
    constexpr int TABM = EOShape<N>::SE + EOShape<N>::SO;
    __shared__ TI slab[Slab<N>::size];
    __shared__ TI stab[TABM + N];
    TI T[TABM];
    load_inverse_tables<N, TI>(tab, stab, T);
    const double alpha = st->alpha;
    const int64_t c = blockIdx.x;
    const Pencil<N> pc(1);
    const int lb = G.logB;
    const int64_t pb = G.offset + block_base(c, lb, N * N * N) +
                       (static_cast<int64_t>((pc.pa * N + pc.pb) * N) << lb);
    double rv[N], rr = 0.0;
    if (pc.act) {
        double xv[N], pv[N], qv[N];
        pencil_load<N, VP>(xv, x + pb, lb);
        pencil_load<N, VP>(pv, p + pb, lb);
        pencil_load<N, VP>(qv, q + pb, lb);
        pencil_load<N, VP>(rv, r + pb, lb);
#pragma unroll
        for (int k = 0; k < N; ++k) {
            xv[k] = fma(alpha, pv[k], xv[k]);
            rv[k] = fma(-alpha, qv[k], rv[k]);
            rr = fma(rv[k], rv[k], rr);
        }
        pencil_store<N, VP>(x + pb, xv, lb);
        pencil_store<N, VP>(r + pb, rv, lb);
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) rv[k] = 0.0;
    }
    double rz = wave_precondition<N, TI, VP, HERM>(rv, z + pb, lb, pc, slab, T, stab + TABM, static_cast<TI>(G.sx),
                                             static_cast<TI>(G.sy), static_cast<TI>(G.sz));
    rz = wave_sum(rz);
    rr = wave_sum(rr);
    if (threadIdx.x == 0) {
        part[c] = rz;
        part[count + c] = rr;
    }
}

tp_status check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, what);
    return TP_OK;
}

template <int N, typename T>
Eig<N, T> mesh_eig(const RefData& ref) {
    Eig<N, T> E;
    for (int i = 0; i < N * N; ++i) E.s[i] = static_cast<T>(ref.S[i]);
    for (int i = 0; i < N; ++i) E.lam[i] = static_cast<T>(ref.lam[i]);
    return E;
}

}  // namespace
}  // namespace tpfdm

using namespace tpfdm;

// The same two residual kernels for n >= 5, one cell per wave (lane (a, b)
// owns the z-pencil (a, b, 0..n-1); per-cell partials).
template <int N, bool VP>
__global__ __launch_bounds__(64) void k_pcg_start_res_wave(const double* __restrict__ b,
                                                           const double* __restrict__ q,
                                                           const double* __restrict__ x0, double* __restrict__ x,
                                                           double* __restrict__ r, MeshArgs G,
                                                           double* __restrict__ part, int64_t count) {
    const int64_t c = blockIdx.x;
    const Pencil<N> pc(1);
    const int lb = G.logB;
    double rr = 0.0, bb = 0.0;
    if (pc.act) {
        const int64_t pb = G.offset + block_base(c, lb, N * N * N) +
                           (static_cast<int64_t>((pc.pa * N + pc.pb) * N) << lb);
        double bv[N], rv[N], xv[N];
        pencil_load<N, VP>(bv, b + pb, lb);
        if (q) {
            double qv[N];
            pencil_load<N, VP>(qv, q + pb, lb);
            pencil_load<N, VP>(xv, x0 + pb, lb);
#pragma unroll
            for (int k = 0; k < N; ++k) rv[k] = bv[k] - qv[k];
        } else {
#pragma unroll
            for (int k = 0; k < N; ++k) rv[k] = bv[k], xv[k] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < N; ++k) {
            rr = fma(rv[k], rv[k], rr);
            bb = fma(bv[k], bv[k], bb);
        }
        pencil_store<N, VP>(x + pb, xv, lb);
        pencil_store<N, VP>(r + pb, rv, lb);
    }
    rr = wave_sum(rr);
    bb = wave_sum(bb);
    if (threadIdx.x == 0) {
        part[count + c] = rr;
        part[2 * count + c] = bb;
    }
}

template <int N, bool VP>
__global__ __launch_bounds__(64) void k_pcg_axpy_wave(double* __restrict__ x, double* __restrict__ r,
                                                      const double* __restrict__ p, const double* __restrict__ q,
                                                      MeshArgs G, const PcgState* __restrict__ st,
                                                      double* __restrict__ part, int64_t count) {
    if (st->done) return;
    const double alpha = st->alpha;
    const int64_t c = blockIdx.x;
    const Pencil<N> pc(1);
    const int lb = G.logB;
    double rr = 0.0;
    if (pc.act) {
        const int64_t pb = G.offset + block_base(c, lb, N * N * N) +
                           (static_cast<int64_t>((pc.pa * N + pc.pb) * N) << lb);
        double xv[N], rv[N], pv[N], qv[N];
        pencil_load<N, VP>(xv, x + pb, lb);
        pencil_load<N, VP>(rv, r + pb, lb);
        pencil_load<N, VP>(pv, p + pb, lb);
        pencil_load<N, VP>(qv, q + pb, lb);
#pragma unroll
        for (int k = 0; k < N; ++k) {
            xv[k] = fma(alpha, pv[k], xv[k]);
            rv[k] = fma(-alpha, qv[k], rv[k]);
            rr = fma(rv[k], rv[k], rr);
        }
        pencil_store<N, VP>(x + pb, xv, lb);
        pencil_store<N, VP>(r + pb, rv, lb);
    }
    rr = wave_sum(rr);
    if (threadIdx.x == 0) part[count + c] = rr;
}

// Workspace of one solver instance (plan-sized vectors and partials).
struct tp_pcg {
    tp_plan* plan = nullptr;
    double* r = nullptr;
    double* z = nullptr;
    double* p = nullptr;
    double* q = nullptr;
    double* xw = nullptr;       // the iterate (copied to the caller's x at the end)
    double* part = nullptr;     // [3][nwg]
    PcgState* st = nullptr;     // device
    PcgState* host = nullptr;   // pinned host copy
    int64_t nwg = 0;
    int64_t elems = 0;
    // one captured chunk of iterations per preconditioner precision (F64, F32)
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    int exec_chunk[2] = {0, 0};
    // non-blocking solves (tp_pcg_begin / tp_pcg_poll)
    hipEvent_t ev = nullptr;    // recorded after each enqueued step
    hipStream_t stream = nullptr;
    double* xout = nullptr;     // the caller's x
    int ti = 0;                 // precision of the running solve
    int phase = 0;              // 0 idle, 1 iterating, 2 copying the result out
    tp_mg* mg = nullptr;        // V-cycle preconditioner (null: block-Jacobi)
    int norm = TP_PCG_RESIDUAL; // stopping test
};

namespace {

void free_pcg(tp_pcg* s) {
    if (s->ev) (void)hipEventDestroy(s->ev), s->ev = nullptr;
    for (hipGraphExec_t& ex : s->exec)
        if (ex) (void)hipGraphExecDestroy(ex), ex = nullptr;
    for (void* ptr : {static_cast<void*>(s->r), static_cast<void*>(s->z), static_cast<void*>(s->p),
                      static_cast<void*>(s->q), static_cast<void*>(s->xw), static_cast<void*>(s->part),
                      static_cast<void*>(s->st)})
        if (ptr) (void)hipFree(ptr);
    if (s->host) (void)hipHostFree(s->host);
}

// Enqueues the start of a solve on stream (x = x0 or 0, r, z, p and the
// first reduction) and makes sure the chunk graph of this precision exists.
template <int N, typename TI, int LB>
tp_status pcg_prepare(const Plan& plan, const GroupInfo& g, tp_pcg* s, const double* b, const double* x,
                      bool x_zero, double rtol, int maxit, int chunk, hipStream_t stream) {
    const MeshArgs G = mesh_args(plan, g);
    Pair<N, double> R;
    FaceRef<N, double> F;
    sipg_tables<N, double>(plan, false, R, F);
    const Eig<N, TI> E = mesh_eig<N, TI>(plan.ref[N]);
    const unsigned nwg = static_cast<unsigned>(s->nwg);
    const int64_t cnt = s->nwg;
    const unsigned dgrid = static_cast<unsigned>(std::min<int64_t>((s->elems + 255) / 256, 8192));
    constexpr bool kLane = N <= kLaneMaxN;
    const double* tabA = reinterpret_cast<const double*>(eo_table(plan, N, EO_APPLY_A, 0));
    const TI* tabS = reinterpret_cast<const TI*>(eo_table(plan, N, EO_INV, sizeof(TI) == 8 ? 0 : 1));
    // 16-byte pencils for the wave body: block-contiguous layout (the
    // solver's vectors are allocation-aligned)
    const bool vp = g.logB == 0 && (N * sizeof(double)) % 16 == 0;
    // the wave kernels of the Hermite-type basis use sign-flipped tables and
    // endpoint derivatives (see wave_sipg_cell)
    const bool herm = !kLane && plan.basis == TP_BASIS_HERMITE;
    FaceRef<N, double> Fw = F;
    if (herm) flip_face_ref<N, double>(Fw);
    if (!x_zero) {
        tp_status st = launch_sipg(plan, g, false, x, s->q, TP_F64, stream);
        if (st != TP_OK) return st;
    }
    const bool f32 = sizeof(TI) == 4;
    if (s->mg) {
        if constexpr (kLane) {
            hipLaunchKernelGGL((k_pcg_start_res<N, LB>), dim3(nwg), dim3(64), 0, stream, b,
                               x_zero ? nullptr : s->q, x, s->xw, s->r, G, s->part, cnt);
            // with FP32 level storage z stays in the hierarchy's FP32 vector
            const bool z32 = mg_storage(s->mg) == TP_F32;
            const void* zp = z32 ? static_cast<const void*>(mg_result32(s->mg)) : static_cast<const void*>(s->z);
            tp_status st = mg_enqueue_vcycle(s->mg, s->r, z32 ? nullptr : s->z, nullptr, f32, stream);
            if (st == TP_OK) st = mg_enqueue_dot(s->mg, s->r, zp, z32, s->part, nullptr, stream);
            if (st != TP_OK) return st;
            if (z32) {
                st = mg_enqueue_widen(s->mg, s->p, stream);
                if (st != TP_OK) return st;
            } else {
                const hipError_t e = hipMemcpyAsync(s->p, s->z, static_cast<size_t>(s->elems) * sizeof(double),
                                                    hipMemcpyDeviceToDevice, stream);
                if (e != hipSuccess) return hip_error(e, "PCG start");
            }
        } else {
            if (vp)
                hipLaunchKernelGGL((k_pcg_start_res_wave<N, true>), dim3(nwg), dim3(64), 0, stream, b,
                                   x_zero ? nullptr : s->q, x, s->xw, s->r, G, s->part, cnt);
            else
                hipLaunchKernelGGL((k_pcg_start_res_wave<N, false>), dim3(nwg), dim3(64), 0, stream, b,
                                   x_zero ? nullptr : s->q, x, s->xw, s->r, G, s->part, cnt);
            const bool z32 = mg_storage(s->mg) == TP_F32;
            const void* zp = z32 ? static_cast<const void*>(mg_result32(s->mg)) : static_cast<const void*>(s->z);
            tp_status st = mg_enqueue_vcycle(s->mg, s->r, z32 ? nullptr : s->z, nullptr, f32, stream);
            if (st == TP_OK) st = mg_enqueue_dot(s->mg, s->r, zp, z32, s->part, nullptr, stream);
            if (st != TP_OK) return st;
            if (z32) {
                st = mg_enqueue_widen(s->mg, s->p, stream);
                if (st != TP_OK) return st;
            } else {
                const hipError_t e = hipMemcpyAsync(s->p, s->z, static_cast<size_t>(s->elems) * sizeof(double),
                                                    hipMemcpyDeviceToDevice, stream);
                if (e != hipSuccess) return hip_error(e, "PCG start");
            }
        }
    } else if constexpr (kLane)
        hipLaunchKernelGGL((k_pcg_start<N, TI, LB>), dim3(nwg), dim3(64), 0, stream, b, x_zero ? nullptr : s->q, x,
                           s->xw, s->r, s->z, s->p, G, E, s->part, cnt);
    else if (herm)
        hipLaunchKernelGGL((k_pcg_start_wave<N, TI, true>), dim3(nwg), dim3(64), 0, stream, b,
                           x_zero ? nullptr : s->q, x, s->xw, s->r, s->z, s->p, G, tabS, s->part, cnt);
    else
        hipLaunchKernelGGL((k_pcg_start_wave<N, TI, false>), dim3(nwg), dim3(64), 0, stream, b,
                           x_zero ? nullptr : s->q, x, s->xw, s->r, s->z, s->p, G, tabS, s->part, cnt);
    hipLaunchKernelGGL(k_pcg_reduce_start, dim3(1), dim3(256), 0, stream, s->part, cnt, s->st, rtol, maxit,
                       s->norm);
    tp_status st = check_launch("PCG start");
    if (st != TP_OK) return st;
    // one chunk of iterations, captured once per solver and precision: every
    // argument is solver-owned, so the graph replays for any b, x
    const int ti = sizeof(TI) == 8 ? 0 : 1;
    if (!s->exec[ti] || s->exec_chunk[ti] != chunk) {
        if (s->exec[ti]) (void)hipGraphExecDestroy(s->exec[ti]), s->exec[ti] = nullptr;
        hipStream_t cs = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_error(e, "PCG capture stream");
        hipGraph_t gr = nullptr;
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            for (int i = 0; i < chunk; ++i) {
                if constexpr (kLane) {
                    bool herm = false;
                    if constexpr (N == 4) herm = plan.basis == TP_BASIS_HERMITE;
                    if (herm) {
                        if constexpr (N == 4)
                            hipLaunchKernelGGL((k_pcg_aq<N, LB, true>), dim3(nwg), dim3(64), 0, cs, s->p, s->q, G, R,
                                               F, s->st, s->part);
                    } else {
                        hipLaunchKernelGGL((k_pcg_aq<N, LB>), dim3(nwg), dim3(64), 0, cs, s->p, s->q, G, R, F, s->st,
                                           s->part);
                    }
                } else if (herm) {
                    if (vp)
                        hipLaunchKernelGGL((k_pcg_aq_wave<N, true, true>), dim3(nwg), dim3(64), 0, cs, s->p, s->q, G,
                                           tabA, Fw, s->st, s->part);
                    else
                        hipLaunchKernelGGL((k_pcg_aq_wave<N, false, true>), dim3(nwg), dim3(64), 0, cs, s->p, s->q,
                                           G, tabA, Fw, s->st, s->part);
                } else if (vp)
                    hipLaunchKernelGGL((k_pcg_aq_wave<N, true, false>), dim3(nwg), dim3(64), 0, cs, s->p, s->q, G,
                                       tabA, F, s->st, s->part);
                else
                    hipLaunchKernelGGL((k_pcg_aq_wave<N, false, false>), dim3(nwg), dim3(64), 0, cs, s->p, s->q, G,
                                       tabA, F, s->st, s->part);
                hipLaunchKernelGGL(k_pcg_reduce_alpha, dim3(1), dim3(256), 0, cs, s->part, cnt, s->st);
                if (s->mg) {
                    if constexpr (!kLane) {
                        if (vp)
                            hipLaunchKernelGGL((k_pcg_axpy_wave<N, true>), dim3(nwg), dim3(64), 0, cs, s->xw, s->r,
                                               s->p, s->q, G, s->st, s->part, cnt);
                        else
                            hipLaunchKernelGGL((k_pcg_axpy_wave<N, false>), dim3(nwg), dim3(64), 0, cs, s->xw, s->r,
                                               s->p, s->q, G, s->st, s->part, cnt);
                        const bool z32 = mg_storage(s->mg) == TP_F32;
                        (void)mg_enqueue_vcycle(s->mg, s->r, z32 ? nullptr : s->z, s->st, f32, cs);
                        (void)mg_enqueue_dot(s->mg, s->r,
                                             z32 ? static_cast<const void*>(mg_result32(s->mg))
                                                 : static_cast<const void*>(s->z),
                                             z32, s->part, s->st, cs);
                    } else {
                        hipLaunchKernelGGL((k_pcg_axpy<N, LB>), dim3(nwg), dim3(64), 0, cs, s->xw, s->r, s->p, s->q,
                                           G, s->st, s->part, cnt);
                        const bool z32 = mg_storage(s->mg) == TP_F32;
                        (void)mg_enqueue_vcycle(s->mg, s->r, z32 ? nullptr : s->z, s->st, f32, cs);
                        (void)mg_enqueue_dot(s->mg, s->r,
                                             z32 ? static_cast<const void*>(mg_result32(s->mg))
                                                 : static_cast<const void*>(s->z),
                                             z32, s->part, s->st, cs);
                    }
                } else if constexpr (kLane)
                    hipLaunchKernelGGL((k_pcg_update<N, TI, LB>), dim3(nwg), dim3(64), 0, cs, s->xw, s->r, s->z,
                                       s->p, s->q, G, E, s->st, s->part, cnt);
                else if (herm) {
                    if (vp)
                        hipLaunchKernelGGL((k_pcg_update_wave<N, TI, true, true>), dim3(nwg), dim3(64), 0, cs, s->xw,
                                           s->r, s->z, s->p, s->q, G, tabS, s->st, s->part, cnt);
                    else
                        hipLaunchKernelGGL((k_pcg_update_wave<N, TI, false, true>), dim3(nwg), dim3(64), 0, cs,
                                           s->xw, s->r, s->z, s->p, s->q, G, tabS, s->st, s->part, cnt);
                } else if (vp)
                    hipLaunchKernelGGL((k_pcg_update_wave<N, TI, true, false>), dim3(nwg), dim3(64), 0, cs, s->xw,
                                       s->r, s->z, s->p, s->q, G, tabS, s->st, s->part, cnt);
                else
                    hipLaunchKernelGGL((k_pcg_update_wave<N, TI, false, false>), dim3(nwg), dim3(64), 0, cs, s->xw,
                                       s->r, s->z, s->p, s->q, G, tabS, s->st, s->part, cnt);
                hipLaunchKernelGGL(k_pcg_reduce_beta, dim3(1), dim3(256), 0, cs, s->part, cnt, s->st);
                if (s->mg && mg_storage(s->mg) == TP_F32)
                    hipLaunchKernelGGL(k_pcg_dir<float>, dim3(dgrid), dim3(256), 0, cs, mg_result32(s->mg), s->p,
                                       s->elems, s->st);
                else
                    hipLaunchKernelGGL(k_pcg_dir<double>, dim3(dgrid), dim3(256), 0, cs, s->z, s->p, s->elems, s->st);
            }
            const hipError_t e2 = hipStreamEndCapture(cs, &gr);
            if (e2 != hipSuccess) e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&s->exec[ti], gr, nullptr, nullptr, 0);
        if (gr) (void)hipGraphDestroy(gr);
        (void)hipStreamDestroy(cs);
        if (e != hipSuccess) {
            s->exec[ti] = nullptr;
            return hip_error(e, "PCG iteration graph");
        }
        s->exec_chunk[ti] = chunk;
    }
    s->ti = ti;
    return TP_OK;
}

template <typename TI>
tp_status pcg_prepare_dispatch(const Plan& plan, const GroupInfo& g, tp_pcg* s, const double* b, const double* x,
                               bool x_zero, double rtol, int maxit, int chunk, hipStream_t stream) {
    const bool b64 = g.logB == 6;
    switch (g.n) {
        case 2: return b64 ? pcg_prepare<2, TI, 6>(plan, g, s, b, x, x_zero, rtol, maxit, chunk, stream)
                           : pcg_prepare<2, TI, -1>(plan, g, s, b, x, x_zero, rtol, maxit, chunk, stream);
        case 3: return b64 ? pcg_prepare<3, TI, 6>(plan, g, s, b, x, x_zero, rtol, maxit, chunk, stream)
                           : pcg_prepare<3, TI, -1>(plan, g, s, b, x, x_zero, rtol, maxit, chunk, stream);
        case 4: return b64 ? pcg_prepare<4, TI, 6>(plan, g, s, b, x, x_zero, rtol, maxit, chunk, stream)
                           : pcg_prepare<4, TI, -1>(plan, g, s, b, x, x_zero, rtol, maxit, chunk, stream);
        case 5: return pcg_prepare<5, TI, -1>(plan, g, s, b, x, x_zero, rtol, maxit, chunk, stream);
        case 6: return pcg_prepare<6, TI, -1>(plan, g, s, b, x, x_zero, rtol, maxit, chunk, stream);
        case 7: return pcg_prepare<7, TI, -1>(plan, g, s, b, x, x_zero, rtol, maxit, chunk, stream);
        case 8: return pcg_prepare<8, TI, -1>(plan, g, s, b, x, x_zero, rtol, maxit, chunk, stream);
        default: break;
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported n");
}

// Argument checks shared by the blocking and the non-blocking solve.
tp_status pcg_validate(const tp_pcg* s, const double* b, const double* x, tp_dtype inner, double rtol, int maxit) {
    if (!s) return set_error(TP_ERR_ARG, "solver is null");
    const Plan& plan = *s->plan;
    if (s->phase != 0) return set_error(TP_ERR_STATE, "a non-blocking solve is still running on this solver");
    if (plan.vec_elems > 0 && (!b || !x)) return set_error(TP_ERR_ARG, "b and x must be non-null");
    if (static_cast<const void*>(b) == static_cast<const void*>(x) && b)
        return set_error(TP_ERR_ARG, "b and x must not alias");
    if (!(rtol > 0.0) || !std::isfinite(rtol)) return set_error(TP_ERR_ARG, "rtol must be finite and > 0");
    if (maxit < 0) return set_error(TP_ERR_ARG, "maxit must be >= 0");
    if (inner != TP_F64 && inner != TP_F32)
        return set_error(TP_ERR_UNSUPPORTED, "the preconditioner runs in TP_F64 or TP_F32");
    if (plan.inverse_op != TP_OP_CELL || plan.factor_mode != TP_FACTOR_SCALED)
        return set_error(TP_ERR_STATE, "the PCG solver needs tp_setup_inverse(TP_OP_CELL, TP_FACTOR_SCALED) first");
    return TP_OK;
}

tp_status pcg_start(tp_pcg* s, const double* b, double* x, bool x_zero, tp_dtype inner, double rtol, int maxit,
                    int chunk, hipStream_t stream) {
    const Plan& plan = *s->plan;
    const GroupInfo& g = plan.groups[0];
    return inner == TP_F64 ? pcg_prepare_dispatch<double>(plan, g, s, b, x, x_zero, rtol, maxit, chunk, stream)
                           : pcg_prepare_dispatch<float>(plan, g, s, b, x, x_zero, rtol, maxit, chunk, stream);
}

// Summary and status of a finished solve from the host copy of the state.
tp_status pcg_finish(const tp_pcg* s, tp_pcg_summary* summary) {
    const PcgState h = *s->host;
    if (summary) {
        summary->iterations = h.iter;
        summary->converged = h.done == 1 ? 1 : 0;
        summary->relres = h.bb > 0.0 ? std::sqrt(h.rr / h.bb) : 0.0;
    }
    if (h.done == 2) return set_error(TP_ERR_NONFINITE, "PCG breakdown or non-finite value after " +
                                                            std::to_string(h.iter) + " iterations");
    if (h.done == 3)
        return set_error(TP_ERR_NOT_CONVERGED, "PCG reached maxit = " + std::to_string(h.iter) +
                                                   " with relative residual " +
                                                   std::to_string(h.bb > 0.0 ? std::sqrt(h.rr / h.bb) : 0.0));
    return TP_OK;
}

tp_status enqueue_state_copy(tp_pcg* s, hipStream_t stream) {
    hipError_t e = hipMemcpyAsync(s->host, s->st, sizeof(PcgState), hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return hip_error(e, "PCG state read-back");
    return TP_OK;
}

tp_status enqueue_result_copy(tp_pcg* s, double* x, hipStream_t stream) {
    hipError_t e = hipMemcpyAsync(x, s->xw, static_cast<size_t>(s->elems) * sizeof(double), hipMemcpyDeviceToDevice,
                                  stream);
    if (e != hipSuccess) return hip_error(e, "PCG result copy");
    return TP_OK;
}

}  // namespace

extern "C" {

tp_status tp_pcg_create(tp_plan* plan, tp_pcg** out) {
    if (!out) return set_error(TP_ERR_ARG, "out must be non-null");
    *out = nullptr;
    if (!plan) return set_error(TP_ERR_ARG, "plan is null");
    if (!plan->mesh) return set_error(TP_ERR_UNSUPPORTED, "the PCG solver needs a mesh plan");
    tp_pcg* s = new (std::nothrow) tp_pcg();
    if (!s) return set_error(TP_ERR_OOM, "host allocation failed");
    s->plan = plan;
    s->elems = std::max<int64_t>(plan->vec_elems, 1);
    // partial sums: one per 64-cell tile (n <= 4) or per cell (n >= 5)
    const GroupInfo& g0 = plan->groups[0];
    s->nwg = std::max<int64_t>(g0.n <= kLaneMaxN ? (g0.nblocks + 63) / 64 : g0.nblocks, 1);
    const size_t vb = static_cast<size_t>(s->elems) * sizeof(double);
    hipError_t e = hipSuccess;
    for (double** d : {&s->r, &s->z, &s->p, &s->q, &s->xw})
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(d), vb);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s->part), 3 * s->nwg * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s->st), sizeof(PcgState));
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&s->host), sizeof(PcgState), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        free_pcg(s);
        delete s;
        (void)hipGetLastError();
        return set_error(TP_ERR_OOM, "PCG workspace allocation failed");
    }
    *out = s;
    return TP_OK;
}

tp_status tp_pcg_solve(tp_pcg* s, const double* b, double* x, int32_t x_is_zero, tp_dtype inner, double rtol,
                       int32_t maxit, int32_t check_every, tp_pcg_summary* summary, hipStream_t stream) {
    tp_status st = pcg_validate(s, b, x, inner, rtol, maxit);
    if (st != TP_OK) return st;
    if (s->plan->groups[0].nblocks == 0) {
        if (summary) *summary = tp_pcg_summary{0, 1, 0.0};
        return TP_OK;
    }
    const int chunk = check_every > 0 ? check_every : 16;
    st = pcg_start(s, b, x, x_is_zero != 0, inner, rtol, maxit, chunk, stream);
    if (st != TP_OK) return st;
    for (;;) {
        st = enqueue_state_copy(s, stream);
        if (st != TP_OK) return st;
        const hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_error(e, "PCG state read-back");
        if (s->host->done) break;
        const hipError_t e2 = hipGraphLaunch(s->exec[s->ti], stream);
        if (e2 != hipSuccess) return hip_error(e2, "PCG iteration graph launch");
    }
    st = enqueue_result_copy(s, x, stream);
    if (st != TP_OK) return st;
    const hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_error(e, "PCG result copy");
    return pcg_finish(s, summary);
}

tp_status tp_pcg_begin(tp_pcg* s, const double* b, double* x, int32_t x_is_zero, tp_dtype inner, double rtol,
                       int32_t maxit, int32_t check_every, hipStream_t stream) {
    tp_status st = pcg_validate(s, b, x, inner, rtol, maxit);
    if (st != TP_OK) return st;
    s->stream = stream;
    s->xout = x;
    if (s->plan->groups[0].nblocks == 0) {
        *s->host = PcgState{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0, 1, maxit, 0};
        s->phase = 2;
        const hipError_t e = hipEventRecord(s->ev, stream);
        if (e != hipSuccess) return s->phase = 0, hip_error(e, "PCG event");
        return TP_OK;
    }
    const int chunk = check_every > 0 ? check_every : 16;
    st = pcg_start(s, b, x, x_is_zero != 0, inner, rtol, maxit, chunk, stream);
    if (st == TP_OK) st = enqueue_state_copy(s, stream);
    if (st != TP_OK) return st;
    const hipError_t e = hipEventRecord(s->ev, stream);
    if (e != hipSuccess) return hip_error(e, "PCG event");
    s->phase = 1;
    return TP_OK;
}

tp_status tp_pcg_poll(tp_pcg* s, tp_pcg_summary* summary) {
    if (!s) return set_error(TP_ERR_ARG, "solver is null");
    if (s->phase == 0) return set_error(TP_ERR_STATE, "no non-blocking solve is running on this solver");
    const hipError_t q = hipEventQuery(s->ev);
    if (q == hipErrorNotReady) {
        (void)hipGetLastError();   // not an error: keep it out of later launch checks
        return TP_PENDING;
    }
    if (q != hipSuccess) {
        s->phase = 0;
        return hip_error(q, "PCG event query");
    }
    if (s->phase == 2) {
        s->phase = 0;
        return pcg_finish(s, summary);
    }
    // phase 1: the state copy of the last step has landed
    tp_status st = TP_OK;
    if (s->host->done) {
        st = enqueue_result_copy(s, s->xout, s->stream);
        if (st == TP_OK) s->phase = 2;
    } else {
        const hipError_t e = hipGraphLaunch(s->exec[s->ti], s->stream);
        st = e == hipSuccess ? enqueue_state_copy(s, s->stream) : hip_error(e, "PCG iteration graph launch");
    }
    if (st == TP_OK) {
        const hipError_t e = hipEventRecord(s->ev, s->stream);
        if (e != hipSuccess) st = hip_error(e, "PCG event");
    }
    if (st != TP_OK) s->phase = 0;
    return st == TP_OK ? TP_PENDING : st;
}

tp_status tp_pcg_set_norm(tp_pcg* s, int32_t norm) {
    if (!s) return set_error(TP_ERR_ARG, "solver is null");
    if (norm != TP_PCG_RESIDUAL && norm != TP_PCG_PRECONDITIONED) return set_error(TP_ERR_ARG, "invalid norm");
    if (s->phase != 0) return set_error(TP_ERR_STATE, "a non-blocking solve is still running on this solver");
    s->norm = norm;
    return TP_OK;
}

tp_status tp_pcg_set_multigrid(tp_pcg* s, tp_mg* mg) {
    if (!s) return set_error(TP_ERR_ARG, "solver is null");
    if (s->phase != 0) return set_error(TP_ERR_STATE, "a non-blocking solve is still running on this solver");
    if (mg && mg_plan(mg) != s->plan) return set_error(TP_ERR_ARG, "the multigrid belongs to another plan");
    s->mg = mg;
    for (hipGraphExec_t& ex : s->exec)   // the captured iterations depend on the preconditioner
        if (ex) (void)hipGraphExecDestroy(ex), ex = nullptr;
    return TP_OK;
}

tp_status tp_pcg_destroy(tp_pcg* s) {
    if (!s) return TP_OK;
    free_pcg(s);
    delete s;
    return TP_OK;
}

}  // extern "C"
