// Geometric multigrid for the coupled SIPG operator of a mesh plan (n <= 8):
// the V-cycle the paper uses to precondition CG (Sec. 5, Sec. 6.1).
//
// Levels: the plan's box and its uniform coarsenings (cells halved in every
// direction while all three counts are even, cell lengths doubled, the
// operator rediscretized with the level's own lengths and penalty).  On each
// level but the coarsest one smoothing application before and one after
// the coarse correction; a smoothing application is the degree-three
// Chebyshev-accelerated block-Jacobi method, three Richardson updates
//   u <- u + omega_j D^{-1} (b - A u),  omega_j = 1 / (c - d cos((2j-1) pi / 6))
// on the spectral interval [0.2, 2] (eq. (chebyshev_weights),
// eq. (chebyshev_richardson)), with D^{-1} the cell-wise fast-diagonalization
// inverse.  All tables (operator, inverse, transfers) are the plan's, in the
// plan's basis.  Each update is one kernel in the factorized form the paper
// describes (Sec. 5.2): the operator row, the residual, the block inverse
// and the update of the lane's cell in registers, so no residual vector is
// written; the first update from u = 0 needs no operator.  Updates alternate
// between the correction and one scratch vector per level.  Transfers embed
// a coarse cell's polynomial into its eight children (prolongation, added
// to the fine correction) and apply the transpose (restriction).  The coarsest level is solved exactly by a
// dense inverse, assembled once by applying the level operator to unit
// vectors (as the paper assembles its coarse LU) and inverted on the host.
//
// For n <= 4 every vector of a level is in the B = 64 blocked layout, one
// cell per lane; for n >= 5 in the B = 1 layout, one cell per wave.  Every
// kernel returns at once when the solve state passed to it is done,
// so a V-cycle can sit inside a captured chunk of CG iterations.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <type_traits>
#include <vector>

#include "sipg.h"

namespace tpfdm {

constexpr int64_t kMaxCoarse = 2048;   // unknowns of the densely solved coarsest level

template <int N>
struct ProlTab {    // 1D embeddings of the left and right child, row-major
    double p[2][N * N];
};

namespace {

__device__ __forceinline__ bool done_flag(const PcgState* st) { return st && st->done; }

// Level vectors are stored in TS (double, or float for the FP32-storage
// hierarchy).  The operator rows of the smoother and of the residual are
// computed in MgTC<TS>: FP64 for FP64 storage, FP32 for FP32 storage (there
// the level vectors carry FP32 rounding already, and the FP32 rows take half
// the registers and LDS of FP64 ones); the smoother's block inverse runs in
// TI, the transfers and the first update in FP64, and every kernel rounds
// only where it stores.
template <typename TS>
using MgTC = typename std::conditional<std::is_same<TS, float>::value, float, double>::type;

// Minimum resident waves per SIMD the lane operator-row kernels are built
// for: four for the FP32 rows of the Hermite-type basis (126 VGPRs, no
// spills; 3% faster MG-PCG at p = 3 on 128^3 cells than at three waves),
// otherwise two (the FP32 Lagrange rows spill 164 bytes per lane at four).
template <typename TS, bool HERM, typename TI>
constexpr int mg_lane_waves() {
    return sizeof(TS) == 4 && sizeof(TI) == 4 && HERM ? 4 : 2;
}

// t = A u on one level (one cell per lane); the consumers form b - t as
// they load, which keeps b out of this kernel's registers.
template <int N, bool HERM, typename TS>
__global__ __launch_bounds__(64, (mg_lane_waves<TS, HERM, TS>())) void k_mg_apply(const TS* __restrict__ u, TS* __restrict__ t, MeshArgs G,
                                                  Pair<N, MgTC<TS>> R, FaceRef<N, MgTC<TS>> F,
                                                  const PcgState* __restrict__ st) {
    using TC = MgTC<TS>;
    if (done_flag(st)) return;
    constexpr int N3 = N * N * N;
    __shared__ TC sa[N * N][64], sbt[N * N][64];
    const int64_t c = static_cast<int64_t>(lane_tile(blockIdx.x, gridDim.x, plane_tiles<N, TS, HERM>(G))) * 64 + threadIdx.x;
    if (c >= G.ncells) return;
    TC acc[N3];
    sipg_cell<N, TS, TC, -1, HERM>(u, G, R, F, c, acc, sa, sbt);
    const int64_t base = G.offset + block_base(c, 6, N3);
#pragma unroll
    for (int e = 0; e < N3; ++e) {
        const int64_t o = base + (static_cast<int64_t>(e) << 6);
        t[o] = static_cast<TS>(acc[e]);
    }
}

// u = omega D^{-1} b: the first Chebyshev update from u = 0 (no operator
// application), the block inverse in precision TI.
template <int N, typename TI, typename TS>
__global__ __launch_bounds__(64, 2) void k_mg_jacobi0(const TS* __restrict__ b, TS* __restrict__ u,
                                                    MeshArgs G, Eig<N, TI> E, double omega,
                                                    const PcgState* __restrict__ st) {
    if (done_flag(st)) return;
    constexpr int N3 = N * N * N;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 64 + threadIdx.x;
    if (c >= G.ncells) return;
    const int64_t base = G.offset + block_base(c, 6, N3);
    TI v[N3];
#pragma unroll
    for (int e = 0; e < N3; ++e) v[e] = static_cast<TI>(b[base + (static_cast<int64_t>(e) << 6)]);
    lane_fdm_inplace<N, TI>(v, E, static_cast<TI>(G.sx), static_cast<TI>(G.sy), static_cast<TI>(G.sz));
#pragma unroll
    for (int e = 0; e < N3; ++e)
        u[base + (static_cast<int64_t>(e) << 6)] = static_cast<TS>(omega * static_cast<double>(v[e]));
}

// One Chebyshev update in a single pass (the factorized form: no residual
// vector is stored): u_out = u_in + omega D^{-1} (b - A u_in) for the lane's
// cell, A u_in from the cell and its six neighbours, the block inverse in
// precision TI on the residual registers.  u_out must not alias u_in (other
// lanes still read u_in).
template <int N, typename TI, bool HERM, typename TS>
__global__ __launch_bounds__(64, (mg_lane_waves<TS, HERM, TI>())) void k_mg_smooth(const TS* __restrict__ b, const TS* __restrict__ uin,
                                                   TS* __restrict__ uout, MeshArgs G, Pair<N, MgTC<TS>> R,
                                                   FaceRef<N, MgTC<TS>> F, Eig<N, TI> E, double omega,
                                                   const PcgState* __restrict__ st) {
    using TC = MgTC<TS>;
    if (done_flag(st)) return;
    constexpr int N3 = N * N * N;
    __shared__ TC sa[N * N][64], sbt[N * N][64];
    const int64_t c = static_cast<int64_t>(lane_tile(blockIdx.x, gridDim.x, plane_tiles<N, TS, HERM>(G))) * 64 + threadIdx.x;
    if (c >= G.ncells) return;
    TC acc[N3];
    sipg_cell<N, TS, TC, -1, HERM>(uin, G, R, F, c, acc, sa, sbt);
    const int64_t base = G.offset + block_base(c, 6, N3);
    TI v[N3];
#pragma unroll
    for (int e = 0; e < N3; ++e)
        v[e] = static_cast<TI>(static_cast<TC>(b[base + (static_cast<int64_t>(e) << 6)]) - acc[e]);
    lane_fdm_inplace<N, TI>(v, E, static_cast<TI>(G.sx), static_cast<TI>(G.sy), static_cast<TI>(G.sz));
#pragma unroll
    for (int e = 0; e < N3; ++e) {
        const int64_t o = base + (static_cast<int64_t>(e) << 6);
        uout[o] = static_cast<TS>(fma(omega, static_cast<double>(v[e]), static_cast<double>(uin[o])));
    }
}

// acc += (X (x) Y (x) Z) w for one cell, the input streamed one x-plane at
// a time (X acts on x, the slowest index).
template <int N, typename LoadF>
__device__ __forceinline__ void kron3_accumulate(LoadF load, const double* X, const double* Y, const double* Z,
                                                 double (&acc)[N * N * N]) {
#pragma unroll
    for (int ip = 0; ip < N; ++ip) {
        double pl[N * N];
#pragma unroll
        for (int q = 0; q < N * N; ++q) pl[q] = load(ip * N * N + q);
        double t1[N * N];
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
            for (int k = 0; k < N; ++k) {
                double sacc = 0.0;
#pragma unroll
                for (int kk = 0; kk < N; ++kk) sacc = fma(Z[k * N + kk], pl[j * N + kk], sacc);
                t1[j * N + k] = sacc;
            }
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
            for (int k = 0; k < N; ++k) {
                double sacc = 0.0;
#pragma unroll
                for (int jj = 0; jj < N; ++jj) sacc = fma(Y[j * N + jj], t1[jj * N + k], sacc);
#pragma unroll
                for (int i = 0; i < N; ++i) acc[(i * N + j) * N + k] = fma(X[i * N + ip], sacc, acc[(i * N + j) * N + k]);
            }
    }
}

// b_coarse = P^T (b_fine - t_fine), t_fine = A u_fine: one coarse cell per
// lane, summed over its children.
template <int N, typename TS>
__global__ __launch_bounds__(64, 2) void k_mg_restrict(const TS* __restrict__ bf, const TS* __restrict__ tf,
                                                     TS* __restrict__ bc,
                                                     MeshArgs Gf, MeshArgs Gc, ProlTab<N> PT,
                                                     const PcgState* __restrict__ st) {
    if (done_flag(st)) return;
    constexpr int N3 = N * N * N;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 64 + threadIdx.x;
    if (c >= Gc.ncells) return;
    const uint32_t cu = static_cast<uint32_t>(c);
    const uint32_t cz = cu % static_cast<uint32_t>(Gc.mz);
    const uint32_t rr = cu / static_cast<uint32_t>(Gc.mz);
    const uint32_t cy = rr % static_cast<uint32_t>(Gc.my);
    const uint32_t cx = rr / static_cast<uint32_t>(Gc.my);
    double acc[N3];
#pragma unroll
    for (int e = 0; e < N3; ++e) acc[e] = 0.0;
#pragma unroll
    for (int ch = 0; ch < 8; ++ch) {
        const int bx = ch >> 2, by = (ch >> 1) & 1, bz = ch & 1;
        const int64_t f = (static_cast<int64_t>(2 * cx + bx) * Gf.my + (2 * cy + by)) * Gf.mz + (2 * cz + bz);
        const int64_t fb = Gf.offset + block_base(f, 6, N3);
        kron3_accumulate<N>(
            [&](int q) {
                const int64_t o = fb + (static_cast<int64_t>(q) << 6);
                return static_cast<double>(bf[o]) - static_cast<double>(tf[o]);
            },
            PT.p[bx], PT.p[by], PT.p[bz], acc);
    }
    const int64_t base = Gc.offset + block_base(c, 6, N3);
#pragma unroll
    for (int e = 0; e < N3; ++e) bc[base + (static_cast<int64_t>(e) << 6)] = static_cast<TS>(acc[e]);
}

// u_out = u_fine + P u_coarse: one fine cell per lane, the child's embedding
// selected per lane.
template <int N, typename TS>
__global__ __launch_bounds__(64, 2) void k_mg_prolong(const TS* __restrict__ uc, const TS* __restrict__ uf,
                                                    TS* __restrict__ uout,
                                                    MeshArgs Gf, MeshArgs Gc, ProlTab<N> P,
                                                    const PcgState* __restrict__ st) {
    if (done_flag(st)) return;
    constexpr int N3 = N * N * N, N2 = N * N;
    const int64_t f = static_cast<int64_t>(blockIdx.x) * 64 + threadIdx.x;
    if (f >= Gf.ncells) return;
    const uint32_t fu = static_cast<uint32_t>(f);
    const uint32_t fz = fu % static_cast<uint32_t>(Gf.mz);
    const uint32_t rr = fu / static_cast<uint32_t>(Gf.mz);
    const uint32_t fy = rr % static_cast<uint32_t>(Gf.my);
    const uint32_t fx = rr / static_cast<uint32_t>(Gf.my);
    const int64_t c = (static_cast<int64_t>(fx / 2) * Gc.my + fy / 2) * Gc.mz + fz / 2;
    double X[N2], Y[N2], Z[N2];
#pragma unroll
    for (int e = 0; e < N2; ++e) {
        X[e] = (fx & 1) ? P.p[1][e] : P.p[0][e];
        Y[e] = (fy & 1) ? P.p[1][e] : P.p[0][e];
        Z[e] = (fz & 1) ? P.p[1][e] : P.p[0][e];
    }
    const TS* w = uc + Gc.offset + block_base(c, 6, N3);
    double acc[N3];
#pragma unroll
    for (int e = 0; e < N3; ++e) acc[e] = 0.0;
    kron3_accumulate<N>([&](int q) { return static_cast<double>(w[static_cast<int64_t>(q) << 6]); }, X, Y, Z, acc);
    const int64_t base = Gf.offset + block_base(f, 6, N3);
#pragma unroll
    for (int e = 0; e < N3; ++e) {
        const int64_t o = base + (static_cast<int64_t>(e) << 6);
        uout[o] = static_cast<TS>(static_cast<double>(uf[o]) + acc[e]);
    }
}

// u = A0^{-1} b on the coarsest level: b gathered into LDS in canonical
// order, one row of the (column-major) inverse per thread.
template <int N, typename TS>
__global__ __launch_bounds__(256) void k_mg_coarse(const double* __restrict__ inv, const TS* __restrict__ b,
                                                   TS* __restrict__ u, int64_t n0, int64_t offset, int lb,
                                                   const PcgState* __restrict__ st) {
    if (done_flag(st)) return;
    constexpr int N3 = N * N * N;
    __shared__ double sb[kMaxCoarse];
    for (int64_t e = threadIdx.x; e < n0; e += 256)
        sb[e] = static_cast<double>(b[offset + block_base(e / N3, lb, N3) + ((e % N3) << lb)]);
    __syncthreads();
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n0) return;
    double s = 0.0;
    for (int64_t j = 0; j < n0; ++j) s = fma(inv[j * n0 + i], sb[j], s);
    u[offset + block_base(i / N3, lb, N3) + ((i % N3) << lb)] = static_cast<TS>(s);
}

// Partial (a, b) per 64-cell tile (the layout of the PCG partials).
template <int N, typename TS>
__global__ __launch_bounds__(64) void k_mg_dot(const double* __restrict__ a, const TS* __restrict__ b,
                                               MeshArgs G, double* __restrict__ part,
                                               const PcgState* __restrict__ st) {
    if (done_flag(st)) return;
    constexpr int N3 = N * N * N;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 64 + threadIdx.x;
    double s = 0.0;
    if (c < G.ncells) {
        const int64_t base = G.offset + block_base(c, 6, N3);
#pragma unroll
        for (int e = 0; e < N3; ++e) {
            const int64_t o = base + (static_cast<int64_t>(e) << 6);
            s = fma(a[o], static_cast<double>(b[o]), s);
        }
    }
    s = wave_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// ---------------------------------------------------------------- n >= 5
// One cell per wave (layout B = 1, FP64 or FP32 level vectors; the
// operator rows in the storage type, the transfers in FP64): lane (a, b) owns
// the z-pencil (a, b, 0..n-1) of the cell for loads and stores; the
// operator row is the wave body of the coupled operator (wave_sipg_cell,
// output by x-pencils), the block inverse the even-odd fast
// diagonalization in an LDS slab, and the transfers three 1D contractions
// through an LDS slab.

// Pencil base of lane (pa, pb)'s z-pencil of cell c.
template <int N>
__device__ __forceinline__ int64_t zpencil_base(const MeshArgs& G, int64_t c, const Pencil<N>& pc) {
    return G.offset + block_base(c, G.logB, N * N * N) + (static_cast<int64_t>((pc.pa * N + pc.pb) * N) << G.logB);
}

// The even-odd tables of a wave operator row: FP64 ones are read where they
// are used at wave-uniform global addresses (scalar loads), FP32 ones are
// loaded into registers once.
template <typename T, int TAB>
__device__ __forceinline__ const T* wave_row_tables(T (&regs)[sizeof(T) == 8 ? 1 : TAB], const T* tab) {
    if constexpr (sizeof(T) == 8) {
        return tab;
    } else {
        load_table<T, TAB>(regs, tab, nullptr);
        return regs;
    }
}

// t = A u, one cell per wave; the row in the level storage type T.
template <int N, bool VP, typename T = double>
__global__ __launch_bounds__(64, 2) void k_mg_apply_wave(const T* __restrict__ u, T* __restrict__ t,
                                                       MeshArgs G, const T* __restrict__ tab,
                                                       FaceRef<N, T> F, const PcgState* __restrict__ st) {
    if (done_flag(st)) return;
    constexpr int TAB = 2 * (EOShape<N>::SE + EOShape<N>::SO);
    __shared__ WaveLds<N, T> L;
    T regs[sizeof(T) == 8 ? 1 : TAB];
    const T* tb = wave_row_tables<T, TAB>(regs, tab);
    const int64_t c = xcd_tile(blockIdx.x, gridDim.x);
    T y[N];
    wave_sipg_cell<N, T, VP, false>(u, G, tb, F, c, L, y);
    const Pencil<N> pc(1);
    if (pc.act) {
        T* out = t + G.offset + block_base(c, G.logB, N * N * N);
#pragma unroll
        for (int i = 0; i < N; ++i) out[static_cast<int64_t>((i * N + pc.pa) * N + pc.pb) << G.logB] = y[i];
    }
}

// z-pencil in, z = omega D^{-1} r of the wave's cell in precision TI in the
// slab, the lane's z-pencil of it returned (every lane of the wave calls it).
template <int N, typename TI>
__device__ __forceinline__ void wave_block_inverse(const Pencil<N>& pc, TI* slab, const TI* T, const TI* lam,
                                                   const MeshArgs& G, double (&r)[N]) {
    using SL = Slab<N>;
    eo_inverse_lds<N, TI>(pc, slab, T, T + EOShape<N>::SE, lam, static_cast<TI>(G.sx), static_cast<TI>(G.sy),
                          static_cast<TI>(G.sz));
    if (pc.act)
#pragma unroll
        for (int k = 0; k < N; ++k) r[k] = static_cast<double>(slab[SL::at(pc.pa, pc.pb, k)]);
}

// u = omega D^{-1} b (the first Chebyshev update from u = 0), one cell per wave.
template <int N, typename TI, bool VP, typename TS = double>
__global__ __launch_bounds__(64, 2) void k_mg_jacobi0_wave(const TS* __restrict__ b, TS* __restrict__ u,
                                                         MeshArgs G, const TI* __restrict__ tabS, double omega,
                                                         const PcgState* __restrict__ st) {
    if (done_flag(st)) return;
    using SL = Slab<N>;
    constexpr int TABM = EOShape<N>::SE + EOShape<N>::SO;
    __shared__ TI slab[SL::size];
    __shared__ TI stab[TABM + N];
    for (int e = threadIdx.x; e < TABM + N; e += 64) stab[e] = tabS[e];
    const int64_t c = blockIdx.x;
    const Pencil<N> pc(1);
    const int64_t pb = zpencil_base<N>(G, c, pc);
    double v[N];
    if (pc.act) {
        pencil_load<N, VP>(v, b + pb, G.logB);
#pragma unroll
        for (int k = 0; k < N; ++k) slab[SL::at(pc.pa, pc.pb, k)] = static_cast<TI>(v[k]);
    }
    wave_sync();
    wave_block_inverse<N, TI>(pc, slab, stab, stab + TABM, G, v);
    if (pc.act) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] *= omega;
        pencil_store<N, VP>(u + pb, v, G.logB);
    }
}

// One Chebyshev update u_out = u_in + omega D^{-1} (b - A u_in) of the
// wave's cell: the operator row by x-pencils, the residual into the slab in
// precision TI, the block inverse, the update by z-pencils.
template <int N, typename TI, bool VP, typename T = double>
__global__ __launch_bounds__(64, 2) void k_mg_smooth_wave(const T* __restrict__ b,
                                                        const T* __restrict__ uin, T* __restrict__ uout,
                                                        MeshArgs G, const T* __restrict__ tab,
                                                        FaceRef<N, T> F, const TI* __restrict__ tabS,
                                                        double omega, const PcgState* __restrict__ st) {
    if (done_flag(st)) return;
    using SL = Slab<N>;
    constexpr int TAB = 2 * (EOShape<N>::SE + EOShape<N>::SO);
    constexpr int TABM = EOShape<N>::SE + EOShape<N>::SO;
    __shared__ __align__(16) WaveLds<N, T> L;
    // the inverse's slab: the face scratch when it fits there, else the
    // whole (by then free) operator scratch, block slab included
    constexpr bool kInT = SL::size * sizeof(TI) <= sizeof(WaveLds<N, T>::t);
    static_assert(SL::size * sizeof(TI) <= sizeof(WaveLds<N, T>), "slab exceeds the operator scratch");
    __shared__ TI stab[TABM + N];
    for (int e = threadIdx.x; e < TABM + N; e += 64) stab[e] = tabS[e];
    T regs[sizeof(T) == 8 ? 1 : TAB];
    const T* tb = wave_row_tables<T, TAB>(regs, tab);
    const int64_t c = xcd_tile(blockIdx.x, gridDim.x);
    const Pencil<N> pc(1);
    const T* bb = b + G.offset + block_base(c, G.logB, N * N * N);
    // FP32: the lane's x-pencil of b and z-pencil of u_in are loaded before
    // the operator row, so that their latency overlaps it (measured at p = 7
    // on 48^3 cells: MG-PCG 84.8 -> 74.8 ms, at five waves per SIMD instead
    // of seven); in FP64 the 32 more registers cost a wave per SIMD and the
    // solve time stays the same, so FP64 loads them where they are used
    constexpr bool kPre = sizeof(T) == 4;
    T bx[kPre ? N : 1];
    T uz[kPre ? N : 1];
    if constexpr (kPre) {
        if (pc.act) {
#pragma unroll
            for (int i = 0; i < N; ++i) bx[i] = bb[static_cast<int64_t>((i * N + pc.pa) * N + pc.pb) << G.logB];
            pencil_load<N, VP>(uz, uin + zpencil_base<N>(G, c, pc), G.logB);
        }
    }
    T y[N];
    wave_sipg_cell<N, T, VP, false>(uin, G, tb, F, c, L, y);   // ends synced
    TI* slab = kInT ? reinterpret_cast<TI*>(L.t) : reinterpret_cast<TI*>(&L);
    if (pc.act)
#pragma unroll
        for (int i = 0; i < N; ++i) {
            T bv;
            if constexpr (kPre) bv = bx[i];
            else bv = bb[static_cast<int64_t>((i * N + pc.pa) * N + pc.pb) << G.logB];
            slab[SL::at(i, pc.pa, pc.pb)] = static_cast<TI>(bv - y[i]);
        }
    wave_sync();
    double d[N];
    wave_block_inverse<N, TI>(pc, slab, stab, stab + TABM, G, d);
    if (pc.act) {
        const int64_t pb = zpencil_base<N>(G, c, pc);
        double uv[N];
        if constexpr (kPre) {
#pragma unroll
            for (int k = 0; k < N; ++k) uv[k] = static_cast<double>(uz[k]);
        } else {
            pencil_load<N, VP>(uv, uin + pb, G.logB);
        }
#pragma unroll
        for (int k = 0; k < N; ++k) uv[k] = fma(omega, d[k], uv[k]);
        pencil_store<N, VP>(uout + pb, uv, G.logB);
    }
}

// (X (x) Y (x) Z) applied to the slab's block, in place, X acting on x:
// the lane's z-pencil z enters in registers; on return the lane holds its
// x-pencil (x0..x_{n-1} at (pa, pb) = (j, k)) of the result in out.
template <int N>
__device__ __forceinline__ void wave_kron3(const Pencil<N>& pc, double* slab, const double* X, const double* Y,
                                           const double* Z, const double (&z)[N], double (&out)[N]) {
    using SL = Slab<N>;
    if (pc.act) {   // z: lane (i, j)
#pragma unroll
        for (int k = 0; k < N; ++k) {
            double sacc = 0.0;
#pragma unroll
            for (int kk = 0; kk < N; ++kk) sacc = fma(Z[k * N + kk], z[kk], sacc);
            slab[SL::at(pc.pa, pc.pb, k)] = sacc;
        }
    }
    wave_sync();
    if (pc.act) {   // y: lane (i, k)
        double v[N];
#pragma unroll
        for (int j = 0; j < N; ++j) v[j] = slab[SL::at(pc.pa, j, pc.pb)];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double sacc = 0.0;
#pragma unroll
            for (int jj = 0; jj < N; ++jj) sacc = fma(Y[j * N + jj], v[jj], sacc);
            slab[SL::at(pc.pa, j, pc.pb)] = sacc;
        }
    }
    wave_sync();
    if (pc.act) {   // x: lane (j, k)
        double v[N];
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = slab[SL::at(i, pc.pa, pc.pb)];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double sacc = 0.0;
#pragma unroll
            for (int ii = 0; ii < N; ++ii) sacc = fma(X[i * N + ii], v[ii], sacc);
            out[i] = sacc;
        }
    }
    wave_sync();
}

// b_coarse = P^T (b_fine - t_fine), one coarse cell per wave, summed over
// its eight children.
template <int N, bool VP, typename TS = double>
__global__ __launch_bounds__(64, 2) void k_mg_restrict_wave(const TS* __restrict__ bf,
                                                          const TS* __restrict__ tf, TS* __restrict__ bc,
                                                          MeshArgs Gf, MeshArgs Gc, ProlTab<N> PT,
                                                          const PcgState* __restrict__ st) {
    if (done_flag(st)) return;
    __shared__ double slab[Slab<N>::size];
    __shared__ double tabs[2 * N * N];
    for (int e = threadIdx.x; e < 2 * N * N; e += 64) tabs[e] = PT.p[e / (N * N)][e % (N * N)];
    wave_sync();
    const int64_t c = blockIdx.x;
    const uint32_t cu = static_cast<uint32_t>(c);
    const uint32_t cz = cu % static_cast<uint32_t>(Gc.mz);
    const uint32_t rr = cu / static_cast<uint32_t>(Gc.mz);
    const uint32_t cy = rr % static_cast<uint32_t>(Gc.my);
    const uint32_t cx = rr / static_cast<uint32_t>(Gc.my);
    const Pencil<N> pc(1);
    double acc[N];
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] = 0.0;
    for (int ch = 0; ch < 8; ++ch) {
        const int bx = ch >> 2, by = (ch >> 1) & 1, bz = ch & 1;
        const int64_t f = (static_cast<int64_t>(2 * cx + bx) * Gf.my + (2 * cy + by)) * Gf.mz + (2 * cz + bz);
        double z[N], out[N];
        if (pc.act) {
            const int64_t pb = zpencil_base<N>(Gf, f, pc);
            double tv[N];
            pencil_load<N, VP>(z, bf + pb, Gf.logB);
            pencil_load<N, VP>(tv, tf + pb, Gf.logB);
#pragma unroll
            for (int k = 0; k < N; ++k) z[k] -= tv[k];
        }
        wave_kron3<N>(pc, slab, tabs + bx * N * N, tabs + by * N * N, tabs + bz * N * N, z, out);
        if (pc.act)
#pragma unroll
            for (int i = 0; i < N; ++i) acc[i] += out[i];
    }
    if (pc.act) {
        TS* cb = bc + Gc.offset + block_base(c, Gc.logB, N * N * N);
#pragma unroll
        for (int i = 0; i < N; ++i)
            cb[static_cast<int64_t>((i * N + pc.pa) * N + pc.pb) << Gc.logB] = static_cast<TS>(acc[i]);
    }
}

// u_out = u_fine + P u_coarse, one fine cell per wave.
template <int N, bool VP, typename TS = double>
__global__ __launch_bounds__(64, 2) void k_mg_prolong_wave(const TS* __restrict__ uc,
                                                         const TS* __restrict__ uf, TS* __restrict__ uout,
                                                         MeshArgs Gf, MeshArgs Gc, ProlTab<N> P,
                                                         const PcgState* __restrict__ st) {
    if (done_flag(st)) return;
    __shared__ double slab[Slab<N>::size];
    __shared__ double tabs[2 * N * N];
    for (int e = threadIdx.x; e < 2 * N * N; e += 64) tabs[e] = P.p[e / (N * N)][e % (N * N)];
    wave_sync();
    const int64_t f = blockIdx.x;
    const uint32_t fu = static_cast<uint32_t>(f);
    const uint32_t fz = fu % static_cast<uint32_t>(Gf.mz);
    const uint32_t rr = fu / static_cast<uint32_t>(Gf.mz);
    const uint32_t fy = rr % static_cast<uint32_t>(Gf.my);
    const uint32_t fx = rr / static_cast<uint32_t>(Gf.my);
    const int64_t c = (static_cast<int64_t>(fx / 2) * Gc.my + fy / 2) * Gc.mz + fz / 2;
    const Pencil<N> pc(1);
    double z[N], out[N];
    if (pc.act) pencil_load<N, VP>(z, uc + zpencil_base<N>(Gc, c, pc), Gc.logB);
    wave_kron3<N>(pc, slab, tabs + (fx & 1) * N * N, tabs + (fy & 1) * N * N, tabs + (fz & 1) * N * N, z, out);
    if (pc.act) {
        const int64_t base = Gf.offset + block_base(f, Gf.logB, N * N * N);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int64_t o = base + (static_cast<int64_t>((i * N + pc.pa) * N + pc.pb) << Gf.logB);
            uout[o] = static_cast<TS>(static_cast<double>(uf[o]) + out[i]);
        }
    }
}

// Partial (a, b) per cell, one cell per wave.
template <int N, bool VP, typename TB = double>
__global__ __launch_bounds__(64) void k_mg_dot_wave(const double* __restrict__ a, const TB* __restrict__ b,
                                                    MeshArgs G, double* __restrict__ part,
                                                    const PcgState* __restrict__ st) {
    if (done_flag(st)) return;
    const int64_t c = blockIdx.x;
    const Pencil<N> pc(1);
    double s = 0.0;
    if (pc.act) {
        const int64_t pb = zpencil_base<N>(G, c, pc);
        double av[N], bv[N];
        pencil_load<N, VP>(av, a + pb, G.logB);
        pencil_load<N, VP>(bv, b + pb, G.logB);
#pragma unroll
        for (int k = 0; k < N; ++k) s = fma(av[k], bv[k], s);
    }
    s = wave_sum(s);
    if (threadIdx.x == 0) part[c] = s;
}

// The degree-coarsened coarsest level (n >= 5, Lagrange basis), used when
// the coarsest geometric level is too large for the dense solve: on the
// same cells the degree drops to 1 (eight unknowns per cell in canonical
// order, contiguous per cell), reached by the cellwise embedding
// E = E1 (x) E1 (x) E1 of Q_1 into Q_p, E1[i] = (1 - x_i, x_i) at the nodes
// x_i of [0, 1]; its operator is the Galerkin product E^T A E.
template <int N>
struct DegTab {
    double e[N][2];
};

// bc = E^T (b - t), one thread per coarse unknown (cell, jx, jy, jz).
template <int N, typename TS = double>
__global__ __launch_bounds__(64) void k_mg_deg_restrict(const TS* __restrict__ b, const TS* __restrict__ t,
                                                        double* __restrict__ bc, MeshArgs G, DegTab<N> E,
                                                        const PcgState* __restrict__ st) {
    if (done_flag(st)) return;
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * 64 + threadIdx.x;
    if (idx >= G.ncells * 8) return;
    const int64_t c = idx >> 3;
    const int jx = static_cast<int>(idx >> 2) & 1, jy = static_cast<int>(idx >> 1) & 1, jz = static_cast<int>(idx) & 1;
    const int64_t base = G.offset + block_base(c, G.logB, N * N * N);
    double s = 0.0;
    for (int a = 0; a < N; ++a)
        for (int q = 0; q < N; ++q) {
            const double wab = E.e[a][jx] * E.e[q][jy];
            for (int k = 0; k < N; ++k) {
                const int64_t o = base + (static_cast<int64_t>((a * N + q) * N + k) << G.logB);
                s = fma(wab * E.e[k][jz], static_cast<double>(b[o]) - static_cast<double>(t[o]), s);
            }
        }
    bc[idx] = s;
}

// uout = u + E uc, one thread per fine unknown.
template <int N, typename TS = double>
__global__ __launch_bounds__(64) void k_mg_deg_prolong(const double* __restrict__ uc, const TS* __restrict__ u,
                                                       TS* __restrict__ uout, MeshArgs G, DegTab<N> E,
                                                       const PcgState* __restrict__ st) {
    if (done_flag(st)) return;
    constexpr int N3 = N * N * N;
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * 64 + threadIdx.x;
    if (idx >= G.ncells * N3) return;
    const int64_t c = idx / N3;
    const int q = static_cast<int>(idx % N3);
    const int a = q / (N * N), y = (q / N) % N, k = q % N;
    const double* v = uc + c * 8;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s = fma(E.e[a][j >> 2] * E.e[y][(j >> 1) & 1] * E.e[k][j & 1], v[j], s);
    const int64_t o = G.offset + block_base(c, G.logB, N3) + (static_cast<int64_t>(q) << G.logB);
    uout[o] = static_cast<TS>(static_cast<double>(u[o]) + s);
}

template <int N>
DegTab<N> deg_table() {
    DegTab<N> E;
    double x[N];
    gll_points(N, x);
    for (int i = 0; i < N; ++i) E.e[i][0] = 1.0 - x[i], E.e[i][1] = x[i];
    return E;
}

// dst = src converted element by element (the finest level's right-hand
// side into the FP32-storage hierarchy, its result back to FP64).
template <typename TD, typename TSRC>
__global__ __launch_bounds__(256) void k_mg_convert(const TSRC* __restrict__ src, TD* __restrict__ dst, int64_t n,
                                                    const PcgState* __restrict__ st) {
    if (done_flag(st)) return;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * 256)
        dst[i] = static_cast<TD>(src[i]);
}

tp_status check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, what);
    return TP_OK;
}

// Cholesky factorization and inverse of a symmetric positive definite
// matrix (row-major), the triangular solves spread over host threads;
// the inverse is returned column-major (equal to row-major: symmetric).
bool spd_inverse(int64_t n, std::vector<double>& A, std::vector<double>& inv) {
    for (int64_t j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (int64_t k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
        if (!(d > 0.0)) return false;
        const double l = std::sqrt(d);
        A[j * n + j] = l;
        for (int64_t i = j + 1; i < n; ++i) {
            double s = A[i * n + j];
            for (int64_t k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = s / l;
        }
    }
    inv.assign(static_cast<size_t>(n * n), 0.0);
    const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    auto work = [&](unsigned tid) {
        std::vector<double> y(static_cast<size_t>(n));
        for (int64_t col = tid; col < n; col += nt) {
            for (int64_t i = 0; i < n; ++i) {       // L y = e_col
                double s = i == col ? 1.0 : 0.0;
                for (int64_t k = 0; k < i; ++k) s -= A[i * n + k] * y[k];
                y[i] = s / A[i * n + i];
            }
            for (int64_t i = n - 1; i >= 0; --i) {  // L^T x = y
                double s = y[i];
                for (int64_t k = i + 1; k < n; ++k) s -= A[k * n + i] * inv[col * n + k];
                inv[col * n + i] = s / A[i * n + i];
            }
        }
    };
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t) th.emplace_back(work, t);
    for (auto& t : th) t.join();
    return true;
}

}  // namespace

// Coarse inverses are shared by every hierarchy with the same coarsest level
// on a device and kept until the process ends.
struct CoarseKey {
    int device, n, basis, deg, mx, my, mz;
    double hx, hy, hz, C;
    bool operator<(const CoarseKey& o) const {
        return std::tie(device, n, basis, deg, mx, my, mz, hx, hy, hz, C) <
               std::tie(o.device, o.n, o.basis, o.deg, o.mx, o.my, o.mz, o.hx, o.hy, o.hz, o.C);
    }
};
static std::mutex g_coarse_mutex;
static std::map<CoarseKey, double*> g_coarse;

}  // namespace tpfdm

using namespace tpfdm;

struct MgLevel {
    MeshArgs G;
    int64_t elems = 0;
    void* t = nullptr;     // residual scratch
    void* b = nullptr;     // right-hand side (levels below the finest; every level with FP32 storage)
    void* u = nullptr;     // correction (levels below the finest; every level with FP32 storage)
};

struct tp_mg {
    tp_plan* plan = nullptr;
    int n = 0;
    int storage = TP_F64;           // element type of the level vectors (TP_F64 or TP_F32)
    std::vector<MgLevel> lv;
    double omega[3] = {0.0, 0.0, 0.0};
    double* coarse_inv = nullptr;   // shared, not owned
    int64_t n0 = 0;
    // degree-coarsened coarsest level (n >= 5): degree 1 on the last
    // geometric level's cells, right-hand side and correction of n0 values
    bool deg = false;
    double* deg_b = nullptr;
    double* deg_u = nullptr;
};

namespace {

template <int N, typename TI, bool HERM, typename TS>
tp_status vcycle_level(const tp_mg* m, size_t l, const TS* b, TS* u, const PcgState* st, hipStream_t s) {
    const Plan& plan = *m->plan;
    const MgLevel& L = m->lv[l];
    TS* Lt = static_cast<TS*>(L.t);
    const unsigned grid = static_cast<unsigned>((L.G.ncells + 63) / 64);
    if (l + 1 == m->lv.size()) {
        const unsigned cg = static_cast<unsigned>((m->n0 + 255) / 256);
        hipLaunchKernelGGL((k_mg_coarse<N, TS>), dim3(cg), dim3(256), 0, s, m->coarse_inv, b, u, m->n0, L.G.offset,
                           L.G.logB, st);
        return check_launch("coarse solve");
    }
    Pair<N, MgTC<TS>> R;
    FaceRef<N, MgTC<TS>> F;
    sipg_tables<N, MgTC<TS>>(plan, false, R, F);
    Eig<N, TI> E;
    for (int i = 0; i < N * N; ++i) E.s[i] = static_cast<TI>(plan.ref[N].S[i]);
    for (int i = 0; i < N; ++i) E.lam[i] = static_cast<TI>(plan.ref[N].lam[i]);
    ProlTab<N> P, PT;
    for (int i = 0; i < N * N; ++i) P.p[0][i] = plan.ref[N].P0[i], P.p[1][i] = plan.ref[N].P1[i];
    for (int c = 0; c < 2; ++c)
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) PT.p[c][i * N + j] = P.p[c][j * N + i];
    // Chebyshev updates ping-pong between u and the level's scratch t; the
    // prolongation writes out of place so that the last update lands in u.
    auto step = [&](const TS* from, TS* to, int j) {
        hipLaunchKernelGGL((k_mg_smooth<N, TI, HERM, TS>), dim3(grid), dim3(64), 0, s, b, from, to, L.G, R, F, E,
                           m->omega[j], st);
    };
    hipLaunchKernelGGL((k_mg_jacobi0<N, TI, TS>), dim3(grid), dim3(64), 0, s, b, u, L.G, E, m->omega[0], st);
    step(u, Lt, 1);
    step(Lt, u, 2);
    const MgLevel& C = m->lv[l + 1];
    TS* Cb = static_cast<TS*>(C.b);
    TS* Cu = static_cast<TS*>(C.u);
    hipLaunchKernelGGL((k_mg_apply<N, HERM, TS>), dim3(grid), dim3(64), 0, s, u, Lt, L.G, R, F, st);
    hipLaunchKernelGGL((k_mg_restrict<N, TS>), dim3(static_cast<unsigned>((C.G.ncells + 63) / 64)), dim3(64), 0, s, b,
                       Lt, Cb, L.G, C.G, PT, st);
    tp_status stt = check_launch("level transfer");
    if (stt != TP_OK) return stt;
    stt = vcycle_level<N, TI, HERM, TS>(m, l + 1, Cb, Cu, st, s);
    if (stt != TP_OK) return stt;
    hipLaunchKernelGGL((k_mg_prolong<N, TS>), dim3(grid), dim3(64), 0, s, Cu, u, Lt, L.G, C.G, P, st);
    step(Lt, u, 0);
    step(u, Lt, 1);
    step(Lt, u, 2);
    return check_launch("smoothing");
}

// The same V-cycle for n >= 5 on the wave kernels (layout B = 1: pencils
// move as 16-byte vectors where VP), level vectors and operator rows in TS
// (FP64, or FP32 for the FP32-storage hierarchy).
template <int N, typename TI, bool VP, typename TS>
tp_status vcycle_level_wave(const tp_mg* m, size_t l, const TS* b, TS* u, const PcgState* st,
                            hipStream_t s) {
    const Plan& plan = *m->plan;
    const MgLevel& L = m->lv[l];
    TS* Lt = static_cast<TS*>(L.t);
    const unsigned grid = static_cast<unsigned>(L.G.ncells);
    const bool last = l + 1 == m->lv.size();
    if (last && !m->deg) {
        const unsigned cg = static_cast<unsigned>((m->n0 + 255) / 256);
        hipLaunchKernelGGL((k_mg_coarse<N, TS>), dim3(cg), dim3(256), 0, s, m->coarse_inv, b, u, m->n0,
                           L.G.offset, L.G.logB, st);
        return check_launch("coarse solve");
    }
    FaceRef<N, TS> F;
    {
        Pair<N, TS> R;
        sipg_tables<N, TS>(plan, false, R, F);
    }
    const TS* tabA = reinterpret_cast<const TS*>(eo_table(plan, N, EO_APPLY_A, sizeof(TS) == 8 ? 0 : 1));
    const TI* tabS = reinterpret_cast<const TI*>(eo_table(plan, N, EO_INV, sizeof(TI) == 8 ? 0 : 1));
    ProlTab<N> P, PT;
    for (int i = 0; i < N * N; ++i) P.p[0][i] = plan.ref[N].P0[i], P.p[1][i] = plan.ref[N].P1[i];
    for (int c = 0; c < 2; ++c)
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) PT.p[c][i * N + j] = P.p[c][j * N + i];
    auto step = [&](const TS* from, TS* to, int j) {
        hipLaunchKernelGGL((k_mg_smooth_wave<N, TI, VP, TS>), dim3(grid), dim3(64), 0, s, b, from, to, L.G, tabA, F,
                           tabS, m->omega[j], st);
    };
    hipLaunchKernelGGL((k_mg_jacobi0_wave<N, TI, VP, TS>), dim3(grid), dim3(64), 0, s, b, u, L.G, tabS, m->omega[0],
                       st);
    step(u, Lt, 1);
    step(Lt, u, 2);
    if (last) {
        // coarse correction on the degree-1 level: E^T (b - A u), its dense
        // solve, u + E u_c
        const DegTab<N> E = deg_table<N>();
        hipLaunchKernelGGL((k_mg_apply_wave<N, VP, TS>), dim3(grid), dim3(64), 0, s, u, Lt, L.G, tabA, F, st);
        hipLaunchKernelGGL((k_mg_deg_restrict<N, TS>), dim3(static_cast<unsigned>((m->n0 + 63) / 64)), dim3(64), 0, s,
                           b, Lt, m->deg_b, L.G, E, st);
        hipLaunchKernelGGL((k_mg_coarse<2, double>), dim3(static_cast<unsigned>((m->n0 + 255) / 256)), dim3(256), 0, s,
                           m->coarse_inv, m->deg_b, m->deg_u, m->n0, int64_t(0), 0, st);
        hipLaunchKernelGGL((k_mg_deg_prolong<N, TS>),
                           dim3(static_cast<unsigned>((L.G.ncells * N * N * N + 63) / 64)), dim3(64), 0, s, m->deg_u,
                           u, Lt, L.G, E, st);
        tp_status stt = check_launch("degree-level correction");
        if (stt != TP_OK) return stt;
        step(Lt, u, 0);
        step(u, Lt, 1);
        step(Lt, u, 2);
        return check_launch("smoothing");
    }
    const MgLevel& C = m->lv[l + 1];
    TS* Cb = static_cast<TS*>(C.b);
    TS* Cu = static_cast<TS*>(C.u);
    hipLaunchKernelGGL((k_mg_apply_wave<N, VP, TS>), dim3(grid), dim3(64), 0, s, u, Lt, L.G, tabA, F, st);
    hipLaunchKernelGGL((k_mg_restrict_wave<N, VP, TS>), dim3(static_cast<unsigned>(C.G.ncells)), dim3(64), 0, s, b,
                       Lt, Cb, L.G, C.G, PT, st);
    tp_status stt = check_launch("level transfer");
    if (stt != TP_OK) return stt;
    stt = vcycle_level_wave<N, TI, VP, TS>(m, l + 1, Cb, Cu, st, s);
    if (stt != TP_OK) return stt;
    hipLaunchKernelGGL((k_mg_prolong_wave<N, VP, TS>), dim3(grid), dim3(64), 0, s, Cu, u, Lt, L.G, C.G, P, st);
    step(Lt, u, 0);
    step(u, Lt, 1);
    step(Lt, u, 2);
    return check_launch("smoothing");
}

template <typename TI, typename TS>
tp_status vcycle_dispatch(const tp_mg* m, const TS* b, TS* u, const PcgState* st, hipStream_t s) {
    switch (m->n) {
        case 2: return vcycle_level<2, TI, false, TS>(m, 0, b, u, st, s);
        case 3: return vcycle_level<3, TI, false, TS>(m, 0, b, u, st, s);
        case 4:
            return m->plan->basis == TP_BASIS_HERMITE ? vcycle_level<4, TI, true, TS>(m, 0, b, u, st, s)
                                                      : vcycle_level<4, TI, false, TS>(m, 0, b, u, st, s);
        default: break;
    }
    {
        // 16-byte pencil accesses when the caller's finest b and u allow them
        // (the level vectors are allocation-aligned) and a pencil is a whole
        // number of 16-byte vectors
        const bool vp = reinterpret_cast<uintptr_t>(b) % 16 == 0 && reinterpret_cast<uintptr_t>(u) % 16 == 0;
        constexpr bool v6 = (6 * sizeof(TS)) % 16 == 0;
        switch (m->n) {
            case 5: return vcycle_level_wave<5, TI, false, TS>(m, 0, b, u, st, s);
            case 6: return vp && v6 ? vcycle_level_wave<6, TI, v6, TS>(m, 0, b, u, st, s)
                                    : vcycle_level_wave<6, TI, false, TS>(m, 0, b, u, st, s);
            case 7: return vcycle_level_wave<7, TI, false, TS>(m, 0, b, u, st, s);
            case 8: return vp ? vcycle_level_wave<8, TI, true, TS>(m, 0, b, u, st, s)
                              : vcycle_level_wave<8, TI, false, TS>(m, 0, b, u, st, s);
            default: break;
        }
    }
    return set_error(TP_ERR_UNSUPPORTED, "multigrid supports n <= 8");
}

template <int N>
tp_status coarse_probe_n(const tp_mg* m, std::vector<double>& A) {
    const Plan& plan = *m->plan;
    const MgLevel& L = m->lv.back();
    Pair<N, double> R;
    FaceRef<N, double> F;
    sipg_tables<N, double>(plan, false, R, F);
    constexpr int N3 = N * N * N;
    const int64_t n0 = m->n0;
    A.assign(static_cast<size_t>(n0 * n0), 0.0);
    std::vector<double> col(static_cast<size_t>(L.elems));
    const unsigned grid = static_cast<unsigned>((L.G.ncells + 63) / 64);
    // FP64 probe vectors of the coarsest level (freed on return)
    double *pu = nullptr, *pt = nullptr;
    const size_t vb = static_cast<size_t>(L.elems) * sizeof(double);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&pu), vb);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&pt), vb);
    tp_status st = e == hipSuccess ? TP_OK : hip_error(e, "coarse probe vectors");
    // column j = A e_j, with pu = e_j as the probe
    for (int64_t j = 0; st == TP_OK && j < n0; ++j) {
        st = launch_fill(pu, L.elems, TP_F64, 0, true, nullptr);
        if (st != TP_OK) break;
        const double one = 1.0;
        const int64_t pos = L.G.offset + block_base(j / N3, L.G.logB, N3) + ((j % N3) << L.G.logB);
        e = hipMemcpy(pu + pos, &one, sizeof(double), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            st = hip_error(e, "coarse probe");
            break;
        }
        if constexpr (N <= kLaneMaxN)
            hipLaunchKernelGGL((k_mg_apply<N, false, double>), dim3(grid), dim3(64), 0, nullptr, pu, pt, L.G, R, F,
                               static_cast<const PcgState*>(nullptr));
        else
            hipLaunchKernelGGL((k_mg_apply_wave<N, false>), dim3(static_cast<unsigned>(L.G.ncells)), dim3(64), 0,
                               nullptr, pu, pt, L.G, reinterpret_cast<const double*>(eo_table(plan, N, EO_APPLY_A, 0)),
                               F, static_cast<const PcgState*>(nullptr));
        e = hipMemcpy(col.data(), pt, vb, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            st = hip_error(e, "coarse probe");
            break;
        }
        for (int64_t i = 0; i < n0; ++i)
            A[i * n0 + j] =
                col[static_cast<size_t>(L.G.offset + block_base(i / N3, L.G.logB, N3) + ((i % N3) << L.G.logB))];
    }
    if (pu) (void)hipFree(pu);
    if (pt) (void)hipFree(pt);
    return st;
}

// The Galerkin operator E^T A E of the degree-1 level, column by column:
// E e_j on the last geometric level, A of it, then E^T of that.
template <int N>
tp_status coarse_probe_deg(const tp_mg* m, std::vector<double>& A) {
    const Plan& plan = *m->plan;
    const MgLevel& L = m->lv.back();
    FaceRef<N, double> F;
    {
        Pair<N, double> R;
        sipg_tables<N, double>(plan, false, R, F);
    }
    const double* tabA = reinterpret_cast<const double*>(eo_table(plan, N, EO_APPLY_A, 0));
    const DegTab<N> E = deg_table<N>();
    const int64_t n0 = m->n0;
    A.assign(static_cast<size_t>(n0 * n0), 0.0);
    std::vector<double> col(static_cast<size_t>(n0));
    // FP64 probe vectors (freed on return): zero, E e_j and A E e_j on the
    // last geometric level, e_j and the column on the degree-1 level
    double *zf = nullptr, *pu = nullptr, *pt = nullptr, *ec = nullptr, *cc = nullptr;
    const size_t vb = static_cast<size_t>(L.elems) * sizeof(double);
    const size_t cb = static_cast<size_t>(n0) * sizeof(double);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&zf), vb);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&pu), vb);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&pt), vb);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&ec), cb);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&cc), cb);
    tp_status st = e == hipSuccess ? TP_OK : hip_error(e, "degree-level probe vectors");
    if (st == TP_OK) st = launch_fill(zf, L.elems, TP_F64, 0, true, nullptr);
    if (st == TP_OK) st = launch_fill(pu, L.elems, TP_F64, 0, true, nullptr);
    const PcgState* none = nullptr;
    const unsigned gf = static_cast<unsigned>((L.G.ncells * N * N * N + 63) / 64);
    const unsigned gc = static_cast<unsigned>((n0 + 63) / 64);
    for (int64_t j = 0; st == TP_OK && j < n0; ++j) {
        st = launch_fill(ec, n0, TP_F64, 0, true, nullptr);
        if (st != TP_OK) break;
        const double one = 1.0;
        e = hipMemcpy(ec + j, &one, sizeof(double), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            st = hip_error(e, "degree-level probe");
            break;
        }
        hipLaunchKernelGGL((k_mg_deg_prolong<N>), dim3(gf), dim3(64), 0, nullptr, ec, zf, pu, L.G, E, none);
        hipLaunchKernelGGL((k_mg_apply_wave<N, false>), dim3(static_cast<unsigned>(L.G.ncells)), dim3(64), 0, nullptr,
                           pu, pt, L.G, tabA, F, none);
        hipLaunchKernelGGL((k_mg_deg_restrict<N>), dim3(gc), dim3(64), 0, nullptr, pt, zf, cc, L.G, E, none);
        st = check_launch("degree-level probe");
        if (st != TP_OK) break;
        e = hipMemcpy(col.data(), cc, cb, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            st = hip_error(e, "degree-level probe");
            break;
        }
        for (int64_t i = 0; i < n0; ++i) A[i * n0 + j] = col[static_cast<size_t>(i)];
    }
    for (double* q : {zf, pu, pt, ec, cc})
        if (q) (void)hipFree(q);
    return st;
}

void free_mg(tp_mg* m) {
    for (auto& L : m->lv)
        for (void* p : {L.t, L.b, L.u})
            if (p) (void)hipFree(p);
    m->lv.clear();
    for (double* p : {m->deg_b, m->deg_u})
        if (p) (void)hipFree(p);
    m->deg_b = m->deg_u = nullptr;
}

template <int N, bool VP>
void launch_dot_wave(const MgLevel& L, const double* a, const void* b, bool b32, double* part, const PcgState* ps,
                     hipStream_t s) {
    const unsigned grid = static_cast<unsigned>(L.G.ncells);
    if (b32)
        hipLaunchKernelGGL((k_mg_dot_wave<N, VP, float>), dim3(grid), dim3(64), 0, s, a, static_cast<const float*>(b),
                           L.G, part, ps);
    else
        hipLaunchKernelGGL((k_mg_dot_wave<N, VP, double>), dim3(grid), dim3(64), 0, s, a, static_cast<const double*>(b),
                           L.G, part, ps);
}

tp_status convert_launch(const void* src, void* dst, bool to_f32, int64_t n, const PcgState* st, hipStream_t s) {
    const unsigned grid = static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 8192));
    if (to_f32)
        hipLaunchKernelGGL((k_mg_convert<float, double>), dim3(grid), dim3(256), 0, s, static_cast<const double*>(src),
                           static_cast<float*>(dst), n, st);
    else
        hipLaunchKernelGGL((k_mg_convert<double, float>), dim3(grid), dim3(256), 0, s, static_cast<const float*>(src),
                           static_cast<double*>(dst), n, st);
    return check_launch("multigrid conversion");
}

}  // namespace

namespace tpfdm {
tp_status mg_enqueue_vcycle(const tp_mg* m, const double* b, double* u, const void* st, bool f32, hipStream_t s) {
    // the smoother reads the plan's cell-block eigen tables at every enqueue
    if (m->plan->inverse_op != TP_OP_CELL || m->plan->factor_mode != TP_FACTOR_SCALED)
        return set_error(TP_ERR_STATE, "the plan's inverse setup is no longer TP_OP_CELL, TP_FACTOR_SCALED");
    const PcgState* ps = static_cast<const PcgState*>(st);
    if (m->storage == TP_F32) {
        // b into the hierarchy's FP32 right-hand side, the cycle, and (when
        // u is given) the FP32 result back to FP64
        const MgLevel& L0 = m->lv[0];
        tp_status r = convert_launch(b, L0.b, true, L0.elems, ps, s);
        if (r != TP_OK) return r;
        const float* b32 = static_cast<const float*>(L0.b);
        float* u32 = static_cast<float*>(L0.u);
        r = f32 ? vcycle_dispatch<float, float>(m, b32, u32, ps, s) : vcycle_dispatch<double, float>(m, b32, u32, ps, s);
        if (r != TP_OK || !u) return r;
        return convert_launch(u32, u, false, L0.elems, ps, s);
    }
    return f32 ? vcycle_dispatch<float, double>(m, b, u, ps, s) : vcycle_dispatch<double, double>(m, b, u, ps, s);
}

int mg_storage(const tp_mg* m) { return m->storage; }

const float* mg_result32(const tp_mg* m) {
    return m->storage == TP_F32 ? static_cast<const float*>(m->lv[0].u) : nullptr;
}

tp_status mg_enqueue_dot(const tp_mg* m, const double* a, const void* b, bool b32, double* part, const void* st,
                         hipStream_t s) {
    const MgLevel& L = m->lv[0];
    // 16-byte pencil loads for n = 8 (and n = 6 with FP64 b) when both
    // vectors are 16-byte aligned (solver and level vectors are)
    const bool vp = reinterpret_cast<uintptr_t>(a) % 16 == 0 && reinterpret_cast<uintptr_t>(b) % 16 == 0;
    const unsigned grid = static_cast<unsigned>((L.G.ncells + 63) / 64);
    const PcgState* ps = static_cast<const PcgState*>(st);
    const double* bd = static_cast<const double*>(b);
    const float* bf = static_cast<const float*>(b);
    switch (m->n) {
        case 2:
            if (b32) hipLaunchKernelGGL((k_mg_dot<2, float>), dim3(grid), dim3(64), 0, s, a, bf, L.G, part, ps);
            else hipLaunchKernelGGL((k_mg_dot<2, double>), dim3(grid), dim3(64), 0, s, a, bd, L.G, part, ps);
            break;
        case 3:
            if (b32) hipLaunchKernelGGL((k_mg_dot<3, float>), dim3(grid), dim3(64), 0, s, a, bf, L.G, part, ps);
            else hipLaunchKernelGGL((k_mg_dot<3, double>), dim3(grid), dim3(64), 0, s, a, bd, L.G, part, ps);
            break;
        case 4:
            if (b32) hipLaunchKernelGGL((k_mg_dot<4, float>), dim3(grid), dim3(64), 0, s, a, bf, L.G, part, ps);
            else hipLaunchKernelGGL((k_mg_dot<4, double>), dim3(grid), dim3(64), 0, s, a, bd, L.G, part, ps);
            break;
        case 5: launch_dot_wave<5, false>(L, a, b, b32, part, ps, s); break;
        case 6:
            if (vp && !b32) launch_dot_wave<6, true>(L, a, b, b32, part, ps, s);
            else launch_dot_wave<6, false>(L, a, b, b32, part, ps, s);
            break;
        case 7: launch_dot_wave<7, false>(L, a, b, b32, part, ps, s); break;
        case 8:
            if (vp) launch_dot_wave<8, true>(L, a, b, b32, part, ps, s);
            else launch_dot_wave<8, false>(L, a, b, b32, part, ps, s);
            break;
        default: return set_error(TP_ERR_UNSUPPORTED, "multigrid supports n <= 8");
    }
    return check_launch("dot");
}

tp_status mg_enqueue_widen(const tp_mg* m, double* dst, hipStream_t s) {
    if (m->storage != TP_F32) return set_error(TP_ERR_STATE, "the multigrid stores its levels in FP64");
    return convert_launch(m->lv[0].u, dst, false, m->lv[0].elems, nullptr, s);
}

const tp_plan* mg_plan(const tp_mg* m) { return m->plan; }
}  // namespace tpfdm

extern "C" {

tp_status tp_mg_create(tp_plan* plan, tp_mg** out) { return tp_mg_create_typed(plan, TP_F64, out); }

tp_status tp_mg_create_typed(tp_plan* plan, tp_dtype storage, tp_mg** out) {
    if (!out) return set_error(TP_ERR_ARG, "out must be non-null");
    *out = nullptr;
    if (!plan) return set_error(TP_ERR_ARG, "plan is null");
    if (storage != TP_F64 && storage != TP_F32)
        return set_error(TP_ERR_UNSUPPORTED, "multigrid level vectors are stored in FP64 or FP32");
    if (!plan->mesh) return set_error(TP_ERR_UNSUPPORTED, "multigrid needs a mesh plan");
    const GroupInfo& g = plan->groups[0];
    if (g.n <= kLaneMaxN && g.logB != 6)
        return set_error(TP_ERR_UNSUPPORTED, "multigrid needs the layout B = 64 for n <= 4");
    if (g.n > kLaneMaxN && g.logB != 0)
        return set_error(TP_ERR_UNSUPPORTED, "multigrid needs the layout B = 1 for n >= 5");
    if (g.n > kLaneMaxN && plan->basis == TP_BASIS_HERMITE)
        return set_error(TP_ERR_UNSUPPORTED, "multigrid in the Hermite-type basis supports n = 4");
    if (plan->inverse_op != TP_OP_CELL || plan->factor_mode != TP_FACTOR_SCALED)
        return set_error(TP_ERR_STATE, "multigrid needs tp_setup_inverse(TP_OP_CELL, TP_FACTOR_SCALED) first");
    tp_mg* m = new (std::nothrow) tp_mg();
    if (!m) return set_error(TP_ERR_OOM, "host allocation failed");
    m->plan = plan;
    m->n = g.n;
    m->storage = storage;
    const size_t es = storage == TP_F32 ? sizeof(float) : sizeof(double);
    const double a = 0.2, b = 2.0, c = 0.5 * (a + b), d = 0.5 * (b - a);
    for (int j = 1; j <= 3; ++j) m->omega[j - 1] = 1.0 / (c - d * std::cos((2 * j - 1) * 3.141592653589793 / 6.0));
    // levels
    int mx = plan->mesh_m[0], my = plan->mesh_m[1], mz = plan->mesh_m[2];
    double hx = plan->mesh_h[0], hy = plan->mesh_h[1], hz = plan->mesh_h[2];
    const int64_t n3 = int64_t(g.n) * g.n * g.n;
    hipError_t e = hipSuccess;
    for (;;) {
        MgLevel L;
        L.G.ncells = int64_t(mx) * my * mz;
        L.G.offset = 0;
        L.G.logB = g.logB;
        L.G.mx = mx;
        L.G.my = my;
        L.G.mz = mz;
        L.G.sx = hy * hz / hx;
        L.G.sy = hx * hz / hy;
        L.G.sz = hx * hy / hz;
        const int64_t B = int64_t(1) << g.logB;
        L.elems = (L.G.ncells + B - 1) / B * n3 * B;
        const size_t vb = static_cast<size_t>(L.elems) * es;
        if (e == hipSuccess) e = hipMalloc(&L.t, vb);
        // the finest level works on the caller's b and u, except with FP32
        // storage, whose finest level has its own FP32 copies
        if (!m->lv.empty() || storage == TP_F32) {
            if (e == hipSuccess) e = hipMalloc(&L.b, vb);
            if (e == hipSuccess) e = hipMalloc(&L.u, vb);
        }
        m->lv.push_back(L);
        if (e != hipSuccess || mx % 2 || my % 2 || mz % 2) break;
        mx /= 2, my /= 2, mz /= 2;
        hx *= 2, hy *= 2, hz *= 2;
    }
    if (e != hipSuccess) {
        free_mg(m);
        delete m;
        (void)hipGetLastError();
        return set_error(TP_ERR_OOM, "multigrid workspace allocation failed");
    }
    const MgLevel& Lc = m->lv.back();
    m->n0 = Lc.G.ncells * n3;
    if (m->n0 > kMaxCoarse && g.n > kLaneMaxN && Lc.G.ncells * 8 <= kMaxCoarse) {
        // too large for the dense solve at degree p: one more level of
        // degree 1 on the same cells (Lagrange basis; n >= 5 only)
        m->deg = true;
        m->n0 = Lc.G.ncells * 8;
        const size_t cb = static_cast<size_t>(m->n0) * sizeof(double);
        e = hipMalloc(reinterpret_cast<void**>(&m->deg_b), cb);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&m->deg_u), cb);
        if (e != hipSuccess) {
            free_mg(m);
            delete m;
            (void)hipGetLastError();
            return set_error(TP_ERR_OOM, "multigrid workspace allocation failed");
        }
    }
    if (m->n0 > kMaxCoarse) {
        free_mg(m);
        delete m;
        return set_error(TP_ERR_UNSUPPORTED, "the coarsest level (" + std::to_string(m->n0) +
                                                 " unknowns) is too large for its dense solve");
    }
    if (m->lv.size() == 1 && !m->lv[0].b && !m->deg) {   // no coarser level: the finest is solved densely; it needs b and u scratch
        MgLevel& L0 = m->lv[0];
        const size_t vb = static_cast<size_t>(L0.elems) * es;
        e = hipMalloc(&L0.b, vb);
        if (e == hipSuccess) e = hipMalloc(&L0.u, vb);
        if (e != hipSuccess) {
            free_mg(m);
            delete m;
            (void)hipGetLastError();
            return set_error(TP_ERR_OOM, "multigrid workspace allocation failed");
        }
    }
    // the coarse inverse, shared per device and coarsest level
    int dev = 0;
    (void)hipGetDevice(&dev);
    const CoarseKey key{dev, g.n, plan->basis, m->deg ? 1 : 0, Lc.G.mx, Lc.G.my, Lc.G.mz, hx, hy, hz, plan->penalty_C};
    std::lock_guard<std::mutex> lock(g_coarse_mutex);
    auto it = g_coarse.find(key);
    if (it != g_coarse.end()) {
        m->coarse_inv = it->second;
    } else {
        std::vector<double> A, inv;
        tp_status st = TP_OK;
        if (m->deg) {
            switch (g.n) {
                case 5: st = coarse_probe_deg<5>(m, A); break;
                case 6: st = coarse_probe_deg<6>(m, A); break;
                case 7: st = coarse_probe_deg<7>(m, A); break;
                default: st = coarse_probe_deg<8>(m, A); break;
            }
        } else {
            switch (g.n) {
                case 2: st = coarse_probe_n<2>(m, A); break;
                case 3: st = coarse_probe_n<3>(m, A); break;
                case 4: st = coarse_probe_n<4>(m, A); break;
                case 5: st = coarse_probe_n<5>(m, A); break;
                case 6: st = coarse_probe_n<6>(m, A); break;
                case 7: st = coarse_probe_n<7>(m, A); break;
                default: st = coarse_probe_n<8>(m, A); break;
            }
        }
        if (st == TP_OK && !spd_inverse(m->n0, A, inv))
            st = set_error(TP_ERR_NOT_SPD, "the coarsest level operator is not positive definite");
        double* dinv = nullptr;
        if (st == TP_OK) {
            e = hipMalloc(reinterpret_cast<void**>(&dinv), inv.size() * sizeof(double));
            if (e == hipSuccess)
                e = hipMemcpy(dinv, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice);
            if (e != hipSuccess) st = hip_error(e, "coarse inverse upload");
        }
        if (st != TP_OK) {
            if (dinv) (void)hipFree(dinv);
            free_mg(m);
            delete m;
            return st;
        }
        g_coarse[key] = dinv;
        m->coarse_inv = dinv;
    }
    *out = m;
    return TP_OK;
}

tp_status tp_mg_vcycle(tp_mg* m, const double* b, double* x, hipStream_t stream) {
    if (!m) return set_error(TP_ERR_ARG, "multigrid is null");
    if (!b || !x) return set_error(TP_ERR_ARG, "b and x must be non-null");
    if (static_cast<const void*>(b) == static_cast<const void*>(x)) return set_error(TP_ERR_ARG, "b and x must not alias");
    return mg_enqueue_vcycle(m, b, x, nullptr, false, stream);
}

tp_status tp_mg_destroy(tp_mg* m) {
    if (!m) return TP_OK;
    free_mg(m);
    delete m;
    return TP_OK;
}

}  // extern "C"
