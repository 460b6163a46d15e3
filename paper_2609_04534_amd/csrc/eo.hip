// Wave-per-tile kernels for n >= 5 (and any n on request) with even-odd
// factored 1D matrices.
//
// The 1D mass, stiffness and penalized stiffness matrices of the
// Gauss-Lobatto basis are centrosymmetric (A[i][j] = A[n-1-i][n-1-j]), so a
// product y = A x splits into the even part e_j = x_j + x_{n-1-j} and the odd
// part o_j = x_j - x_{n-1-j}:  y_i = E_i + O_i,  y_{n-1-i} = E_i - O_i with
// E = A_E e (ceil(n/2) x ceil(n/2)) and O = A_O o (floor(n/2) x floor(n/2)).
// The generalized eigenvectors of such a pencil are symmetric or
// antisymmetric, so S^T x and S y split the same way.  This halves the
// multiply-adds and the size of the matrices; the halved matrices are read
// at wave-uniform addresses (FP32, and FP64 from n = 5 on: scalar
// registers) or held in VGPRs (FP64 below n = 5).
//
// Mapping: one wave per tile of BPW blocks, each block's slab in LDS, one
// pencil per lane and phase (see Slab/Pencil); a persistent grid loops over
// tiles and loads tile t + grid into registers while tile t is computed.
#include <algorithm>
#include <climits>
#include <type_traits>

#include "eo.h"

namespace tpfdm {

namespace {

// From this n on, the FP64 apply and inverse read their halved matrices at
// wave-uniform global addresses (scalar loads into SGPRs, served by the
// scalar cache) instead of holding them in VGPRs: at n = 8 that frees 125
// of 232 VGPRs in apply and 60 of 148 in the inverse, for two more waves
// per SIMD (measured on 16.8 M DoF: apply 10-22 % and inverse up to 8 %
// faster for n = 5..8, results bit-identical).
constexpr int kEoScalarTabN = 5;

// v = A u.  Table: ME | MO | PE | PO.
// Per tile: z-phase from the prefetched pencil registers, y-phase and
// x-phase through LDS, x-phase results stored straight to global memory
// (lanes (j, k) of one output plane are consecutive addresses).
template <int N, typename TS, typename TC, bool VP>
__global__ __launch_bounds__(64, 2) void k_apply_eo(const TS* __restrict__ u, TS* __restrict__ v, GArgs G,
                                                    const TC* __restrict__ tab, int64_t ntiles) {
    using L = Slab<N>;
    using S = EOShape<N>;
    constexpr int HC = S::HC, H = S::H;
    constexpr int TAB = 2 * (S::SE + S::SO);
    __shared__ TC s1[L::BPW * L::size], s2[L::BPW * L::size];
    // FP64 tables at n = 8 (64 values) are read at wave-uniform global
    // addresses (scalar loads into SGPRs, from the scalar cache) instead of
    // being held in 128 VGPRs; smaller or FP32 tables stay in registers
    constexpr bool kScalarTab = sizeof(TC) == 8 && N >= kEoScalarTabN;
    __shared__ TC stab[kScalarTab ? 1 : TAB];
    TC T[kScalarTab ? 1 : TAB];
    if constexpr (!kScalarTab) load_table<TC, TAB>(T, tab, stab);
    const TC* Tb = kScalarTab ? tab : T;
    const TC* ME = Tb;
    const TC* MO = Tb + S::SE;
    const TC* PE = Tb + S::SE + S::SO;
    const TC* PO = Tb + 2 * S::SE + S::SO;
    int64_t t = blockIdx.x;
    if (t >= ntiles) return;
    const int lane = threadIdx.x;
    const int lw = lane / L::N2;
    const int lp = lane - lw * L::N2;
    const int li = lp / N, lj = lp - (lp / N) * N;
    const int so = (lw < L::BPW ? lw : 0) * L::size;
    TC* A1 = s1 + so;
    TC* A2 = s2 + so;
    TC pre[N];
    {
        const bool ok = lw < L::BPW && lw < nvalid_of<N>(G, t);
        if (ok) pencil_load<N, VP>(pre, pencil_ptr<N>(u, G, t * L::BPW + lw, li, lj), G.logB);
    }
    for (; t < ntiles; t += gridDim.x) {
        const int64_t g0 = t * L::BPW;
        const Pencil<N> pc(nvalid_of<N>(G, t));
        TC x[N];
#pragma unroll
        for (int k = 0; k < N; ++k) x[k] = pre[k];
        const int64_t tn = t + gridDim.x;
        if (tn < ntiles && lw < L::BPW && lw < nvalid_of<N>(G, tn))
            pencil_load<N, VP>(pre, pencil_ptr<N>(u, G, tn * L::BPW + lw, li, lj), G.logB);
        TC sx = TC(1), sy = TC(1), sz = TC(1);
        if (pc.act) block_scales(G.h, g0 + pc.w, sx, sy, sz);
        eo_apply_body<N>(pc, x, v, G, g0, A1, A2, ME, MO, PE, PO, sx, sy, sz);
    }
}

// x = D^{-1} r.  Table: SE | SO | lam (eigenvalues in split spectral order).
template <int N, typename TS, typename TC, bool VP>
__global__ __launch_bounds__(64, 2) void k_inverse_eo(const TS* __restrict__ r, TS* __restrict__ x, GArgs G,
                                                      const TC* __restrict__ tab, int64_t ntiles) {
    using L = Slab<N>;
    using S = EOShape<N>;
    constexpr int TABM = S::SE + S::SO;
    __shared__ TC s1[L::BPW * L::size];
    __shared__ TC stab[TABM + N];
    for (int e = threadIdx.x; e < TABM + N; e += 64) stab[e] = tab[e];
    wave_sync();
    constexpr bool kScalarTab = sizeof(TC) == 8 && N >= kEoScalarTabN;
    TC T[kScalarTab ? 1 : TABM];
    if constexpr (kScalarTab) {
    } else if constexpr (sizeof(TC) == 8) {
#pragma unroll
        for (int i = 0; i < TABM; ++i) T[i] = stab[i];
    } else {
#pragma unroll
        for (int i = 0; i < TABM; ++i) T[i] = tab[i];
    }
    const TC* SE = kScalarTab ? tab : T;
    const TC* SO = (kScalarTab ? tab : T) + S::SE;
    const TC* lam = stab + TABM;
    int64_t t = blockIdx.x;
    if (t >= ntiles) return;
    const int lane = threadIdx.x;
    const int lw = lane / L::N2;
    const int lp = lane - lw * L::N2;
    const int li = lp / N, lj = lp - (lp / N) * N;
    const int so = (lw < L::BPW ? lw : 0) * L::size;
    TC* A1 = s1 + so;
    TC pre[N];
    {
        const bool ok = lw < L::BPW && lw < nvalid_of<N>(G, t);
        if (ok) pencil_load<N, VP>(pre, pencil_ptr<N>(r, G, t * L::BPW + lw, li, lj), G.logB);
    }
    for (; t < ntiles; t += gridDim.x) {
        const int64_t g0 = t * L::BPW;
        const Pencil<N> pc(nvalid_of<N>(G, t));
        TC xin[N];
#pragma unroll
        for (int k = 0; k < N; ++k) xin[k] = pre[k];
        const int64_t tn = t + gridDim.x;
        if (tn < ntiles && lw < L::BPW && lw < nvalid_of<N>(G, tn))
            pencil_load<N, VP>(pre, pencil_ptr<N>(r, G, tn * L::BPW + lw, li, lj), G.logB);
        TC sx = TC(1), sy = TC(1), sz = TC(1);
        if (pc.act) block_scales(G.h, g0 + pc.w, sx, sy, sz);
        eo_inverse_body<N, VP>(pc, xin, x, G, g0, A1, SE, SO, lam, sx, sy, sz);
    }
}

// Minimum resident waves per SIMD the solve kernel is compiled for.  FP64
// inner inverse: n <= 6 fits 128 VGPRs (four waves); at n = 7 that spills,
// and at n = 8 three waves with more registers measured faster (125 vs
// 144 us on 32768 blocks) than four.  The FP32 inner one measured faster at
// 165 VGPRs (n = 8) than squeezed into 128.
template <int N, typename TI>
constexpr int solve_min_waves() {
    return sizeof(TI) == 8 ? (N >= 7 ? 3 : 4) : 2;
}

// Block-local iterative refinement over all tiles of a group (persistent grid).
template <int N, typename TI, int RND, bool VP>
__global__ __launch_bounds__(64, (solve_min_waves<N, TI>())) void k_solve_eo(const double* __restrict__ b, double* __restrict__ x, GArgs G,
                                                    const double* __restrict__ tabA, const TI* __restrict__ tabS,
                                                    int64_t ntiles, double rtol, int maxit,
                                                    int32_t* __restrict__ iters, double* __restrict__ relres,
                                                    int64_t block0, SolvePartial* parts) {
    using L = Slab<N>;
    using S = EOShape<N>;
    __shared__ SolveLdsR<N> lds;
    __shared__ TI stabS[S::SE + S::SO + N];
    // the 1D tables are read where they are used at wave-uniform addresses
    // (scalar loads into SGPRs); in VGPRs the FP64 ones would take 192
    // registers at n = 8 and halve the resident waves, from LDS every
    // contraction would wait on LDS.  Only the eigenvalues, indexed per
    // lane, go through LDS.
    stage_table<TI, S::SE + S::SO + N>(tabS, stabS);
    const TI* lam = stabS + S::SE + S::SO;
    SolveAcc acc;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x)
        eo_solve_tile<N, TI, RND, VP>(b, x, G, t * L::BPW, nvalid_of<N>(G, t), lds, tabA, tabS, lam, rtol, maxit,
                                      iters, relres, block0, acc);
    acc.flush(parts + blockIdx.x);
}

template <typename TS>
constexpr int dtype_code() {
    return std::is_same<TS, double>::value ? TP_F64
           : std::is_same<TS, float>::value ? TP_F32
           : std::is_same<TS, _Float16>::value ? TP_F16
                                               : TP_BF16;
}

tp_status check(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, what);
    return TP_OK;
}

// Pencils can move as 16-byte vectors: B = 1, n a multiple of the vector
// width and both buffers (with the group offset) 16-byte aligned.
template <int N, typename TS>
bool vector_pencils(const GroupInfo& g, const void* a, const void* b) {
    constexpr int VEC = 16 / static_cast<int>(sizeof(TS));
    if (g.logB != 0 || N % VEC != 0) return false;
    const uintptr_t pa = reinterpret_cast<uintptr_t>(static_cast<const TS*>(a) + g.offset);
    const uintptr_t pb = reinterpret_cast<uintptr_t>(static_cast<const TS*>(b) + g.offset);
    return (pa % 16) == 0 && (pb % 16) == 0;
}

// Persistent grid: as many one-wave workgroups as fit on the device at once.
int64_t persistent_grid(const Plan& plan, const void* kernel, int64_t ntiles) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, 64, 0) != hipSuccess || occ <= 0) occ = 8;
    return std::max<int64_t>(1, std::min<int64_t>(ntiles, static_cast<int64_t>(plan.cus) * occ));
}

template <int N>
int64_t eo_tiles(const GroupInfo& g) {
    return (g.nblocks + Slab<N>::BPW - 1) / Slab<N>::BPW;
}

template <int N, typename TS, typename TC>
tp_status apply_eo_n(const Plan& plan, const GroupInfo& g, int op, const void* u, void* v, hipStream_t s) {
    const int64_t ntiles = eo_tiles<N>(g);
    const TC* tab = reinterpret_cast<const TC*>(eo_table(plan, N, op == TP_OP_CELL ? EO_APPLY_A : EO_APPLY_K,
                                                         sizeof(TC) == 8 ? 0 : 1));
    GArgs a{g.h, g.nblocks, g.offset, g.logB};
    const bool vp = vector_pencils<N, TS>(g, u, v);
    const void* kern = vp ? reinterpret_cast<const void*>(&k_apply_eo<N, TS, TC, true>)
                          : reinterpret_cast<const void*>(&k_apply_eo<N, TS, TC, false>);
    static int64_t grid_cache[2] = {0, 0};
    int64_t& gc = grid_cache[vp ? 1 : 0];
    if (gc == 0) gc = persistent_grid(plan, kern, INT64_MAX);
    const int div = g.div_apply[dtype_code<TS>()];  // 0: one workgroup per tile
    const int64_t grid = div == 0 ? ntiles : std::min(std::max<int64_t>(1, gc / div), ntiles);
    if (vp)
        hipLaunchKernelGGL((k_apply_eo<N, TS, TC, true>), dim3(static_cast<unsigned>(grid)), dim3(64), 0, s,
                           static_cast<const TS*>(u), static_cast<TS*>(v), a, tab, ntiles);
    else
        hipLaunchKernelGGL((k_apply_eo<N, TS, TC, false>), dim3(static_cast<unsigned>(grid)), dim3(64), 0, s,
                           static_cast<const TS*>(u), static_cast<TS*>(v), a, tab, ntiles);
    return check("apply (even-odd) launch");
}

template <int N, typename TS, typename TC>
tp_status inverse_eo_n(const Plan& plan, const GroupInfo& g, const void* r, void* x, hipStream_t s) {
    const int64_t ntiles = eo_tiles<N>(g);
    const TC* tab = reinterpret_cast<const TC*>(eo_table(plan, N, EO_INV, sizeof(TC) == 8 ? 0 : 1));
    GArgs a{g.h, g.nblocks, g.offset, g.logB};
    const bool vp = vector_pencils<N, TS>(g, r, x);
    const void* kern = vp ? reinterpret_cast<const void*>(&k_inverse_eo<N, TS, TC, true>)
                          : reinterpret_cast<const void*>(&k_inverse_eo<N, TS, TC, false>);
    static int64_t grid_cache[2] = {0, 0};
    int64_t& gc = grid_cache[vp ? 1 : 0];
    if (gc == 0) gc = persistent_grid(plan, kern, INT64_MAX);
    const int div = g.div_inverse[dtype_code<TS>()];
    const int64_t grid = div == 0 ? ntiles : std::min(std::max<int64_t>(1, gc / div), ntiles);
    if (vp)
        hipLaunchKernelGGL((k_inverse_eo<N, TS, TC, true>), dim3(static_cast<unsigned>(grid)), dim3(64), 0, s,
                           static_cast<const TS*>(r), static_cast<TS*>(x), a, tab, ntiles);
    else
        hipLaunchKernelGGL((k_inverse_eo<N, TS, TC, false>), dim3(static_cast<unsigned>(grid)), dim3(64), 0, s,
                           static_cast<const TS*>(r), static_cast<TS*>(x), a, tab, ntiles);
    return check("apply_inverse (even-odd) launch");
}

template <int N, typename TI, int RND>
tp_status solve_eo_n(const Plan& plan, const GroupInfo& g, const double* b, double* x, double rtol, int maxit,
                     int32_t* iters, double* relres, const SolveWork& w, int64_t part_base, int64_t* nparts,
                     hipStream_t s) {
    const int64_t ntiles = eo_tiles<N>(g);
    const double* tabA = reinterpret_cast<const double*>(eo_table(plan, N, EO_APPLY_A, 0));
    const TI* tabS = reinterpret_cast<const TI*>(eo_table(plan, N, EO_INV, sizeof(TI) == 8 ? 0 : 1));
    GArgs a{g.h, g.nblocks, g.offset, g.logB};
    const bool vp = vector_pencils<N, double>(g, b, x);
    const void* kern = vp ? reinterpret_cast<const void*>(&k_solve_eo<N, TI, RND, true>)
                          : reinterpret_cast<const void*>(&k_solve_eo<N, TI, RND, false>);
    static int64_t grid_cache[2] = {0, 0};
    int64_t& gc = grid_cache[vp ? 1 : 0];
    if (gc == 0) gc = persistent_grid(plan, kern, INT64_MAX);
    const int64_t grid = std::min(gc, ntiles);
    if (part_base + grid > w.cap) return set_error(TP_ERR_UNSUPPORTED, "too many solve workgroups");
    *nparts = grid;
    SolvePartial* parts = w.parts + part_base;
    if (vp)
        hipLaunchKernelGGL((k_solve_eo<N, TI, RND, true>), dim3(static_cast<unsigned>(grid)), dim3(64), 0, s, b, x, a,
                           tabA, tabS, ntiles, rtol, maxit, iters, relres, g.block0, parts);
    else
        hipLaunchKernelGGL((k_solve_eo<N, TI, RND, false>), dim3(static_cast<unsigned>(grid)), dim3(64), 0, s, b, x,
                           a, tabA, tabS, ntiles, rtol, maxit, iters, relres, g.block0, parts);
    return check("solve launch");
}

template <typename TI, int RND>
tp_status solve_eo_dispatch(const Plan& plan, const GroupInfo& g, const double* b, double* x, double rtol,
                            int maxit, int32_t* iters, double* relres, const SolveWork& w, int64_t pb, int64_t* np,
                            hipStream_t s) {
    switch (g.n) {
        case 2: return solve_eo_n<2, TI, RND>(plan, g, b, x, rtol, maxit, iters, relres, w, pb, np, s);
        case 3: return solve_eo_n<3, TI, RND>(plan, g, b, x, rtol, maxit, iters, relres, w, pb, np, s);
        case 4: return solve_eo_n<4, TI, RND>(plan, g, b, x, rtol, maxit, iters, relres, w, pb, np, s);
        case 5: return solve_eo_n<5, TI, RND>(plan, g, b, x, rtol, maxit, iters, relres, w, pb, np, s);
        case 6: return solve_eo_n<6, TI, RND>(plan, g, b, x, rtol, maxit, iters, relres, w, pb, np, s);
        case 7: return solve_eo_n<7, TI, RND>(plan, g, b, x, rtol, maxit, iters, relres, w, pb, np, s);
        case 8: return solve_eo_n<8, TI, RND>(plan, g, b, x, rtol, maxit, iters, relres, w, pb, np, s);
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported n");
}

template <typename TS, typename TC>
tp_status apply_eo_dispatch(const Plan& plan, const GroupInfo& g, int op, const void* u, void* v, hipStream_t s) {
    switch (g.n) {
        case 2: return apply_eo_n<2, TS, TC>(plan, g, op, u, v, s);
        case 3: return apply_eo_n<3, TS, TC>(plan, g, op, u, v, s);
        case 4: return apply_eo_n<4, TS, TC>(plan, g, op, u, v, s);
        case 5: return apply_eo_n<5, TS, TC>(plan, g, op, u, v, s);
        case 6: return apply_eo_n<6, TS, TC>(plan, g, op, u, v, s);
        case 7: return apply_eo_n<7, TS, TC>(plan, g, op, u, v, s);
        case 8: return apply_eo_n<8, TS, TC>(plan, g, op, u, v, s);
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported n");
}

template <typename TS, typename TC>
tp_status inverse_eo_dispatch(const Plan& plan, const GroupInfo& g, const void* r, void* x, hipStream_t s) {
    switch (g.n) {
        case 2: return inverse_eo_n<2, TS, TC>(plan, g, r, x, s);
        case 3: return inverse_eo_n<3, TS, TC>(plan, g, r, x, s);
        case 4: return inverse_eo_n<4, TS, TC>(plan, g, r, x, s);
        case 5: return inverse_eo_n<5, TS, TC>(plan, g, r, x, s);
        case 6: return inverse_eo_n<6, TS, TC>(plan, g, r, x, s);
        case 7: return inverse_eo_n<7, TS, TC>(plan, g, r, x, s);
        case 8: return inverse_eo_n<8, TS, TC>(plan, g, r, x, s);
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported n");
}

}  // namespace

tp_status launch_apply_eo(const Plan& plan, const GroupInfo& g, int op, const void* u, void* v, tp_dtype dt,
                          hipStream_t s) {
    if (g.nblocks == 0) return TP_OK;
    switch (dt) {
        case TP_F64: return apply_eo_dispatch<double, double>(plan, g, op, u, v, s);
        case TP_F32: return apply_eo_dispatch<float, float>(plan, g, op, u, v, s);
        case TP_F16: return apply_eo_dispatch<_Float16, float>(plan, g, op, u, v, s);
        case TP_BF16: return apply_eo_dispatch<bf16_t, float>(plan, g, op, u, v, s);
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported dtype");
}

tp_status launch_solve(const Plan& plan, const GroupInfo& g, const double* b, double* x, tp_dtype inner,
                       double rtol, int maxit, int32_t* iters, double* relres, const SolveWork& w, int64_t part_base,
                       int64_t* nparts,
                       hipStream_t s) {
    *nparts = 0;
    if (g.nblocks == 0) return TP_OK;
    switch (inner) {
        case TP_F64:
            return solve_eo_dispatch<double, RND_NONE>(plan, g, b, x, rtol, maxit, iters, relres, w, part_base, nparts, s);
        case TP_F32:
            return solve_eo_dispatch<float, RND_NONE>(plan, g, b, x, rtol, maxit, iters, relres, w, part_base, nparts, s);
        case TP_F16:
            return solve_eo_dispatch<float, RND_F16>(plan, g, b, x, rtol, maxit, iters, relres, w, part_base, nparts, s);
        case TP_BF16:
            return solve_eo_dispatch<float, RND_BF16>(plan, g, b, x, rtol, maxit, iters, relres, w, part_base, nparts, s);
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported inner precision");
}

tp_status launch_inverse_eo(const Plan& plan, const GroupInfo& g, const void* r, void* x, tp_dtype dt,
                            hipStream_t s) {
    if (g.nblocks == 0) return TP_OK;
    switch (dt) {
        case TP_F64: return inverse_eo_dispatch<double, double>(plan, g, r, x, s);
        case TP_F32: return inverse_eo_dispatch<float, float>(plan, g, r, x, s);
        case TP_F16: return inverse_eo_dispatch<_Float16, float>(plan, g, r, x, s);
        case TP_BF16: return inverse_eo_dispatch<bf16_t, float>(plan, g, r, x, s);
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported dtype");
}

}  // namespace tpfdm
