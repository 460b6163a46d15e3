// Kernels for blocks with their own per-direction factors (GENERAL mode).
//
// Every block b carries three 1D pairs (M_d, P_d), d = x, y, z, of its own
// (Sec. 5.2: the cell block is the Kronecker sum of per-direction mass and
// penalized stiffness; on a deformed or non-scaled cell these differ per
// cell), and after the GENERAL setup its own eigen-decompositions
// P_d S_d = M_d S_d Lambda_d.  Nothing is assumed about symmetry or the
// even-odd structure, so the 1D products are plain n x n matrix-vector
// products on pencils.
//
// Mapping: one wave per tile of BPW blocks (as the wave kernels), the tile's
// factors staged once in LDS and read there with per-block broadcast
// addresses, the block slab in LDS between the direction phases.
//
// Device layouts (plan-owned):
//   fac[b][d][0 = M, 1 = P][n][n]          row-major
//   eig[b][d][ S[n][n] (column c = eigenvector c) | lam[n] ]
#include <algorithm>

#include "eo.h"

namespace tpfdm {

namespace {

template <int N>
struct GenShape {
    static constexpr int F = 6 * N * N;        // factor entries per block
    static constexpr int E = 3 * (N * N + N);  // eigen entries per block
};

// y = A x and y = A^T x for a row-major N x N matrix in LDS.
template <int N, typename T>
__device__ __forceinline__ void mv(const T* A, const T (&x)[N], T (&y)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
        T s = T(0);
#pragma unroll
        for (int j = 0; j < N; ++j) s = fma(A[i * N + j], x[j], s);
        y[i] = s;
    }
}
template <int N, typename T>
__device__ __forceinline__ void mvt(const T* A, const T (&x)[N], T (&y)[N]) {
#pragma unroll
    for (int c = 0; c < N; ++c) {
        T s = T(0);
#pragma unroll
        for (int k = 0; k < N; ++k) s = fma(A[k * N + c], x[k], s);
        y[c] = s;
    }
}

// dst = A src on the lane's block slab, A the Kronecker sum of the block's
// factors F (in LDS); dst may alias src; t1, t2 scratch slabs.
//   z: t = M_z src, w = P_z src;  y: a = M_y t, b = P_y t + M_y w;
//   x: dst = P_x a + M_x b.
template <int N, typename T>
__device__ __forceinline__ void gen_apply_lds(const Pencil<N>& pc, const T* src, T* dst, T* t1, T* t2, const T* F) {
    using L = Slab<N>;
    constexpr int N2 = N * N;
    const T *Mx = F, *Px = F + N2, *My = F + 2 * N2, *Py = F + 3 * N2, *Mz = F + 4 * N2, *Pz = F + 5 * N2;
    const int pa = pc.pa, pb = pc.pb;
    if (pc.act) {
        T x[N], y[N];
#pragma unroll
        for (int k = 0; k < N; ++k) x[k] = src[L::at(pa, pb, k)];
        mv<N>(Mz, x, y);
#pragma unroll
        for (int k = 0; k < N; ++k) t1[L::at(pa, pb, k)] = y[k];
        mv<N>(Pz, x, y);
#pragma unroll
        for (int k = 0; k < N; ++k) t2[L::at(pa, pb, k)] = y[k];
    }
    wave_sync();
    if (pc.act) {
        T t[N], w[N], a[N], b1[N], b2[N];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            t[j] = t1[L::at(pa, j, pb)];
            w[j] = t2[L::at(pa, j, pb)];
        }
        mv<N>(My, t, a);
        mv<N>(Py, t, b1);
        mv<N>(My, w, b2);
#pragma unroll
        for (int j = 0; j < N; ++j) {
            t1[L::at(pa, j, pb)] = a[j];
            t2[L::at(pa, j, pb)] = b1[j] + b2[j];
        }
    }
    wave_sync();
    if (pc.act) {
        T a[N], b[N], y1[N], y2[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            a[i] = t1[L::at(i, pa, pb)];
            b[i] = t2[L::at(i, pa, pb)];
        }
        mv<N>(Px, a, y1);
        mv<N>(Mx, b, y2);
#pragma unroll
        for (int i = 0; i < N; ++i) dst[L::at(i, pa, pb)] = y1[i] + y2[i];
    }
    wave_sync();
}

// slab <- D^{-1} slab with the block's eigen-decompositions E (in LDS):
// S_z^T, S_y^T, S_x^T, scaling by 1/(lam_x[i] + lam_y[j] + lam_z[k]),
// S_x, S_y, S_z, each phase on its own pencils.
template <int N, typename T>
__device__ __forceinline__ void gen_inverse_lds(const Pencil<N>& pc, T* slab, const T* E) {
    using L = Slab<N>;
    constexpr int NE = N * N + N;
    const T *Sx = E, *lx = E + N * N, *Sy = E + NE, *ly = E + NE + N * N, *Sz = E + 2 * NE, *lz = E + 2 * NE + N * N;
    const int pa = pc.pa, pb = pc.pb;
    T a[N], y[N];
    if (pc.act) {  // z forward
#pragma unroll
        for (int k = 0; k < N; ++k) a[k] = slab[L::at(pa, pb, k)];
        mvt<N>(Sz, a, y);
#pragma unroll
        for (int c = 0; c < N; ++c) slab[L::at(pa, pb, c)] = y[c];
    }
    wave_sync();
    if (pc.act) {  // y forward
#pragma unroll
        for (int j = 0; j < N; ++j) a[j] = slab[L::at(pa, j, pb)];
        mvt<N>(Sy, a, y);
#pragma unroll
        for (int b = 0; b < N; ++b) slab[L::at(pa, b, pb)] = y[b];
    }
    wave_sync();
    if (pc.act) {  // x forward, scaling, x backward: lane (b, c) = (pa, pb)
#pragma unroll
        for (int i = 0; i < N; ++i) a[i] = slab[L::at(i, pa, pb)];
        mvt<N>(Sx, a, y);
        const T mu = ly[pa] + lz[pb];
#pragma unroll
        for (int i = 0; i < N; ++i) y[i] *= recip(lx[i] + mu);
        mv<N>(Sx, y, a);
#pragma unroll
        for (int i = 0; i < N; ++i) slab[L::at(i, pa, pb)] = a[i];
    }
    wave_sync();
    if (pc.act) {  // y backward
#pragma unroll
        for (int b = 0; b < N; ++b) y[b] = slab[L::at(pa, b, pb)];
        mv<N>(Sy, y, a);
#pragma unroll
        for (int j = 0; j < N; ++j) slab[L::at(pa, j, pb)] = a[j];
    }
    wave_sync();
    if (pc.act) {  // z backward
#pragma unroll
        for (int c = 0; c < N; ++c) y[c] = slab[L::at(pa, pb, c)];
        mv<N>(Sz, y, a);
#pragma unroll
        for (int k = 0; k < N; ++k) slab[L::at(pa, pb, k)] = a[k];
    }
    wave_sync();
}

// Copies `count` consecutive elements starting at src into LDS.
template <typename T>
__device__ __forceinline__ void stage(T* dst, const T* __restrict__ src, int count) {
    for (int e = threadIdx.x; e < count; e += 64) dst[e] = src[e];
}

// The tile's input z-pencils into the slab (storage -> compute type).
template <int N, bool VP, typename TS, typename TC>
__device__ __forceinline__ void slab_in(const Pencil<N>& pc, TC* slab, const TS* __restrict__ u, const GArgs& G,
                                        int64_t g0) {
    using L = Slab<N>;
    if (pc.act) {
        TC x[N];
        pencil_load<N, VP>(x, pencil_ptr<N>(u, G, g0 + pc.w, pc.pa, pc.pb), G.logB);
#pragma unroll
        for (int k = 0; k < N; ++k) slab[L::at(pc.pa, pc.pb, k)] = x[k];
    }
}

template <int N, typename TS, typename TC, bool VP>
__global__ __launch_bounds__(64, 2) void k_apply_gen(const TS* __restrict__ u, TS* __restrict__ v, GArgs G,
                                                     const TC* __restrict__ fac, int64_t ntiles) {
    using L = Slab<N>;
    constexpr int F = GenShape<N>::F;
    __shared__ TC sf[L::BPW * F];
    __shared__ TC s0[L::BPW * L::size], s1[L::BPW * L::size], s2[L::BPW * L::size];
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t g0 = t * L::BPW;
        const int nvalid = nvalid_of<N>(G, t);
        const Pencil<N> pc(nvalid);
        const int so = (pc.w < L::BPW ? pc.w : 0) * L::size;
        stage(sf, fac + g0 * F, nvalid * F);
        slab_in<N, VP, TS, TC>(pc, s0 + so, u, G, g0);
        wave_sync();
        gen_apply_lds<N, TC>(pc, s0 + so, s0 + so, s1 + so, s2 + so, sf + (pc.w < L::BPW ? pc.w : 0) * F);
        if (pc.act) {  // x-planes to global memory: lanes (j, k) of a plane are consecutive
            TS* out = v + G.offset + block_base(g0 + pc.w, G.logB, L::N3);
#pragma unroll
            for (int i = 0; i < N; ++i)
                stc(out + (static_cast<int64_t>((i * N + pc.pa) * N + pc.pb) << G.logB), s0[so + L::at(i, pc.pa, pc.pb)]);
        }
        wave_sync();
    }
}

template <int N, typename TS, typename TC, bool VP>
__global__ __launch_bounds__(64, 2) void k_inverse_gen(const TS* __restrict__ r, TS* __restrict__ x, GArgs G,
                                                       const TC* __restrict__ eig, int64_t ntiles) {
    using L = Slab<N>;
    constexpr int E = GenShape<N>::E;
    __shared__ TC se[L::BPW * E];
    __shared__ TC s0[L::BPW * L::size];
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t g0 = t * L::BPW;
        const int nvalid = nvalid_of<N>(G, t);
        const Pencil<N> pc(nvalid);
        const int so = (pc.w < L::BPW ? pc.w : 0) * L::size;
        stage(se, eig + g0 * E, nvalid * E);
        slab_in<N, VP, TS, TC>(pc, s0 + so, r, G, g0);
        wave_sync();
        gen_inverse_lds<N, TC>(pc, s0 + so, se + (pc.w < L::BPW ? pc.w : 0) * E);
        if (pc.act) {
            TC y[N];
#pragma unroll
            for (int k = 0; k < N; ++k) y[k] = s0[so + L::at(pc.pa, pc.pb, k)];
            pencil_store<N, VP>(const_cast<TS*>(pencil_ptr<N>(x, G, g0 + pc.w, pc.pa, pc.pb)), y, G.logB);
        }
        wave_sync();
    }
}

template <int N, typename TI, int RND>
__global__ __launch_bounds__(64, 2) void k_solve_gen(const double* __restrict__ b, double* __restrict__ x, GArgs G,
                                                     const double* __restrict__ fac, const TI* __restrict__ eig,
                                                     int64_t ntiles, double rtol, int maxit,
                                                     int32_t* __restrict__ iters, double* __restrict__ relres,
                                                     int64_t block0, SolvePartial* parts) {
    using L = Slab<N>;
    constexpr int F = GenShape<N>::F, E = GenShape<N>::E;
    __shared__ SolveLds<N, TI> lds;
    __shared__ double sf[L::BPW * F];
    __shared__ TI se[L::BPW * E];
    SolveAcc acc;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t g0 = t * L::BPW;
        const int nvalid = nvalid_of<N>(G, t);
        wave_sync();  // the previous tile is done with the staged factors
        stage(sf, fac + g0 * F, nvalid * F);
        stage(se, eig + g0 * E, nvalid * E);
        const int w = static_cast<int>(threadIdx.x) / L::N2;
        const double* Fw = sf + (w < L::BPW ? w : 0) * F;
        const TI* Ew = se + (w < L::BPW ? w : 0) * E;
        solve_tile<N, TI, RND>(
            b, x, G, g0, nvalid, lds,
            [&](const Pencil<N>& p, const double* src, double* dst, double* t1, double* t2) {
                gen_apply_lds<N, double>(p, src, dst, t1, t2, Fw);
            },
            [&](const Pencil<N>& p, TI* slab) { gen_inverse_lds<N, TI>(p, slab, Ew); }, rtol, maxit, iters, relres,
            block0, acc);
    }
    acc.flush(parts + blockIdx.x);
}

tp_status check_gen(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, what);
    return TP_OK;
}

template <int N, typename TS>
bool gen_vector_pencils(const GroupInfo& g, const void* a, const void* b) {
    constexpr int VEC = 16 / static_cast<int>(sizeof(TS));
    if (g.logB != 0 || N % VEC != 0) return false;
    const uintptr_t pa = reinterpret_cast<uintptr_t>(static_cast<const TS*>(a) + g.offset);
    const uintptr_t pb = reinterpret_cast<uintptr_t>(static_cast<const TS*>(b) + g.offset);
    return (pa % 16) == 0 && (pb % 16) == 0;
}

int64_t gen_grid(const Plan& plan, int64_t ntiles) {
    return std::max<int64_t>(1, std::min<int64_t>(ntiles, static_cast<int64_t>(plan.cus) * 16));
}

template <int N, typename TS, typename TC>
tp_status apply_gen_n(const Plan& plan, const GroupInfo& g, const void* u, void* v, hipStream_t s) {
    const int64_t ntiles = (g.nblocks + Slab<N>::BPW - 1) / Slab<N>::BPW;
    const TC* fac = static_cast<const TC*>(sizeof(TC) == 8 ? static_cast<const void*>(g.fac)
                                                           : static_cast<const void*>(g.fac32));
    GArgs a{g.h, g.nblocks, g.offset, g.logB};
    const unsigned grid = static_cast<unsigned>(gen_grid(plan, ntiles));
    if (gen_vector_pencils<N, TS>(g, u, v))
        hipLaunchKernelGGL((k_apply_gen<N, TS, TC, true>), dim3(grid), dim3(64), 0, s, static_cast<const TS*>(u),
                           static_cast<TS*>(v), a, fac, ntiles);
    else
        hipLaunchKernelGGL((k_apply_gen<N, TS, TC, false>), dim3(grid), dim3(64), 0, s, static_cast<const TS*>(u),
                           static_cast<TS*>(v), a, fac, ntiles);
    return check_gen("apply (block factors) launch");
}

template <int N, typename TS, typename TC>
tp_status inverse_gen_n(const Plan& plan, const GroupInfo& g, const void* r, void* x, hipStream_t s) {
    const int64_t ntiles = (g.nblocks + Slab<N>::BPW - 1) / Slab<N>::BPW;
    const TC* eig = static_cast<const TC*>(sizeof(TC) == 8 ? static_cast<const void*>(g.eig)
                                                           : static_cast<const void*>(g.eig32));
    GArgs a{g.h, g.nblocks, g.offset, g.logB};
    const unsigned grid = static_cast<unsigned>(gen_grid(plan, ntiles));
    if (gen_vector_pencils<N, TS>(g, r, x))
        hipLaunchKernelGGL((k_inverse_gen<N, TS, TC, true>), dim3(grid), dim3(64), 0, s, static_cast<const TS*>(r),
                           static_cast<TS*>(x), a, eig, ntiles);
    else
        hipLaunchKernelGGL((k_inverse_gen<N, TS, TC, false>), dim3(grid), dim3(64), 0, s, static_cast<const TS*>(r),
                           static_cast<TS*>(x), a, eig, ntiles);
    return check_gen("apply_inverse (block factors) launch");
}

template <int N, typename TI, int RND>
tp_status solve_gen_n(const Plan& plan, const GroupInfo& g, const double* b, double* x, double rtol, int maxit,
                      int32_t* iters, double* relres, const SolveWork& w, int64_t part_base, int64_t* nparts,
                       hipStream_t s) {
    const int64_t ntiles = (g.nblocks + Slab<N>::BPW - 1) / Slab<N>::BPW;
    const TI* eig = static_cast<const TI*>(sizeof(TI) == 8 ? static_cast<const void*>(g.eig)
                                                           : static_cast<const void*>(g.eig32));
    GArgs a{g.h, g.nblocks, g.offset, g.logB};
    const int64_t grid = std::min<int64_t>(gen_grid(plan, ntiles), static_cast<int64_t>(plan.cus) * kMaxWgPerCu);
    if (part_base + grid > w.cap) return set_error(TP_ERR_UNSUPPORTED, "too many solve workgroups");
    hipLaunchKernelGGL((k_solve_gen<N, TI, RND>), dim3(static_cast<unsigned>(grid)), dim3(64), 0, s, b, x, a, g.fac,
                       eig, ntiles, rtol, maxit, iters, relres, g.block0,
                       w.parts + part_base);
    *nparts = grid;
    return check_gen("solve (block factors) launch");
}

template <typename TS, typename TC>
tp_status apply_gen_dispatch(const Plan& plan, const GroupInfo& g, const void* u, void* v, hipStream_t s) {
    switch (g.n) {
        case 2: return apply_gen_n<2, TS, TC>(plan, g, u, v, s);
        case 3: return apply_gen_n<3, TS, TC>(plan, g, u, v, s);
        case 4: return apply_gen_n<4, TS, TC>(plan, g, u, v, s);
        case 5: return apply_gen_n<5, TS, TC>(plan, g, u, v, s);
        case 6: return apply_gen_n<6, TS, TC>(plan, g, u, v, s);
        case 7: return apply_gen_n<7, TS, TC>(plan, g, u, v, s);
        case 8: return apply_gen_n<8, TS, TC>(plan, g, u, v, s);
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported n");
}

template <typename TS, typename TC>
tp_status inverse_gen_dispatch(const Plan& plan, const GroupInfo& g, const void* r, void* x, hipStream_t s) {
    switch (g.n) {
        case 2: return inverse_gen_n<2, TS, TC>(plan, g, r, x, s);
        case 3: return inverse_gen_n<3, TS, TC>(plan, g, r, x, s);
        case 4: return inverse_gen_n<4, TS, TC>(plan, g, r, x, s);
        case 5: return inverse_gen_n<5, TS, TC>(plan, g, r, x, s);
        case 6: return inverse_gen_n<6, TS, TC>(plan, g, r, x, s);
        case 7: return inverse_gen_n<7, TS, TC>(plan, g, r, x, s);
        case 8: return inverse_gen_n<8, TS, TC>(plan, g, r, x, s);
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported n");
}

template <typename TI, int RND>
tp_status solve_gen_dispatch(const Plan& plan, const GroupInfo& g, const double* b, double* x, double rtol, int maxit,
                             int32_t* iters, double* relres, const SolveWork& w, int64_t pb, int64_t* np,
                             hipStream_t s) {
    switch (g.n) {
        case 2: return solve_gen_n<2, TI, RND>(plan, g, b, x, rtol, maxit, iters, relres, w, pb, np, s);
        case 3: return solve_gen_n<3, TI, RND>(plan, g, b, x, rtol, maxit, iters, relres, w, pb, np, s);
        case 4: return solve_gen_n<4, TI, RND>(plan, g, b, x, rtol, maxit, iters, relres, w, pb, np, s);
        case 5: return solve_gen_n<5, TI, RND>(plan, g, b, x, rtol, maxit, iters, relres, w, pb, np, s);
        case 6: return solve_gen_n<6, TI, RND>(plan, g, b, x, rtol, maxit, iters, relres, w, pb, np, s);
        case 7: return solve_gen_n<7, TI, RND>(plan, g, b, x, rtol, maxit, iters, relres, w, pb, np, s);
        case 8: return solve_gen_n<8, TI, RND>(plan, g, b, x, rtol, maxit, iters, relres, w, pb, np, s);
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported n");
}

}  // namespace

tp_status launch_apply_gen(const Plan& plan, const GroupInfo& g, const void* u, void* v, tp_dtype dt, hipStream_t s) {
    if (g.nblocks == 0) return TP_OK;
    if (!g.fac) return set_error(TP_ERR_STATE, "group has no block factors");
    switch (dt) {
        case TP_F64: return apply_gen_dispatch<double, double>(plan, g, u, v, s);
        case TP_F32: return apply_gen_dispatch<float, float>(plan, g, u, v, s);
        case TP_F16: return apply_gen_dispatch<_Float16, float>(plan, g, u, v, s);
        case TP_BF16: return apply_gen_dispatch<bf16_t, float>(plan, g, u, v, s);
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported dtype");
}

tp_status launch_inverse_gen(const Plan& plan, const GroupInfo& g, const void* r, void* x, tp_dtype dt,
                             hipStream_t s) {
    if (g.nblocks == 0) return TP_OK;
    if (!g.eig) return set_error(TP_ERR_STATE, "group has no block eigen-decompositions");
    switch (dt) {
        case TP_F64: return inverse_gen_dispatch<double, double>(plan, g, r, x, s);
        case TP_F32: return inverse_gen_dispatch<float, float>(plan, g, r, x, s);
        case TP_F16: return inverse_gen_dispatch<_Float16, float>(plan, g, r, x, s);
        case TP_BF16: return inverse_gen_dispatch<bf16_t, float>(plan, g, r, x, s);
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported dtype");
}

tp_status launch_solve_gen(const Plan& plan, const GroupInfo& g, const double* b, double* x, tp_dtype inner,
                           double rtol, int maxit, int32_t* iters, double* relres, const SolveWork& w,
                           int64_t part_base, int64_t* nparts, hipStream_t s) {
    *nparts = 0;
    if (g.nblocks == 0) return TP_OK;
    if (!g.eig || !g.fac) return set_error(TP_ERR_STATE, "group has no block factors");
    switch (inner) {
        case TP_F64:
            return solve_gen_dispatch<double, RND_NONE>(plan, g, b, x, rtol, maxit, iters, relres, w, part_base, nparts, s);
        case TP_F32:
            return solve_gen_dispatch<float, RND_NONE>(plan, g, b, x, rtol, maxit, iters, relres, w, part_base, nparts, s);
        case TP_F16:
            return solve_gen_dispatch<float, RND_F16>(plan, g, b, x, rtol, maxit, iters, relres, w, part_base, nparts, s);
        case TP_BF16:
            return solve_gen_dispatch<float, RND_BF16>(plan, g, b, x, rtol, maxit, iters, relres, w, part_base, nparts, s);
    }
    return set_error(TP_ERR_UNSUPPORTED, "unsupported inner precision");
}

}  // namespace tpfdm
