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
// multiply-adds and the size of the matrices; the halved matrices live in
// VGPRs (loaded once per workgroup through LDS), which keeps the scalar
// register file free for addressing.
//
// Mapping: one wave per tile of BPW blocks, each block's slab in LDS, one
// pencil per lane and phase (see Slab/Pencil); a persistent grid loops over
// tiles and loads tile t + grid into registers while tile t is computed.
#include "device.h"

namespace tpfdm {

namespace {

template <int N>
struct EOShape {
    static constexpr int H = N / 2;
    static constexpr int HC = (N + 1) / 2;
    static constexpr int SE = HC * HC;
    static constexpr int SO = H * H;
};

// e, o parts of a pencil.
template <int N, typename T>
__device__ __forceinline__ void eo_split(const T (&x)[N], T (&e)[EOShape<N>::HC], T (&o)[EOShape<N>::H]) {
    constexpr int H = EOShape<N>::H;
#pragma unroll
    for (int j = 0; j < H; ++j) {
        e[j] = x[j] + x[N - 1 - j];
        o[j] = x[j] - x[N - 1 - j];
    }
    if constexpr (N % 2 == 1) e[H] = x[H];
}

// E = AE e (HC outputs), O = AO o (H outputs); matrices row-major.
template <int N, typename T>
__device__ __forceinline__ void eo_mul(const T* AE, const T* AO, const T (&e)[EOShape<N>::HC],
                                       const T (&o)[EOShape<N>::H], T (&E)[EOShape<N>::HC],
                                       T (&O)[EOShape<N>::H]) {
    constexpr int H = EOShape<N>::H, HC = EOShape<N>::HC;
#pragma unroll
    for (int i = 0; i < HC; ++i) {
        T s = T(0);
#pragma unroll
        for (int j = 0; j < HC; ++j) s = fma(AE[i * HC + j], e[j], s);
        E[i] = s;
    }
#pragma unroll
    for (int i = 0; i < H; ++i) {
        T s = T(0);
#pragma unroll
        for (int j = 0; j < H; ++j) s = fma(AO[i * H + j], o[j], s);
        O[i] = s;
    }
}

template <int N, typename T>
__device__ __forceinline__ void eo_join(const T (&E)[EOShape<N>::HC], const T (&O)[EOShape<N>::H], T (&y)[N]) {
    constexpr int H = EOShape<N>::H;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        y[i] = E[i] + O[i];
        y[N - 1 - i] = E[i] - O[i];
    }
    if constexpr (N % 2 == 1) y[H] = E[H];
}

// Forward spectral transform y = S^T x along a pencil: the first HC outputs
// are the coefficients of the symmetric eigenvectors, the last H those of
// the antisymmetric ones (SE[k][c] = S[k][sym c] for k < HC, SO likewise).
template <int N, typename T>
__device__ __forceinline__ void eo_fwd(const T* SE, const T* SO, const T (&x)[N], T (&y)[N]) {
    constexpr int H = EOShape<N>::H, HC = EOShape<N>::HC;
    T e[HC], o[H];
    eo_split<N>(x, e, o);
#pragma unroll
    for (int c = 0; c < HC; ++c) {
        T s = T(0);
#pragma unroll
        for (int k = 0; k < HC; ++k) s = fma(SE[k * HC + c], e[k], s);
        y[c] = s;
    }
#pragma unroll
    for (int c = 0; c < H; ++c) {
        T s = T(0);
#pragma unroll
        for (int k = 0; k < H; ++k) s = fma(SO[k * H + c], o[k], s);
        y[HC + c] = s;
    }
}

// Backward transform x = S y (y in the split spectral order of eo_fwd).
template <int N, typename T>
__device__ __forceinline__ void eo_bwd(const T* SE, const T* SO, const T (&y)[N], T (&x)[N]) {
    constexpr int H = EOShape<N>::H, HC = EOShape<N>::HC;
    T E[HC], O[H];
#pragma unroll
    for (int k = 0; k < HC; ++k) {
        T s = T(0);
#pragma unroll
        for (int c = 0; c < HC; ++c) s = fma(SE[k * HC + c], y[c], s);
        E[k] = s;
    }
#pragma unroll
    for (int k = 0; k < H; ++k) {
        T s = T(0);
#pragma unroll
        for (int c = 0; c < H; ++c) s = fma(SO[k * H + c], y[HC + c], s);
        O[k] = s;
    }
    eo_join<N>(E, O, x);
}

// Per-lane prefetch buffer of one tile (BPW blocks, block-linear order).
template <int N, typename TC>
struct TileBuf {
    static constexpr int PER = (Slab<N>::BPW * Slab<N>::N3 + 63) / 64;
    TC v[PER];
};

template <int N, typename TS, typename TC>
__device__ __forceinline__ void tile_load(TileBuf<N, TC>& buf, const TS* __restrict__ src, const GArgs& G,
                                          int64_t g0, int nvalid) {
    using L = Slab<N>;
#pragma unroll
    for (int r = 0; r < TileBuf<N, TC>::PER; ++r) {
        const int e = r * 64 + static_cast<int>(threadIdx.x);
        const int w = e / L::N3;
        const int q = e - w * L::N3;
        buf.v[r] = (w < nvalid)
                       ? ldc<TC>(src + G.offset + block_base(g0 + w, G.logB, L::N3) + (static_cast<int64_t>(q) << G.logB))
                       : TC(0);
    }
}

template <int N, typename TC>
__device__ __forceinline__ void tile_to_lds(const TileBuf<N, TC>& buf, TC* slabs, int nvalid) {
    using L = Slab<N>;
#pragma unroll
    for (int r = 0; r < TileBuf<N, TC>::PER; ++r) {
        const int e = r * 64 + static_cast<int>(threadIdx.x);
        const int w = e / L::N3;
        const int q = e - w * L::N3;
        if (w < nvalid) slabs[w * L::size + L::lin(q)] = buf.v[r];
    }
}

template <int N, typename TS, typename TC>
__device__ __forceinline__ void tile_store(TS* __restrict__ dst, const TC* slabs, const GArgs& G, int64_t g0,
                                           int nvalid) {
    using L = Slab<N>;
#pragma unroll
    for (int r = 0; r < TileBuf<N, TC>::PER; ++r) {
        const int e = r * 64 + static_cast<int>(threadIdx.x);
        const int w = e / L::N3;
        const int q = e - w * L::N3;
        if (w < nvalid)
            stc(dst + G.offset + block_base(g0 + w, G.logB, L::N3) + (static_cast<int64_t>(q) << G.logB),
                slabs[w * L::size + L::lin(q)]);
    }
}

// v = A u.  Table: ME | MO | PE | PO.
template <int N, typename TS, typename TC>
__global__ __launch_bounds__(64, 2) void k_apply_eo(const TS* __restrict__ u, TS* __restrict__ v, GArgs G,
                                                 const TC* __restrict__ tab, int64_t ntiles) {
    using L = Slab<N>;
    using S = EOShape<N>;
    constexpr int HC = S::HC, H = S::H;
    constexpr int TAB = 2 * (S::SE + S::SO);
    __shared__ TC s0[L::BPW * L::size], s1[L::BPW * L::size], s2[L::BPW * L::size];
    __shared__ TC stab[TAB];
    for (int e = threadIdx.x; e < TAB; e += 64) stab[e] = tab[e];
    __syncthreads();
    TC ME[S::SE], MO[S::SO], PE[S::SE], PO[S::SO];
#pragma unroll
    for (int i = 0; i < S::SE; ++i) {
        ME[i] = stab[i];
        PE[i] = stab[S::SE + S::SO + i];
    }
#pragma unroll
    for (int i = 0; i < S::SO; ++i) {
        MO[i] = stab[S::SE + i];
        PO[i] = stab[2 * S::SE + S::SO + i];
    }
    int64_t t = blockIdx.x;
    if (t >= ntiles) return;
    TileBuf<N, TC> buf;
    auto nvalid_of = [&](int64_t tt) {
        const int64_t g0 = tt * L::BPW;
        return static_cast<int>(G.nblocks - g0 < L::BPW ? G.nblocks - g0 : L::BPW);
    };
    tile_load<N>(buf, u, G, t * L::BPW, nvalid_of(t));
    for (; t < ntiles; t += gridDim.x) {
        const int64_t g0 = t * L::BPW;
        const int nvalid = nvalid_of(t);
        tile_to_lds<N>(buf, s0, nvalid);
        const int64_t tn = t + gridDim.x;
        if (tn < ntiles) tile_load<N>(buf, u, G, tn * L::BPW, nvalid_of(tn));
        const Pencil<N> pc(nvalid);
        TC sx = TC(1), sy = TC(1), sz = TC(1);
        if (pc.act) block_scales(G.h, g0 + pc.w, sx, sy, sz);
        const int so = (pc.w < L::BPW ? pc.w : 0) * L::size;
        TC* A0 = s0 + so;
        TC* A1 = s1 + so;
        TC* A2 = s2 + so;
        const int pa = pc.pa, pb = pc.pb;
        __syncthreads();
        if (pc.act) {  // z: lane (i, j); t = M x, w = P x
            TC x[N], e[HC], o[H], E[HC], O[H], y[N];
#pragma unroll
            for (int k = 0; k < N; ++k) x[k] = A0[L::at(pa, pb, k)];
            eo_split<N>(x, e, o);
            eo_mul<N>(ME, MO, e, o, E, O);
            eo_join<N>(E, O, y);
#pragma unroll
            for (int k = 0; k < N; ++k) A1[L::at(pa, pb, k)] = y[k];
            eo_mul<N>(PE, PO, e, o, E, O);
            eo_join<N>(E, O, y);
#pragma unroll
            for (int k = 0; k < N; ++k) A2[L::at(pa, pb, k)] = y[k];
        }
        __syncthreads();
        if (pc.act) {  // y: lane (i, k); a = s_x M t, b = s_y P t + s_z M w
            TC x[N], et[HC], ot[H], ew[HC], ow[H], E[HC], O[H], E2[HC], O2[H], y[N];
#pragma unroll
            for (int j = 0; j < N; ++j) x[j] = A1[L::at(pa, j, pb)];
            eo_split<N>(x, et, ot);
#pragma unroll
            for (int j = 0; j < N; ++j) x[j] = A2[L::at(pa, j, pb)];
            eo_split<N>(x, ew, ow);
            eo_mul<N>(ME, MO, et, ot, E, O);
            eo_join<N>(E, O, y);
#pragma unroll
            for (int j = 0; j < N; ++j) A1[L::at(pa, j, pb)] = y[j] * sx;
            eo_mul<N>(PE, PO, et, ot, E, O);
            eo_mul<N>(ME, MO, ew, ow, E2, O2);
#pragma unroll
            for (int i = 0; i < HC; ++i) E[i] = fma(sy, E[i], sz * E2[i]);
#pragma unroll
            for (int i = 0; i < H; ++i) O[i] = fma(sy, O[i], sz * O2[i]);
            eo_join<N>(E, O, y);
#pragma unroll
            for (int j = 0; j < N; ++j) A2[L::at(pa, j, pb)] = y[j];
        }
        __syncthreads();
        if (pc.act) {  // x: lane (j, k); v = P a + M b
            TC x[N], ea[HC], oa[H], eb[HC], ob[H], E[HC], O[H], E2[HC], O2[H], y[N];
#pragma unroll
            for (int i = 0; i < N; ++i) x[i] = A1[L::at(i, pa, pb)];
            eo_split<N>(x, ea, oa);
#pragma unroll
            for (int i = 0; i < N; ++i) x[i] = A2[L::at(i, pa, pb)];
            eo_split<N>(x, eb, ob);
            eo_mul<N>(PE, PO, ea, oa, E, O);
            eo_mul<N>(ME, MO, eb, ob, E2, O2);
#pragma unroll
            for (int i = 0; i < HC; ++i) E[i] += E2[i];
#pragma unroll
            for (int i = 0; i < H; ++i) O[i] += O2[i];
            eo_join<N>(E, O, y);
#pragma unroll
            for (int i = 0; i < N; ++i) A0[L::at(i, pa, pb)] = y[i];
        }
        __syncthreads();
        tile_store<N>(v, s0, G, g0, nvalid);
        __syncthreads();
    }
}

// x = D^{-1} r.  Table: SE | SO | lamP (eigenvalues in split spectral order).
template <int N, typename TS, typename TC>
__global__ __launch_bounds__(64) void k_inverse_eo(const TS* __restrict__ r, TS* __restrict__ x, GArgs G,
                                                   const TC* __restrict__ tab, int64_t ntiles) {
    using L = Slab<N>;
    using S = EOShape<N>;
    constexpr int TAB = S::SE + S::SO + N;
    __shared__ TC s0[L::BPW * L::size], s1[L::BPW * L::size];
    __shared__ TC stab[TAB];
    for (int e = threadIdx.x; e < TAB; e += 64) stab[e] = tab[e];
    __syncthreads();
    TC SE[S::SE], SO[S::SO];
#pragma unroll
    for (int i = 0; i < S::SE; ++i) SE[i] = stab[i];
#pragma unroll
    for (int i = 0; i < S::SO; ++i) SO[i] = stab[S::SE + i];
    const TC* lam = stab + S::SE + S::SO;
    int64_t t = blockIdx.x;
    if (t >= ntiles) return;
    TileBuf<N, TC> buf;
    auto nvalid_of = [&](int64_t tt) {
        const int64_t g0 = tt * L::BPW;
        return static_cast<int>(G.nblocks - g0 < L::BPW ? G.nblocks - g0 : L::BPW);
    };
    tile_load<N>(buf, r, G, t * L::BPW, nvalid_of(t));
    for (; t < ntiles; t += gridDim.x) {
        const int64_t g0 = t * L::BPW;
        const int nvalid = nvalid_of(t);
        tile_to_lds<N>(buf, s0, nvalid);
        const int64_t tn = t + gridDim.x;
        if (tn < ntiles) tile_load<N>(buf, r, G, tn * L::BPW, nvalid_of(tn));
        const Pencil<N> pc(nvalid);
        TC sx = TC(1), sy = TC(1), sz = TC(1);
        if (pc.act) block_scales(G.h, g0 + pc.w, sx, sy, sz);
        const int so = (pc.w < L::BPW ? pc.w : 0) * L::size;
        TC* A0 = s0 + so;
        TC* A1 = s1 + so;
        const int pa = pc.pa, pb = pc.pb;
        __syncthreads();
        if (pc.act) {  // z forward: lane (i, j)
            TC xin[N], y[N];
#pragma unroll
            for (int k = 0; k < N; ++k) xin[k] = A0[L::at(pa, pb, k)];
            eo_fwd<N>(SE, SO, xin, y);
#pragma unroll
            for (int c = 0; c < N; ++c) A1[L::at(pa, pb, c)] = y[c];
        }
        __syncthreads();
        if (pc.act) {  // y forward: lane (i, c)
            TC xin[N], y[N];
#pragma unroll
            for (int j = 0; j < N; ++j) xin[j] = A1[L::at(pa, j, pb)];
            eo_fwd<N>(SE, SO, xin, y);
#pragma unroll
            for (int b = 0; b < N; ++b) A1[L::at(pa, b, pb)] = y[b];
        }
        __syncthreads();
        if (pc.act) {  // x forward, scale, x backward: lane (b, c)
            TC xin[N], y[N];
#pragma unroll
            for (int i = 0; i < N; ++i) xin[i] = A1[L::at(i, pa, pb)];
            eo_fwd<N>(SE, SO, xin, y);
            const TC mu_bc = lam[pa] * sy + lam[pb] * sz;
#pragma unroll
            for (int a = 0; a < N; ++a) y[a] *= recip(fma(lam[a], sx, mu_bc));
            eo_bwd<N>(SE, SO, y, xin);
#pragma unroll
            for (int i = 0; i < N; ++i) A1[L::at(i, pa, pb)] = xin[i];
        }
        __syncthreads();
        if (pc.act) {  // y backward: lane (i, c)
            TC y[N], xo[N];
#pragma unroll
            for (int b = 0; b < N; ++b) y[b] = A1[L::at(pa, b, pb)];
            eo_bwd<N>(SE, SO, y, xo);
#pragma unroll
            for (int j = 0; j < N; ++j) A1[L::at(pa, j, pb)] = xo[j];
        }
        __syncthreads();
        if (pc.act) {  // z backward: lane (i, j)
            TC y[N], xo[N];
#pragma unroll
            for (int c = 0; c < N; ++c) y[c] = A1[L::at(pa, pb, c)];
            eo_bwd<N>(SE, SO, y, xo);
#pragma unroll
            for (int k = 0; k < N; ++k) A0[L::at(pa, pb, k)] = xo[k];
        }
        __syncthreads();
        tile_store<N>(x, s0, G, g0, nvalid);
        __syncthreads();
    }
}

tp_status check(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, what);
    return TP_OK;
}

template <int N>
int64_t eo_tiles(const GroupInfo& g) {
    return (g.nblocks + Slab<N>::BPW - 1) / Slab<N>::BPW;
}

template <int N, typename TS, typename TC>
tp_status apply_eo_n(const Plan& plan, const GroupInfo& g, int op, const void* u, void* v, hipStream_t s) {
    const int64_t ntiles = eo_tiles<N>(g);
    const int64_t grid = std::min<int64_t>(ntiles, plan.wave_grid);
    const TC* tab = reinterpret_cast<const TC*>(eo_table(plan, N, op == TP_OP_CELL ? EO_APPLY_A : EO_APPLY_K,
                                                         sizeof(TC) == 8 ? 0 : 1));
    GArgs a{g.h, g.nblocks, g.offset, g.logB};
    hipLaunchKernelGGL((k_apply_eo<N, TS, TC>), dim3(static_cast<unsigned>(grid)), dim3(64), 0, s,
                       static_cast<const TS*>(u), static_cast<TS*>(v), a, tab, ntiles);
    return check("apply (even-odd) launch");
}

template <int N, typename TS, typename TC>
tp_status inverse_eo_n(const Plan& plan, const GroupInfo& g, const void* r, void* x, hipStream_t s) {
    const int64_t ntiles = eo_tiles<N>(g);
    const int64_t grid = std::min<int64_t>(ntiles, plan.wave_grid);
    const TC* tab = reinterpret_cast<const TC*>(eo_table(plan, N, EO_INV, sizeof(TC) == 8 ? 0 : 1));
    GArgs a{g.h, g.nblocks, g.offset, g.logB};
    hipLaunchKernelGGL((k_inverse_eo<N, TS, TC>), dim3(static_cast<unsigned>(grid)), dim3(64), 0, s,
                       static_cast<const TS*>(r), static_cast<TS*>(x), a, tab, ntiles);
    return check("apply_inverse (even-odd) launch");
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
