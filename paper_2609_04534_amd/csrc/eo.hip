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
#include <algorithm>
#include <climits>
#include <type_traits>

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

// ------------------------------------------------------------ pencil I/O
// Lane (w, i, j) of a tile owns the z-pencil (i, j, 0..n-1) of block w.  For
// the block-contiguous layout (B = 1) a pencil is n consecutive elements and
// is moved with 16-byte vector accesses when the address allows it.
template <int N, typename TS>
__device__ __forceinline__ const TS* pencil_ptr(const TS* base, const GArgs& G, int64_t g, int i, int j) {
    return base + G.offset + block_base(g, G.logB, N * N * N) + (static_cast<int64_t>((i * N + j) * N) << G.logB);
}

// 16 bytes of storage elements.
template <typename TS>
union Pack16 {
    static constexpr int n = 16 / static_cast<int>(sizeof(TS));
    uint4 u;
    TS s[16 / sizeof(TS)];
};

// With VP the caller guarantees B = 1 and 16-byte aligned pencils.
template <int N, bool VP, typename TS, typename TC>
__device__ __forceinline__ void pencil_load(TC (&x)[N], const TS* __restrict__ p, int logB) {
    constexpr int VEC = Pack16<TS>::n;
    if constexpr (VP && N % VEC == 0) {
        {
            const uint4* vp = reinterpret_cast<const uint4*>(p);
#pragma unroll
            for (int c = 0; c < N / VEC; ++c) {
                Pack16<TS> pk;
                pk.u = vp[c];
#pragma unroll
                for (int l = 0; l < VEC; ++l) x[c * VEC + l] = ldc<TC>(&pk.s[l]);
            }
            return;
        }
    }
#pragma unroll
    for (int k = 0; k < N; ++k) x[k] = ldc<TC>(p + (static_cast<int64_t>(k) << logB));
}

template <int N, bool VP, typename TS, typename TC>
__device__ __forceinline__ void pencil_store(TS* __restrict__ p, const TC (&x)[N], int logB) {
    constexpr int VEC = Pack16<TS>::n;
    if constexpr (VP && N % VEC == 0) {
        {
            uint4* vp = reinterpret_cast<uint4*>(p);
#pragma unroll
            for (int c = 0; c < N / VEC; ++c) {
                Pack16<TS> pk;
#pragma unroll
                for (int l = 0; l < VEC; ++l) stc(&pk.s[l], x[c * VEC + l]);
                vp[c] = pk.u;
            }
            return;
        }
    }
#pragma unroll
    for (int k = 0; k < N; ++k) stc(p + (static_cast<int64_t>(k) << logB), x[k]);
}

template <int N>
__device__ __forceinline__ int nvalid_of(const GArgs& G, int64_t t) {
    const int64_t g0 = t * Slab<N>::BPW;
    return static_cast<int>(G.nblocks - g0 < Slab<N>::BPW ? G.nblocks - g0 : Slab<N>::BPW);
}

// Loads the 1D factor table into registers.  FP64 tables go through LDS so
// that they land in VGPRs; FP32 tables are read with wave-uniform addresses
// and stay in scalar registers.
template <typename TC, int COUNT>
__device__ __forceinline__ void load_table(TC (&dst)[COUNT], const TC* __restrict__ tab, TC* stab) {
    if constexpr (sizeof(TC) == 8) {
        for (int e = threadIdx.x; e < COUNT; e += 64) stab[e] = tab[e];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < COUNT; ++i) dst[i] = stab[i];
    } else {
#pragma unroll
        for (int i = 0; i < COUNT; ++i) dst[i] = tab[i];
    }
}

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
    __shared__ TC stab[TAB];
    TC T[TAB];
    load_table<TC, TAB>(T, tab, stab);
    const TC* ME = T;
    const TC* MO = T + S::SE;
    const TC* PE = T + S::SE + S::SO;
    const TC* PO = T + 2 * S::SE + S::SO;
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
        const int pa = pc.pa, pb = pc.pb;
        if (pc.act) {  // z: lane (i, j); t = M x, w = P x
            TC e[HC], o[H], E[HC], O[H], y[N];
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
            TC et[HC], ot[H], ew[HC], ow[H], E[HC], O[H], E2[HC], O2[H], y[N];
#pragma unroll
            for (int j = 0; j < N; ++j) y[j] = A1[L::at(pa, j, pb)];
            eo_split<N>(y, et, ot);
#pragma unroll
            for (int j = 0; j < N; ++j) y[j] = A2[L::at(pa, j, pb)];
            eo_split<N>(y, ew, ow);
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
        if (pc.act) {  // x: lane (j, k); v = P a + M b, stored to global
            TC y[N], ea[HC], oa[H], eb[HC], ob[H], E[HC], O[H], E2[HC], O2[H];
#pragma unroll
            for (int i = 0; i < N; ++i) y[i] = A1[L::at(i, pa, pb)];
            eo_split<N>(y, ea, oa);
#pragma unroll
            for (int i = 0; i < N; ++i) y[i] = A2[L::at(i, pa, pb)];
            eo_split<N>(y, eb, ob);
            eo_mul<N>(PE, PO, ea, oa, E, O);
            eo_mul<N>(ME, MO, eb, ob, E2, O2);
#pragma unroll
            for (int i = 0; i < HC; ++i) E[i] += E2[i];
#pragma unroll
            for (int i = 0; i < H; ++i) O[i] += O2[i];
            eo_join<N>(E, O, y);
            TS* out = v + G.offset + block_base(g0 + pc.w, G.logB, L::N3);
#pragma unroll
            for (int i = 0; i < N; ++i) stc(out + (static_cast<int64_t>((i * N + pa) * N + pb) << G.logB), y[i]);
        }
        __syncthreads();
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
    __syncthreads();
    TC T[TABM];
    if constexpr (sizeof(TC) == 8) {
#pragma unroll
        for (int i = 0; i < TABM; ++i) T[i] = stab[i];
    } else {
#pragma unroll
        for (int i = 0; i < TABM; ++i) T[i] = tab[i];
    }
    const TC* SE = T;
    const TC* SO = T + S::SE;
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
        const int pa = pc.pa, pb = pc.pb;
        if (pc.act) {  // z forward: lane (i, j)
            TC y[N];
            eo_fwd<N>(SE, SO, xin, y);
#pragma unroll
            for (int c = 0; c < N; ++c) A1[L::at(pa, pb, c)] = y[c];
        }
        __syncthreads();
        if (pc.act) {  // y forward: lane (i, c)
            TC a[N], y[N];
#pragma unroll
            for (int j = 0; j < N; ++j) a[j] = A1[L::at(pa, j, pb)];
            eo_fwd<N>(SE, SO, a, y);
#pragma unroll
            for (int b = 0; b < N; ++b) A1[L::at(pa, b, pb)] = y[b];
        }
        __syncthreads();
        if (pc.act) {  // x forward, scale, x backward: lane (b, c)
            TC a[N], y[N];
#pragma unroll
            for (int i = 0; i < N; ++i) a[i] = A1[L::at(i, pa, pb)];
            eo_fwd<N>(SE, SO, a, y);
            const TC mu_bc = lam[pa] * sy + lam[pb] * sz;
#pragma unroll
            for (int c = 0; c < N; ++c) y[c] *= recip(fma(lam[c], sx, mu_bc));
            eo_bwd<N>(SE, SO, y, a);
#pragma unroll
            for (int i = 0; i < N; ++i) A1[L::at(i, pa, pb)] = a[i];
        }
        __syncthreads();
        if (pc.act) {  // y backward: lane (i, c)
            TC y[N], a[N];
#pragma unroll
            for (int b = 0; b < N; ++b) y[b] = A1[L::at(pa, b, pb)];
            eo_bwd<N>(SE, SO, y, a);
#pragma unroll
            for (int j = 0; j < N; ++j) A1[L::at(pa, j, pb)] = a[j];
        }
        __syncthreads();
        if (pc.act) {  // z backward: lane (i, j), pencil stored to global
            TC y[N], a[N];
#pragma unroll
            for (int c = 0; c < N; ++c) y[c] = A1[L::at(pa, pb, c)];
            eo_bwd<N>(SE, SO, y, a);
            pencil_store<N, VP>(const_cast<TS*>(pencil_ptr<N>(x, G, g0 + pc.w, pa, pb)), a, G.logB);
        }
        __syncthreads();
    }
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
    const int64_t grid = std::min(gc, ntiles);
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
    const int64_t grid = std::min(gc, ntiles);
    if (vp)
        hipLaunchKernelGGL((k_inverse_eo<N, TS, TC, true>), dim3(static_cast<unsigned>(grid)), dim3(64), 0, s,
                           static_cast<const TS*>(r), static_cast<TS*>(x), a, tab, ntiles);
    else
        hipLaunchKernelGGL((k_inverse_eo<N, TS, TC, false>), dim3(static_cast<unsigned>(grid)), dim3(64), 0, s,
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
